// Internal declarations of libefie (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/efie.h"

namespace efie {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
void clear_error();

struct Error {
    int code;
    std::string msg;
};

#define EFIE_HIP_CHECK(expr)                                                          \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess)                                                         \
            throw ::efie::Error{EFIE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

#define EFIE_REQUIRE(cond, code, msg)                                                 \
    do {                                                                              \
        if (!(cond)) throw ::efie::Error{(code), (msg)};                              \
    } while (0)

// Wrap an ABI body: converts Error / std::exception into status + message.
template <class F>
int guarded(F&& f) {
    try {
        clear_error();
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(std::string("internal: ") + e.what());
        return EFIE_ERR_ARG;
    }
}

constexpr int NQ = 7;   // points of the triangle rule

// --------------------------------------------------- device geometry tables
// Structure-of-arrays tables of one mesh, all device pointers into the caller's
// blob.  Index conventions: per-triangle arrays of length T; per (point, tri)
// arrays are [a * T + t]; per (local vertex i, tri) arrays are [i * T + t].
// Local edge i of a triangle is the edge opposite its local vertex i, so that
// vertex i is the free vertex of the RWG half-function carried by that edge.
struct DevMesh {
    int32_t T, N;               // triangles, RWGs
    int32_t n_near;             // ordered near pairs
    int32_t n_up;               // of them with q >= p
    double nf;                  // near factor: distance rule of near_by_distance
    double diam;                // bounding-box diagonal of the vertices (host use: FP32 phase range)
    // FP64.  Positions are stored relative to the triangle centroid (cx, cy, cz):
    // offsets are O(h), so products of offsets keep their relative precision.
    const double *cx, *cy, *cz;          // centroids [T]
    const double *qx, *qy, *qz, *qw;     // quadrature point offsets and weights*area [7][T]
    const double *vx, *vy, *vz;          // vertex offsets [3][T]
    const double *cf;                    // s l / (2A)            [3][T]
    const double *dv;                    // s l / A (divergence)  [3][T]
    const double *nx, *ny, *nz;          // unit normal [T]
    const double *hm;                    // longest edge [T]
    // FP32 copies for the complex64 far-pair kernel
    const float *qx32, *qy32, *qz32, *qw32, *vx32, *vy32, *vz32, *cf32, *dv32;
    // topology
    const int32_t* te;                   // RWG index of local edge i [3][T]
    const int32_t* tv;                   // vertex id of local vertex i [3][T]
    const int32_t *near_p, *near_q;      // ordered near pairs (incl. p == q)
    const int32_t *et;                   // RWG -> (T+, T-) [2][N]
    const int32_t *el;                   // RWG -> local edge index in T+ / T- [2][N]
    // distance-adaptive far rule: pairs with centroid distance D >= far3 * (larger
    // longest edge) take the 3x3 product of the interior 3-point rule (far3 = 0: off)
    const double *q3x, *q3y, *q3z, *q3w;       // its point offsets and weights*area [3][T]
    const float *q3x32, *q3y32, *q3z32, *q3w32;
    double far3;
    const int32_t* near_up;              // indices e of the ordered near pairs with q >= p, increasing
};

}  // namespace efie

struct efie_mesh_s {
    int64_t nv = 0, T = 0, N = 0;
    double near_factor = 2.0;
    double far3 = 0.0;                       // ratio of the distance-adaptive far rule (0: off)
    double diam = 0.0;                       // bounding-box diagonal of the vertices
    std::vector<double> xyz;                 // nv*3
    std::vector<int32_t> tri;                // T*3
    std::vector<int32_t> edge_v, edge_t, edge_l;  // N*2 each (edge_l: local index in T+/T-)
    std::vector<double> edge_len;            // N
    std::vector<int32_t> tri_edge, tri_sign; // T*3
    std::vector<double> area, normal, centroid, hmax;
    std::vector<int32_t> near_p, near_q;     // ordered near pairs, sorted by p then q
    std::vector<int32_t> near_up;            // indices of the pairs with q >= p
    // device tables (caller-owned blob)
    void* dev = nullptr;
    size_t dev_bytes = 0;
    efie::DevMesh dm{};
    std::vector<char> host_blob;             // packed image of the device tables
    std::vector<size_t> offs;                // byte offsets of each table in the blob
};

namespace efie {
// The distance part of the near-pair rule: |c_p - c_q|^2 < (nf max(h_p, h_q))^2,
// every operation rounded on its own (no fused multiply-add), in the order
// ((dx dx + dy dy) + dz dz), so that the host list and the device test decide
// every pair alike.  A pair is near if this holds or the triangles share a vertex.
__host__ __device__ inline bool near_by_distance(double cpx, double cpy, double cpz, double cqx, double cqy,
                                                 double cqz, double hp, double hq, double nf) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double dx = __dsub_rn(cpx, cqx), dy = __dsub_rn(cpy, cqy), dz = __dsub_rn(cpz, cqz);
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const double thr = __dmul_rn(nf, hp > hq ? hp : hq);
    return d2 < __dmul_rn(thr, thr);
#else
#pragma clang fp contract(off)
    const double dx = cpx - cqx, dy = cpy - cqy, dz = cpz - cqz;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double thr = nf * (hp > hq ? hp : hq);
    return d2 < thr * thr;
#endif
}

// The FP32 far-pair kernels take the phase Re(k) R in revolutions to the hardware
// sine and cosine, whose argument must stay below 256 revolutions in magnitude.
// Every distance between two points of a mesh is at most its bounding-box
// diagonal, so complex64 assembly is accepted for |Re k| < fp32_kmax(diam).
inline double fp32_kmax(double diam) { return 256.0 * 2.0 * 3.14159265358979323846 / diam; }
inline void require_fp32_phase(double diam, double kr, const char* who) {
    if (!(std::fabs(kr) < fp32_kmax(diam)))
        throw Error{EFIE_ERR_ARG, std::string(who) + ": |Re k| * (mesh diameter) / 2 pi reaches 256 revolutions, "
                                                     "beyond the FP32 phase range of complex64 assembly; use EFIE_C128"};
}

// mesh.cpp
void build_mesh(efie_mesh_s& m, const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                double near_factor);
void pack_tables(efie_mesh_s& m);            // fills host_blob, offs, returns size via host_blob.size()
void bind_tables(efie_mesh_s& m, void* dev); // sets m.dm pointers into dev
// the tables of pack_tables one by one (the batched assembly concatenates them)
int table_count();
size_t table_bytes_of(const efie_mesh_s& m, int t);             // bytes of table t of m
void bind_pointers(DevMesh& d, const void* base, const std::vector<size_t>& offs);  // table t at base + offs[t]
// Radon's 7-point degree-5 triangle rule: barycentric points and weights (sum 1),
// in the order the quadrature tables use.
void radon7(double bary[7][3], double w[7]);
}  // namespace efie

namespace efie {
// ------------------------------------------------------- launch timing
// Optional HIP-event timing of the library's main kernels, for measurement
// (enabled through efie_prof_enable).  Each begin/end pair brackets one launch
// on the launch stream.
enum ProfId { PROF_FAR = 0, PROF_NEAR = 1, PROF_MFMA = 2, PROF_GEMV = 3, PROF_ZGEMM = 4, PROF_KRYLOV = 5,
              PROF_EXCITE = 6, PROF_FARFIELD = 7, PROF_GRAD_FAR = 8, PROF_GRAD_NEAR = 9, PROF_GRAD_TRI = 10,
              PROF_ROWS_NEAR = 11, PROF_MFMA_SMALL = 12, PROF_COUNT = 13 };
void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s, double work = 0.0);   // work: algorithmic flops or bytes of the launch
}  // namespace efie

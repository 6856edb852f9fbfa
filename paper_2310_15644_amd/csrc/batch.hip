// Many uneven meshes at once: the tile assembly of every mesh and a grouped
// Krylov solve.
//
// Assembly.  Every mesh is assembled by the single-mesh tile kernels
// (tile_kernels.h: its near blocks, then its tiles of Z written once), the meshes
// in order of decreasing cost dealt round-robin to four streams of the device
// forked from and joined back into the caller's stream, so that the small meshes'
// launches run beside each other.  The kernels and their arguments are those of
// efie_assemble_ws, so every batched matrix is bit-identical to its single-mesh
// assembly; Z is written once and no atomics touch it.  (A persistent work-queue
// launch over all meshes' tiles reads each mesh's tables through pointers loaded
// from device memory, generic loads that cost the tile code a third of its
// occupancy; the kernel-argument launches keep the single-mesh code as it is.)
//
// Solve.  One right-hand side per mesh; Z of the meshes concatenated
// (Z_i at element offset sum_{j<i} N_j^2), vectors concatenated (offset
// sum_{j<i} N_j).  COCG per mesh with FP64 vectors; each iteration is one grouped
// GEMV launch over the rows of all still-active meshes (FP64 accumulation for both
// storage types) and one grouped step launch (one block per mesh).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "linalg.h"

namespace efie {

void assemble_tiles(const DevMesh& m, double kr, double ki, double eta, int dtype, void* Z, void* NB, size_t nb_bytes,
                    hipStream_t s);

struct BatchMeshDev {
    DevMesh m;
    int64_t zoff;     // element offset of this mesh's Z
    int64_t pad[3];
};

// the streams of the batched assembly: four per device, created on first use and
// kept until the process ends; host threads take turns
constexpr int BATCH_STREAMS = 4;
struct BatchStreams {
    hipStream_t s[BATCH_STREAMS] = {};
    hipEvent_t fork = nullptr, join[BATCH_STREAMS] = {};
    std::mutex mu;
};
static BatchStreams& batch_streams() {
    constexpr int MAXDEV = 64;
    static BatchStreams bs[MAXDEV];
    static std::mutex create_mu;
    int dev = 0;
    EFIE_HIP_CHECK(hipGetDevice(&dev));
    EFIE_REQUIRE(dev >= 0 && dev < MAXDEV, EFIE_ERR_STATE, "batch streams: device index out of range");
    BatchStreams& x = bs[dev];
    std::lock_guard<std::mutex> g(create_mu);
    if (!x.fork) {
        for (int i = 0; i < BATCH_STREAMS; ++i) {
            EFIE_HIP_CHECK(hipStreamCreateWithFlags(&x.s[i], hipStreamNonBlocking));
            EFIE_HIP_CHECK(hipEventCreateWithFlags(&x.join[i], hipEventDisableTiming));
        }
        EFIE_HIP_CHECK(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
    }
    return x;
}

// rows of all meshes: y[voff_s + i] = sum_k Z_s[i][k] x[voff_s + k] for active meshes
template <typename ZT>
__global__ __launch_bounds__(256) void grouped_gemv_kernel(const ZT* __restrict__ Zcat, const int64_t* __restrict__ zoff,
                                                           const int64_t* __restrict__ voff, int nmesh,
                                                           const int* __restrict__ active, const double2* __restrict__ x,
                                                           double2* __restrict__ y, int64_t rows) {
    const int64_t g = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= rows) return;
    int lo = 0, hi = nmesh;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (voff[mid] <= g) lo = mid;
        else hi = mid;
    }
    if (active && !active[lo]) return;
    const int n = int(voff[lo + 1] - voff[lo]);
    const int i = int(g - voff[lo]);
    const ZT* zr = Zcat + zoff[lo] + int64_t(i) * n;
    const double2* xs = x + voff[lo];
    double ar = 0, ai = 0;
    for (int k = lane; k < n; k += 64) {
        const ZT z = zr[k];
        const double2 v = xs[k];
        ar += double(z.x) * v.x - double(z.y) * v.y;
        ai += double(z.x) * v.y + double(z.y) * v.x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o, 64);
        ai += __shfl_xor(ai, o, 64);
    }
    if (lane == 0) y[g] = make_double2(ar, ai);
}

// ------------------------------------------------------------- grouped COCG
// One block per mesh; vectors of mesh s at [voff[s], voff[s+1]).  Same recurrences
// as the single-mesh COCG (CG with the unconjugated bilinear form).
constexpr int BKB = 256;

__device__ void bsum(double (&v)[4], double* sh) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) sh[4 * w + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double t = 0.0;
        for (int u = 0; u < BKB / 64; ++u) t += sh[4 * u + k];
        v[k] = t;
    }
}

__global__ __launch_bounds__(BKB) void bcocg_init(const double2* b, double2* x, double2* r, double2* p, BatchCol* cols,
                                                  int* active, const int64_t* voff, double tol) {
    __shared__ double sh[4 * BKB / 64];
    const int s = blockIdx.x;
    const int64_t o = voff[s];
    const int n = int(voff[s + 1] - o);
    double v[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += BKB) {
        const double2 e = b[o + k];
        x[o + k] = make_double2(0, 0);
        r[o + k] = e;
        p[o + k] = e;
        v[0] += e.x * e.x - e.y * e.y;
        v[1] += 2.0 * e.x * e.y;
        v[2] += e.x * e.x + e.y * e.y;
    }
    bsum(v, sh);
    if (threadIdx.x == 0) {
        BatchCol c{};
        c.rho_r = v[0];
        c.rho_i = v[1];
        c.bn2 = c.rn2 = v[2];
        c.tol2 = tol * tol * v[2];
        c.status = v[2] > 0.0 ? EFIE_NOT_CONVERGED : EFIE_OK;
        cols[s] = c;
        active[s] = v[2] > 0.0;
    }
}

__global__ __launch_bounds__(BKB) void bcocg_step(double2* x, double2* r, double2* p, const double2* q,
                                                  BatchCol* cols, int* active, const int64_t* voff, int* nact) {
    __shared__ double sh[4 * BKB / 64];
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int64_t o = voff[s];
    const int n = int(voff[s + 1] - o);
    const BatchCol c0 = cols[s];   // read before the barriers; thread 0 rewrites it after them
    double v[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += BKB) {
        const double2 pp = p[o + k], qq = q[o + k];
        v[0] += pp.x * qq.x - pp.y * qq.y;
        v[1] += pp.x * qq.y + pp.y * qq.x;
    }
    bsum(v, sh);
    const double d = v[0] * v[0] + v[1] * v[1];
    if (d == 0.0) {
        if (threadIdx.x == 0) {
            cols[s].status = EFIE_ERR_BREAKDOWN;
            active[s] = 0;
        }
        return;
    }
    const double ar = (c0.rho_r * v[0] + c0.rho_i * v[1]) / d, ai = (c0.rho_i * v[0] - c0.rho_r * v[1]) / d;
    double u[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += BKB) {
        const double2 pp = p[o + k], qq = q[o + k];
        double2 xx = x[o + k], rr = r[o + k];
        xx.x += ar * pp.x - ai * pp.y;
        xx.y += ar * pp.y + ai * pp.x;
        rr.x -= ar * qq.x - ai * qq.y;
        rr.y -= ar * qq.y + ai * qq.x;
        x[o + k] = xx;
        r[o + k] = rr;
        u[0] += rr.x * rr.x - rr.y * rr.y;
        u[1] += 2.0 * rr.x * rr.y;
        u[2] += rr.x * rr.x + rr.y * rr.y;
    }
    bsum(u, sh);
    const double dd = c0.rho_r * c0.rho_r + c0.rho_i * c0.rho_i;
    const double br = (u[0] * c0.rho_r + u[1] * c0.rho_i) / dd, bi = (u[1] * c0.rho_r - u[0] * c0.rho_i) / dd;
    for (int k = threadIdx.x; k < n; k += BKB) {
        const double2 rr = r[o + k];
        double2 pp = p[o + k];
        const double px = rr.x + br * pp.x - bi * pp.y, py = rr.y + br * pp.y + bi * pp.x;
        p[o + k] = make_double2(px, py);
    }
    if (threadIdx.x == 0) {
        BatchCol c = c0;
        c.rho_r = u[0];
        c.rho_i = u[1];
        c.rn2 = u[2];
        c.iters += 1;
        int still = 1;
        if (!(u[2] == u[2])) {
            c.status = EFIE_ERR_NAN;
            still = 0;
        } else if (u[2] <= c.tol2) {
            c.status = EFIE_OK;
            still = 0;
        }
        cols[s] = c;
        active[s] = still;
        if (still) atomicAdd(nact, 1);
    }
}

// out[2s] = ||b_s - y_s||^2, out[2s+1] = ||b_s||^2 (doubles)
__global__ __launch_bounds__(BKB) void bresidual(const double2* b, const double2* y, const int64_t* voff, double* out) {
    __shared__ double sh[4 * BKB / 64];
    const int s = blockIdx.x;
    const int64_t o = voff[s];
    const int n = int(voff[s + 1] - o);
    double v[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += BKB) {
        const double2 bb = b[o + k], yy = y[o + k];
        const double dx = bb.x - yy.x, dy = bb.y - yy.y;
        v[0] += dx * dx + dy * dy;
        v[1] += bb.x * bb.x + bb.y * bb.y;
    }
    bsum(v, sh);
    if (threadIdx.x == 0) {
        out[2 * s] = v[0];
        out[2 * s + 1] = v[1];
    }
}

void batch_cocg_init(const double2* b, double2* x, double2* r, double2* p, BatchCol* cols, int* active,
                     const int64_t* voff, int nm, double tol, hipStream_t s) {
    hipLaunchKernelGGL(bcocg_init, dim3(nm), dim3(BKB), 0, s, b, x, r, p, cols, active, voff, tol);
}
void batch_cocg_step(double2* x, double2* r, double2* p, const double2* q, BatchCol* cols, int* active,
                     const int64_t* voff, int nm, int* nact, hipStream_t s) {
    hipLaunchKernelGGL(bcocg_step, dim3(nm), dim3(BKB), 0, s, x, r, p, q, cols, active, voff, nact);
}
void batch_residual_norms(const double2* b, const double2* y, const int64_t* voff, int nm, double2* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(bresidual, dim3(nm), dim3(BKB), 0, s, b, y, voff, reinterpret_cast<double*>(out));
}

namespace {
size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

struct BatchWs {
    char* NB;                      // near blocks of every mesh
    double2 *r, *p, *q, *y;
    BatchCol* cols;
    int* active;
    int* nact;
};

// byte offsets of every mesh's near blocks (complex128 size, 256-aligned), caller
// order; total in [nm]
std::vector<size_t> batch_nb_offsets(const efie_batch_s& B) {
    const size_t nm = B.meshes.size();
    std::vector<size_t> off(nm + 1, 0);
    for (size_t i = 0; i < nm; ++i)
        off[i + 1] = off[i] + a256(std::max<size_t>(256, B.meshes[i]->near_p.size() * 9 * 16));
    return off;
}

size_t batch_ws_layout(const efie_batch_s& B, BatchWs* w, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += a256(bytes);
        return p;
    };
    BatchWs x{};
    const size_t nm = B.meshes.size();
    const size_t vec = size_t(B.v_total) * 16;
    x.NB = take(batch_nb_offsets(B)[nm]);
    x.r = (double2*)take(vec);
    x.p = (double2*)take(vec);
    x.q = (double2*)take(vec);
    x.y = (double2*)take(vec);
    x.cols = (BatchCol*)take(sizeof(BatchCol) * nm);
    x.active = (int*)take(sizeof(int) * nm);
    x.nact = (int*)take(64);
    if (w) *w = x;
    return off;
}
}  // namespace

void batch_prepare(efie_batch_s& B) {
    const int nm = int(B.meshes.size());
    B.zoff.assign(size_t(nm), 0);
    B.voff.assign(size_t(nm) + 1, 0);
    int64_t z = 0;
    for (int i = 0; i < nm; ++i) {
        B.zoff[size_t(i)] = z;
        z += B.meshes[size_t(i)]->N * B.meshes[size_t(i)]->N;
        B.voff[size_t(i) + 1] = B.voff[size_t(i)] + B.meshes[size_t(i)]->N;
    }
    B.z_total = z;
    B.v_total = B.voff[size_t(nm)];
    // processing order: decreasing cost (pass-1 blocks and near pairs)
    std::vector<int64_t> items(static_cast<size_t>(nm));
    for (int i = 0; i < nm; ++i) {
        const efie_mesh_s& m = *B.meshes[size_t(i)];
        const int64_t nq = (m.T + 255) / 256;
        items[size_t(i)] = m.T * nq + (int64_t(m.near_p.size()) + 255) / 256;
    }
    B.order.resize(size_t(nm));
    std::iota(B.order.begin(), B.order.end(), 0);
    std::stable_sort(B.order.begin(), B.order.end(), [&](int a, int b) { return items[size_t(a)] > items[size_t(b)]; });
}

}  // namespace efie

using namespace efie;

extern "C" int efie_batch_create(const efie_mesh* meshes, int32_t nmesh, efie_batch* out) {
    return guarded([&]() {
        EFIE_REQUIRE(meshes && out && nmesh >= 1, EFIE_ERR_ARG, "batch_create: bad argument");
        auto* B = new efie_batch_s();
        for (int i = 0; i < nmesh; ++i) {
            if (!meshes[i] || !meshes[i]->dev) {
                delete B;
                throw Error{EFIE_ERR_STATE, "batch_create: every mesh must exist and be uploaded"};
            }
            B->meshes.push_back(meshes[i]);
        }
        batch_prepare(*B);
        *out = B;
        return int(EFIE_OK);
    });
}

extern "C" void efie_batch_destroy(efie_batch b) { delete b; }

extern "C" int efie_batch_sizes(efie_batch b, size_t* table_bytes, size_t* ws_bytes, int64_t* z_elems,
                                int64_t* v_elems, int64_t* items) {
    return guarded([&]() {
        EFIE_REQUIRE(b != nullptr, EFIE_ERR_ARG, "batch_sizes: null");
        const size_t nm = b->meshes.size();
        if (table_bytes) *table_bytes = a256(sizeof(BatchMeshDev) * nm) + a256(8 * nm) + a256(8 * (nm + 1));
        if (ws_bytes) *ws_bytes = batch_ws_layout(*b, nullptr, nullptr);
        if (z_elems) *z_elems = b->z_total;
        if (v_elems) *v_elems = b->v_total;
        if (items) {   // launches of the assembly: near blocks and tiles per mesh
            *items = int64_t(2 * nm);
        }
        return int(EFIE_OK);
    });
}

extern "C" int efie_batch_upload(efie_batch b, void* dev, size_t bytes, hipStream_t stream) {
    return guarded([&]() {
        EFIE_REQUIRE(b && dev, EFIE_ERR_ARG, "batch_upload: null argument");
        const size_t nm = b->meshes.size();
        const size_t need = a256(sizeof(BatchMeshDev) * nm) + a256(8 * nm) + a256(8 * (nm + 1));
        EFIE_REQUIRE(bytes >= need, EFIE_ERR_ARG, "batch_upload: buffer too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(dev) & 255) == 0, EFIE_ERR_ARG, "batch_upload: not 256-aligned");
        std::vector<char> blob(need, 0);
        auto* bmd = reinterpret_cast<BatchMeshDev*>(blob.data());
        for (size_t r = 0; r < nm; ++r) {
            const int i = b->order[r];
            const efie_mesh_s& m = *b->meshes[size_t(i)];
            EFIE_REQUIRE(m.dev != nullptr, EFIE_ERR_STATE, "batch_upload: a mesh is not uploaded");
            BatchMeshDev d{};
            d.m = m.dm;
            d.zoff = b->zoff[size_t(i)];
            bmd[r] = d;
        }
        size_t off = a256(sizeof(BatchMeshDev) * nm);
        std::memcpy(blob.data() + off, b->zoff.data(), 8 * nm);
        b->off_zoff = off;
        off += a256(8 * nm);
        std::memcpy(blob.data() + off, b->voff.data(), 8 * (nm + 1));
        b->off_voff = off;
        EFIE_HIP_CHECK(hipMemcpyAsync(dev, blob.data(), need, hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        b->dev = dev;
        return int(EFIE_OK);
    });
}

extern "C" int efie_batch_assemble(efie_batch b, const double* k, double eta, int dtype, void* Zcat, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
    return guarded([&]() {
        EFIE_REQUIRE(b && k && Zcat && ws, EFIE_ERR_ARG, "batch_assemble: null argument");
        EFIE_REQUIRE(b->dev != nullptr, EFIE_ERR_STATE, "batch_assemble: batch tables not uploaded");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "batch_assemble: bad dtype");
        EFIE_REQUIRE(ws_bytes >= batch_ws_layout(*b, nullptr, nullptr), EFIE_ERR_ARG, "batch_assemble: ws too small");
        BatchWs w;
        batch_ws_layout(*b, &w, static_cast<char*>(ws));
        const size_t nm = b->meshes.size();
        for (size_t i = 0; i < nm; ++i)
            EFIE_REQUIRE(b->meshes[i]->dev != nullptr, EFIE_ERR_STATE, "batch_assemble: a mesh is not uploaded");
        for (size_t r = 0; r < nm; ++r) {
            const double kr = k[b->order[r]];
            EFIE_REQUIRE(std::isfinite(kr) && kr > 0.0, EFIE_ERR_ARG, "batch_assemble: k must be real and > 0");
            if (dtype == EFIE_C64) require_fp32_phase(b->meshes[size_t(b->order[r])]->diam, kr, "batch_assemble");
        }
        const std::vector<size_t> nbo = batch_nb_offsets(*b);
        const size_t esz = dtype == EFIE_C128 ? 16 : 8;
        BatchStreams& bs = batch_streams();
        std::lock_guard<std::mutex> g(bs.mu);
        prof_begin(PROF_FAR, stream);
        EFIE_HIP_CHECK(hipEventRecord(bs.fork, stream));
        for (int i = 0; i < BATCH_STREAMS; ++i) EFIE_HIP_CHECK(hipStreamWaitEvent(bs.s[i], bs.fork, 0));
        for (size_t r = 0; r < nm; ++r) {
            const int i = b->order[r];
            const efie_mesh_s& m = *b->meshes[size_t(i)];
            char* z = static_cast<char*>(Zcat) + size_t(b->zoff[size_t(i)]) * esz;
            assemble_tiles(m.dm, k[i], 0.0, eta, dtype, z, w.NB + nbo[size_t(i)], nbo[size_t(i) + 1] - nbo[size_t(i)],
                           bs.s[r % BATCH_STREAMS]);
        }
        for (int i = 0; i < BATCH_STREAMS; ++i) {
            EFIE_HIP_CHECK(hipEventRecord(bs.join[i], bs.s[i]));
            EFIE_HIP_CHECK(hipStreamWaitEvent(stream, bs.join[i], 0));
        }
        prof_end(PROF_FAR, stream);
        EFIE_HIP_CHECK(hipGetLastError());
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        return int(EFIE_OK);
    });
}

extern "C" int efie_batch_solve(efie_batch b, const void* Zcat, int dtype, const void* Vcat, void* Jcat,
                                const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
    return guarded([&]() {
        EFIE_REQUIRE(b && Zcat && Vcat && Jcat && opts && ws, EFIE_ERR_ARG, "batch_solve: null argument");
        EFIE_REQUIRE(b->dev != nullptr, EFIE_ERR_STATE, "batch_solve: batch tables not uploaded");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "batch_solve: bad dtype");
        EFIE_REQUIRE(opts->solver == EFIE_COCG, EFIE_ERR_ARG, "batch_solve: COCG only");
        EFIE_REQUIRE(opts->maxit >= 1 && opts->tol > 0.0, EFIE_ERR_ARG, "batch_solve: bad maxit/tol");
        EFIE_REQUIRE(ws_bytes >= batch_ws_layout(*b, nullptr, nullptr), EFIE_ERR_ARG, "batch_solve: ws too small");
        BatchWs w;
        batch_ws_layout(*b, &w, static_cast<char*>(ws));
        const int nm = int(b->meshes.size());
        const char* base = static_cast<const char*>(b->dev);
        const auto* zoff = reinterpret_cast<const int64_t*>(base + b->off_zoff);
        const auto* voff = reinterpret_cast<const int64_t*>(base + b->off_voff);
        const double2* V = static_cast<const double2*>(Vcat);
        double2* J = static_cast<double2*>(Jcat);
        const int64_t rows = b->v_total;
        const unsigned gblocks = unsigned((rows + 3) / 4);
        auto gemv = [&](const double2* x, double2* y, const int* act) {
            prof_begin(PROF_GEMV, stream);
            if (dtype == EFIE_C64)
                hipLaunchKernelGGL(grouped_gemv_kernel<float2>, dim3(gblocks), dim3(256), 0, stream,
                                   static_cast<const float2*>(Zcat), zoff, voff, nm, act, x, y, rows);
            else
                hipLaunchKernelGGL(grouped_gemv_kernel<double2>, dim3(gblocks), dim3(256), 0, stream,
                                   static_cast<const double2*>(Zcat), zoff, voff, nm, act, x, y, rows);
            prof_end(PROF_GEMV, stream);
        };
        batch_cocg_init(V, J, w.r, w.p, w.cols, w.active, voff, nm, opts->tol, stream);
        int h = nm;
        int it = 0;
        for (; it < opts->maxit && h > 0; ++it) {
            gemv(w.p, w.q, w.active);
            fill_zero_bytes(w.nact, 64, stream);
            batch_cocg_step(J, w.r, w.p, w.q, w.cols, w.active, voff, nm, w.nact, stream);
            EFIE_HIP_CHECK(hipMemcpyAsync(&h, w.nact, sizeof(int), hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        }
        // true residuals
        gemv(J, w.y, nullptr);
        batch_residual_norms(V, w.y, voff, nm, w.r, stream);   // w.r reused: [2 * nm] doubles
        std::vector<BatchCol> cols(static_cast<size_t>(nm));
        std::vector<double> norms(2 * size_t(nm));
        EFIE_HIP_CHECK(hipMemcpyAsync(norms.data(), w.r, sizeof(double) * 2 * nm, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(cols.data(), w.cols, sizeof(BatchCol) * nm, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        int ret = EFIE_OK;
        for (int s = 0; s < nm; ++s) {
            const double rel = norms[2 * s + 1] > 0 ? std::sqrt(norms[2 * s] / norms[2 * s + 1]) : 0.0;
            int st = cols[size_t(s)].status;
            if (!(rel == rel)) st = EFIE_ERR_NAN;
            if (stats) {
                stats[s].iters = cols[size_t(s)].iters;
                stats[s].status = st;
                stats[s].relres_recur = cols[size_t(s)].bn2 > 0 ? std::sqrt(cols[size_t(s)].rn2 / cols[size_t(s)].bn2) : 0;
                stats[s].relres_true = rel;
            }
            if (st != EFIE_OK) ret = EFIE_NOT_CONVERGED;
        }
        EFIE_HIP_CHECK(hipGetLastError());
        return ret;
    });
}

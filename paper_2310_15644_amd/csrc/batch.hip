// Many uneven meshes at once: the tile assembly of every mesh in one persistent
// launch, and a grouped Krylov solve.
//
// Assembly.  At upload the meshes' tables are concatenated table by table into the
// batch's device blob (the meshes in order of decreasing cost).  One launch
// computes the near-pair blocks of every mesh (a block of 256 ordered near pairs
// belongs to one mesh), then one persistent launch (as many blocks as fit on the
// device at once) walks the tiles of all meshes' matrices: tile t goes to block
// t mod grid, which finds its mesh by binary search over the tile offsets and runs
// the single-mesh tile code (tile_kernels.h) on a view of that mesh's tables.  The
// view's pointers are the kernel argument's concatenated bases plus the mesh's
// element offsets, so the tables are read with global (not generic) loads, as in
// the single-mesh kernel.  Every batched matrix is bit-identical to its single-mesh
// assembly; Z is written once and no atomics touch it.
//
// Solve.  One right-hand side per mesh; Z of the meshes concatenated
// (Z_i at element offset sum_{j<i} N_j^2), vectors concatenated (offset
// sum_{j<i} N_j).  COCG per mesh with FP64 vectors; each iteration is one grouped
// GEMV launch over the rows of all still-active meshes (FP64 accumulation for both
// storage types) and one grouped step launch (one block per mesh).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "linalg.h"
#include "tile_kernels.h"

namespace efie {

// one mesh of one batched assembly: where its tables, near blocks, Z and tiles
// start (processing order)
struct BatchItem {
    int32_t T, N, n_near, pad;
    int64_t toff, noff, eoff;   // triangles, RWGs and ordered near pairs of the meshes before it
    int64_t uoff;               // their near pairs with q >= p
    int32_t n_up, pad2;
    int64_t zoff, nboff;        // elements of Z and of the near blocks before it (in the precision of Z)
    int64_t tile0, nblk0;       // its first tile and its first block of the near-block launch
    double kr, nf, far3;
    Scale sc;
};

// the mesh of item `it` as the single-mesh code sees it: the concatenated tables
// offset to its first element
__device__ __forceinline__ DevMesh mesh_view(const DevMesh& c, const BatchItem& it) {
    DevMesh v = c;
    const int64_t t = it.toff, n = it.noff, e = it.eoff;
    v.T = it.T;
    v.N = it.N;
    v.n_near = it.n_near;
    v.nf = it.nf;
    v.far3 = it.far3;
    v.cx = c.cx + t; v.cy = c.cy + t; v.cz = c.cz + t;
    v.qx = c.qx + 7 * t; v.qy = c.qy + 7 * t; v.qz = c.qz + 7 * t; v.qw = c.qw + 7 * t;
    v.vx = c.vx + 3 * t; v.vy = c.vy + 3 * t; v.vz = c.vz + 3 * t; v.cf = c.cf + 3 * t; v.dv = c.dv + 3 * t;
    v.nx = c.nx + t; v.ny = c.ny + t; v.nz = c.nz + t; v.hm = c.hm + t;
    v.qx32 = c.qx32 + 7 * t; v.qy32 = c.qy32 + 7 * t; v.qz32 = c.qz32 + 7 * t; v.qw32 = c.qw32 + 7 * t;
    v.vx32 = c.vx32 + 3 * t; v.vy32 = c.vy32 + 3 * t; v.vz32 = c.vz32 + 3 * t;
    v.cf32 = c.cf32 + 3 * t; v.dv32 = c.dv32 + 3 * t;
    v.te = c.te + 3 * t; v.tv = c.tv + 3 * t;
    v.near_p = c.near_p + e; v.near_q = c.near_q + e;
    v.n_up = it.n_up;
    v.near_up = c.near_up + it.uoff;
    v.et = c.et + 2 * n; v.el = c.el + 2 * n;
    v.q3x = c.q3x + 3 * t; v.q3y = c.q3y + 3 * t; v.q3z = c.q3z + 3 * t; v.q3w = c.q3w + 3 * t;
    v.q3x32 = c.q3x32 + 3 * t; v.q3y32 = c.q3y32 + 3 * t; v.q3z32 = c.q3z32 + 3 * t; v.q3w32 = c.q3w32 + 3 * t;
    return v;
}

// the last item whose 64-bit field f is <= x (the items in increasing f)
template <int64_t BatchItem::*F>
__device__ __forceinline__ int item_of(const BatchItem* __restrict__ items, int nm, int64_t x) {
    int lo = 0, hi = nm;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid].*F <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// the near-pair blocks of every mesh, a group of NEAR_G lanes per pair: block b
// (NEAR_PER_BLOCK pairs) belongs to one mesh (each mesh's pairs padded to whole
// blocks)
constexpr int NEAR_PER_BLOCK = 256 / NEAR_G;
template <typename R>
__global__ __launch_bounds__(256) void batch_near_kernel(DevMesh cat, const BatchItem* __restrict__ items, int nm,
                                                         typename Cplx<R>::T* __restrict__ NB) {
    const int r = item_of<&BatchItem::nblk0>(items, nm, int64_t(blockIdx.x));
    const BatchItem& it = items[r];
    const int u = int(int64_t(blockIdx.x) - it.nblk0) * NEAR_PER_BLOCK + int(threadIdx.x) / NEAR_G;
    if (u >= it.n_up) return;   // the pairs with q >= p only
    const DevMesh v = mesh_view(cat, it);
    near_block_one<R>(v, it.kr, 0.0, it.sc, NB + it.nboff, v.near_up[u], int(threadIdx.x) % NEAR_G);
}

// the tiles of every mesh's Z: persistent, tile t by block t mod gridDim.x
template <typename R>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 3 : 1) void batch_tiles_kernel(
    DevMesh cat, const BatchItem* __restrict__ items, int nm, int64_t ntiles,
    const typename Cplx<R>::T* __restrict__ NB, typename Cplx<R>::T* __restrict__ Z) {
    __shared__ TileLds<R> L;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int r = item_of<&BatchItem::tile0>(items, nm, t);
        const BatchItem& it = items[r];
        const DevMesh v = mesh_view(cat, it);
        const R kphase = std::is_same<R, float>::value ? R(it.kr / (2.0 * PI)) : R(it.kr);
        tile_block<R, false>(v, tables_of<R>(v), kphase, R(0), it.sc, NB + it.nboff, Z + it.zoff, t - it.tile0, L);
    }
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
    BatchItem* items;              // the assembly's per-mesh items (processing order)
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

// the batch's device tables: Z and vector offsets, then each mesh table
// concatenated over the meshes (256-aligned per table)
size_t batch_table_bytes(const efie_batch_s& B) {
    const size_t nm = B.meshes.size();
    size_t off = a256(8 * nm) + a256(8 * (nm + 1));
    for (int t = 0; t < table_count(); ++t) {
        for (size_t i = 0; i < nm; ++i) off += table_bytes_of(*B.meshes[i], t);
        off = a256(off);
    }
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
    x.items = (BatchItem*)take(sizeof(BatchItem) * nm);
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
    // the concatenated tables follow the processing order
    B.toff.assign(size_t(nm), 0);
    B.noff.assign(size_t(nm), 0);
    B.eoff.assign(size_t(nm), 0);
    B.uoff.assign(size_t(nm), 0);
    int64_t t = 0, n = 0, e = 0, u = 0;
    for (int r = 0; r < nm; ++r) {
        const int i = B.order[size_t(r)];
        const efie_mesh_s& m = *B.meshes[size_t(i)];
        B.toff[size_t(i)] = t;
        B.noff[size_t(i)] = n;
        B.eoff[size_t(i)] = e;
        B.uoff[size_t(i)] = u;
        u += int64_t(m.near_up.size());
        t += m.T;
        n += m.N;
        e += int64_t(m.near_p.size());
    }
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
        if (table_bytes) *table_bytes = batch_table_bytes(*b);
        if (ws_bytes) *ws_bytes = batch_ws_layout(*b, nullptr, nullptr);
        if (z_elems) *z_elems = b->z_total;
        if (v_elems) *v_elems = b->v_total;
        if (items) {   // work items of the persistent assembly launch: complex64 tiles of all meshes
            int64_t t = 0;
            for (size_t i = 0; i < nm; ++i) t += tile_count<float>(int(b->meshes[i]->N));
            *items = t;
        }
        return int(EFIE_OK);
    });
}

extern "C" int efie_batch_upload(efie_batch b, void* dev, size_t bytes, hipStream_t stream) {
    return guarded([&]() {
        EFIE_REQUIRE(b && dev, EFIE_ERR_ARG, "batch_upload: null argument");
        const size_t nm = b->meshes.size();
        const size_t need = batch_table_bytes(*b);
        EFIE_REQUIRE(bytes >= need, EFIE_ERR_ARG, "batch_upload: buffer too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(dev) & 255) == 0, EFIE_ERR_ARG, "batch_upload: not 256-aligned");
        // per mesh (caller order) the offsets of its Z and of its vectors, read by
        // the grouped solve; then every table of the meshes concatenated (processing
        // order), read by the assembly
        std::vector<char> blob(need, 0);
        size_t off = 0;
        std::memcpy(blob.data() + off, b->zoff.data(), 8 * nm);
        b->off_zoff = off;
        off += a256(8 * nm);
        std::memcpy(blob.data() + off, b->voff.data(), 8 * (nm + 1));
        b->off_voff = off;
        off += a256(8 * (nm + 1));
        const int nt = table_count();
        std::vector<size_t> toffs(size_t(nt), 0);
        for (int t = 0; t < nt; ++t) {
            toffs[size_t(t)] = off;
            for (size_t r = 0; r < nm; ++r) {
                const efie_mesh_s& m = *b->meshes[size_t(b->order[r])];
                const size_t nb = table_bytes_of(m, t);
                EFIE_REQUIRE(m.offs.size() == size_t(nt) && m.offs[size_t(t)] + nb <= m.host_blob.size(),
                             EFIE_ERR_STATE, "batch_upload: mesh tables inconsistent");
                if (nb) std::memcpy(blob.data() + off, m.host_blob.data() + m.offs[size_t(t)], nb);
                off += nb;
            }
            off = a256(off);
        }
        EFIE_REQUIRE(off == need, EFIE_ERR_STATE, "batch_upload: table size mismatch");
        b->cat = DevMesh{};
        bind_pointers(b->cat, dev, toffs);
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
        std::vector<BatchItem> items(nm);
        int64_t tile = 0, nblk = 0;
        for (size_t r = 0; r < nm; ++r) {
            const int i = b->order[r];
            const efie_mesh_s& m = *b->meshes[size_t(i)];
            BatchItem& it = items[r];
            it.T = int32_t(m.T);
            it.N = int32_t(m.N);
            it.n_near = int32_t(m.near_p.size());
            it.toff = b->toff[size_t(i)];
            it.noff = b->noff[size_t(i)];
            it.eoff = b->eoff[size_t(i)];
            it.uoff = b->uoff[size_t(i)];
            it.n_up = int32_t(m.near_up.size());
            it.zoff = b->zoff[size_t(i)];
            it.nboff = int64_t(nbo[size_t(i)] / esz);
            it.tile0 = tile;
            it.nblk0 = nblk;
            it.kr = k[i];
            it.nf = m.near_factor;
            it.far3 = m.far3;
            it.sc = operator_scale(k[i], 0.0, eta);
            tile += dtype == EFIE_C64 ? tile_count<float>(int(m.N)) : tile_count<double>(int(m.N));
            nblk += (int64_t(m.near_up.size()) + NEAR_PER_BLOCK - 1) / NEAR_PER_BLOCK;
        }
        EFIE_REQUIRE(nblk < (int64_t(1) << 31), EFIE_ERR_ARG, "batch_assemble: too many near pairs");
        EFIE_HIP_CHECK(hipMemcpyAsync(w.items, items.data(), sizeof(BatchItem) * nm, hipMemcpyHostToDevice, stream));
        int dev = 0, ncu = 0, per_cu = 0;
        EFIE_HIP_CHECK(hipGetDevice(&dev));
        EFIE_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        auto run = [&](auto tag) {
            using R = decltype(tag);
            using C2 = typename Cplx<R>::T;
            C2* NB = reinterpret_cast<C2*>(w.NB);
            if (nblk > 0) {
                prof_begin(PROF_NEAR, stream);
                hipLaunchKernelGGL(batch_near_kernel<R>, dim3(unsigned(nblk)), dim3(256), 0, stream, b->cat, w.items,
                                   int(nm), NB);
                prof_end(PROF_NEAR, stream);
            }
            EFIE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_tiles_kernel<R>, 256, 0));
            const int64_t grid = std::min<int64_t>(tile, int64_t(std::max(1, per_cu)) * std::max(1, ncu));
            prof_begin(PROF_FAR, stream);
            hipLaunchKernelGGL(batch_tiles_kernel<R>, dim3(unsigned(grid)), dim3(256), 0, stream, b->cat, w.items,
                               int(nm), tile, NB, static_cast<C2*>(Zcat));
            prof_end(PROF_FAR, stream);
        };
        if (dtype == EFIE_C64) run(float{});
        else run(double{});
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

// Many uneven meshes at once: persistent work-queue assembly and a grouped
// Krylov solve.
//
// Assembly.  The atomic-free two-pass scheme of the single-mesh assembly
// (assemble.hip), run as work items of persistent launches: the meshes, ordered
// by decreasing cost, are cut into segments (chunks of test triangles) whose rows
// W[p][i][n][side] fit one workspace; per group of segments four launches take
// items from their own atomic counter until all are done (every block leaves when
// the counter passes the total):
//   A  rows: a far item is one block of the single-mesh pass-1 kernel (FAR_PB test
//      triangles against 256 source triangles); a near item 256 ordered near pairs
//      (their own launch, whose FP64 code would otherwise take the far items'
//      registers);
//   B  gather: a block per (test triangle, local edge) row of a segment;
//   C  mirror: the mirror tile pairs of every mesh whose last segment is in the group.
// Each item runs the same device code as the single-mesh kernels (rows_kernels.h),
// with the same scale factors, so every batched matrix is bit-identical to its
// single-mesh assembly; no atomics touch Z.
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
#include "rows_kernels.h"

namespace efie {

struct BatchMeshDev {
    DevMesh m;
    int64_t zoff;     // element offset of this mesh's Z
    int64_t pad[2];
};

struct BatchParam {
    Scale sc;         // operator_scale(k, 0, eta), as the single-mesh assembly
    double kr;
    float kphase32;   // k / 2 pi in FP32 (the complex64 pass 1)
    float pad;
};

// a chunk [c0, c0 + np) of the test triangles of mesh r (processing order)
struct BatchSeg {
    int r, c0, np, nqblk;
    int e0, e1;       // its ordered near pairs
    int64_t woff;     // element offset of its rows in the workspace
    int64_t nfar;     // pass-1 far items: ceil(np / FAR_PB) nqblk
};

// the item of a block: one shared load, uniform over the block
__device__ inline long long next_item(unsigned long long* counter) {
    __shared__ long long item_s;
    if (threadIdx.x == 0) item_s = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long item = item_s;
    __syncthreads();
    return item;
}

// pref[lo] <= item < pref[lo + 1]
__device__ inline int find_seg(const int64_t* __restrict__ pref, int n, long long item) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// phase A: pass-1 far blocks (NEAR false) or the near pairs, 256 per item (NEAR
// true), of every segment of the group (two launches: the FP64 near-pair code
// would take the far blocks' registers)
template <typename ZT, bool NEAR>
__global__ __launch_bounds__(256) void batch_rows_kernel(const BatchMeshDev* __restrict__ bm,
                                                         const BatchParam* __restrict__ prm,
                                                         const BatchSeg* __restrict__ seg,
                                                         const int64_t* __restrict__ pref, int nseg, int64_t total,
                                                         unsigned long long* counter, ZT* __restrict__ W) {
    using R = typename std::conditional<sizeof(ZT) == 8, float, double>::type;
    for (;;) {
        const long long item = next_item(counter);
        if (item >= total) return;
        const int s = find_seg(pref, nseg, item);
        const BatchSeg& g = seg[s];
        const DevMesh& m = bm[g.r].m;
        const BatchParam& pm = prm[g.r];
        const long long li = item - pref[s];
        ZT* w = W + g.woff;
        if (!NEAR) {
            const R kphase = sizeof(ZT) == 8 ? R(pm.kphase32) : R(pm.kr);
            far_rows_block<R, false, true>(m, tables_of<R>(m), kphase, R(0), pm.sc, w, g.c0, g.np, g.nqblk, int(li));
        } else {
            const long long e = g.e0 + li * 256 + threadIdx.x;
            if (e < g.e1) near_rows_one<R>(m, pm.kr, 0.0, pm.sc, w, g.c0, g.c0 + g.np, int(e), 1);
        }
    }
}

// phase B: the gather blocks of every segment (3 np per segment)
template <typename ZT>
__global__ __launch_bounds__(256) void batch_gather_kernel(const BatchMeshDev* __restrict__ bm,
                                                           const BatchSeg* __restrict__ seg,
                                                           const int64_t* __restrict__ pref, int nseg, int64_t total,
                                                           unsigned long long* counter, const ZT* __restrict__ W,
                                                           ZT* __restrict__ Zcat) {
    using R = typename std::conditional<sizeof(ZT) == 8, float, double>::type;
    for (;;) {
        const long long item = next_item(counter);
        if (item >= total) return;
        const int s = find_seg(pref, nseg, item);
        const BatchSeg& g = seg[s];
        const BatchMeshDev& b = bm[g.r];
        gather_rows_block<R, true>(b.m, W + g.woff, g.c0, g.c0 + g.np, Zcat + b.zoff, int(item - pref[s]));
    }
}

// phase C: the mirror tile pairs of the meshes completed by the group (mesh ranks mr[])
template <typename ZT>
__global__ __launch_bounds__(256) void batch_mirror_kernel(const BatchMeshDev* __restrict__ bm,
                                                           const int* __restrict__ mr,
                                                           const int64_t* __restrict__ pref, int nmr, int64_t total,
                                                           unsigned long long* counter, ZT* __restrict__ Zcat) {
    for (;;) {
        const long long item = next_item(counter);
        if (item >= total) return;
        const int s = find_seg(pref, nmr, item);
        const BatchMeshDev& b = bm[mr[s]];
        const int N = b.m.N;
        mirror_add_block<ZT>(Zcat + b.zoff, N, (N + 31) / 32, item - pref[s]);
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

// rows of one group of segments: at most this many bytes (a chunk of one test
// triangle is the minimum)
constexpr size_t BATCH_W_BUDGET = size_t(2) << 30;

// The assembly plan for one storage type: segments in processing order, cut into
// groups whose rows fit BATCH_W_BUDGET; per group the item prefixes of the three
// phases (concatenated, nseg + 1 / nmr + 1 entries per group).
struct BatchPlan {
    struct Group {
        int s0, ns, m0, nmr;         // its segments and mirror meshes
        size_t a0, c0;               // first entry of its prefixes in apref / bpref, cpref
        int64_t atot, ntot, btot, ctot;   // item totals: far rows, near rows, gather, mirror
    };
    std::vector<BatchSeg> segs;
    std::vector<int64_t> apref, npref, bpref, cpref;
    std::vector<int> mr;
    std::vector<Group> groups;
    size_t w_bytes = 0;
    int64_t pass1_items = 0;
};

BatchPlan batch_plan(const efie_batch_s& B, size_t esz) {
    BatchPlan P;
    const int nm = int(B.meshes.size());
    std::vector<BatchSeg> cur;
    std::vector<int> cur_mr;
    size_t gbytes = 0;
    auto close = [&]() {
        if (cur.empty() && cur_mr.empty()) return;
        BatchPlan::Group g{};
        g.s0 = int(P.segs.size());
        g.ns = int(cur.size());
        g.m0 = int(P.mr.size());
        g.nmr = int(cur_mr.size());
        g.a0 = P.apref.size();
        g.c0 = P.cpref.size();
        int64_t a = 0, nn = 0, b = 0, c = 0;
        for (const BatchSeg& x : cur) {
            P.apref.push_back(a);
            P.npref.push_back(nn);
            P.bpref.push_back(b);
            a += x.nfar;
            nn += (x.e1 - x.e0 + 255) / 256;
            b += 3 * int64_t(x.np);
            P.segs.push_back(x);
        }
        P.apref.push_back(a);
        P.npref.push_back(nn);
        P.bpref.push_back(b);
        for (int r : cur_mr) {
            P.cpref.push_back(c);
            const int64_t nt = (B.meshes[size_t(B.order[size_t(r)])]->N + 31) / 32;
            c += nt * (nt + 1) / 2;
            P.mr.push_back(r);
        }
        P.cpref.push_back(c);
        g.atot = a;
        g.ntot = nn;
        g.btot = b;
        g.ctot = c;
        P.pass1_items += a + nn;
        P.groups.push_back(g);
        P.w_bytes = std::max(P.w_bytes, gbytes);
        cur.clear();
        cur_mr.clear();
        gbytes = 0;
    };
    for (int r = 0; r < nm; ++r) {
        const efie_mesh_s& m = *B.meshes[size_t(B.order[size_t(r)])];
        const size_t per_tri = size_t(6) * size_t(m.N) * esz;
        EFIE_REQUIRE(per_tri <= BATCH_W_BUDGET, EFIE_ERR_ARG, "batch: a mesh too large for the row workspace");
        const int T = int(m.T);
        const int chunk = int(std::max<size_t>(1, std::min<size_t>(size_t(T), BATCH_W_BUDGET / per_tri)));
        const int nqblk = (T + FAR_BLOCK - 1) / FAR_BLOCK;
        for (int c0 = 0; c0 < T; c0 += chunk) {
            const int np = std::min(chunk, T - c0);
            const size_t bytes = a256(size_t(np) * per_tri);
            if (!cur.empty() && gbytes + bytes > BATCH_W_BUDGET) close();
            BatchSeg x{};
            x.r = r;
            x.c0 = c0;
            x.np = np;
            x.nqblk = nqblk;
            x.e0 = int(std::lower_bound(m.near_p.begin(), m.near_p.end(), c0) - m.near_p.begin());
            x.e1 = int(std::lower_bound(m.near_p.begin(), m.near_p.end(), c0 + np) - m.near_p.begin());
            x.woff = int64_t(gbytes / esz);
            x.nfar = int64_t((np + FAR_PB - 1) / FAR_PB) * nqblk;
            cur.push_back(x);
            gbytes += bytes;
        }
        cur_mr.push_back(r);   // the mesh's last segment is in the current group
    }
    close();
    return P;
}

struct BatchWs {
    BatchParam* prm;
    unsigned long long* counter;   // [0] far rows, [1] near rows, [2] gather, [3] mirror
    BatchSeg* segs;
    int64_t *apref, *npref, *bpref, *cpref;
    int* mr;
    void* W;
    double2 *r, *p, *q, *y;
    BatchCol* cols;
    int* active;
    int* nact;
};

// sizes of the plan arrays and rows: the larger of the two storage types
struct BatchPlanMax {
    size_t nseg = 0, npref = 0, ncpref = 0, nmr = 0, w_bytes = 0;
};
BatchPlanMax batch_plan_max(const efie_batch_s& B) {
    BatchPlanMax x;
    for (size_t esz : {size_t(8), size_t(16)}) {
        const BatchPlan P = batch_plan(B, esz);
        x.nseg = std::max(x.nseg, P.segs.size());
        x.npref = std::max(x.npref, P.apref.size());
        x.ncpref = std::max(x.ncpref, P.cpref.size());
        x.nmr = std::max(x.nmr, P.mr.size());
        x.w_bytes = std::max(x.w_bytes, P.w_bytes);
    }
    return x;
}

size_t batch_ws_layout(const efie_batch_s& B, BatchWs* w, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += a256(bytes);
        return p;
    };
    const BatchPlanMax pm = batch_plan_max(B);
    BatchWs x{};
    const size_t nm = B.meshes.size();
    const size_t vec = size_t(B.v_total) * 16;
    x.prm = (BatchParam*)take(sizeof(BatchParam) * nm);
    x.counter = (unsigned long long*)take(64);
    x.segs = (BatchSeg*)take(sizeof(BatchSeg) * pm.nseg);
    x.apref = (int64_t*)take(8 * pm.npref);
    x.npref = (int64_t*)take(8 * pm.npref);
    x.bpref = (int64_t*)take(8 * pm.npref);
    x.cpref = (int64_t*)take(8 * pm.ncpref);
    x.mr = (int*)take(4 * pm.nmr);
    x.W = take(pm.w_bytes);
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
            if (meshes[i]->far3 != 0.0) {
                delete B;
                throw Error{EFIE_ERR_ARG, "batch_create: the batch takes the 7x7 rule only (a mesh has the far rule on)"};
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
        if (items) *items = batch_plan(*b, 8).pass1_items;
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
        b->mesh_dev.assign(nm, nullptr);
        for (size_t r = 0; r < nm; ++r) {
            const int i = b->order[r];
            const efie_mesh_s& m = *b->meshes[size_t(i)];
            EFIE_REQUIRE(m.dev != nullptr, EFIE_ERR_STATE, "batch_upload: a mesh is not uploaded");
            EFIE_REQUIRE(m.far3 == 0.0, EFIE_ERR_ARG, "batch_upload: the batch takes the 7x7 rule only (a mesh has "
                                                      "the far rule on)");
            BatchMeshDev d{};
            d.m = m.dm;
            d.zoff = b->zoff[size_t(i)];
            bmd[r] = d;
            b->mesh_dev[size_t(i)] = m.dev;
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
        for (size_t i = 0; i < nm; ++i) {
            const efie_mesh_s& m = *b->meshes[i];
            EFIE_REQUIRE(m.far3 == 0.0, EFIE_ERR_ARG, "batch_assemble: the batch takes the 7x7 rule only (a mesh "
                                                      "has the far rule on)");
            EFIE_REQUIRE(m.dev != nullptr && m.dev == b->mesh_dev[i], EFIE_ERR_STATE,
                         "batch_assemble: a mesh was uploaded again after the batch; upload the batch again");
        }
        std::vector<BatchParam> prm(nm);
        for (size_t r = 0; r < nm; ++r) {
            const double kr = k[b->order[r]];
            EFIE_REQUIRE(std::isfinite(kr) && kr > 0.0, EFIE_ERR_ARG, "batch_assemble: k must be real and > 0");
            if (dtype == EFIE_C64) require_fp32_phase(b->meshes[size_t(b->order[r])]->diam, kr, "batch_assemble");
            BatchParam p{};
            p.sc = operator_scale(kr, 0.0, eta);   // the single-mesh assembly's factors, bit for bit
            p.kr = kr;
            p.kphase32 = float(kr / (2.0 * PI));
            prm[r] = p;
        }
        const size_t esz = dtype == EFIE_C128 ? 16 : 8;
        const BatchPlan plan = batch_plan(*b, esz);
        EFIE_HIP_CHECK(hipMemcpyAsync(w.prm, prm.data(), sizeof(BatchParam) * nm, hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.segs, plan.segs.data(), sizeof(BatchSeg) * plan.segs.size(),
                                      hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.apref, plan.apref.data(), 8 * plan.apref.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.npref, plan.npref.data(), 8 * plan.npref.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.bpref, plan.bpref.data(), 8 * plan.bpref.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.cpref, plan.cpref.data(), 8 * plan.cpref.size(), hipMemcpyHostToDevice, stream));
        if (!plan.mr.empty())
            EFIE_HIP_CHECK(hipMemcpyAsync(w.mr, plan.mr.data(), 4 * plan.mr.size(), hipMemcpyHostToDevice, stream));
        int dev_id = 0, ncu = 0;
        EFIE_HIP_CHECK(hipGetDevice(&dev_id));
        EFIE_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev_id));
        const auto* bmd = static_cast<const BatchMeshDev*>(b->dev);
        auto grid_of = [&](const void* fn) {   // persistent grid: every CU full
            int per_cu = 0;
            EFIE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
            return dim3(unsigned(std::max(1, ncu * std::max(1, per_cu))));
        };
        auto run = [&](auto tag) {
            using ZT = decltype(tag);
            ZT* W = static_cast<ZT*>(w.W);
            ZT* Z = static_cast<ZT*>(Zcat);
            const dim3 ga = grid_of(reinterpret_cast<const void*>(batch_rows_kernel<ZT, false>));
            const dim3 gn = grid_of(reinterpret_cast<const void*>(batch_rows_kernel<ZT, true>));
            const dim3 gb = grid_of(reinterpret_cast<const void*>(batch_gather_kernel<ZT>));
            const dim3 gc = grid_of(reinterpret_cast<const void*>(batch_mirror_kernel<ZT>));
            for (const BatchPlan::Group& g : plan.groups) {
                fill_zero_bytes(w.counter, 64, stream);
                if (g.atot > 0)
                    hipLaunchKernelGGL((batch_rows_kernel<ZT, false>), ga, dim3(256), 0, stream, bmd, w.prm,
                                       w.segs + g.s0, w.apref + g.a0, g.ns, g.atot, w.counter, W);
                if (g.ntot > 0)
                    hipLaunchKernelGGL((batch_rows_kernel<ZT, true>), gn, dim3(256), 0, stream, bmd, w.prm,
                                       w.segs + g.s0, w.npref + g.a0, g.ns, g.ntot, w.counter + 1, W);
                if (g.btot > 0)
                    hipLaunchKernelGGL(batch_gather_kernel<ZT>, gb, dim3(256), 0, stream, bmd, w.segs + g.s0,
                                       w.bpref + g.a0, g.ns, g.btot, w.counter + 2, W, Z);
                if (g.ctot > 0)
                    hipLaunchKernelGGL(batch_mirror_kernel<ZT>, gc, dim3(256), 0, stream, bmd, w.mr + g.m0,
                                       w.cpref + g.c0, g.nmr, g.ctot, w.counter + 3, Z);
            }
        };
        prof_begin(PROF_FAR, stream);
        if (dtype == EFIE_C64) run(float2{});
        else run(double2{});
        prof_end(PROF_FAR, stream);
        EFIE_HIP_CHECK(hipGetLastError());
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));   // the host staging lives on this stack frame
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

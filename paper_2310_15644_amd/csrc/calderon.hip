// Device side of the Calderon preconditioner (structure of the paper's Sec. III,
// eq. 16: second operator at k~, times a Gram inverse, times the first operator).
//
//   T_BC = R^T T_bary(k~) R   without forming T_bary (N_b x N_b, 543 GB in complex128
//       for the level-5 sphere): per chunk of barycentric test triangles p,
//         W[p][i][f][side]       every pair value (the pair rows of rows_kernels.h,
//                                complex k~),
//         Yw[(p,i)][n] = sum_f (W[p][i][f][0] + W[p][i][f][1]) R[f][n]
//                                (R by BC function n, CSC: a gather along the row),
//         T_BC[m][:] += sum R[e(p,i)][m] Yw[(p,i)][:]
//                                (one block per BC row m touched by the chunk, from
//                                host-built lists; no atomics);
//   P = T_BC G_mix^{-1}       row s of P solves G_mix^T p_s = row s of T_BC = column s
//       (T_BC is symmetric), by BiCGStab for a batch of columns at once in column
//       layout X[j][s], so that every sparse product reads rows of the batch
//       coalesced; the solution block is then transposed into P.
// The preconditioned operator P Z is applied as two dense products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "calderon.h"
#include "linalg.h"
#include "mfie_pair.h"

namespace efie {

void pair_rows_chunk(const DevMesh& m, double kr, double ki, double eta, int dtype, void* W, int c0, int c1,
                     const std::vector<int32_t>& near_p, const std::vector<int32_t>& near_up, bool upper,
                     hipStream_t s);
bool verbose();
double now_s();

struct DevCald {
    int N, Nb;
    const int32_t *r_ptr, *r_idx;   // CSC of R by BC function
    const double* r_val;
    const int32_t *g_ptr, *g_idx, *gt_ptr, *gt_idx;   // G and G^T, rows stored in n_order order
    const double *g_val, *gt_val;
    const int32_t* n_order;         // primal RWGs in a spatially coherent order
    const int32_t* run_t0;          // runs of BC functions: first position in n_order
    const int32_t *u_ptr, *u_idx;   // per run: its distinct barycentric RWGs
    const int32_t* r_loc;           // per entry of R's CSC: local position in its run's list
};

// Yw[row][n] = sum_k (W[row][f][0] + W[row][f][1]) r_val[k], f = r_idx[k], k over
// column n of R (row = 3 (p - c0) + i; W rows hold 2 N_b elements, the two sides
// of an RWG adjacent).  A block takes one run of BC functions (blockIdx.y: the
// positions run_t0[b] .. run_t0[b+1] of n_order, spatially coherent) and RRL
// rows; it gathers once per row the distinct barycentric RWGs the run reads
// (u_idx, sorted, so that runs of neighbouring indices coalesce), sums the two
// sides of each into LDS, and then every thread contracts the column of R of one
// BC function from LDS through the local positions r_loc.  The row groups of a
// run are neighbouring blocks, so that the run's list and columns of R stay in L2
// while its rows stream past.  L2 fetches about 1.7 times the bytes of W written
// (lines shared by neighbouring runs, lists that overlap), instead of once per BC
// function that uses an entry.
// two sides of barycentric RWG f in row wr, summed, each only where its flag is
// set (a select, so that unwritten entries never enter; complex64: one 16-byte load)
// (lanes with neither side wanted issue no load)
__device__ inline float2 bc_pair_sum(const float2* wr, int f, bool s0, bool s1) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (s0 || s1) v = *reinterpret_cast<const float4*>(wr + 2 * size_t(f));
    return make_float2((s0 ? v.x : 0.f) + (s1 ? v.z : 0.f), (s0 ? v.y : 0.f) + (s1 ? v.w : 0.f));
}
__device__ inline double2 bc_pair_sum(const double2* wr, int f, bool s0, bool s1) {
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (s0) a = wr[2 * size_t(f)];
    if (s1) b = wr[2 * size_t(f) + 1];
    return make_double2((s0 ? a.x : 0.0) + (s1 ? b.x : 0.0), (s0 ? a.y : 0.0) + (s1 ? b.y : 0.0));
}

constexpr int BC_NQ = BC_UMAX / 256;   // list entries per thread
constexpr int BC_KG = 8;               // column entries per group
// The rows hold the pairs with source triangle q >= p only (p the row's test
// triangle c0 + row / 3): side s of RWG f (triangle et[s Nb + f]) is read only
// where that triangle is not below p.
template <typename C2, int RRL>
__global__ __launch_bounds__(256) void bc_src_kernel(DevCald c, const C2* __restrict__ W, double2* __restrict__ Yw,
                                                     int nrows, const int32_t* __restrict__ et, int c0) {
    static_assert(BC_UMAX % 256 == 0, "list bound must be a multiple of the block");
    // the RRL rows of one list entry adjacent, so that a thread reads them with a
    // few wide LDS loads (random entries meet bank conflicts once per load, not once
    // per row)
    __shared__ C2 lw[BC_UMAX][RRL];
    const int b = blockIdx.y;
    const int r0 = blockIdx.x * RRL;
    const int u0 = c.u_ptr[b], nu = c.u_ptr[b + 1] - u0;   // 1 <= nu <= BC_UMAX by construction
    // the run's list, once for all rows; entries past the end repeat the last one
    // (loaded, not stored), so every load below is in bounds and unconditional
    int fl[BC_NQ], tp[BC_NQ], tm[BC_NQ];
#pragma unroll
    for (int q = 0; q < BC_NQ; ++q) fl[q] = c.u_idx[u0 + min(int(threadIdx.x) + 256 * q, nu - 1)];
#pragma unroll
    for (int q = 0; q < BC_NQ; ++q) {
        tp[q] = et[fl[q]];
        tm[q] = et[size_t(c.Nb) + fl[q]];
    }
    // rows past the end read a valid row (result dropped); the loads of row u + 1
    // are in flight while row u is written to LDS
    auto wrow = [&](int u) { return W + size_t(min(r0 + u, nrows - 1)) * 2 * size_t(c.Nb); };
    auto ptri = [&](int u) { return c0 + min(r0 + u, nrows - 1) / 3; };
    C2 x[BC_NQ], y[BC_NQ];
    {
        const int p = ptri(0);
#pragma unroll
        for (int q = 0; q < BC_NQ; ++q) x[q] = bc_pair_sum(wrow(0), fl[q], tp[q] >= p, tm[q] >= p);
    }
#pragma unroll
    for (int u = 0; u < RRL; ++u) {
        if (u + 1 < RRL) {
            const int p = ptri(u + 1);
#pragma unroll
            for (int q = 0; q < BC_NQ; ++q) y[q] = bc_pair_sum(wrow(u + 1), fl[q], tp[q] >= p, tm[q] >= p);
        }
#pragma unroll
        for (int q = 0; q < BC_NQ; ++q)
            if (int(threadIdx.x) + 256 * q < nu) lw[threadIdx.x + 256 * q][u] = x[q];
#pragma unroll
        for (int q = 0; q < BC_NQ; ++q) x[q] = y[q];
    }
    __syncthreads();
    const int t = c.run_t0[b] + int(threadIdx.x);
    if (t >= c.run_t0[b + 1]) return;
    const int n = c.n_order[t];
    double ar[RRL], ai[RRL];
#pragma unroll
    for (int u = 0; u < RRL; ++u) ar[u] = ai[u] = 0.0;
    // the column in groups: all index and coefficient loads of a group first
    for (int kb = c.r_ptr[n], ke = c.r_ptr[n + 1]; kb < ke; kb += BC_KG) {
        int l[BC_KG];
        double v[BC_KG];
#pragma unroll
        for (int q = 0; q < BC_KG; ++q) {
            const int k = min(kb + q, ke - 1);
            l[q] = c.r_loc[k];
            v[q] = kb + q < ke ? c.r_val[k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < BC_KG; ++q) {
            const C2* e = lw[l[q]];
#pragma unroll
            for (int u = 0; u < RRL; ++u) {
                const C2 xx = e[u];
                ar[u] += v[q] * double(xx.x);
                ai[u] += v[q] * double(xx.y);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RRL; ++u)
        if (r0 + u < nrows) Yw[size_t(r0 + u) * c.N + n] = make_double2(ar[u], ai[u]);
}
// rows per block x list bound: 10 x 1024 complex64 (80 KB of LDS) lets two blocks
// share a CU, one computing while the other loads, and still amortizes the run's
// list and index loads over 10 rows (level 5, source-side contraction per P
// build: 429 ms with 8 x 2304 and one block per CU; 387 / 392 / 406 / 455 / 470 ms
// with 10 x 1024, 8 x 768, 12 x 768, 6 x 1024, 16 x 512)
constexpr int BC_RRL32 = 10, BC_RRL64 = 4;

// Tbc[m][n] += sum_k coef[k] Yw[rows[k]][n] over the list of BC row m = ml[blockIdx.y]
__global__ __launch_bounds__(256) void bc_test_kernel(const int32_t* __restrict__ ml, const int32_t* __restrict__ mptr,
                                                      const int32_t* __restrict__ rows,
                                                      const double* __restrict__ coef,
                                                      const double2* __restrict__ Yw, double2* __restrict__ Tbc,
                                                      int N) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int mi = blockIdx.y;
    if (n >= N) return;
    const size_t o = size_t(ml[mi]) * N + n;
    double2 acc = Tbc[o];
    for (int k = mptr[mi]; k < mptr[mi + 1]; ++k) {
        const double2 y = Yw[size_t(rows[k]) * N + n];
        acc.x += coef[k] * y.x;
        acc.y += coef[k] * y.y;
    }
    Tbc[o] = acc;
}

// T <- T + T^T in place (N x N complex128): one block per pair of mirror 32 x 32
// tiles (bi <= bj), both read into LDS before either is written
__global__ __launch_bounds__(256) void sym_add_kernel(double2* __restrict__ T, int N, int nt) {
    __shared__ double2 a[32][33], b[32][33];
    // blockIdx.x -> (bi, bj), bi <= bj, row by row of the upper triangle of tiles
    int k = int(blockIdx.x), bi = 0;
    while (k >= nt - bi) {
        k -= nt - bi;
        ++bi;
    }
    const int bj = bi + k;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
        if (i < N && j < N) a[r][tx] = T[size_t(i) * N + j];
        if (i2 < N && j2 < N) b[r][tx] = T[size_t(i2) * N + j2];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        if (i < N && j < N) {   // (i, j) += (j, i): element (r, tx) of a plus element (tx, r) of b
            const double2 u = a[r][tx], v = b[tx][r];
            T[size_t(i) * N + j] = make_double2(u.x + v.x, u.y + v.y);
        }
        if (bi != bj) {
            const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
            if (i2 < N && j2 < N) {
                const double2 u = b[r][tx], v = a[tx][r];
                T[size_t(i2) * N + j2] = make_double2(u.x + v.x, u.y + v.y);
            }
        }
    }
}

// ------------------------------------------- BiCGStab on column tiles
// The Gram systems (G_mix^T y = b for P, G_mix y = b for Q) are solved column by
// column with BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13(2) 1992):
// two sparse products per step and no transpose.  On these well-conditioned
// systems it reaches 1e-3 in three steps where CG on the normal equations takes
// about ten (two products each).
// The vectors are stored as V (double2, or float2 when the requested tolerance
// is loose: GRAM_C64_TOL); every sum, norm and update is evaluated in FP64.
// A batch of S columns is split into tiles of CG_W = 64 columns, each tile stored
// row by row: element (j, s) sits at ((s / CG_W) N + j) CG_W + s % CG_W, so a
// wave reads a row of a tile as 512 contiguous bytes (complex64).  A block takes
// CG_R consecutive rows of one tile (a slice), a wave every fourth of them.  The
// padding columns of the last tile stay zero.
constexpr double GRAM_C64_TOL = 1e-4;
constexpr int CG_W = 64;   // columns per tile: one per lane
constexpr int CG_R = 64;   // rows per block
__device__ inline double2 ld2(const double2& v) { return v; }
__device__ inline double2 ld2(const float2& v) { return make_double2(double(v.x), double(v.y)); }
template <typename V>
__device__ inline V st2(double x, double y);
template <>
__device__ inline double2 st2<double2>(double x, double y) { return make_double2(x, y); }
template <>
__device__ inline float2 st2<float2>(double x, double y) { return make_float2(float(x), float(y)); }

inline int cg_pad(int S) { return (S + CG_W - 1) / CG_W * CG_W; }
__host__ __device__ inline int cg_slices(int N) { return (N + CG_R - 1) / CG_R; }
// blocks of a batch of S columns: every slice of every tile, the tile count
// rounded up to a multiple of 8
inline unsigned cg_blocks(int S, int N) { return unsigned((cg_pad(S) / CG_W + 7) / 8 * 8) * unsigned(cg_slices(N)); }

// Block b runs on XCD b % 8 (round-robin dispatch).  That XCD's blocks, in
// dispatch order, take tile b % 8, then tile b % 8 + 8, ..., every slice of one
// tile before the next: the rows a sparse product gathers then come from the
// XCD's own tile, and its L2 is not shared among all the columns.
struct CgBlock {
    int tile, c, wv, s, j0, j1, slice;
};
__device__ inline CgBlock cg_block(int N) {
    const int ns = (N + CG_R - 1) / CG_R;
    const int b = blockIdx.x, idx = b >> 3;
    CgBlock k;
    k.tile = (b & 7) + 8 * (idx / ns);
    k.slice = idx % ns;
    k.c = int(threadIdx.x) & 63;
    k.wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    k.s = k.tile * CG_W + k.c;
    k.j0 = k.slice * CG_R + k.wv;   // the wave's rows: j0, j0 + 4, ... < j1
    k.j1 = min(N, (k.slice + 1) * CG_R);
    return k;
}
__device__ inline size_t cg_at(int tile, int j, int c, int N) { return (size_t(tile) * N + j) * CG_W + c; }

// part[slice][s] = the block's sum over its waves of sq (a column's squared norm
// over the slice), for s < S
__device__ inline void cg_part(double sq, const CgBlock& k, int S, double* part) {
    __shared__ double sh[4][CG_W];
    sh[k.wv][k.c] = sq;
    __syncthreads();
    if (k.wv == 0 && k.s < S) part[size_t(k.slice) * S + k.s] = sh[0][k.c] + sh[1][k.c] + sh[2][k.c] + sh[3][k.c];
}

// ar + j ai += sum of val[e] Xt[idx[e] CG_W] over e = kb .. min(kb + G, ke) - 1
// (indices past ke repeat the last entry with weight 0)
template <int G, typename V>
__device__ inline void csp_group(const int32_t* __restrict__ idx, const double* __restrict__ val,
                                 const V* __restrict__ Xt, int kb, int ke, double& ar, double& ai) {
    int ix[G];
    double vv[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int e = min(kb + q, ke - 1);
        ix[q] = idx[e];
        vv[q] = kb + q < ke ? val[e] : 0.0;
    }
    double2 x[G];
#pragma unroll
    for (int q = 0; q < G; ++q) x[q] = ld2(Xt[size_t(ix[q]) * CG_W]);
#pragma unroll
    for (int q = 0; q < G; ++q) {
        ar += vv[q] * x[q].x;
        ai += vv[q] * x[q].y;
    }
}

// Out[j] = sum_q val[q] X[idx[q]] for the rows of a real CSR matrix A stored in
// the spatially coherent order (stored row t is row j = order[t]), over the stored
// rows of the block's slice, for the columns of the block's tile; and the slice
// sums of three column reductions over those rows: part[0] and part[1] the real
// and imaginary parts of sum_j conj(Y[j]) Out[j], part[2] sum_j |Out[j]|^2
// (part[v] = part + v ns S)
template <typename V>
__global__ __launch_bounds__(256) void cspmm_dot_kernel(const int32_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ idx,
                                                        const double* __restrict__ val, const V* __restrict__ X,
                                                        V* __restrict__ Out, int S, const int32_t* __restrict__ order,
                                                        int N, const V* __restrict__ Y, double* __restrict__ part) {
    const CgBlock k = cg_block(N);
    if (k.tile * CG_W >= S) return;
    const V* Xt = X + cg_at(k.tile, 0, k.c, N);
    double dr = 0.0, di = 0.0, sq = 0.0;
    for (int t = k.j0; t < k.j1; t += 4) {
        double ar = 0, ai = 0;
        int kb = ptr[t];
        const int ke = ptr[t + 1];
        for (; kb + 8 <= ke; kb += 8) csp_group<8>(idx, val, Xt, kb, ke, ar, ai);
        for (; kb < ke; kb += 4) csp_group<4>(idx, val, Xt, kb, ke, ar, ai);
        const V o = st2<V>(ar, ai);
        const size_t e = cg_at(k.tile, order[t], k.c, N);
        Out[e] = o;
        const double2 od = ld2(o), yv = ld2(Y[e]);
        dr += yv.x * od.x + yv.y * od.y;
        di += yv.x * od.y - yv.y * od.x;
        sq += od.x * od.x + od.y * od.y;
    }
    const size_t ps = size_t(cg_slices(N)) * S;
    cg_part(dr, k, S, part);
    __syncthreads();
    cg_part(di, k, S, part + ps);
    __syncthreads();
    cg_part(sq, k, S, part + 2 * ps);
}

// out[y S + s] = sum over the ns slices of part[(y ns + slice) S + s] for the
// reductions y = blockIdx.y; block = 16 columns x 16 slice stripes, grid
// (ceil(S / 16), reductions)
__global__ __launch_bounds__(256) void colsq_final_kernel(const double* __restrict__ part, int S, int ns,
                                                          double* __restrict__ out) {
    __shared__ double sh[16][17];
    part += size_t(blockIdx.y) * size_t(ns) * S;
    out += size_t(blockIdx.y) * S;
    const int c = threadIdx.x & 15, st = threadIdx.x >> 4;
    const int s = blockIdx.x * 16 + c;
    double a = 0.0;
    if (s < S)
        for (int js = st; js < ns; js += 16) a += part[size_t(js) * S + s];
    sh[st][c] = a;
    __syncthreads();
    if (st == 0 && s < S) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += sh[q][c];
        out[s] = t;
    }
}

// per column: rho = <r^, r>, alpha, omega, beta of the current step (complex),
// ||b||^2, ||r||^2, the target tol^2 ||b||^2
struct BicgCol {
    double rho_r, rho_i, al_r, al_i, om_r, om_i, be_r, be_i;
    double bn2, rn2, tol2;
    int active, iters;
};

// x = 0, r = r^ = p = b (b[j][s] with leading dimension ldb; zero in the padding
// columns); part = slice sums of |r|^2
template <typename V>
__global__ __launch_bounds__(256) void bicg_init_kernel(const double2* __restrict__ b, int ldb, V* __restrict__ x,
                                                        V* __restrict__ r, V* __restrict__ rh, V* __restrict__ p,
                                                        int N, int S, double* __restrict__ part) {
    const CgBlock k = cg_block(N);
    if (k.tile * CG_W >= S) return;
    double sq = 0.0;
    for (int j = k.j0; j < k.j1; j += 4) {
        const double2 v = k.s < S ? b[size_t(j) * ldb + k.s] : make_double2(0.0, 0.0);
        const size_t e = cg_at(k.tile, j, k.c, N);
        x[e] = st2<V>(0.0, 0.0);
        const V rv = st2<V>(v.x, v.y);
        r[e] = rv;
        rh[e] = rv;
        p[e] = rv;
        const double2 rd = ld2(rv);
        sq += rd.x * rd.x + rd.y * rd.y;
    }
    cg_part(sq, k, S, part);
}
// red = ||b||^2 (of the stored b)
__global__ void bicg_setup_kernel(BicgCol* cols, const double* bn2, double tol, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    BicgCol c{};
    c.rho_r = bn2[s];
    c.bn2 = bn2[s];
    c.rn2 = bn2[s];
    c.tol2 = tol * tol * bn2[s];
    c.active = bn2[s] > c.tol2;
    cols[s] = c;
}
// after v = A p and d = <r^, v> (red[0] + j red[1]): alpha = rho / d
__global__ void bicg_alpha_kernel(BicgCol* cols, const double* red, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || !cols[s].active) return;
    BicgCol c = cols[s];
    const double dr = red[s], di = red[S + s], dd = dr * dr + di * di;
    if (!(dd > 0.0)) {   // breakdown: the column keeps its last iterate
        c.active = 0;
    } else {
        c.al_r = (c.rho_r * dr + c.rho_i * di) / dd;
        c.al_i = (c.rho_i * dr - c.rho_r * di) / dd;
    }
    cols[s] = c;
}
// s = r - alpha v, in place of r (active columns)
template <typename V>
__global__ __launch_bounds__(256) void bicg_s_kernel(V* __restrict__ r, const V* __restrict__ v,
                                                     const BicgCol* __restrict__ cols, int N, int S) {
    const CgBlock k = cg_block(N);
    if (k.s >= S || !cols[k.s].active) return;
    const double ar = cols[k.s].al_r, ai = cols[k.s].al_i;
    for (int j = k.j0; j < k.j1; j += 4) {
        const size_t e = cg_at(k.tile, j, k.c, N);
        const double2 rr = ld2(r[e]), vv = ld2(v[e]);
        r[e] = st2<V>(rr.x - (ar * vv.x - ai * vv.y), rr.y - (ar * vv.y + ai * vv.x));
    }
}
// after t = A s with red = (<s, t> re, im, ||t||^2): omega = <t, s> / ||t||^2 =
// conj(<s, t>) / ||t||^2 (zero when t = 0: then s is the residual and x += alpha p)
__global__ void bicg_omega_kernel(BicgCol* cols, const double* red, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || !cols[s].active) return;
    const double tt = red[2 * S + s];
    cols[s].om_r = tt > 0.0 ? red[s] / tt : 0.0;
    cols[s].om_i = tt > 0.0 ? -red[S + s] / tt : 0.0;
}
// x += alpha p + omega s, r = s - omega t (active columns); part = slice sums of
// <r^, r> (re, im) and |r|^2 for every column
template <typename V>
__global__ __launch_bounds__(256) void bicg_xr_kernel(V* __restrict__ x, V* __restrict__ r, const V* __restrict__ p,
                                                      const V* __restrict__ t, const V* __restrict__ rh,
                                                      const BicgCol* __restrict__ cols, int N, int S,
                                                      double* __restrict__ part) {
    const CgBlock k = cg_block(N);
    if (k.tile * CG_W >= S) return;
    const bool act = k.s < S && cols[k.s].active;
    double ar = 0, ai = 0, wr = 0, wi = 0;
    if (act) {
        ar = cols[k.s].al_r;
        ai = cols[k.s].al_i;
        wr = cols[k.s].om_r;
        wi = cols[k.s].om_i;
    }
    double dr = 0.0, di = 0.0, sq = 0.0;
    for (int j = k.j0; j < k.j1; j += 4) {
        const size_t e = cg_at(k.tile, j, k.c, N);
        double2 rr = ld2(r[e]);
        if (act) {
            const double2 pp = ld2(p[e]), tv = ld2(t[e]), xx = ld2(x[e]);
            x[e] = st2<V>(xx.x + (ar * pp.x - ai * pp.y) + (wr * rr.x - wi * rr.y),
                          xx.y + (ar * pp.y + ai * pp.x) + (wr * rr.y + wi * rr.x));
            const V rn = st2<V>(rr.x - (wr * tv.x - wi * tv.y), rr.y - (wr * tv.y + wi * tv.x));
            r[e] = rn;
            rr = ld2(rn);
        }
        const double2 hv = ld2(rh[e]);
        dr += hv.x * rr.x + hv.y * rr.y;
        di += hv.x * rr.y - hv.y * rr.x;
        sq += rr.x * rr.x + rr.y * rr.y;
    }
    const size_t ps = size_t(cg_slices(N)) * S;
    cg_part(dr, k, S, part);
    __syncthreads();
    cg_part(di, k, S, part + ps);
    __syncthreads();
    cg_part(sq, k, S, part + 2 * ps);
}
// red = (<r^, r> re, im, ||r||^2): convergence, then beta = (rho' / rho)(alpha /
// omega) and rho = rho'; nactive counts the columns still active
__global__ void bicg_check_kernel(BicgCol* cols, const double* red, int S, int* nactive) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    BicgCol c = cols[s];
    if (!c.active) return;
    const double rr = red[s], ri = red[S + s], rn2 = red[2 * S + s];
    c.rn2 = rn2;
    c.iters += 1;
    const double oo = c.om_r * c.om_r + c.om_i * c.om_i, hh = c.rho_r * c.rho_r + c.rho_i * c.rho_i;
    if (rn2 <= c.tol2 || !(rn2 == rn2) || !(oo > 0.0) || !(hh > 0.0)) {
        c.active = 0;
    } else {
        // (rho' / rho) (alpha / omega)
        const double qr = (rr * c.rho_r + ri * c.rho_i) / hh, qi = (ri * c.rho_r - rr * c.rho_i) / hh;
        const double ur = (c.al_r * c.om_r + c.al_i * c.om_i) / oo, ui = (c.al_i * c.om_r - c.al_r * c.om_i) / oo;
        c.be_r = qr * ur - qi * ui;
        c.be_i = qr * ui + qi * ur;
        c.rho_r = rr;
        c.rho_i = ri;
    }
    cols[s] = c;
    if (c.active) atomicAdd(nactive, 1);
}
// p = r + beta (p - omega v) (active columns)
template <typename V>
__global__ __launch_bounds__(256) void bicg_p_kernel(V* __restrict__ p, const V* __restrict__ r, const V* __restrict__ v,
                                                     const BicgCol* __restrict__ cols, int N, int S) {
    const CgBlock k = cg_block(N);
    if (k.s >= S || !cols[k.s].active) return;
    const double br = cols[k.s].be_r, bi = cols[k.s].be_i, wr = cols[k.s].om_r, wi = cols[k.s].om_i;
    for (int j = k.j0; j < k.j1; j += 4) {
        const size_t e = cg_at(k.tile, j, k.c, N);
        const double2 pp = ld2(p[e]), rr = ld2(r[e]), vv = ld2(v[e]);
        const double ux = pp.x - (wr * vv.x - wi * vv.y), uy = pp.y - (wr * vv.y + wi * vv.x);
        p[e] = st2<V>(rr.x + (br * ux - bi * uy), rr.y + (br * uy + bi * ux));
    }
}

// P[s0 + s][j] = w[j][s] for s < S, 32 x 32 tiles through LDS; grid (ceil(N / 32),
// padded columns / 32)
template <typename V>
__global__ __launch_bounds__(256) void tile_out_kernel(const V* __restrict__ w, int S, int N, double2* __restrict__ P,
                                                       int s0) {
    __shared__ double2 tl[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int jb = blockIdx.x * 32, cb = blockIdx.y * 32;
    for (int r = ty; r < 32; r += 8) {
        const int j = jb + r, sc = cb + tx;
        if (j < N) tl[r][tx] = ld2(w[cg_at(sc / CG_W, j, sc % CG_W, N)]);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int sc = cb + r, j = jb + tx;
        if (sc < S && j < N) P[size_t(s0 + sc) * N + j] = tl[tx][r];
    }
}

// ------------------------------------------ the MFIE operator of the 3-D CFIE
// K_BC(k) = R^T K_mix(k) without forming K_mix (N_b x N): per chunk of
// barycentric test triangles p, every pair value into W[p][i][n][side] (source
// RWG n primal, side 0 where the source triangle is T+(n)), then the test-side
// contraction K_BC[m][n] += sum R[e(p, i)][m] (W[p][i][n][0] + W[p][i][n][1]) by
// the BC-row lists of the T_BC build (no atomics; chunks in order).
constexpr int K_PB = 4;   // barycentric test triangles per block of k_rows_kernel

// block = (K_PB test triangles of the chunk, 256 primal source triangles), the
// blocks of consecutive test triangles kept on one XCD (as in the far-row kernel);
// every slot of a row is written: the three local edges of the source triangles
// cover each (n, side) once
template <bool CK>
__global__ __launch_bounds__(256) void k_rows_kernel(DevMesh mb, DevMesh m, double kr, double ki,
                                                     double2* __restrict__ W, int c0, int np, int nqblk) {
    const int nblk = int(gridDim.x);
    const int xcd = int(blockIdx.x) & 7, idx = int(blockIdx.x) >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    const int logical = xcd * per + min(xcd, rem) + idx;
    const int pg = logical / nqblk, qb = logical - pg * nqblk;
    const int q = qb * 256 + int(threadIdx.x);
    const int T = m.T;
    if (q >= T) return;
    const size_t N = size_t(m.N);
    const int pl1 = min(np, (pg + 1) * K_PB);
    for (int pl = pg * K_PB; pl < pl1; ++pl) {
        const int p = c0 + pl, t = p / 6;   // the refinement's triangle p lies in primal triangle p / 6
        double2* rows = W + size_t(pl) * 6 * N;
        auto put = [&](int i, int j, double re, double im) {
            const size_t n = size_t(m.te[j * T + q]);
            const int side = m.cf[j * T + q] > 0.0 ? 0 : 1;
            rows[(size_t(i) * N + n) * 2 + side] = make_double2(re, im);
        };
        if (q == t) {   // coplanar: the principal value vanishes
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) put(i, j, 0.0, 0.0);
            continue;
        }
        mfie_pair<CK>(mb, m, p, q, kr, ki, is_near(m, t, q), put);
    }
}

// K[m][n] += sum_k coef[k] (W[rows[k]][n][0] + W[rows[k]][n][1]) over the list of
// BC row m = ml[blockIdx.y]
__global__ __launch_bounds__(256) void kbc_test_kernel(const int32_t* __restrict__ ml,
                                                       const int32_t* __restrict__ mptr,
                                                       const int32_t* __restrict__ rows,
                                                       const double* __restrict__ coef,
                                                       const double2* __restrict__ W, double2* __restrict__ K, int N) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int mi = blockIdx.y;
    if (n >= N) return;
    const size_t o = size_t(ml[mi]) * N + n;
    double2 acc = K[o];
    for (int k = mptr[mi]; k < mptr[mi + 1]; ++k) {
        const double2* w = W + size_t(rows[k]) * 2 * size_t(N) + 2 * size_t(n);
        const double2 a = w[0], b = w[1];
        acc.x += coef[k] * (a.x + b.x);
        acc.y += coef[k] * (a.y + b.y);
    }
    K[o] = acc;
}

// Y = a X (n complex elements; Y may be X)
__global__ void scale_c_kernel(const double2* X, double2* Y, double a, size_t n) {
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) {
        const double2 v = X[i];
        Y[i] = make_double2(a * v.x, a * v.y);
    }
}

// Y[order[t]][idx[e]] += a val[e] over the stored rows t of a real CSR matrix whose
// rows are stored in the order `order` (one thread per row: no two threads touch
// one element)
__global__ void add_csr_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                               const double* __restrict__ val, const int32_t* __restrict__ order, int N, double a,
                               double2* __restrict__ Y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    double2* row = Y + size_t(order[t]) * N;
    for (int e = ptr[t]; e < ptr[t + 1]; ++e) row[idx[e]].x += a * val[e];
}

// T <- T^T in place (N x N complex128): one block per pair of mirror 32 x 32
// tiles (bi <= bj), both read into LDS before either is written
__global__ __launch_bounds__(256) void transpose_inplace_kernel(double2* __restrict__ T, int N, int nt) {
    __shared__ double2 a[32][33], b[32][33];
    int k = int(blockIdx.x), bi = 0;
    while (k >= nt - bi) {
        k -= nt - bi;
        ++bi;
    }
    const int bj = bi + k;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
        if (i < N && j < N) a[r][tx] = T[size_t(i) * N + j];
        if (i2 < N && j2 < N) b[r][tx] = T[size_t(i2) * N + j2];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        // (bi*32 + r, bj*32 + tx) <- old (bj*32 + tx, bi*32 + r) = b[tx][r]
        const int i = bi * 32 + r, j = bj * 32 + tx;
        if (i < N && j < N) T[size_t(i) * N + j] = b[tx][r];
        if (bi != bj) {   // (bj*32 + r, bi*32 + tx) <- old (bi*32 + tx, bj*32 + r) = a[tx][r]
            const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
            if (i2 < N && j2 < N) T[size_t(i2) * N + j2] = a[tx][r];
        }
    }
}

// out[s] = khat_s x pol_s
__global__ void cross3_kernel(const double* __restrict__ kh, const double* __restrict__ po, double* __restrict__ out,
                              int nrhs) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nrhs) return;
    const double* a = kh + 3 * s;
    const double* b = po + 3 * s;
    out[3 * s] = a[1] * b[2] - a[2] * b[1];
    out[3 * s + 1] = a[2] * b[0] - a[0] * b[2];
    out[3 * s + 2] = a[0] * b[1] - a[1] * b[0];
}

// H[s][n] = sum over column n of R of r_val[k] Vb[s][r_idx[k]]: BC-tested values
// from barycentric-RWG-tested ones
__global__ void bc_contract_kernel(DevCald c, const double2* __restrict__ Vb, int nrhs, double2* __restrict__ H) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(c.N) * nrhs) return;
    const int s = int(idx / c.N), n = int(idx - size_t(s) * c.N);
    const double2* v = Vb + size_t(s) * c.Nb;
    double ar = 0.0, ai = 0.0;
    for (int k = c.r_ptr[n]; k < c.r_ptr[n + 1]; ++k) {
        const double2 x = v[c.r_idx[k]];
        ar += c.r_val[k] * x.x;
        ai += c.r_val[k] * x.y;
    }
    H[idx] = make_double2(ar, ai);
}

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr size_t CALD_W_BUDGET = size_t(2) << 30;    // workspace rows of one chunk of test triangles
constexpr size_t CALD_CG_BUDGET = size_t(6) << 30;   // Gram-solve vectors of one column batch

struct CaldPlan {
    int chunk = 1, nchunks = 1, Sb = 1;
    size_t entries = 0;   // (BC row, workspace row, coefficient) list entries over all chunks
    size_t vsz = 16;      // bytes per complex element of the Gram-solve vectors
};

CaldPlan cald_plan(const efie_calderon_s& C, int bary_dtype, double tol) {
    CaldPlan pl;
    pl.vsz = tol >= GRAM_C64_TOL ? 8 : 16;
    const size_t esz = bary_dtype == EFIE_C64 ? 8 : 16;
    const size_t per_tri = size_t(6) * size_t(C.bary.N) * esz;
    const size_t Tb = size_t(C.bary.T);
    // grid limits: 3 rows per triangle (bc_src) and at most 18 BC rows per triangle (bc_test)
    pl.chunk = int(std::max<size_t>(1, std::min<size_t>({Tb, CALD_W_BUDGET / per_tri, 3640})));
    pl.nchunks = int((Tb + size_t(pl.chunk) - 1) / size_t(pl.chunk));
    const size_t N = size_t(C.N);
    pl.Sb = int(std::max<size_t>(64, std::min<size_t>(N, CALD_CG_BUDGET / (6 * N * pl.vsz))));
    pl.entries = 2 * C.re_idx.size();
    return pl;
}

struct CaldWs {
    void* W;
    double2* Yw;
    int32_t *ml, *mptr, *rows;
    double* coef;
    double2* Tbc;
    void *x, *r, *rh, *p, *v, *t;   // BiCGStab vectors (complex64 or complex128)
    double *part, *red;             // slice sums and column sums of three reductions
    BicgCol* cols;
    int* counter;
};

size_t cald_layout(const efie_calderon_s& C, const CaldPlan& pl, int bary_dtype, CaldWs* w, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += a256(bytes);
        return p;
    };
    const size_t N = size_t(C.N), Nb = size_t(C.bary.N), Sb = size_t(pl.Sb);
    const size_t esz = bary_dtype == EFIE_C64 ? 8 : 16;
    CaldWs x{};
    x.W = take(size_t(pl.chunk) * 6 * Nb * esz);
    x.Yw = (double2*)take(size_t(pl.chunk) * 3 * N * 16);
    x.ml = (int32_t*)take(4 * pl.entries);
    x.mptr = (int32_t*)take(4 * (pl.entries + size_t(pl.nchunks)));
    x.rows = (int32_t*)take(4 * pl.entries);
    x.coef = (double*)take(8 * pl.entries);
    x.Tbc = (double2*)take(N * N * 16);
    const size_t vb = N * size_t(cg_pad(pl.Sb)) * pl.vsz;
    x.x = take(vb);
    x.r = take(vb);
    x.rh = take(vb);
    x.p = take(vb);
    x.v = take(vb);
    x.t = take(vb);
    x.part = (double*)take(3 * 8 * size_t(cg_slices(int(N))) * Sb);
    x.red = (double*)take(3 * 8 * Sb);
    x.cols = (BicgCol*)take(sizeof(BicgCol) * Sb);
    x.counter = (int*)take(16);
    if (w) *w = x;
    return off;
}

// Host lists of the test-side contraction, per chunk of barycentric test triangles:
// for every BC row m touched by the chunk, the workspace rows 3 (p - c0) + i whose
// barycentric RWG e(p, i) has R[e][m] != 0, with that coefficient.
struct CaldLists {
    std::vector<int32_t> ml, mptr, rows;
    std::vector<double> coef;
    std::vector<int64_t> m0, nm, mp0;   // per chunk: first entry in ml, count, first entry in mptr
};

CaldLists cald_lists(const efie_calderon_s& C, const CaldPlan& pl) {
    CaldLists L;
    const int64_t Tb = C.bary.T;
    struct E {
        int32_t m, row;
        double c;
    };
    std::vector<E> es;
    for (int ch = 0; ch < pl.nchunks; ++ch) {
        const int64_t c0 = int64_t(ch) * pl.chunk, c1 = std::min<int64_t>(Tb, c0 + pl.chunk);
        es.clear();
        for (int64_t p = c0; p < c1; ++p)
            for (int i = 0; i < 3; ++i) {
                const int32_t e = C.bary.tri_edge[size_t(3 * p + i)];
                for (int32_t k = C.re_ptr[size_t(e)]; k < C.re_ptr[size_t(e) + 1]; ++k)
                    es.push_back({C.re_idx[size_t(k)], int32_t(3 * (p - c0) + i), C.re_val[size_t(k)]});
            }
        std::stable_sort(es.begin(), es.end(), [](const E& a, const E& b) { return a.m < b.m; });
        L.m0.push_back(int64_t(L.ml.size()));
        L.mp0.push_back(int64_t(L.mptr.size()));
        for (size_t q = 0; q < es.size(); ++q) {
            if (q == 0 || es[q].m != es[q - 1].m) {
                L.ml.push_back(es[q].m);
                L.mptr.push_back(int32_t(L.rows.size()));
            }
            L.rows.push_back(es[q].row);
            L.coef.push_back(es[q].c);
        }
        L.mptr.push_back(int32_t(L.rows.size()));
        L.nm.push_back(int64_t(L.ml.size()) - L.m0.back());
    }
    return L;
}

DevCald dev_cald(const efie_calderon_s& C) {
    const char* b = static_cast<const char*>(C.dev);
    const auto& o = C.offs;
    DevCald d{};
    d.N = int(C.N);
    d.Nb = int(C.bary.N);
    d.r_ptr = reinterpret_cast<const int32_t*>(b + o[0]);
    d.r_idx = reinterpret_cast<const int32_t*>(b + o[1]);
    d.r_val = reinterpret_cast<const double*>(b + o[2]);
    d.g_ptr = reinterpret_cast<const int32_t*>(b + o[3]);
    d.g_idx = reinterpret_cast<const int32_t*>(b + o[4]);
    d.g_val = reinterpret_cast<const double*>(b + o[5]);
    d.gt_ptr = reinterpret_cast<const int32_t*>(b + o[6]);
    d.gt_idx = reinterpret_cast<const int32_t*>(b + o[7]);
    d.gt_val = reinterpret_cast<const double*>(b + o[8]);
    d.n_order = reinterpret_cast<const int32_t*>(b + o[9]);
    d.run_t0 = reinterpret_cast<const int32_t*>(b + o[10]);
    d.u_ptr = reinterpret_cast<const int32_t*>(b + o[11]);
    d.u_idx = reinterpret_cast<const int32_t*>(b + o[12]);
    d.r_loc = reinterpret_cast<const int32_t*>(b + o[13]);
    return d;
}

template <class T>
size_t put(std::vector<char>& blob, std::vector<size_t>& offs, const std::vector<T>& v) {
    size_t off = a256(blob.size());
    blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    offs.push_back(off);
    return off;
}

// BiCGStab on A Y = B for the columns of B (N x N, row-major) in batches of pl.Sb
// (vectors stored as V), each batch transposed into the rows of Pout; A = G^T
// (opG false) or G (opG true).  Returns the worst final relative residual.
template <typename V>
double cald_gram_solve(const DevCald& d, const CaldWs& w, const CaldPlan& pl, int N, double tol, int maxit,
                       double2* Pout, const double2* B, bool opG, hipStream_t stream) {
    // A with the CSR of A (stored rows in n_order)
    const int32_t *a_ptr = opG ? d.g_ptr : d.gt_ptr, *a_idx = opG ? d.g_idx : d.gt_idx;
    const double* a_val = opG ? d.g_val : d.gt_val;
    V* const xv = static_cast<V*>(w.x);
    V* const rv = static_cast<V*>(w.r);
    V* const hv = static_cast<V*>(w.rh);
    V* const pv = static_cast<V*>(w.p);
    V* const vv = static_cast<V*>(w.v);
    V* const tv = static_cast<V*>(w.t);
    double worst = 0.0;
    for (int s0 = 0; s0 < N; s0 += pl.Sb) {
        const int S = std::min(pl.Sb, N - s0);
        const dim3 gs(cg_blocks(S, N)), gc(unsigned((S + 255) / 256));
        const int ns = cg_slices(N);
        auto finish = [&](int nred) {   // slice sums -> column sums red[y S + s], y < nred
            hipLaunchKernelGGL(colsq_final_kernel, dim3(unsigned((S + 15) / 16), unsigned(nred)), dim3(256), 0, stream,
                               w.part, S, ns, w.red);
        };
        hipLaunchKernelGGL(bicg_init_kernel<V>, gs, dim3(256), 0, stream, B + s0, N, xv, rv, hv, pv, N, S, w.part);
        finish(1);
        hipLaunchKernelGGL(bicg_setup_kernel, gc, dim3(256), 0, stream, w.cols, w.red, tol, S);
        int h_active = S;
        for (int it = 0; it < maxit && h_active > 0; ++it) {
            // v = A p, alpha = rho / <r^, v>, s = r - alpha v
            hipLaunchKernelGGL(cspmm_dot_kernel<V>, gs, dim3(256), 0, stream, a_ptr, a_idx, a_val, pv, vv, S,
                               d.n_order, N, hv, w.part);
            finish(2);
            hipLaunchKernelGGL(bicg_alpha_kernel, gc, dim3(256), 0, stream, w.cols, w.red, S);
            hipLaunchKernelGGL(bicg_s_kernel<V>, gs, dim3(256), 0, stream, rv, vv, w.cols, N, S);
            // t = A s, omega = <t, s> / <t, t>, x += alpha p + omega s, r = s - omega t
            hipLaunchKernelGGL(cspmm_dot_kernel<V>, gs, dim3(256), 0, stream, a_ptr, a_idx, a_val, rv, tv, S,
                               d.n_order, N, rv, w.part);
            finish(3);
            hipLaunchKernelGGL(bicg_omega_kernel, gc, dim3(256), 0, stream, w.cols, w.red, S);
            hipLaunchKernelGGL(bicg_xr_kernel<V>, gs, dim3(256), 0, stream, xv, rv, pv, tv, hv, w.cols, N, S, w.part);
            finish(3);
            fill_zero_bytes(w.counter, 8, stream);
            hipLaunchKernelGGL(bicg_check_kernel, gc, dim3(256), 0, stream, w.cols, w.red, S, w.counter);
            // p = r + beta (p - omega v)
            hipLaunchKernelGGL(bicg_p_kernel<V>, gs, dim3(256), 0, stream, pv, rv, vv, w.cols, N, S);
            EFIE_HIP_CHECK(hipMemcpyAsync(&h_active, w.counter, sizeof(int), hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        }
        hipLaunchKernelGGL(tile_out_kernel<V>, dim3(unsigned((N + 31) / 32), unsigned(cg_pad(S) / 32)), dim3(256), 0,
                           stream, xv, S, N, Pout, s0);
        if (verbose())
            std::fprintf(stderr, "[efie] calderon Gram solve columns %d..%d done t=%.3f\n", s0, s0 + S, now_s()),
                std::fflush(stderr);
        std::vector<BicgCol> cols(static_cast<size_t>(S));
        EFIE_HIP_CHECK(hipMemcpyAsync(cols.data(), w.cols, sizeof(BicgCol) * size_t(S), hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        for (const auto& cc : cols) worst = std::max(worst, cc.bn2 > 0 ? std::sqrt(cc.rn2 / cc.bn2) : 0.0);
    }
    return worst;
}

// CSR rows in the order ord: stored row t is row ord[t]
void permute_rows(const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx, const std::vector<double>& val,
                  const std::vector<int32_t>& ord, std::vector<int32_t>& pp, std::vector<int32_t>& pi,
                  std::vector<double>& pv) {
    pp.assign(ord.size() + 1, 0);
    pi.clear();
    pv.clear();
    for (size_t t = 0; t < ord.size(); ++t) {
        const size_t j = size_t(ord[t]);
        for (int32_t q = ptr[j]; q < ptr[j + 1]; ++q) {
            pi.push_back(idx[size_t(q)]);
            pv.push_back(val[size_t(q)]);
        }
        pp[t + 1] = int32_t(pi.size());
    }
}

}  // namespace
}  // namespace efie

extern "C" {

int efie_calderon_create(efie_mesh mesh, efie_calderon* out) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh && out, EFIE_ERR_ARG, "calderon_create: null argument");
        auto* C = new efie_calderon_s();
        try {
            C->primal = mesh;
            efie::build_calderon(*C, *mesh);
            // sparse arrays after the barycentric tables
            std::vector<char> blob;
            std::vector<size_t> offs;
            efie::put(blob, offs, C->r_ptr);
            efie::put(blob, offs, C->r_idx);
            efie::put(blob, offs, C->r_val);
            // the device copies of G and G^T store their rows in n_order order
            std::vector<int32_t> pp, pi;
            std::vector<double> pv;
            efie::permute_rows(C->g_ptr, C->g_idx, C->g_val, C->n_order, pp, pi, pv);
            efie::put(blob, offs, pp);
            efie::put(blob, offs, pi);
            efie::put(blob, offs, pv);
            efie::permute_rows(C->gt_ptr, C->gt_idx, C->gt_val, C->n_order, pp, pi, pv);
            efie::put(blob, offs, pp);
            efie::put(blob, offs, pi);
            efie::put(blob, offs, pv);
            efie::put(blob, offs, C->n_order);
            efie::put(blob, offs, C->run_t0);
            efie::put(blob, offs, C->u_ptr);
            efie::put(blob, offs, C->u_idx);
            efie::put(blob, offs, C->r_loc);
            blob.resize(efie::a256(blob.size()));
            C->host_blob.swap(blob);
            C->offs.swap(offs);
            C->bary_bytes = C->bary.host_blob.size();
        } catch (...) {
            delete C;
            throw;
        }
        *out = C;
        return int(EFIE_OK);
    });
}

void efie_calderon_destroy(efie_calderon c) { delete c; }

int efie_calderon_set_far_rule(efie_calderon c, double ratio) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c != nullptr && std::isfinite(ratio), EFIE_ERR_ARG, "calderon_set_far_rule: bad argument");
        c->far3 = ratio < 0.0 ? -1.0 : ratio;
        return int(EFIE_OK);
    });
}

int efie_calderon_sizes(efie_calderon c, int64_t* n_bary_rwg, int64_t* n_bary_tri, size_t* table_bytes,
                        size_t* ws_bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c != nullptr, EFIE_ERR_ARG, "calderon_sizes: null");
        if (n_bary_rwg) *n_bary_rwg = c->bary.N;
        if (n_bary_tri) *n_bary_tri = c->bary.T;
        if (table_bytes) *table_bytes = efie::a256(c->bary_bytes) + c->host_blob.size();
        if (ws_bytes) {
            size_t mx = 0;
            for (int dt : {EFIE_C128, EFIE_C64})
                for (double tl : {1.0, 0.0})
                    mx = std::max(mx, efie::cald_layout(*c, efie::cald_plan(*c, dt, tl), dt, nullptr, nullptr));
            *ws_bytes = mx;
        }
        return int(EFIE_OK);
    });
}

int efie_calderon_upload(efie_calderon c, void* dev, size_t bytes, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c && dev, EFIE_ERR_ARG, "calderon_upload: null argument");
        const size_t off = efie::a256(c->bary_bytes);
        EFIE_REQUIRE(bytes >= off + c->host_blob.size(), EFIE_ERR_ARG, "calderon_upload: buffer too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(dev) & 255) == 0, EFIE_ERR_ARG, "calderon_upload: not 256-aligned");
        char* d = static_cast<char*>(dev);
        EFIE_HIP_CHECK(hipMemcpyAsync(d, c->bary.host_blob.data(), c->bary_bytes, hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(d + off, c->host_blob.data(), c->host_blob.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        efie::bind_tables(c->bary, d);
        c->dev = d + off;
        return int(EFIE_OK);
    });
}

int efie_calderon_host_matrices(efie_calderon c, double* R, double* G) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c != nullptr, EFIE_ERR_ARG, "calderon_host_matrices: null");
        const size_t N = size_t(c->N), Nb = size_t(c->bary.N);
        if (R) {
            std::memset(R, 0, sizeof(double) * Nb * N);
            for (size_t n = 0; n < N; ++n)
                for (int32_t k = c->r_ptr[n]; k < c->r_ptr[n + 1]; ++k) {
                    const int32_t e = c->r_idx[size_t(k)];
                    R[size_t(c->bary_canon[size_t(e)]) * N + n] = c->bary_flip[size_t(e)] ? -c->r_val[size_t(k)]
                                                                                          : c->r_val[size_t(k)];
                }
        }
        if (G) {
            std::memset(G, 0, sizeof(double) * N * N);
            for (size_t m = 0; m < N; ++m)
                for (int32_t k = c->g_ptr[m]; k < c->g_ptr[m + 1]; ++k) G[m * N + size_t(c->g_idx[size_t(k)])] = c->g_val[size_t(k)];
        }
        return int(EFIE_OK);
    });
}

int efie_calderon_assemble_ex(efie_calderon c, double kt_re, double kt_im, double eta, int bary_dtype, void* P,
                              void* Tbc_out, double tol, int32_t maxit, double* relres, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE(c && P && ws, EFIE_ERR_ARG, "calderon_assemble: null argument");
        EFIE_REQUIRE(c->dev != nullptr, EFIE_ERR_STATE, "calderon_assemble: tables not uploaded");
        EFIE_REQUIRE(bary_dtype == EFIE_C128 || bary_dtype == EFIE_C64, EFIE_ERR_ARG, "calderon_assemble: bad dtype");
        EFIE_REQUIRE(kt_im <= 0.0 && (kt_re != 0.0 || kt_im != 0.0), EFIE_ERR_ARG, "calderon_assemble: bad k~");
        EFIE_REQUIRE(tol > 0.0 && maxit >= 1, EFIE_ERR_ARG, "calderon_assemble: bad tol/maxit");
        if (bary_dtype == EFIE_C64) require_fp32_phase(c->bary.diam, kt_re, "calderon_assemble");
        const int N = int(c->N);
        const CaldPlan pl = cald_plan(*c, bary_dtype, tol);
        const size_t need = cald_layout(*c, pl, bary_dtype, nullptr, nullptr);
        EFIE_REQUIRE(ws_bytes >= need, EFIE_ERR_ARG, "calderon_assemble: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "calderon_assemble: ws not aligned");
        CaldWs w;
        cald_layout(*c, pl, bary_dtype, &w, static_cast<char*>(ws));
        const DevCald d = dev_cald(*c);
        // ---- T_BC = R^T T_bary(k~) R, streamed over chunks of barycentric test triangles
        const CaldLists L = cald_lists(*c, pl);
        EFIE_HIP_CHECK(hipMemcpyAsync(w.ml, L.ml.data(), 4 * L.ml.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.mptr, L.mptr.data(), 4 * L.mptr.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.rows, L.rows.data(), 4 * L.rows.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.coef, L.coef.data(), 8 * L.coef.size(), hipMemcpyHostToDevice, stream));
        fill_zero_bytes(w.Tbc, size_t(N) * N * 16, stream);
        const int Tb = int(c->bary.T);
        const unsigned nx = unsigned((N + 255) / 256);
        static_assert(BC_BLOCK == 256, "one thread per BC function of a run");
        EFIE_REQUIRE(c->u_max <= BC_UMAX, EFIE_ERR_STATE, "calderon_assemble: BC run lists too long");
        const unsigned nruns = unsigned(c->run_t0.size() - 1);
        EFIE_REQUIRE(nruns <= 65535, EFIE_ERR_STATE, "calderon_assemble: too many BC runs for one launch");
        // the barycentric operator's far rule: its own, else the primal mesh's
        const double f3 = c->far3 >= 0.0 ? c->far3 : c->primal->far3;
        c->bary.far3 = f3;
        c->bary.dm.far3 = f3;
        for (int ch = 0; ch < pl.nchunks; ++ch) {
            const int c0 = ch * pl.chunk, c1 = std::min(Tb, c0 + pl.chunk), np = c1 - c0;
            pair_rows_chunk(c->bary.dm, kt_re, kt_im, eta, bary_dtype, w.W, c0, c1, c->bary.near_p, c->bary.near_up,
                            true, stream);
            const int nr = 3 * np;
            if (bary_dtype == EFIE_C64)
                hipLaunchKernelGGL((bc_src_kernel<float2, BC_RRL32>),
                                   dim3(unsigned((nr + BC_RRL32 - 1) / BC_RRL32), nruns), dim3(256), 0, stream, d,
                                   static_cast<const float2*>(w.W), w.Yw, nr, c->bary.dm.et, c0);
            else
                hipLaunchKernelGGL((bc_src_kernel<double2, BC_RRL64>),
                                   dim3(unsigned((nr + BC_RRL64 - 1) / BC_RRL64), nruns), dim3(256), 0, stream, d,
                                   static_cast<const double2*>(w.W), w.Yw, nr, c->bary.dm.et, c0);
            if (L.nm[size_t(ch)] > 0)
                hipLaunchKernelGGL(bc_test_kernel, dim3(nx, unsigned(L.nm[size_t(ch)])), dim3(256), 0, stream,
                                   w.ml + L.m0[size_t(ch)], w.mptr + L.mp0[size_t(ch)], w.rows, w.coef, w.Yw, w.Tbc, N);
            if (verbose() && (ch % 64 == 63 || ch + 1 == pl.nchunks)) {
                EFIE_HIP_CHECK(hipStreamSynchronize(stream));
                std::fprintf(stderr, "[efie] calderon T_BC chunk %d/%d t=%.3f\n", ch + 1, pl.nchunks, now_s());
                std::fflush(stderr);
            }
        }
        // the chunks held the rows of U + D/2 (pairs with source triangle above the
        // test triangle, halved diagonal blocks): T_BC = A + A^T
        {
            const int nt = (N + 31) / 32;
            const size_t npairs = size_t(nt) * size_t(nt + 1) / 2;
            EFIE_REQUIRE(npairs < (size_t(1) << 31), EFIE_ERR_ARG, "calderon_assemble: N too large");
            hipLaunchKernelGGL(sym_add_kernel, dim3(unsigned(npairs)), dim3(256), 0, stream, w.Tbc, N, nt);
        }
        if (Tbc_out)
            EFIE_HIP_CHECK(hipMemcpyAsync(Tbc_out, w.Tbc, size_t(N) * N * 16, hipMemcpyDeviceToDevice, stream));
        // ---- P = T_BC G^{-1}: column batches of G^T Y = T_BC (column s = row s of T_BC), P = Y^T
        const double worst =
            pl.vsz == 8
                ? cald_gram_solve<float2>(d, w, pl, N, tol, maxit, static_cast<double2*>(P), w.Tbc, false, stream)
                : cald_gram_solve<double2>(d, w, pl, N, tol, maxit, static_cast<double2*>(P), w.Tbc, false, stream);
        if (relres) *relres = worst;
        EFIE_HIP_CHECK(hipGetLastError());
        return worst <= tol ? int(EFIE_OK) : int(EFIE_NOT_CONVERGED);
    });
}

int efie_calderon_assemble(efie_calderon c, double kt_re, double kt_im, double eta, void* P, void* Tbc_out,
                           double tol, int32_t maxit, double* relres, void* ws, size_t ws_bytes, hipStream_t stream) {
    return efie_calderon_assemble_ex(c, kt_re, kt_im, eta, EFIE_C128, P, Tbc_out, tol, maxit, relres, ws, ws_bytes,
                                     stream);
}

int efie_calderon_cfie_assemble(efie_calderon c, double k, double kt_re, double kt_im, double eta, void* M, void* Q,
                                void* K_out, void* Kt_out, double tol, int32_t maxit, double* relres, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE(c && M && Q && ws, EFIE_ERR_ARG, "calderon_cfie_assemble: null argument");
        EFIE_REQUIRE(c->dev != nullptr && c->primal->dev != nullptr, EFIE_ERR_STATE,
                     "calderon_cfie_assemble: tables not uploaded (mesh and Calderon)");
        EFIE_REQUIRE(std::isfinite(k) && k > 0.0, EFIE_ERR_ARG, "calderon_cfie_assemble: need k > 0");
        EFIE_REQUIRE(std::isfinite(kt_re) && std::isfinite(kt_im) && kt_im <= 0.0 && (kt_re != 0.0 || kt_im != 0.0),
                     EFIE_ERR_ARG, "calderon_cfie_assemble: bad k~");
        EFIE_REQUIRE(std::isfinite(eta) && eta > 0.0, EFIE_ERR_ARG, "calderon_cfie_assemble: need eta > 0");
        EFIE_REQUIRE(tol > 0.0 && maxit >= 1, EFIE_ERR_ARG, "calderon_cfie_assemble: bad tol/maxit");
        const int N = int(c->N);
        const CaldPlan pl = cald_plan(*c, EFIE_C128, tol);
        const size_t need = cald_layout(*c, pl, EFIE_C128, nullptr, nullptr);
        EFIE_REQUIRE(ws_bytes >= need, EFIE_ERR_ARG, "calderon_cfie_assemble: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG,
                     "calderon_cfie_assemble: ws not aligned");
        CaldWs w;
        cald_layout(*c, pl, EFIE_C128, &w, static_cast<char*>(ws));
        const DevCald d = dev_cald(*c);
        const CaldLists L = cald_lists(*c, pl);
        EFIE_HIP_CHECK(hipMemcpyAsync(w.ml, L.ml.data(), 4 * L.ml.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.mptr, L.mptr.data(), 4 * L.mptr.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.rows, L.rows.data(), 4 * L.rows.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(w.coef, L.coef.data(), 8 * L.coef.size(), hipMemcpyHostToDevice, stream));
        const DevMesh& mb = c->bary.dm;
        const DevMesh& m = c->primal->dm;
        const int Tb = int(c->bary.T);
        const int nqblk = (m.T + 255) / 256;
        const unsigned nx = unsigned((N + 255) / 256);
        const size_t nn = size_t(N) * size_t(N);
        const unsigned gsc = unsigned(std::min<size_t>((nn + 255) / 256, 65536));
        auto build_k = [&](double kr, double ki) {   // K_BC(kr + j ki) into w.Tbc
            fill_zero_bytes(w.Tbc, nn * 16, stream);
            for (int ch = 0; ch < pl.nchunks; ++ch) {
                const int c0 = ch * pl.chunk, c1 = std::min(Tb, c0 + pl.chunk), np = c1 - c0;
                const size_t nblk = size_t((np + K_PB - 1) / K_PB) * size_t(nqblk);
                EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "calderon_cfie_assemble: chunk too large");
                if (ki != 0.0)
                    hipLaunchKernelGGL(k_rows_kernel<true>, dim3(unsigned(nblk)), dim3(256), 0, stream, mb, m, kr, ki,
                                       static_cast<double2*>(w.W), c0, np, nqblk);
                else
                    hipLaunchKernelGGL(k_rows_kernel<false>, dim3(unsigned(nblk)), dim3(256), 0, stream, mb, m, kr,
                                       ki, static_cast<double2*>(w.W), c0, np, nqblk);
                if (L.nm[size_t(ch)] > 0)
                    hipLaunchKernelGGL(kbc_test_kernel, dim3(nx, unsigned(L.nm[size_t(ch)])), dim3(256), 0, stream,
                                       w.ml + L.m0[size_t(ch)], w.mptr + L.mp0[size_t(ch)], w.rows, w.coef,
                                       static_cast<const double2*>(w.W), w.Tbc, N);
            }
            if (verbose()) {
                EFIE_HIP_CHECK(hipStreamSynchronize(stream));
                std::fprintf(stderr, "[efie] cfie K_BC(%g%+gj) t=%.3f\n", kr, ki, now_s());
                std::fflush(stderr);
            }
        };
        const unsigned gr = unsigned((N + 255) / 256);
        // M = eta (-G^T / 2 - K_BC(k))
        build_k(k, 0.0);
        if (K_out) EFIE_HIP_CHECK(hipMemcpyAsync(K_out, w.Tbc, nn * 16, hipMemcpyDeviceToDevice, stream));
        hipLaunchKernelGGL(scale_c_kernel, dim3(gsc), dim3(256), 0, stream, w.Tbc, static_cast<double2*>(M), -eta, nn);
        hipLaunchKernelGGL(add_csr_kernel, dim3(gr), dim3(256), 0, stream, d.gt_ptr, d.gt_idx, d.gt_val, d.n_order, N,
                           -0.5 * eta, static_cast<double2*>(M));
        // M~ = eta (-G^T / 2 + K_BC(k~)), transposed in place: its rows are the
        // right-hand sides of G Q^T = M~^T
        build_k(kt_re, kt_im);
        if (Kt_out) EFIE_HIP_CHECK(hipMemcpyAsync(Kt_out, w.Tbc, nn * 16, hipMemcpyDeviceToDevice, stream));
        hipLaunchKernelGGL(scale_c_kernel, dim3(gsc), dim3(256), 0, stream, w.Tbc, w.Tbc, eta, nn);
        hipLaunchKernelGGL(add_csr_kernel, dim3(gr), dim3(256), 0, stream, d.gt_ptr, d.gt_idx, d.gt_val, d.n_order, N,
                           -0.5 * eta, w.Tbc);
        {
            const int nt = (N + 31) / 32;
            const size_t npairs = size_t(nt) * size_t(nt + 1) / 2;
            EFIE_REQUIRE(npairs < (size_t(1) << 31), EFIE_ERR_ARG, "calderon_cfie_assemble: N too large");
            hipLaunchKernelGGL(transpose_inplace_kernel, dim3(unsigned(npairs)), dim3(256), 0, stream, w.Tbc, N, nt);
        }
        // Q = M~ G^-T: row s of Q solves G y = row s of M~
        const double worst =
            pl.vsz == 8
                ? cald_gram_solve<float2>(d, w, pl, N, tol, maxit, static_cast<double2*>(Q), w.Tbc, true, stream)
                : cald_gram_solve<double2>(d, w, pl, N, tol, maxit, static_cast<double2*>(Q), w.Tbc, true, stream);
        if (relres) *relres = worst;
        EFIE_HIP_CHECK(hipGetLastError());
        return worst <= tol ? int(EFIE_OK) : int(EFIE_NOT_CONVERGED);
    });
}

int efie_calderon_mfie_rhs_workspace_size(efie_calderon c, int64_t nrhs, size_t* bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c && bytes && nrhs >= 1, EFIE_ERR_ARG, "calderon_mfie_rhs_workspace_size: bad argument");
        *bytes = efie::a256(size_t(24) * size_t(nrhs)) + size_t(nrhs) * size_t(c->bary.N) * 16;
        return int(EFIE_OK);
    });
}

int efie_calderon_mfie_rhs(efie_calderon c, double k, const double* khat, const double* pol, int64_t nrhs, void* H,
                           void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE(c && khat && pol && H && ws, EFIE_ERR_ARG, "calderon_mfie_rhs: null argument");
        EFIE_REQUIRE(c->dev != nullptr, EFIE_ERR_STATE, "calderon_mfie_rhs: tables not uploaded");
        EFIE_REQUIRE(std::isfinite(k) && k > 0.0, EFIE_ERR_ARG, "calderon_mfie_rhs: need k > 0");
        EFIE_REQUIRE(nrhs >= 1 && nrhs * c->bary.N < (int64_t(1) << 31), EFIE_ERR_ARG, "calderon_mfie_rhs: bad nrhs");
        const size_t off = a256(size_t(24) * size_t(nrhs));
        EFIE_REQUIRE(ws_bytes >= off + size_t(nrhs) * size_t(c->bary.N) * 16, EFIE_ERR_ARG,
                     "calderon_mfie_rhs: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "calderon_mfie_rhs: ws not aligned");
        double* kxp = static_cast<double*>(ws);
        auto* Vb = reinterpret_cast<double2*>(static_cast<char*>(ws) + off);
        const int S = int(nrhs);
        hipLaunchKernelGGL(cross3_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, khat, pol, kxp, S);
        const int code = efie_excite_planewave(&c->bary, k, khat, kxp, nrhs, 1.0, Vb, stream);
        if (code != EFIE_OK) return code;
        const DevCald d = dev_cald(*c);
        const size_t tot = size_t(c->N) * size_t(S);
        hipLaunchKernelGGL(bc_contract_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, stream, d, Vb, S,
                           static_cast<double2*>(H));
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

}  // extern "C"

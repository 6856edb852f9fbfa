// Device bodies of the atomic-free two-pass assembly (see assemble.hip for the
// scheme): pass 1 writes every pair value of a chunk of test triangles into
// rows W[p][i][n][side], pass 2 adds the rows of each RWG's two triangles into Z,
// the mirror completes Z = U + U^T.  The single-mesh kernels (assemble.hip) and the
// batched work-queue kernels (batch.hip) call the same bodies, so a batched
// matrix is bit-identical to the single-mesh one.
#pragma once

#include <hip/hip_runtime.h>

#include "efie_internal.h"
#include "pair_kernels.h"

namespace efie {

template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
    using T = float2;
};
template <>
struct Cplx<double> {
    using T = double2;
};

// Z = A T_A + P T_Phi: A = eta j k / (4 pi), P = eta / (j k) / (4 pi) = -j eta conj(k) / (|k|^2 4 pi)
inline Scale operator_scale(double kr, double ki, double eta) {
    Scale sc{};
    const double f = eta / (4.0 * PI);
    sc.ar = -f * ki;
    sc.ai = f * kr;
    const double k2 = kr * kr + ki * ki;
    sc.pr = -f * ki / k2;
    sc.pi = -f * kr / k2;
    return sc;
}

template <typename R>
__host__ __device__ Tables<R> tables_of(const DevMesh& m);
template <>
__host__ __device__ inline Tables<double> tables_of<double>(const DevMesh& m) {
    return {m.qx, m.qy, m.qz, m.qw, m.vx, m.vy, m.vz, m.cf, m.dv, m.q3x, m.q3y, m.q3z, m.q3w};
}
template <>
__host__ __device__ inline Tables<float> tables_of<float>(const DevMesh& m) {
    return {m.qx32, m.qy32, m.qz32, m.qw32, m.vx32, m.vy32, m.vz32, m.cf32, m.dv32,
            m.q3x32, m.q3y32, m.q3z32, m.q3w32};
}

// pass 1, one block (FAR_BLOCK threads) of logical index `logical` = (group of
// FAR_PB test triangles of the chunk, 256 source triangles).  A block takes FAR_PB
// test triangles against its source triangles: the source triangles' tables, read
// for the first, are cache hits for the others.  UPPER: only the far pairs with
// source triangle q > p are written; the entries of the pairs q < p are left
// unwritten and those of near pairs to the near rows (the reader takes only the
// entries of triangles q >= p and restores the other half from the symmetry of
// the operator).
template <typename R, bool CK, bool UPPER>
__device__ __forceinline__ void far_rows_block(const DevMesh& m, const Tables<R>& tb, R kphase, R ki, const Scale& sc,
                                               typename Cplx<R>::T* __restrict__ W, int c0, int np, int nqblk,
                                               int logical) {
    using C2 = typename Cplx<R>::T;
    const int pg = logical / nqblk, qb = logical - pg * nqblk;
    const int q = qb * FAR_BLOCK + int(threadIdx.x);
    const int T = m.T;
    if (q >= T) return;
    const size_t N = size_t(m.N);
    const int pl1 = min(np, (pg + 1) * FAR_PB);
    for (int pl = pg * FAR_PB; pl < pl1; ++pl) {
        const int p = c0 + pl;
        C2* rows = W + size_t(pl) * 3 * 2 * N;
        auto put = [&](int i, int j, R re, R im) {
            const size_t n = size_t(m.te[j * T + q]);
            const int side = tb.cf[j * T + q] > R(0) ? 0 : 1;
            rows[(size_t(i) * N + n) * 2 + side] = C2{re, im};
        };
        if (UPPER && q < p) continue;
        const bool near = is_near(m, p, q);
        if (UPPER && near) continue;
        if (near) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) put(i, j, R(0), R(0));
            continue;
        }
        far_pair_emit<R, CK, false>(m, tb, p, q, kphase, ki, sc, put, put);
    }
}

// the ordered near pair e = (p, q) with p in the chunk [c0, c1): its values replace
// the zeros pass 1 wrote (FP64 arithmetic, all nine entries).  upper: pairs with
// q < p are not written and the diagonal blocks (q = p) are halved.
template <typename R>
__device__ __forceinline__ void near_rows_one(const DevMesh& m, double kr, double ki, const Scale& sc,
                                              typename Cplx<R>::T* __restrict__ W, int c0, int c1, int e, int upper) {
    using C2 = typename Cplx<R>::T;
    const int p = m.near_p[e], q = m.near_q[e];
    if (p < c0 || p >= c1) return;
    if (upper && q < p) return;
    const double f = upper && q == p ? 0.5 : 1.0;
    const int T = m.T;
    const size_t N = size_t(m.N);
    C2* rows = W + size_t(p - c0) * 3 * 2 * N;
    auto put = [&](int i, int j, double re, double im) {
        const size_t n = size_t(m.te[j * T + q]);
        const int side = m.cf[j * T + q] > 0.0 ? 0 : 1;
        rows[(size_t(i) * N + n) * 2 + side] = C2{R(f * re), R(f * im)};
    };
    near_pair_emit<false>(m, e, kr, ki, sc, put, put);
}

// pass 2, one block (256 threads) of index blk = (test triangle p of the chunk,
// local edge i) -> RWG row mm; the block of mm's T+ adds both triangles' rows when
// both are in the chunk, so every row is updated by one block per chunk.  UPPER:
// the rows hold the pairs with source triangle q >= p only (q = p halved); side t
// of RWG n enters the row of test triangle p only where its triangle et[t N + n]
// >= p, and the result is the U of Z = U + U^T
template <typename R, bool UPPER>
__device__ __forceinline__ void gather_rows_block(const DevMesh& m, const typename Cplx<R>::T* __restrict__ W, int c0,
                                                  int c1, typename Cplx<R>::T* __restrict__ Z, int blk) {
    using C2 = typename Cplx<R>::T;
    const int pl = blk / 3, i = blk - 3 * pl;
    const int p = c0 + pl;
    const int T = m.T, N = m.N;
    const int mm = m.te[i * T + p];
    const int tp = m.et[mm], tm = m.et[N + mm];
    const int ip = m.el[mm], im = m.el[N + mm];
    const bool in_p = tp >= c0 && tp < c1, in_m = tm >= c0 && tm < c1;
    if (p != tp && in_p) return;          // the T+ block of this chunk owns the row
    // chunks run in increasing order: a row none of whose triangles lies in an earlier
    // chunk is written here for the first time (no zero fill, no read of Z)
    const bool first = tp >= c0 && tm >= c0;
    const C2* wp = in_p ? W + (size_t(tp - c0) * 3 + ip) * 2 * size_t(N) : nullptr;
    const C2* wm = in_m ? W + (size_t(tm - c0) * 3 + im) * 2 * size_t(N) : nullptr;
    C2* zr = Z + size_t(mm) * N;
    // U elements per thread per step, all loads issued before the adds
    constexpr int U = 4;
    const int step = int(blockDim.x) * U;
    for (int n0 = threadIdx.x; n0 < N; n0 += step) {
        C2 acc[U], a[U], b[U], c[U], d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int n = n0 + u * int(blockDim.x);
            if (n < N) {
                acc[u] = first ? C2{0, 0} : zr[n];
                if (UPPER) {
                    const int s0 = m.et[n], s1 = m.et[N + n];   // source triangles of the two sides
                    a[u] = b[u] = c[u] = d[u] = C2{0, 0};
                    if (wp && s0 >= tp) a[u] = wp[2 * n];
                    if (wp && s1 >= tp) b[u] = wp[2 * n + 1];
                    if (wm && s0 >= tm) c[u] = wm[2 * n];
                    if (wm && s1 >= tm) d[u] = wm[2 * n + 1];
                } else {
                    if (wp) { a[u] = wp[2 * n]; b[u] = wp[2 * n + 1]; }
                    if (wm) { c[u] = wm[2 * n]; d[u] = wm[2 * n + 1]; }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int n = n0 + u * int(blockDim.x);
            if (n < N) {
                if (wp) { acc[u].x += a[u].x + b[u].x; acc[u].y += a[u].y + b[u].y; }
                if (wm) { acc[u].x += c[u].x + d[u].x; acc[u].y += c[u].y + d[u].y; }
                zr[n] = acc[u];
            }
        }
    }
}

// Z <- Z + Z^T in place (N x N) for the pair k of mirror 32 x 32 tiles (bi <= bj,
// numbered row by row of the upper triangle of tiles), both read into LDS before
// either is written; one block of 256 threads
template <typename C2>
__device__ __forceinline__ void mirror_add_block(C2* __restrict__ Z, int N, int nt, long long k) {
    __shared__ C2 a[32][33], b[32][33];
    // tile row bi starts at S(bi) = bi nt - bi (bi - 1) / 2: the root of S(r) = k,
    // corrected for its rounding
    auto S = [&](long long r) { return r * nt - r * (r - 1) / 2; };
    const double b2 = 2.0 * nt + 1.0;
    long long bi = (long long)((b2 - sqrt(b2 * b2 - 8.0 * double(k))) * 0.5);
    bi = bi < 0 ? 0 : (bi > nt - 1 ? nt - 1 : bi);
    while (bi > 0 && S(bi) > k) --bi;
    while (bi + 1 < nt && S(bi + 1) <= k) ++bi;
    const int bj = int(bi + (k - S(bi)));
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = int(bi) * 32 + r, j = bj * 32 + tx;
        const int i2 = bj * 32 + r, j2 = int(bi) * 32 + tx;
        if (i < N && j < N) a[r][tx] = Z[size_t(i) * N + j];
        if (i2 < N && j2 < N) b[r][tx] = Z[size_t(i2) * N + j2];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = int(bi) * 32 + r, j = bj * 32 + tx;
        if (i < N && j < N) {   // (i, j) += (j, i): element (r, tx) of a plus element (tx, r) of b
            const C2 u = a[r][tx], v = b[tx][r];
            Z[size_t(i) * N + j] = C2{u.x + v.x, u.y + v.y};
        }
        if (bi != bj) {
            const int i2 = bj * 32 + r, j2 = int(bi) * 32 + tx;
            if (i2 < N && j2 < N) {
                const C2 u = b[r][tx], v = a[tx][r];
                Z[size_t(i2) * N + j2] = C2{u.x + v.x, u.y + v.y};
            }
        }
    }
}

}  // namespace efie

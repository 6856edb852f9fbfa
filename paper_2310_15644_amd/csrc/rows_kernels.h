// Device bodies of the pair rows W[p][i][n][side] of a chunk of test triangles
// (every pair value, the source RWG n and its side 0/1 = the source triangle is
// n's T+ / T-), the first step of the Calderon build, and helpers shared with the
// tile assembly: the operator scale factors and the quadrature tables of a mesh.
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

// the far pair rows, one block (FAR_BLOCK threads) of logical index `logical` = (group of
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

// the ordered near pair e = (p, q) with p in the chunk [c0, c1), by the group of
// NEAR_G lanes (lane g): its values replace the zeros the far rows wrote (FP64
// arithmetic, all nine entries).  upper: pairs with q < p are not written and the
// diagonal blocks (q = p) are halved.
template <typename R>
__device__ __forceinline__ void near_rows_one(const DevMesh& m, double kr, double ki, const Scale& sc,
                                              typename Cplx<R>::T* __restrict__ W, int c0, int c1, int e, int g,
                                              int upper) {
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
    near_pair_group<false>(m, e, g, kr, ki, sc, put, put);
}

}  // namespace efie

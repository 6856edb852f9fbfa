// Owner-computes assembly of Z by tiles of RWG functions: one block of 256
// threads owns a TS x TS tile of Z (rows r0.., columns c0.., r0 <= c0 by tiles)
// and writes it, and its mirror, exactly once.
//
//   * the tile's row RWGs have at most 2 TS distinct triangles P, its column RWGs
//     at most 2 TS distinct triangles Q (collected and deduplicated in LDS);
//   * every triangle pair of P x Q is evaluated once per tile, four row triangles
//     per step (one per wave) against all of Q (one per lane): far pairs by the
//     7 x 7 rule (or the adaptive 3 x 3 rule), near pairs copied from their FP64
//     blocks (computed once per assembly into NB by near_block_one for the pairs
//     q >= p, the others transposed; found by binary search in the ordered near
//     list);
//   * entry (m, n) adds its four pair values B[T_a(m)][T_b(n)][i_a][j_b] (a, b the
//     sides of the two RWGs) as their row triangles come up, steps in order and
//     sides in order: a fixed order, so the result is deterministic and does not
//     depend on timing; the diagonal tiles compute m <= n only, and every tile
//     writes (m, n) and (n, m) with the same value, so Z = Z^T exactly.
// No workspace rows and no atomics: Z is written once (and NB, n_near x 9
// values, is the only scratch).  The pairs per tile depend on how compact the
// tile's RWGs are on the surface: with vertex ids in a spatially coherent order
// (RWGs are numbered lexicographically by their vertex ids) a 64-RWG tile touches
// about 57 triangles, so the tiles evaluate about 1.8 times the T^2 / 2 pairs of
// the symmetric operator.
#pragma once

#include <hip/hip_runtime.h>

#include "efie_internal.h"
#include "pair_kernels.h"
#include "rows_kernels.h"

namespace efie {

template <typename R>
struct TileCfg;
template <>
struct TileCfg<float> {
    static constexpr int TS = 64;   // complex64: 64 x 64 tiles, 16 accumulators per thread
};
template <>
struct TileCfg<double> {
    static constexpr int TS = 32;   // complex128: 32 x 32 tiles (the pair code's registers)
};

template <typename R>
struct TileLds {
    static constexpr int TS = TileCfg<R>::TS, NC = 2 * TS;
    using C2 = typename Cplx<R>::T;
    int cand[2][NC];    // [0] rows, [1] columns: triangle of (RWG, side), -1 past the end
    int first[2][NC];   // first position holding the same triangle
    int pos[2][NC];     // unique triangles before this position
    int uniq[2][NC];    // the distinct triangles
    int loc[2][NC];     // position of (RWG, side)'s triangle in uniq
    int el[2][NC];      // local edge index of the RWG in that triangle
    int nu[2];
    // the pair values of one step: wave w's row triangle against every column
    // triangle, [w][column triangle][3 i + j]; reused for the mirror at the end
    C2 val[4][NC][9];
};
static_assert(sizeof(typename Cplx<float>::T) * 4 * 128 * 9 >= sizeof(typename Cplx<float>::T) * 64 * 65,
              "the mirror staging fits the pair values");
static_assert(sizeof(typename Cplx<double>::T) * 4 * 64 * 9 >= sizeof(typename Cplx<double>::T) * 32 * 33,
              "the mirror staging fits the pair values");

// ordered near pair index of (p, q), -1 if absent: binary search in the list sorted
// by (p, q)
__device__ inline int find_near(const DevMesh& m, int p, int q) {
    int lo = 0, hi = m.n_near;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int mp = m.near_p[mid], mq = m.near_q[mid];
        if (mp < p || (mp == p && mq < q)) lo = mid + 1;
        else hi = mid;
    }
    return (lo < m.n_near && m.near_p[lo] == p && m.near_q[lo] == q) ? lo : -1;
}

// NB[9 e + 3 i + j]: the FP64 block of ordered near pair e = (p, q), q >= p (the
// others are not written), stored in the precision of Z; by the group of NEAR_G
// lanes, lane g
template <typename R>
__device__ __forceinline__ void near_block_one(const DevMesh& m, double kr, double ki, const Scale& sc,
                                               typename Cplx<R>::T* __restrict__ NB, int e, int g) {
    using C2 = typename Cplx<R>::T;
    if (m.near_q[e] < m.near_p[e]) return;
    C2* out = NB + size_t(e) * 9;
    auto put = [&](int i, int j, double re, double im) { out[3 * i + j] = C2{R(re), R(im)}; };
    near_pair_group<false>(m, e, g, kr, ki, sc, put, put);
}

// (bi, bj), bi <= bj, of tile k numbered row by row of the upper triangle of nt x nt
__device__ inline void tile_decode(long long k, int nt, int& bi_out, int& bj_out) {
    auto S = [&](long long r) { return r * nt - r * (r - 1) / 2; };
    const double b2 = 2.0 * nt + 1.0;
    long long bi = (long long)((b2 - sqrt(b2 * b2 - 8.0 * double(k))) * 0.5);
    bi = bi < 0 ? 0 : (bi > nt - 1 ? nt - 1 : bi);
    while (bi > 0 && S(bi) > k) --bi;
    while (bi + 1 < nt && S(bi + 1) <= k) ++bi;
    bi_out = int(bi);
    bj_out = int(bi + (k - S(bi)));
}

template <typename R>
inline long long tile_count(int N) {
    const long long nt = (N + TileCfg<R>::TS - 1) / TileCfg<R>::TS;
    return nt * (nt + 1) / 2;
}

// the tile k of Z (one block of 256 threads = 4 waves; L in LDS, free again on
// return).  Step s: wave w takes row triangle 4 s + w (wave-uniform, so its
// quadrature data are scalar loads) against every column triangle (one per lane,
// a second pass for lanes past 64); then every thread adds, for the entries it
// owns (entry tid + 256 u: for 64-wide tiles column = lane, row = w + 4 u), the
// values of the step's row triangles, sides in order.  The accumulators stay in
// registers; the pair values pass through LDS.
template <typename R, bool CK>
__device__ __forceinline__ void tile_block(const DevMesh& m, const Tables<R>& tb, R kphase, R ki, const Scale& sc,
                                           const typename Cplx<R>::T* __restrict__ NB,
                                           typename Cplx<R>::T* __restrict__ Z, long long k, TileLds<R>& L) {
    using C2 = typename Cplx<R>::T;
    constexpr int TS = TileCfg<R>::TS, NC = 2 * TS, NE = TS * TS / 256;
    const int N = m.N, tid = int(threadIdx.x);
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nt = (N + TS - 1) / TS;
    int bi, bj;
    tile_decode(k, nt, bi, bj);
    const int r0 = bi * TS, c0 = bj * TS;
    const int nr = min(TS, N - r0), nc = min(TS, N - c0);
    const bool diag = bi == bj;
    // the triangles of the rows' and the columns' RWGs, both sides
    for (int t = tid; t < 2 * NC; t += 256) {
        const int ww = t / NC, x = t - ww * NC;
        const int e = x >> 1, sd = x & 1;
        const int base = ww ? c0 : r0, cnt = ww ? nc : nr;
        L.cand[ww][x] = e < cnt ? m.et[sd * N + base + e] : -1;
        L.el[ww][x] = e < cnt ? m.el[sd * N + base + e] : 0;
    }
    __syncthreads();
    for (int t = tid; t < 2 * NC; t += 256) {
        const int ww = t / NC, x = t - ww * NC;
        const int v = L.cand[ww][x];
        int f = x;
        if (v >= 0)
            for (int y = 0; y < x; ++y)
                if (L.cand[ww][y] == v) {
                    f = y;
                    break;
                }
        L.first[ww][x] = f;
    }
    __syncthreads();
    for (int t = tid; t < 2 * NC; t += 256) {
        const int ww = t / NC, x = t - ww * NC;
        int c = 0;
        for (int y = 0; y < x; ++y) c += (L.cand[ww][y] >= 0 && L.first[ww][y] == y) ? 1 : 0;
        L.pos[ww][x] = c;
        if (x == NC - 1) L.nu[ww] = c + ((L.cand[ww][x] >= 0 && L.first[ww][x] == x) ? 1 : 0);
    }
    __syncthreads();
    for (int t = tid; t < 2 * NC; t += 256) {
        const int ww = t / NC, x = t - ww * NC;
        const int v = L.cand[ww][x];
        if (v >= 0 && L.first[ww][x] == x) L.uniq[ww][L.pos[ww][x]] = v;
        L.loc[ww][x] = v >= 0 ? L.pos[ww][L.first[ww][x]] : -1;
    }
    __syncthreads();
    const int nP = L.nu[0], nQ = L.nu[1];
    // complex64: the lane's first column triangle's 7-point rule stays in
    // registers for every step (complex128 has no registers to spare)
    constexpr bool CACHE = sizeof(R) == 4;
    R pre[4][NQ];
    if (CACHE) {
        const int qq = lane < nQ ? L.uniq[1][lane] : 0;
#pragma unroll
        for (int b = 0; b < NQ; ++b) {
            pre[0][b] = tb.qx[b * m.T + qq];
            pre[1][b] = tb.qy[b * m.T + qq];
            pre[2][b] = tb.qz[b * m.T + qq];
            pre[3][b] = tb.qw[b * m.T + qq];
        }
    }
    C2 acc[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) acc[u] = C2{R(0), R(0)};
    // 64-wide tiles: the rows of a thread's entries (r = w + 4 u) are wave-uniform,
    // so where their row triangles come up is read once, packed as
    // 16 loc + 3 el (loc = 4 step + slot; -16: row past the end), and tested with
    // scalar branches; the column side (c = lane) is per lane, read once too
    constexpr bool UNIFORM_ROWS = TS == 64;
    int rinfo[UNIFORM_ROWS ? NE : 1][2];
    int cidx[2] = {0, 0};   // element of the lane's column side sb in one slot of L.val
    if (UNIFORM_ROWS) {
#pragma unroll
        for (int u = 0; u < (UNIFORM_ROWS ? NE : 1); ++u) {
            const int r = w + 4 * u;
#pragma unroll
            for (int sa = 0; sa < 2; ++sa)
                rinfo[u][sa] = __builtin_amdgcn_readfirstlane(
                    r < nr ? 16 * L.loc[0][2 * r + sa] + 3 * L.el[0][2 * r + sa] : -16);
        }
        // columns past the end read element 0 (valid LDS) into entries never written
#pragma unroll
        for (int sb = 0; sb < 2; ++sb)
            cidx[sb] = lane < nc ? 9 * L.loc[1][2 * lane + sb] + L.el[1][2 * lane + sb] : 0;
    }
    for (int s = 0; 4 * s < nP; ++s) {
        const int pi = 4 * s + w;
        if (pi < nP) {
            const int p = __builtin_amdgcn_readfirstlane(L.uniq[0][pi]);
            for (int ql = lane; ql < nQ; ql += 64) {
                const int q = L.uniq[1][ql];
                C2* out = L.val[w][ql];
                if (is_near(m, p, q)) {
                    // the blocks are stored for q >= p; (p, q) with q < p is the
                    // transpose of (q, p), the operator being symmetric
                    const bool up = q >= p;
                    const int e = up ? find_near(m, p, q) : find_near(m, q, p);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            out[3 * i + j] = e >= 0 ? NB[size_t(e) * 9 + (up ? 3 * i + j : 3 * j + i)] : C2{R(0), R(0)};
                } else {
                    auto put = [&](int i, int j, R re, R im) { out[3 * i + j] = C2{re, im}; };
                    if (CACHE && ql == lane && !(m.far3 > 0.0 && far3_pair(m, p, q)))
                        far_pair_rule<NQ, R, CK, false, true>(m, tb, tb.qx, tb.qy, tb.qz, tb.qw, p, q, kphase, ki, sc,
                                                              put, put, pre);
                    else
                        far_pair_emit<R, CK, false>(m, tb, p, q, kphase, ki, sc, put, put);
                }
            }
        }
        __syncthreads();
        if (UNIFORM_ROWS) {
#pragma unroll
            for (int u = 0; u < (UNIFORM_ROWS ? NE : 1); ++u)
#pragma unroll
                for (int sa = 0; sa < 2; ++sa) {
                    const int info = rinfo[u][sa];
                    if ((info >> 6) != s) continue;
                    // slot (info >> 4) - 4 s: written with s so that the addresses
                    // are formed here, not kept for every (u, sa) across the steps
                    const int so = ((info >> 4) - 4 * s) * (NC * 9) + (info & 15);
#pragma unroll
                    for (int sb = 0; sb < 2; ++sb) {
                        const C2 v = (&L.val[0][0][0])[so + cidx[sb]];
                        acc[u].x += v.x;
                        acc[u].y += v.y;
                    }
                }
            __syncthreads();
            continue;
        }
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            const int r = e / TS, c = e - r * TS;
            if (r >= nr || c >= nc || (diag && r > c)) continue;
#pragma unroll
            for (int sa = 0; sa < 2; ++sa) {
                const int pl = L.loc[0][2 * r + sa] - 4 * s;
                if (pl < 0 || pl >= 4) continue;
                const int ei = 3 * L.el[0][2 * r + sa];
#pragma unroll
                for (int sb = 0; sb < 2; ++sb) {
                    const C2 v = L.val[pl][L.loc[1][2 * c + sb]][ei + L.el[1][2 * c + sb]];
                    acc[u].x += v.x;
                    acc[u].y += v.y;
                }
            }
        }
        __syncthreads();
    }
    // the tile, then its mirror through LDS (diagonal tiles: the entries above the
    // diagonal)
    C2(*st)[TS + 1] = reinterpret_cast<C2(*)[TS + 1]>(&L.val[0][0][0]);
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int e = tid + 256 * u;
        const int r = e / TS, c = e - r * TS;
        st[r][c] = acc[u];
        if (r < nr && c < nc && !(diag && r > c)) Z[size_t(r0 + r) * N + (c0 + c)] = acc[u];
    }
    __syncthreads();
    for (int e = tid; e < TS * TS; e += 256) {
        const int rr = e / TS, cc = e - rr * TS;   // Z row c0 + rr, column r0 + cc: entry (r0 + cc, c0 + rr)
        if (cc < nr && rr < nc && !(diag && cc >= rr)) Z[size_t(c0 + rr) * N + (r0 + cc)] = st[cc][rr];
    }
    __syncthreads();
}

}  // namespace efie

// Dense EFIE operator assembly on gfx950.
//
// Z_mn = eta (j k T_A + T_Phi / (j k)) over RWG functions (Galerkin matrices as
// in the paper's Sec. III, time factor e^{+j omega t} from its Sec. II eq. 5),
// (T_A)_mn = <f_m, G f_n>, (T_Phi)_mn = <div f_m, G div f_n>, G = exp(-jkR)/(4 pi R).
//
// Work decomposition.  One thread owns one triangle pair (p, q): it evaluates
// the 7 x 7 Green's function values of the pair, reduces them to the moments
//   M0 = sum W_a W_b G,   Md = sum W_a W_b G d_a,   Md' = sum W_a W_b G d'_b,
//   Mdd' = sum W_a W_b G (d_a . d'_b)
// (d, d' quadrature points relative to the triangle centroids), and forms the
// nine RWG half-function products from them:
//   T_A(i,j)   = c_i c'_j [Mdd' - u'_j . Md - u_i . Md' + (u_i . u'_j) M0],
//   T_Phi(i,j) = g_i g'_j M0,
// with u the vertex offsets, c = s l/(2A), g = s l/A.  The nine results are added
// to Z with atomics: every Z entry receives exactly four such contributions.
// The test triangle is uniform over a block (scalar loads), the source triangle
// varies across lanes (coalesced structure-of-arrays loads).
//
// Without atomics (efie_assemble_ws): owner-computes tiles (tile_kernels.h).  A
// block owns a tile of Z (64 x 64 RWGs in complex64, 32 x 32 in complex128, the
// tiles on and above the diagonal), evaluates every triangle pair between the
// triangles of its row RWGs and those of its column RWGs once, adds each entry's
// four pair values in a fixed order and writes the tile and its mirror: Z is
// written once, no workspace rows, no atomics, deterministic and exactly
// symmetric.  The near pairs' FP64 blocks are computed first (one thread per
// ordered near pair) into the caller's workspace, where the tiles read them.
// The pair rows W[p][i][n][side] of a chunk of test triangles (far_rows_kernel,
// near_rows_kernel: the pairs with source triangle q >= p, q = p halved) remain
// the first step of the Calderon build, which contracts rows without forming the
// matrix (pair_rows_chunk).
//
// Near pairs (a shared vertex, or centroids closer than the near factor times the
// larger longest edge; decided on the device as on the host) are skipped by the
// far kernels and handled by the near kernels in FP64: the smooth part (exp(-jkR)-1)/(4 pi R) with the same
// 7 x 7 rule, and the 1/(4 pi R) part with closed-form inner integrals over the
// source triangle (Wilton et al., IEEE TAP 32(3) 1984; Graglia, IEEE TAP 41(10)
// 1993) and the 7-point rule over the test triangle, averaged with the
// transposed (q, p) block so that Z = Z^T exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "efie_internal.h"
#include "pair_kernels.h"
#include "rows_kernels.h"
#include "tile_kernels.h"

namespace efie {

template <typename R, bool CK, bool PARTS>
__global__ __launch_bounds__(FAR_BLOCK) void far_pairs_kernel(DevMesh m, Tables<R> tb, R kphase, R ki,
                                                              Scale sc, void* Z, void* Z2, int nqblk) {
    const int p = blockIdx.x / nqblk;
    const int q = (blockIdx.x - p * nqblk) * FAR_BLOCK + threadIdx.x;
    if (q >= m.T) return;
    far_pair<R, CK, PARTS>(m, tb, p, q, kphase, ki, sc, Z, Z2);
}

template <typename ZT, bool PARTS>
__global__ __launch_bounds__(128) void near_pairs_kernel(DevMesh m, double kr, double ki, Scale sc, void* Z,
                                                         void* Z2) {
    // a group of NEAR_G lanes per ordered near pair
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = t / NEAR_G;
    if (e >= m.n_near) return;
    near_pair<ZT, PARTS>(m, e, t % NEAR_G, kr, ki, sc, Z, Z2);
}

// the pair rows of a chunk of test triangles (the first step of the Calderon
// build): the bodies live in rows_kernels.h
template <typename R, bool CK, bool UPPER>
__global__ __launch_bounds__(FAR_BLOCK) void far_rows_kernel(DevMesh m, Tables<R> tb, R kphase, R ki, Scale sc,
                                                             typename Cplx<R>::T* __restrict__ W, int c0, int np,
                                                             int nqblk) {
    // blocks are dealt to the 8 XCDs round-robin: remap so that each XCD runs the
    // blocks of consecutive test triangles, all blocks of one group together
    const int nblk = int(gridDim.x);
    const int xcd = int(blockIdx.x) & 7, idx = int(blockIdx.x) >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    const int logical = xcd * per + min(xcd, rem) + idx;
    far_rows_block<R, CK, UPPER>(m, tb, kphase, ki, sc, W, c0, np, nqblk, logical);
}

template <typename R>
__global__ __launch_bounds__(128) void near_rows_kernel(DevMesh m, double kr, double ki, Scale sc,
                                                        typename Cplx<R>::T* __restrict__ W, int c0, int c1, int e0,
                                                        int e1, int upper) {
    // [e0, e1): ordered near pairs, or with upper positions in the list of the
    // pairs with q >= p
    const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
    const int x = e0 + t / NEAR_G;
    if (x >= e1) return;
    near_rows_one<R>(m, kr, ki, sc, W, c0, c1, upper ? m.near_up[x] : x, t % NEAR_G, upper);
}

// the FP64 blocks of every ordered near pair, in the precision of Z
template <typename R>
__global__ __launch_bounds__(256) void near_blocks_kernel(DevMesh m, double kr, double ki, Scale sc,
                                                          typename Cplx<R>::T* __restrict__ NB) {
    const int t = int(blockIdx.x) * 256 + int(threadIdx.x);
    const int u = t / NEAR_G;   // the pairs with q >= p only
    if (u >= m.n_up) return;
    near_block_one<R>(m, kr, ki, sc, NB, m.near_up[u], t % NEAR_G);
}

// one block per tile of Z (tiles on and above the diagonal); complex64: three
// blocks per CU (the LDS allows three), so at most 168 VGPRs
template <typename R, bool CK>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 3 : 1) void tile_kernel(DevMesh m, Tables<R> tb, R kphase, R ki, Scale sc,
                                                   const typename Cplx<R>::T* __restrict__ NB,
                                                   typename Cplx<R>::T* __restrict__ Z) {
    __shared__ TileLds<R> L;
    tile_block<R, CK>(m, tb, kphase, ki, sc, NB, Z, (long long)blockIdx.x, L);
}

template <typename R>
__global__ void fill_zero_kernel(R* p, size_t n) {
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = R(0);
}

void fill_zero_bytes(void* p, size_t bytes, hipStream_t s) {
    // bytes is a multiple of 8 for every buffer this library clears
    size_t n = bytes / 8;
    int blocks = int(std::min<size_t>((n + 255) / 256, 65536));
    if (n) hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<double*>(p), n);
}

namespace {

template <typename R, bool PARTS>
void launch_far(const DevMesh& m, double kr, double ki, const Scale& sc, void* Z, void* Z2, hipStream_t s) {
    const int nqblk = (m.T + FAR_BLOCK - 1) / FAR_BLOCK;
    const size_t nblk = size_t(m.T) * nqblk;
    EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "assemble: mesh too large for one launch");
    const bool ck = ki != 0.0;
    const R kphase = std::is_same<R, float>::value ? R(kr / (2.0 * PI)) : R(kr);
    prof_begin(PROF_FAR, s);
    if (ck)
        hipLaunchKernelGGL((far_pairs_kernel<R, true, PARTS>), dim3(unsigned(nblk)), dim3(FAR_BLOCK), 0, s, m,
                           tables_of<R>(m), kphase, R(ki), sc, Z, Z2, nqblk);
    else
        hipLaunchKernelGGL((far_pairs_kernel<R, false, PARTS>), dim3(unsigned(nblk)), dim3(FAR_BLOCK), 0, s, m,
                           tables_of<R>(m), kphase, R(ki), sc, Z, Z2, nqblk);
    prof_end(PROF_FAR, s);
}

// With the pairs q >= p only, the far kernel leaves the entries of near pairs
// alone, so a chunk's near pairs (few, long-running threads) run beside its far
// pairs on a second stream: forked from the caller's stream before the far kernel,
// so that they follow whatever read the workspace before, and joined before
// anything reads the chunk's rows.  One side stream and event pair per device,
// created on first use and kept until the process ends; host threads that
// assemble at once take turns enqueueing (the pair of events is shared).
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::mutex mu;
};

static SideStream& side_stream() {
    constexpr int MAXDEV = 64;
    static SideStream ss[MAXDEV];
    static std::mutex create_mu;
    int dev = 0;
    EFIE_HIP_CHECK(hipGetDevice(&dev));
    EFIE_REQUIRE(dev >= 0 && dev < MAXDEV, EFIE_ERR_STATE, "side stream: device index out of range");
    SideStream& x = ss[dev];
    std::lock_guard<std::mutex> g(create_mu);
    if (!x.s) {
        EFIE_HIP_CHECK(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
        EFIE_HIP_CHECK(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
        EFIE_HIP_CHECK(hipEventCreateWithFlags(&x.join, hipEventDisableTiming));
    }
    return x;
}

// launch near(stream) beside far(stream) as above; returns after both are enqueued,
// with the caller's stream s waiting for the near pairs (timed as PROF_ROWS_NEAR on
// the side stream)
template <typename NearF, typename FarF>
static void near_beside_far(hipStream_t s, NearF near, FarF far) {
    SideStream& x = side_stream();
    std::lock_guard<std::mutex> g(x.mu);
    EFIE_HIP_CHECK(hipEventRecord(x.fork, s));
    EFIE_HIP_CHECK(hipStreamWaitEvent(x.s, x.fork, 0));
    prof_begin(PROF_ROWS_NEAR, x.s);
    near(x.s);
    prof_end(PROF_ROWS_NEAR, x.s);
    EFIE_HIP_CHECK(hipEventRecord(x.join, x.s));
    far(s);
    EFIE_HIP_CHECK(hipStreamWaitEvent(s, x.join, 0));
}

// Z by tiles: the near blocks into the workspace, then one block per tile (each
// launch bracketed for efie_prof_read)
template <typename R>
void launch_tiles(const DevMesh& m, double kr, double ki, const Scale& sc, void* Z, void* ws, size_t ws_bytes,
                  hipStream_t s) {
    using C2 = typename Cplx<R>::T;
    EFIE_REQUIRE(ws_bytes >= size_t(m.n_near) * 9 * sizeof(C2), EFIE_ERR_ARG,
                 "assemble_ws: workspace smaller than the near-pair blocks");
    const long long ntiles = tile_count<R>(m.N);
    EFIE_REQUIRE(ntiles < (1ll << 31), EFIE_ERR_ARG, "assemble_ws: N too large");
    C2* NB = static_cast<C2*>(ws);
    if (m.n_up > 0) {
        prof_begin(PROF_NEAR, s);
        hipLaunchKernelGGL(near_blocks_kernel<R>, dim3(unsigned((int64_t(m.n_up) * NEAR_G + 255) / 256)), dim3(256),
                           0, s, m, kr, ki, sc, NB);
        prof_end(PROF_NEAR, s);
    }
    const R kphase = std::is_same<R, float>::value ? R(kr / (2.0 * PI)) : R(kr);
    prof_begin(PROF_FAR, s);
    if (ki != 0.0)
        hipLaunchKernelGGL((tile_kernel<R, true>), dim3(unsigned(ntiles)), dim3(256), 0, s, m, tables_of<R>(m),
                           kphase, R(ki), sc, NB, static_cast<C2*>(Z));
    else
        hipLaunchKernelGGL((tile_kernel<R, false>), dim3(unsigned(ntiles)), dim3(256), 0, s, m, tables_of<R>(m),
                           kphase, R(ki), sc, NB, static_cast<C2*>(Z));
    prof_end(PROF_FAR, s);
}

template <typename ZT, bool PARTS>
void launch_near(const DevMesh& m, double kr, double ki, const Scale& sc, void* Z, void* Z2, hipStream_t s) {
    if (m.n_near == 0) return;
    prof_begin(PROF_NEAR, s);
    hipLaunchKernelGGL((near_pairs_kernel<ZT, PARTS>), dim3(unsigned((int64_t(m.n_near) * NEAR_G + 127) / 128)),
                       dim3(128), 0, s, m, kr, ki,
                       sc, Z, Z2);
    prof_end(PROF_NEAR, s);
}

}  // namespace


// The pair rows of test triangles [c0, c1): every pair value of Z = eta (j k T_A + T_Phi / (j k)) (far pairs in the storage precision,
// near pairs in FP64) into rows W[p - c0][i][n][side] of complex64 (dtype
// EFIE_C64) or complex128 elements.  Used by the Calderon build, which contracts
// these rows without forming the matrix.  upper: only the pairs with source
// triangle q > p, plus the halved diagonal blocks q = p (rows of U + D/2 for the
// split Z = U + U^T + D of the symmetric operator); the entries of triangles
// q < p are not written, and the reader must skip them.
void pair_rows_chunk(const DevMesh& m, double kr, double ki, double eta, int dtype, void* W, int c0, int c1,
                     const std::vector<int32_t>& near_p, const std::vector<int32_t>& near_up, bool upper,
                     hipStream_t s) {
    const Scale sc = operator_scale(kr, ki, eta);
    if (dtype == EFIE_C64) require_fp32_phase(m.diam, kr, "pair rows");
    const int nqblk = (m.T + FAR_BLOCK - 1) / FAR_BLOCK;
    const int np = c1 - c0;
    EFIE_REQUIRE(np >= 1 && size_t(np) * nqblk < (size_t(1) << 31), EFIE_ERR_ARG, "pair_rows_chunk: bad chunk");
    const bool ck = ki != 0.0;
    const dim3 g1(unsigned(size_t((np + FAR_PB - 1) / FAR_PB) * nqblk));
    int e0 = int(std::lower_bound(near_p.begin(), near_p.end(), c0) - near_p.begin());
    int e1 = int(std::lower_bound(near_p.begin(), near_p.end(), c1) - near_p.begin());
    if (upper) {   // the chunk's pairs with q >= p: a run of the increasing list near_up
        e0 = int(std::lower_bound(near_up.begin(), near_up.end(), e0) - near_up.begin());
        e1 = int(std::lower_bound(near_up.begin(), near_up.end(), e1) - near_up.begin());
    }
    auto run = [&](auto tag) {
        using R = decltype(tag);
        using C2 = typename Cplx<R>::T;
        const R kphase = std::is_same<R, float>::value ? R(kr / (2.0 * PI)) : R(kr);
        C2* w = static_cast<C2*>(W);
        auto far = [&](hipStream_t st) {
            if (ck && upper)
                hipLaunchKernelGGL((far_rows_kernel<R, true, true>), g1, dim3(FAR_BLOCK), 0, st, m, tables_of<R>(m),
                                   kphase, R(ki), sc, w, c0, np, nqblk);
            else if (ck)
                hipLaunchKernelGGL((far_rows_kernel<R, true, false>), g1, dim3(FAR_BLOCK), 0, st, m, tables_of<R>(m),
                                   kphase, R(ki), sc, w, c0, np, nqblk);
            else if (upper)
                hipLaunchKernelGGL((far_rows_kernel<R, false, true>), g1, dim3(FAR_BLOCK), 0, st, m, tables_of<R>(m),
                                   kphase, R(ki), sc, w, c0, np, nqblk);
            else
                hipLaunchKernelGGL((far_rows_kernel<R, false, false>), g1, dim3(FAR_BLOCK), 0, st, m, tables_of<R>(m),
                                   kphase, R(ki), sc, w, c0, np, nqblk);
        };
        auto near = [&](hipStream_t st) {
            hipLaunchKernelGGL((near_rows_kernel<R>), dim3(unsigned((int64_t(e1 - e0) * NEAR_G + 127) / 128)), dim3(128),
                               0, st, m, kr, ki, sc,
                               w, c0, c1, e0, e1, int(upper));
        };
        if (e1 <= e0) {
            far(s);
        } else if (upper) {
            near_beside_far(s, near, far);   // disjoint entries: see near_beside_far
        } else {
            far(s);                          // the far kernel zeroes the near entries first
            near(s);
        }
    };
    if (dtype == EFIE_C64) run(float{});
    else run(double{});
}

// ws != nullptr (and not parts): Z by tiles, the near blocks in that workspace
static void assemble_impl(const DevMesh& m, double kr, double ki, double eta, int dtype, void* Z, void* Z2, int parts,
                          hipStream_t s, void* ws, size_t ws_bytes, const std::vector<int32_t>* near_p) {
    const size_t N = size_t(m.N);
    const size_t esz = dtype == EFIE_C128 ? 16 : 8;
    if (dtype == EFIE_C64) require_fp32_phase(m.diam, kr, "assemble");
    if (!ws || parts) fill_zero_bytes(Z, N * N * esz, s);   // the tiles write every entry
    if (parts) fill_zero_bytes(Z2, N * N * esz, s);
    Scale sc{};
    if (parts) sc.ar = 1.0 / (4.0 * PI);
    else sc = operator_scale(kr, ki, eta);
    if (dtype == EFIE_C128) {
        if (parts) {
            launch_far<double, true>(m, kr, ki, sc, Z, Z2, s);
            launch_near<double, true>(m, kr, ki, sc, Z, Z2, s);
        } else {
            if (ws) {
                launch_tiles<double>(m, kr, ki, sc, Z, ws, ws_bytes, s);   // near pairs included
            } else {
                launch_far<double, false>(m, kr, ki, sc, Z, Z2, s);
                launch_near<double, false>(m, kr, ki, sc, Z, Z2, s);
            }
        }
    } else {
        if (parts) {
            launch_far<float, true>(m, kr, ki, sc, Z, Z2, s);
            launch_near<float, true>(m, kr, ki, sc, Z, Z2, s);
        } else {
            if (ws) {
                launch_tiles<float>(m, kr, ki, sc, Z, ws, ws_bytes, s);    // near pairs included
            } else {
                launch_far<float, false>(m, kr, ki, sc, Z, Z2, s);
                launch_near<float, false>(m, kr, ki, sc, Z, Z2, s);
            }
        }
    }
    EFIE_HIP_CHECK(hipGetLastError());
}

void assemble_into(const DevMesh& m, double kr, double ki, double eta, int dtype, void* Z, void* Z2, int parts,
                   hipStream_t s) {
    assemble_impl(m, kr, ki, eta, dtype, Z, Z2, parts, s, nullptr, 0, nullptr);
}

}  // namespace efie

extern "C" int efie_assemble(efie_mesh mesh, double k_re, double k_im, double eta, int dtype, void* Z, void* Z2,
                             int parts, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr && Z != nullptr, EFIE_ERR_ARG, "assemble: null argument");
        EFIE_REQUIRE(mesh->dev != nullptr, EFIE_ERR_STATE, "assemble: mesh tables not uploaded");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "assemble: bad dtype");
        EFIE_REQUIRE(!parts || Z2 != nullptr, EFIE_ERR_ARG, "assemble: parts mode needs Z2");
        EFIE_REQUIRE(std::isfinite(k_re) && std::isfinite(k_im) && k_im <= 0.0, EFIE_ERR_ARG,
                     "assemble: need finite k with Im k <= 0");
        EFIE_REQUIRE(parts || (k_re != 0.0 || k_im != 0.0), EFIE_ERR_ARG, "assemble: k = 0 needs parts mode");
        efie::assemble_into(mesh->dm, k_re, k_im, eta, dtype, Z, Z2, parts, stream);
        return int(EFIE_OK);
    });
}

extern "C" int efie_assemble_workspace_size(efie_mesh mesh, int dtype, size_t* min_bytes, size_t* full_bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr && min_bytes != nullptr && full_bytes != nullptr, EFIE_ERR_ARG,
                     "assemble_workspace_size: null argument");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "assemble_workspace_size: bad dtype");
        // the FP64 blocks of the ordered near pairs, stored in the precision of Z
        const size_t nb = std::max<size_t>(256, mesh->near_p.size() * 9 * (dtype == EFIE_C128 ? 16 : 8));
        *min_bytes = nb;
        *full_bytes = nb;
        return int(EFIE_OK);
    });
}

extern "C" int efie_assemble_ws(efie_mesh mesh, double k_re, double k_im, double eta, int dtype, void* Z, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr && Z != nullptr && ws != nullptr, EFIE_ERR_ARG, "assemble_ws: null argument");
        EFIE_REQUIRE(mesh->dev != nullptr, EFIE_ERR_STATE, "assemble_ws: mesh tables not uploaded");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "assemble_ws: bad dtype");
        EFIE_REQUIRE(std::isfinite(k_re) && std::isfinite(k_im) && k_im <= 0.0 && (k_re != 0.0 || k_im != 0.0),
                     EFIE_ERR_ARG, "assemble_ws: need finite nonzero k with Im k <= 0");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 15) == 0, EFIE_ERR_ARG, "assemble_ws: workspace not 16-byte aligned");
        efie::assemble_impl(mesh->dm, k_re, k_im, eta, dtype, Z, nullptr, 0, stream, ws, ws_bytes, &mesh->near_p);
        return int(EFIE_OK);
    });
}

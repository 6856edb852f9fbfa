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
// Near pairs (near mask bit set) are skipped by the far kernel and handled by
// near_pairs_kernel in FP64: the smooth part (exp(-jkR)-1)/(4 pi R) with the same
// 7 x 7 rule, and the 1/(4 pi R) part with closed-form inner integrals over the
// source triangle (Wilton et al., IEEE TAP 32(3) 1984; Graglia, IEEE TAP 41(10)
// 1993) and the 7-point rule over the test triangle, averaged with the
// transposed (q, p) block so that Z = Z^T exactly.
#include <hip/hip_runtime.h>

#include <cmath>

#include "efie_internal.h"
#include "pair_kernels.h"

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
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.n_near) return;
    near_pair<ZT, PARTS>(m, e, kr, ki, sc, Z, Z2);
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

template <typename R>
Tables<R> tables(const DevMesh& m);
template <>
Tables<double> tables<double>(const DevMesh& m) {
    return {m.qx, m.qy, m.qz, m.qw, m.vx, m.vy, m.vz, m.cf, m.dv};
}
template <>
Tables<float> tables<float>(const DevMesh& m) {
    return {m.qx32, m.qy32, m.qz32, m.qw32, m.vx32, m.vy32, m.vz32, m.cf32, m.dv32};
}

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
                           tables<R>(m), kphase, R(ki), sc, Z, Z2, nqblk);
    else
        hipLaunchKernelGGL((far_pairs_kernel<R, false, PARTS>), dim3(unsigned(nblk)), dim3(FAR_BLOCK), 0, s, m,
                           tables<R>(m), kphase, R(ki), sc, Z, Z2, nqblk);
    prof_end(PROF_FAR, s);
}

template <typename ZT, bool PARTS>
void launch_near(const DevMesh& m, double kr, double ki, const Scale& sc, void* Z, void* Z2, hipStream_t s) {
    if (m.n_near == 0) return;
    prof_begin(PROF_NEAR, s);
    hipLaunchKernelGGL((near_pairs_kernel<ZT, PARTS>), dim3((m.n_near + 127) / 128), dim3(128), 0, s, m, kr, ki,
                       sc, Z, Z2);
    prof_end(PROF_NEAR, s);
}

}  // namespace

void assemble_into(const DevMesh& m, double kr, double ki, double eta, int dtype, void* Z, void* Z2, int parts,
                   hipStream_t s) {
    const size_t N = size_t(m.N);
    const size_t esz = dtype == EFIE_C128 ? 16 : 8;
    fill_zero_bytes(Z, N * N * esz, s);
    if (parts) fill_zero_bytes(Z2, N * N * esz, s);
    Scale sc{};
    if (parts) {
        sc.ar = 1.0 / (4.0 * PI);
    } else {
        // A = eta j k / (4 pi),  P = eta / (j k) / (4 pi) = -j eta conj(k) / (|k|^2 4 pi)
        const double f = eta / (4.0 * PI);
        sc.ar = -f * ki;
        sc.ai = f * kr;
        const double k2 = kr * kr + ki * ki;
        sc.pr = -f * ki / k2;
        sc.pi = -f * kr / k2;
    }
    if (dtype == EFIE_C128) {
        if (parts) {
            launch_far<double, true>(m, kr, ki, sc, Z, Z2, s);
            launch_near<double, true>(m, kr, ki, sc, Z, Z2, s);
        } else {
            launch_far<double, false>(m, kr, ki, sc, Z, Z2, s);
            launch_near<double, false>(m, kr, ki, sc, Z, Z2, s);
        }
    } else {
        if (parts) {
            launch_far<float, true>(m, kr, ki, sc, Z, Z2, s);
            launch_near<float, true>(m, kr, ki, sc, Z, Z2, s);
        } else {
            launch_far<float, false>(m, kr, ki, sc, Z, Z2, s);
            launch_near<float, false>(m, kr, ki, sc, Z, Z2, s);
        }
    }
    EFIE_HIP_CHECK(hipGetLastError());
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

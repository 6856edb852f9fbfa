// Complex64 Y = X Z^T on FP32 matrix cores (MFMA), FP32 accumulation.
//
// The complex product is carried out as one real product ("4M": every complex
// multiply-add costs four real ones, 8 M n K flops in total):
//   A (M x 2n) = X viewed as floats,  A[s][2j+t] = (Re, Im)[t] X[s][j];
//   B (2n x 2n) built on the fly from the 2 x 2 real blocks of Z,
//     B[2j][2i] = Re Z[i][j], B[2j+1][2i] = -Im Z[i][j],
//     B[2j][2i+1] = Im Z[i][j], B[2j+1][2i+1] = Re Z[i][j];
//   C = A B is then Y viewed as floats, interleaved (re, im), row by row.
// So X and Y keep the ABI's interleaved complex64 layout and no operand is
// converted or copied.
//
// Tiling: a block of 256 threads (4 wavefronts, 2 x 2) owns a BM x BN tile of C
// (BM right-hand sides, BN/2 unknowns).  K is walked in chunks of KC complex
// elements staged in LDS; each wavefront issues v_mfma_f32_16x16x4f32 on 16 x 16
// sub-tiles (K = 4 reals = 2 complex elements per instruction).
// Operand layouts of v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l holds D[4*(l/16)+r][l%16].
#include <hip/hip_runtime.h>

#include "efie_internal.h"
#include "linalg.h"

namespace efie {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int KC>
__global__ __launch_bounds__(256) void cgemm_mfma_kernel(const float2* __restrict__ X, const float2* __restrict__ Z,
                                                         float2* __restrict__ Y, int M, int n) {
    constexpr int AP = 2 * KC + 4;     // floats per LDS row of the X tile (padded)
    constexpr int BNC = BN / 2;        // unknowns per tile
    constexpr int BP = KC + 1;         // float2 per LDS row of the Z tile (padded)
    constexpr int WM = BM / 2, WN = BN / 2;   // wavefront tile
    constexpr int TM = WM / 16, TN = WN / 16;
    __shared__ float As[BM * AP];
    __shared__ float2 Bs[BNC * BP];

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    // XCD-friendly order: consecutive block ids walk the right-hand-side tiles of
    // one column tile first, so blocks sharing a Z tile run close together.
    const int nbm = (M + BM - 1) / BM;
    const int bm = blockIdx.x % nbm, bn = blockIdx.x / nbm;
    const int s0 = bm * BM, i0 = bn * BNC;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int kq = lane >> 4;          // 0..3: real k within an instruction
    const int l16 = lane & 15;
    for (int j0 = 0; j0 < n; j0 += KC) {
        // stage X[s0 .. s0+BM)[j0 .. j0+KC) and Z[i0 .. i0+BNC)[j0 .. j0+KC)
        for (int e = tid; e < BM * KC; e += 256) {
            const int r = e / KC, jj = e % KC;
            const int s = s0 + r, j = j0 + jj;
            float2 v = (s < M && j < n) ? X[size_t(s) * n + j] : make_float2(0.f, 0.f);
            As[r * AP + 2 * jj] = v.x;
            As[r * AP + 2 * jj + 1] = v.y;
        }
        for (int e = tid; e < BNC * KC; e += 256) {
            const int r = e / KC, jj = e % KC;
            const int i = i0 + r, j = j0 + jj;
            Bs[r * BP + jj] = (i < n && j < n) ? Z[size_t(i) * n + j] : make_float2(0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < KC / 2; ++st) {
            const int kf = 4 * st + kq;        // real k index inside the chunk
            const int jj = kf >> 1, t = kf & 1;
            float av[TM], bv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) av[a] = As[(wm * WM + a * 16 + l16) * AP + kf];
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                const int col = wn * WN + b * 16 + l16;     // real column inside the tile
                const float2 z = Bs[(col >> 1) * BP + jj];
                const int u = col & 1;
                bv[b] = u == 0 ? (t == 0 ? z.x : -z.y) : (t == 0 ? z.y : z.x);
            }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    float* Yf = reinterpret_cast<float*>(Y);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int col = 2 * i0 + wn * WN + b * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = s0 + wm * WM + a * 16 + 4 * kq + r;
                if (row < M && col < 2 * n) Yf[size_t(row) * 2 * n + col] = acc[a][b][r];
            }
        }
}

bool cgemm_mfma_supported(int M, int n) { return M >= 1 && n >= 1; }

void cgemm_mfma(const void* X, const void* Z, void* Y, int M, int n, hipStream_t s) {
    constexpr int BM = 128, BN = 128, KC = 16;
    const int nbm = (M + BM - 1) / BM, nbn = (n + BN / 2 - 1) / (BN / 2);
    const size_t nblk = size_t(nbm) * nbn;
    EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "cgemm: problem too large");
    hipLaunchKernelGGL((cgemm_mfma_kernel<BM, BN, KC>), dim3(unsigned(nblk)), dim3(256), 0, s,
                       static_cast<const float2*>(X), static_cast<const float2*>(Z), static_cast<float2*>(Y), M, n);
}

void zx_product(const void* Z, int zdt, int n, const void* X, int xdt, void* Y, int nrhs, hipStream_t s) {
    if (nrhs == 1) {
        gemv(Z, zdt, n, X, xdt, Y, xdt, s);
    } else if (zdt == EFIE_C64 && xdt == EFIE_C64) {
        cgemm_mfma(X, Z, Y, nrhs, n, s);
    } else {
        zgemm_nt(X, xdt, Z, zdt, Y, xdt, nrhs, n, n, n, n, n, 1.0, 0.0, false, s);
    }
}

}  // namespace efie

extern "C" int efie_zx(const void* Z, int dtype, int64_t n, const void* X, void* Y, int64_t nrhs,
                       hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(Z && X && Y, EFIE_ERR_ARG, "zx: null argument");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "zx: bad dtype");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && nrhs >= 1 && nrhs < 65536, EFIE_ERR_ARG, "zx: bad sizes");
        efie::zx_product(Z, dtype, int(n), X, dtype, Y, int(nrhs), stream);
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

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

// ACC64: the FP32 matrix-core partial sums are flushed into FP64 accumulators after
// every K chunk, and the result is written as complex128 to the rows Y[yrow[r]]
// (the Krylov vectors); this bounds the FP32 accumulation error to short partial
// sums.  Otherwise complex64 is written to Y[r].
//
// Pipeline: two LDS buffers; the global loads of chunk c+1 (16-byte loads into
// registers when n is even, 8-byte otherwise) are in flight while chunk c is
// multiplied, then written to the other buffer; one barrier per chunk.
// Block order: workgroups are dealt to the 8 XCDs round-robin by id, so the ids
// are remapped to give each XCD a contiguous run of tiles, walking the
// right-hand-side tiles of one Z column strip first: the blocks that read the
// same strip of Z share one XCD's L2 and run at about the same time.
template <int BM, int BN, int KC, bool ACC64>
__global__ __launch_bounds__(256) void cgemm_mfma_kernel(const float2* __restrict__ X, const float2* __restrict__ Z,
                                                         void* __restrict__ Yv, int M, int n,
                                                         const int* __restrict__ yrow) {
    constexpr int AP = 2 * KC + 4;     // floats per LDS row of the X tile (padded, 16-byte rows)
    constexpr int BNC = BN / 2;        // unknowns per tile
    constexpr int BP = KC + 2;         // float2 per LDS row of the Z tile (padded, 16-byte rows)
    constexpr int WM = BM / 2, WN = BN / 2;   // wavefront tile
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int KV = KC / 2;         // two-element (16-byte) groups per row of a chunk
    constexpr int NA = BM * KV / 256, NB = BNC * KV / 256;
    static_assert(BM * KV % 256 == 0 && BNC * KV % 256 == 0, "tile not divisible by the block");
    __shared__ float As[2][BM * AP];
    __shared__ float2 Bs[2][BNC * BP];

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int nbm = (M + BM - 1) / BM;
    const int nblk = int(gridDim.x);
    const int xcd = int(blockIdx.x) & 7, idx = int(blockIdx.x) >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    const int logical = xcd * per + min(xcd, rem) + idx;
    const int bm = logical % nbm, bn = logical / nbm;
    const int s0 = bm * BM, i0 = bn * BNC;
    const bool vec = (n & 1) == 0 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Z)) & 15) == 0;

    floatx4 acc[TM][TN];
    double acc64[ACC64 ? TM : 1][ACC64 ? TN : 1][4];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (ACC64) {
#pragma unroll
        for (int a = 0; a < (ACC64 ? TM : 1); ++a)
#pragma unroll
            for (int b = 0; b < (ACC64 ? TN : 1); ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
    }

    float4 ra[NA], rb[NB];
    auto load2 = [&](const float2* base, int row, int nrows, int j) -> float4 {
        // elements j and j+1 of row `row` (zero outside the matrix)
        if (row >= nrows || j >= n) return make_float4(0.f, 0.f, 0.f, 0.f);
        const float2* p = base + size_t(row) * n + j;
        if (vec) return *reinterpret_cast<const float4*>(p);
        const float2 u = p[0];
        const float2 v = j + 1 < n ? p[1] : make_float2(0.f, 0.f);
        return make_float4(u.x, u.y, v.x, v.y);
    };
    auto gload = [&](int j0) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q, r = e / KV, c = e % KV;
            ra[q] = load2(X, s0 + r, M, j0 + 2 * c);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q, r = e / KV, c = e % KV;
            rb[q] = load2(Z, i0 + r, n, j0 + 2 * c);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q, r = e / KV, c = e % KV;
            *reinterpret_cast<float4*>(&As[buf][r * AP + 4 * c]) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q, r = e / KV, c = e % KV;
            *reinterpret_cast<float4*>(&Bs[buf][r * BP + 2 * c]) = rb[q];
        }
    };

    const int kq = lane >> 4;          // 0..3: real k within an instruction
    const int l16 = lane & 15;
    const int nch = (n + KC - 1) / KC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) gload((ch + 1) * KC);
        const float* A_ = As[buf];
        const float2* B_ = Bs[buf];
#pragma unroll
        for (int st = 0; st < KC / 2; ++st) {
            const int kf = 4 * st + kq;        // real k index inside the chunk
            const int jj = kf >> 1, t = kf & 1;
            float av[TM], bv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) av[a] = A_[(wm * WM + a * 16 + l16) * AP + kf];
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                const int col = wn * WN + b * 16 + l16;     // real column inside the tile
                const float2 z = B_[(col >> 1) * BP + jj];
                const int u = col & 1;
                bv[b] = u == 0 ? (t == 0 ? z.x : -z.y) : (t == 0 ? z.y : z.x);
            }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        if (ACC64) {
#pragma unroll
            for (int a = 0; a < (ACC64 ? TM : 1); ++a)
#pragma unroll
                for (int b = 0; b < (ACC64 ? TN : 1); ++b) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[a][b][r] += double(acc[a][b][r]);
                    acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
        }
        if (ch + 1 < nch) lstore(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int col = 2 * i0 + wn * WN + b * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = s0 + wm * WM + a * 16 + 4 * kq + r;
                if (row < M && col < 2 * n) {
                    if (ACC64)
                        reinterpret_cast<double*>(Yv)[size_t(yrow[row]) * 2 * n + col] =
                            acc64[ACC64 ? a : 0][ACC64 ? b : 0][r];
                    else
                        reinterpret_cast<float*>(Yv)[size_t(row) * 2 * n + col] = acc[a][b][r];
                }
            }
        }
}

bool cgemm_mfma_supported(int M, int n) { return M >= 1 && n >= 1; }

// ------------------------------------------------------------ tile variants
// Block tile BM (right-hand sides) x BN (real columns = BN/2 unknowns), K chunk KC.
// The FP64-flush path needs 3x the accumulator registers, so smaller wavefront
// tiles win there; efie_gemm_autotune measures and selects per path.
struct Variant {
    int bm, bn, kc;
};
static const Variant kVariants[] = {{128, 128, 16}, {128, 64, 16}, {64, 128, 16}, {64, 64, 16}, {64, 64, 32},
                                    {128, 128, 32}, {64, 128, 32}, {32, 128, 16}};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
static int g_variant[2] = {0, 1};   // defaults: complex64 output, FP64-flush output

template <int BM, int BN, int KC, bool A64>
static void launch_v(const void* X, const void* Z, void* Y, const int* yrow, int M, int n, hipStream_t s) {
    const int nbm = (M + BM - 1) / BM, nbn = (n + BN / 2 - 1) / (BN / 2);
    const size_t nblk = size_t(nbm) * nbn;
    EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "cgemm: problem too large");
    hipLaunchKernelGGL((cgemm_mfma_kernel<BM, BN, KC, A64>), dim3(unsigned(nblk)), dim3(256), 0, s,
                       static_cast<const float2*>(X), static_cast<const float2*>(Z), Y, M, n, yrow);
}

template <bool A64>
static void launch_variant(int v, const void* X, const void* Z, void* Y, const int* yrow, int M, int n,
                           hipStream_t s) {
    switch (v) {
        case 0: launch_v<128, 128, 16, A64>(X, Z, Y, yrow, M, n, s); break;
        case 1: launch_v<128, 64, 16, A64>(X, Z, Y, yrow, M, n, s); break;
        case 2: launch_v<64, 128, 16, A64>(X, Z, Y, yrow, M, n, s); break;
        case 3: launch_v<64, 64, 16, A64>(X, Z, Y, yrow, M, n, s); break;
        case 4: launch_v<64, 64, 32, A64>(X, Z, Y, yrow, M, n, s); break;
        case 5: launch_v<128, 128, 32, A64>(X, Z, Y, yrow, M, n, s); break;
        case 6: launch_v<64, 128, 32, A64>(X, Z, Y, yrow, M, n, s); break;
        default: launch_v<32, 128, 16, A64>(X, Z, Y, yrow, M, n, s); break;
    }
}

void cgemm_mfma(const void* X, const void* Z, void* Y, int M, int n, hipStream_t s) {
    prof_begin(PROF_MFMA, s);
    launch_variant<false>(g_variant[0], X, Z, Y, nullptr, M, n, s);
    prof_end(PROF_MFMA, s, 8.0 * M * double(n) * n);
}

void cgemm_mfma_acc64(const void* X, const void* Z, double2* Y, const int* yrow, int M, int n, hipStream_t s) {
    prof_begin(PROF_MFMA, s);
    launch_variant<true>(g_variant[1], X, Z, Y, yrow, M, n, s);
    prof_end(PROF_MFMA, s, 8.0 * M * double(n) * n);
}

__global__ void iota_rows_kernel(int* idx, int M) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) idx[i] = i;
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

extern "C" int efie_gemm_variants(int* count) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(count != nullptr, EFIE_ERR_ARG, "gemm_variants: null");
        *count = efie::kNumVariants;
        return int(EFIE_OK);
    });
}

extern "C" int efie_gemm_variant_info(int v, int* bm, int* bn, int* kc) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(v >= 0 && v < efie::kNumVariants && bm && bn && kc, EFIE_ERR_ARG, "gemm_variant_info: bad argument");
        *bm = efie::kVariants[v].bm;
        *bn = efie::kVariants[v].bn;
        *kc = efie::kVariants[v].kc;
        return int(EFIE_OK);
    });
}

extern "C" int efie_gemm_select(int acc64, int variant, int* previous) {
    return efie::guarded([&]() {
        EFIE_REQUIRE((acc64 == 0 || acc64 == 1) && variant >= 0 && variant < efie::kNumVariants, EFIE_ERR_ARG,
                     "gemm_select: bad argument");
        if (previous) *previous = efie::g_variant[acc64];
        efie::g_variant[acc64] = variant;
        return int(EFIE_OK);
    });
}

extern "C" int efie_gemm_autotune(const void* Z, int64_t n, const void* X, int64_t M, int acc64, void* ws,
                                  size_t ws_bytes, int reps, double* ms, int* best, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(Z && X && ws && ms && best && reps >= 1, EFIE_ERR_ARG, "gemm_autotune: bad argument");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && M >= 1 && M < 65536, EFIE_ERR_ARG, "gemm_autotune: bad sizes");
        const size_t ybytes = size_t(M) * size_t(n) * (acc64 ? 16 : 8);
        const size_t need = ((ybytes + 255) & ~size_t(255)) + size_t(M) * sizeof(int);
        EFIE_REQUIRE(ws_bytes >= need, EFIE_ERR_ARG, "gemm_autotune: workspace too small");
        void* Y = ws;
        int* idx = reinterpret_cast<int*>(static_cast<char*>(ws) + ((ybytes + 255) & ~size_t(255)));
        hipLaunchKernelGGL(efie::iota_rows_kernel, dim3(int((M + 255) / 256)), dim3(256), 0, stream, idx, int(M));
        hipEvent_t e0, e1;
        EFIE_HIP_CHECK(hipEventCreate(&e0));
        EFIE_HIP_CHECK(hipEventCreate(&e1));
        double best_ms = 1e300;
        *best = 0;
        for (int v = 0; v < efie::kNumVariants; ++v) {
            auto run = [&]() {
                if (acc64)
                    efie::launch_variant<true>(v, X, Z, Y, idx, int(M), int(n), stream);
                else
                    efie::launch_variant<false>(v, X, Z, Y, nullptr, int(M), int(n), stream);
            };
            run();   // warm-up
            EFIE_HIP_CHECK(hipEventRecord(e0, stream));
            for (int r = 0; r < reps; ++r) run();
            EFIE_HIP_CHECK(hipEventRecord(e1, stream));
            EFIE_HIP_CHECK(hipEventSynchronize(e1));
            float t = 0.f;
            EFIE_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
            ms[v] = double(t) / reps;
            if (ms[v] < best_ms) {
                best_ms = ms[v];
                *best = v;
            }
        }
        EFIE_HIP_CHECK(hipEventDestroy(e0));
        EFIE_HIP_CHECK(hipEventDestroy(e1));
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

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

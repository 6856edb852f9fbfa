// Dense complex products for the EFIE operator on gfx950.
//
//   gemv:      y = Z x, one wavefront per row of Z, 16-byte loads, FP64 accumulation
//              (single right-hand side: HBM-bound, 1 or 0.5 flop per byte).
//   zgemm_nt:  C[M][Nc] = sum_k A[M][k] B[Nc][k] with both operands k-contiguous,
//              LDS-tiled, FP64 accumulation; B may be complex64 or complex128.
//              Z X for many right-hand sides is this product with A = X (nrhs x N),
//              B = Z (N x N, symmetric), C = Y (nrhs x N).
//   cast kernels between complex64 and complex128.
#include <hip/hip_runtime.h>

#include "efie_internal.h"
#include "linalg.h"

namespace efie {

// ------------------------------------------------------------------ GEMV
template <typename T>
struct CT;   // complex element traits: load one element as FP64 pair
template <>
struct CT<double2> {
    __device__ static double2 ld(const double2* p, size_t i) { return p[i]; }
};
template <>
struct CT<float2> {
    __device__ static double2 ld(const float2* p, size_t i) {
        float2 v = p[i];
        return make_double2(v.x, v.y);
    }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename YT>
__device__ __forceinline__ void store_c(YT* y, size_t i, double re, double im);
template <>
__device__ __forceinline__ void store_c<double2>(double2* y, size_t i, double re, double im) {
    y[i] = make_double2(re, im);
}
template <>
__device__ __forceinline__ void store_c<float2>(float2* y, size_t i, double re, double im) {
    y[i] = make_float2(float(re), float(im));
}

// one element per lane per load, 4 loads in flight (16-byte loads for complex128;
// also the fallback for complex64 matrices of odd order).
template <typename ZT, typename XT, typename YT>
__global__ __launch_bounds__(256) void gemv_elem_kernel(const ZT* __restrict__ Z, const XT* __restrict__ x,
                                                        YT* __restrict__ y, int n) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const ZT* zr = Z + size_t(row) * n;
    double ar = 0, ai = 0;
    int k = lane;
    for (; k + 192 < n; k += 256) {
        double2 z0 = CT<ZT>::ld(zr, k), z1 = CT<ZT>::ld(zr, k + 64), z2 = CT<ZT>::ld(zr, k + 128),
                z3 = CT<ZT>::ld(zr, k + 192);
        double2 x0 = CT<XT>::ld(x, k), x1 = CT<XT>::ld(x, k + 64), x2 = CT<XT>::ld(x, k + 128),
                x3 = CT<XT>::ld(x, k + 192);
        ar += z0.x * x0.x - z0.y * x0.y + z1.x * x1.x - z1.y * x1.y + z2.x * x2.x - z2.y * x2.y + z3.x * x3.x -
              z3.y * x3.y;
        ai += z0.x * x0.y + z0.y * x0.x + z1.x * x1.y + z1.y * x1.x + z2.x * x2.y + z2.y * x2.x + z3.x * x3.y +
              z3.y * x3.x;
    }
    for (; k < n; k += 64) {
        double2 z0 = CT<ZT>::ld(zr, k), x0 = CT<XT>::ld(x, k);
        ar += z0.x * x0.x - z0.y * x0.y;
        ai += z0.x * x0.y + z0.y * x0.x;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    if (lane == 0) store_c<YT>(y, row, ar, ai);
}

// complex64 Z: each lane reads two elements (16 bytes) per load; needs n even.
template <typename XT, typename YT>
__global__ __launch_bounds__(256) void gemv_c64_kernel(const float2* __restrict__ Z, const XT* __restrict__ x,
                                                       YT* __restrict__ y, int n) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float4* zr = reinterpret_cast<const float4*>(Z + size_t(row) * n);
    const int n2 = n >> 1;
    double ar = 0, ai = 0;
    int k = lane;
    for (; k + 192 < n2; k += 256) {
        float4 z[4] = {zr[k], zr[k + 64], zr[k + 128], zr[k + 192]};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = 2 * (k + 64 * u);
            double2 xa = CT<XT>::ld(x, kk), xb = CT<XT>::ld(x, kk + 1);
            ar += double(z[u].x) * xa.x - double(z[u].y) * xa.y + double(z[u].z) * xb.x - double(z[u].w) * xb.y;
            ai += double(z[u].x) * xa.y + double(z[u].y) * xa.x + double(z[u].z) * xb.y + double(z[u].w) * xb.x;
        }
    }
    for (; k < n2; k += 64) {
        float4 z0 = zr[k];
        double2 xa = CT<XT>::ld(x, 2 * k), xb = CT<XT>::ld(x, 2 * k + 1);
        ar += double(z0.x) * xa.x - double(z0.y) * xa.y + double(z0.z) * xb.x - double(z0.w) * xb.y;
        ai += double(z0.x) * xa.y + double(z0.y) * xa.x + double(z0.z) * xb.y + double(z0.w) * xb.x;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    if (lane == 0) store_c<YT>(y, row, ar, ai);
}

// Y[idx[c]][i] = sum_k Z[i][k] X[idx[c]][k] for c < m <= MC columns of FP64 vectors:
// one wavefront per RW consecutive rows (each loaded X element serves RW rows), Z
// read once for all m columns, FP64 accumulation with explicit FMAs, and the loads
// of the next K step issued before the arithmetic of the current one.
constexpr int GEMV_SLABS = 8;   // K slabs of the split product (three or more columns)
template <int MC>
constexpr int gemv_rw() { return MC >= 8 ? 2 : 4; }

template <typename ZT>
__device__ __forceinline__ double2 to_d2(ZT v) { return make_double2(double(v.x), double(v.y)); }

// SPLIT: blockIdx.y selects a slab of kslab columns of Z and the FP64 partial sums
// go to part[(slab * MC + c) * n + row] (added by gemv_multi_reduce_kernel); the
// row blocks of one slab are dispatched together, so the slab of X they all read
// stays in L2.
template <typename ZT, int MC, bool SPLIT>
__global__ __launch_bounds__(256) void gemv_multi_kernel(const ZT* __restrict__ Z, const double2* __restrict__ X,
                                                         const int* __restrict__ idx, int m,
                                                         double2* __restrict__ Y, int n, int kslab,
                                                         double2* __restrict__ part) {
    constexpr int RW = gemv_rw<MC>();
    const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RW;
    const int lane = threadIdx.x & 63;
    if (row0 >= n) return;
    const int kb = SPLIT ? int(blockIdx.y) * kslab : 0;
    const int ke = SPLIT ? min(n, kb + kslab) : n;
    const ZT* zr[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) zr[r] = Z + size_t(min(row0 + r, n - 1)) * n;   // rows past the end: discarded
    const double2* xc[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) xc[c] = X + size_t(idx[c < m ? c : 0]) * n;   // c >= m: alias, sums dropped
    double ar[RW][MC], ai[RW][MC];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < MC; ++c) ar[r][c] = ai[r][c] = 0.0;
    ZT zc[RW];
    double2 xv[MC];
    int k = kb + lane;
    if (k < ke) {
#pragma unroll
        for (int r = 0; r < RW; ++r) zc[r] = zr[r][k];
#pragma unroll
        for (int c = 0; c < MC; ++c) xv[c] = xc[c][k];
    }
    for (; k < ke; k += 64) {
        const int kn = k + 64;
        ZT zn[RW];
        double2 xn[MC];
        if (kn < ke) {
#pragma unroll
            for (int r = 0; r < RW; ++r) zn[r] = zr[r][kn];
#pragma unroll
            for (int c = 0; c < MC; ++c) xn[c] = xc[c][kn];
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const double2 z = to_d2(zc[r]);
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                ar[r][c] = fma(z.x, xv[c].x, ar[r][c]);
                ar[r][c] = fma(-z.y, xv[c].y, ar[r][c]);
                ai[r][c] = fma(z.x, xv[c].y, ai[r][c]);
                ai[r][c] = fma(z.y, xv[c].x, ai[r][c]);
            }
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) zc[r] = zn[r];
#pragma unroll
        for (int c = 0; c < MC; ++c) xv[c] = xn[c];
    }
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        if (c < m) {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const double re = wave_sum(ar[r][c]), im = wave_sum(ai[r][c]);
                if (lane == 0 && row0 + r < n) {
                    if (SPLIT)
                        part[(size_t(blockIdx.y) * MC + c) * n + row0 + r] = make_double2(re, im);
                    else
                        Y[size_t(idx[c]) * n + row0 + r] = make_double2(re, im);
                }
            }
        }
    }
}

// Y[idx[c]][i] = sum over slabs of part[(slab * MC + c) * n + i], slabs in order
template <int MC>
__global__ void gemv_multi_reduce_kernel(const double2* __restrict__ part, const int* __restrict__ idx, int m, int n,
                                         int ns, double2* __restrict__ Y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || c >= m) return;
    double re = 0.0, im = 0.0;
    for (int sl = 0; sl < ns; ++sl) {
        const double2 v = part[(size_t(sl) * MC + c) * n + i];
        re += v.x;
        im += v.y;
    }
    Y[size_t(idx[c]) * n + i] = make_double2(re, im);
}

// out[r][k] = (complex64) X[idx[r]][k]
__global__ void gather_cast_kernel(const double2* __restrict__ X, const int* __restrict__ idx, int m, int n,
                                   float2* __restrict__ out) {
    const size_t tot = size_t(m) * n;
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
        const size_t r = e / n, k = e - r * n;
        const double2 v = X[size_t(idx[r]) * n + k];
        out[e] = make_float2(float(v.x), float(v.y));
    }
}
// Y[idx[r]][k] = (complex128) in[r][k]
__global__ void scatter_cast_kernel(const float2* __restrict__ in, const int* __restrict__ idx, int m, int n,
                                    double2* __restrict__ Y) {
    const size_t tot = size_t(m) * n;
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
        const size_t r = e / n, k = e - r * n;
        const float2 v = in[e];
        Y[size_t(idx[r]) * n + k] = make_double2(v.x, v.y);
    }
}

// ------------------------------------------------------------- tiled GEMM
// C[M][Nc] (+)= alpha * sum_k A[M][k] B[Nc][k]; 64 x 64 output tile per block of
// 256 threads (4 x 4 complex outputs each), k-chunks of 16 staged in LDS.
constexpr int GT = 64, GK = 16;

template <typename AT, typename BT, typename CTy>
__global__ __launch_bounds__(256) void zgemm_nt_kernel(const AT* __restrict__ A, const BT* __restrict__ B,
                                                       CTy* __restrict__ C, int M, int Nc, int K, int lda, int ldb,
                                                       int ldc, double alr, double ali, int accumulate,
                                                       const int* __restrict__ arow, const int* __restrict__ crow) {
    __shared__ double2 As[GK][GT + 1];
    __shared__ double2 Bs[GK][GT + 1];
    const int tid = threadIdx.x;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int tm = tid / 16, tn = tid % 16;   // 16 x 16 threads, each 4 x 4 outputs (strided by 16)
    double cr[4][4], ci[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cr[i][j] = ci[i][j] = 0.0;
    for (int k0 = 0; k0 < K; k0 += GK) {
        // 64 x 16 elements of A and of B: 1024 each, 4 per thread
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int e = tid + 256 * l;
            const int r = e / GK, kk = e % GK;
            const int gm = m0 + r, gn = n0 + r, gk = k0 + kk;
            const int am = gm < M ? (arow ? arow[gm] : gm) : 0;
            As[kk][r] = (gm < M && gk < K) ? CT<AT>::ld(A, size_t(am) * lda + gk) : make_double2(0, 0);
            Bs[kk][r] = (gn < Nc && gk < K) ? CT<BT>::ld(B, size_t(gn) * ldb + gk) : make_double2(0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            double2 a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    cr[i][j] += a[i].x * b[j].x - a[i].y * b[j].y;
                    ci[i][j] += a[i].x * b[j].y + a[i].y * b[j].x;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + tm + 16 * i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tn + 16 * j;
            if (gn >= Nc) continue;
            double re = alr * cr[i][j] - ali * ci[i][j];
            double im = alr * ci[i][j] + ali * cr[i][j];
            const size_t o = size_t(crow ? crow[gm] : gm) * ldc + gn;
            if (accumulate) {
                double2 old = CT<CTy>::ld(C, o);
                re += old.x;
                im += old.y;
            }
            store_c<CTy>(C, o, re, im);
        }
    }
}

// ------------------------------------------------------------------ casts
__global__ void cast_c128_to_c64_kernel(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        b[i] = make_float2(float(a[i].x), float(a[i].y));
}
__global__ void cast_c64_to_c128_kernel(const float2* __restrict__ a, double2* __restrict__ b, size_t n) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        b[i] = make_double2(a[i].x, a[i].y);
}

static int grid_for(size_t n) { return int(std::min<size_t>((n + 255) / 256, 16384)); }

void cast_c128_to_c64(const void* a, void* b, size_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(cast_c128_to_c64_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                              static_cast<const double2*>(a), static_cast<float2*>(b), n);
}
void cast_c64_to_c128(const void* a, void* b, size_t n, hipStream_t s) {
    if (n) hipLaunchKernelGGL(cast_c64_to_c128_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                              static_cast<const float2*>(a), static_cast<double2*>(b), n);
}

// ------------------------------------------------------------- dispatchers
size_t gemv_multi_part_bytes(int n) { return size_t(GEMV_SLABS) * 8 * size_t(n) * sizeof(double2); }

void gemv_multi(const void* Z, int zdt, int n, const double2* X, const int* idx, int m, double2* Y, hipStream_t s,
                double2* part) {
    EFIE_REQUIRE(m >= 1 && m <= 8, EFIE_ERR_ARG, "gemv_multi: 1..8 columns");
    const int rw = m > 4 ? gemv_rw<8>() : gemv_rw<4>();
    const int rb = (n + 4 * rw - 1) / (4 * rw);
    // three or more columns: split K so that the X slab in use stays in L2
    const bool split = part != nullptr && m >= 3 && n >= 64 * GEMV_SLABS;
    const int kslab = (n + GEMV_SLABS - 1) / GEMV_SLABS;
    const int ns = split ? (n + kslab - 1) / kslab : 1;
    dim3 grid(rb, ns), blk(256);
    prof_begin(PROF_GEMV, s);
#define GM(ZTy, MC)                                                                                                \
    do {                                                                                                           \
        if (split) {                                                                                               \
            hipLaunchKernelGGL((gemv_multi_kernel<ZTy, MC, true>), grid, blk, 0, s, static_cast<const ZTy*>(Z), X, \
                               idx, m, Y, n, kslab, part);                                                         \
            hipLaunchKernelGGL((gemv_multi_reduce_kernel<MC>), dim3((n + 255) / 256, m), dim3(256), 0, s, part, idx, \
                               m, n, ns, Y);                                                                       \
        } else {                                                                                                   \
            hipLaunchKernelGGL((gemv_multi_kernel<ZTy, MC, false>), grid, blk, 0, s, static_cast<const ZTy*>(Z),   \
                               X, idx, m, Y, n, n, nullptr);                                                       \
        }                                                                                                          \
    } while (0)
    if (zdt == EFIE_C128) {
        if (m == 1) GM(double2, 1); else if (m == 2) GM(double2, 2); else if (m <= 4) GM(double2, 4); else GM(double2, 8);
    } else {
        if (m == 1) GM(float2, 1); else if (m == 2) GM(float2, 2); else if (m <= 4) GM(float2, 4); else GM(float2, 8);
    }
#undef GM
    prof_end(PROF_GEMV, s, double(n) * n * (zdt == EFIE_C128 ? 16 : 8));
}

void gather_cast(const double2* X, const int* idx, int m, int n, float2* out, hipStream_t s) {
    const size_t tot = size_t(m) * n;
    if (tot) hipLaunchKernelGGL(gather_cast_kernel, dim3(grid_for(tot)), dim3(256), 0, s, X, idx, m, n, out);
}
void scatter_cast(const float2* in, const int* idx, int m, int n, double2* Y, hipStream_t s) {
    const size_t tot = size_t(m) * n;
    if (tot) hipLaunchKernelGGL(scatter_cast_kernel, dim3(grid_for(tot)), dim3(256), 0, s, in, idx, m, n, Y);
}

void gemv(const void* Z, int zdt, int n, const void* x, int xdt, void* y, int ydt, hipStream_t s) {
    dim3 grid((n + 3) / 4), blk(256);
    prof_begin(PROF_GEMV, s);
#define GEMV_CASE(KER, ZTy, XTy, YTy) \
    hipLaunchKernelGGL((KER), grid, blk, 0, s, static_cast<const ZTy*>(Z), static_cast<const XTy*>(x), \
                       static_cast<YTy*>(y), n)
    if (zdt == EFIE_C128) {
        if (xdt == EFIE_C128 && ydt == EFIE_C128)
            GEMV_CASE((gemv_elem_kernel<double2, double2, double2>), double2, double2, double2);
        else if (xdt == EFIE_C64 && ydt == EFIE_C64)
            GEMV_CASE((gemv_elem_kernel<double2, float2, float2>), double2, float2, float2);
        else throw Error{EFIE_ERR_ARG, "gemv: unsupported dtype combination"};
    } else if (n % 2 == 0) {
        if (xdt == EFIE_C128 && ydt == EFIE_C128) GEMV_CASE((gemv_c64_kernel<double2, double2>), float2, double2, double2);
        else if (xdt == EFIE_C64 && ydt == EFIE_C64) GEMV_CASE((gemv_c64_kernel<float2, float2>), float2, float2, float2);
        else throw Error{EFIE_ERR_ARG, "gemv: unsupported dtype combination"};
    } else {
        if (xdt == EFIE_C128 && ydt == EFIE_C128)
            GEMV_CASE((gemv_elem_kernel<float2, double2, double2>), float2, double2, double2);
        else if (xdt == EFIE_C64 && ydt == EFIE_C64)
            GEMV_CASE((gemv_elem_kernel<float2, float2, float2>), float2, float2, float2);
        else throw Error{EFIE_ERR_ARG, "gemv: unsupported dtype combination"};
    }
    prof_end(PROF_GEMV, s, double(n) * n * (zdt == EFIE_C128 ? 16 : 8));
#undef GEMV_CASE
}

// ------------------------------------------------- FP64 matrix-core product
// C[crow[s]][i] = sum_k A[arow[s]][k] B[i][k] (complex128 A and C, complex128 or
// complex64 B; B square n x n with K = n here) on v_mfma_f64_16x16x4f64, in the
// planar complex form of the complex64 kernel: the K chunks of A and B sit in LDS
// as complex rows, a lane's operand element is one complex value (one 16-byte LDS
// read), and each 16 x 16 complex output block takes four real instructions per 4
// complex K:  Cr += Ar Br + (-Ai) Bi,  Ci += Ar Bi + Ai Br.
// Operand layouts of v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l holds D[l/16 + 4*r][l%16]
// (rows interleaved, unlike the FP32 16x16x4 form).
// Tiling as the complex64 kernel: 4 wavefronts (WGM along the right-hand sides x
// 4/WGM along the columns), a BM x BNC complex tile, K chunks of KC complex
// elements double-buffered in LDS with register prefetch, XCD-aware block order.
// LDS rows hold KC + 1 complex values, which keeps the 16-byte reads of a
// wavefront free of bank conflicts.  Few right-hand sides (the residual products
// of a handful of columns) use a 16-row tile with all four wavefronts along the
// columns, so Z is read once.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int BM, int BNC, int KC, int WGM, typename BT>
__global__ __launch_bounds__(256) void zgemm_mfma_kernel(const double2* __restrict__ A, const BT* __restrict__ B,
                                                         double2* __restrict__ C, int M, int n, int lda, int ldc,
                                                         const int* __restrict__ arow, const int* __restrict__ crow) {
    constexpr int AS = KC + 1;         // double2 per LDS row
    constexpr int WGN = 4 / WGM;
    constexpr int WM = BM / WGM, WN = BNC / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int NA = BM * KC / 256, NB = BNC * KC / 256;
    static_assert(WGM * WGN == 4 && TM >= 1 && TN >= 1, "bad wavefront arrangement");
    static_assert(BM * KC % 256 == 0 && BNC * KC % 256 == 0, "tile not divisible by the block");
    __shared__ double2 As[2][BM * AS];
    __shared__ double2 Bs[2][BNC * AS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w / WGN, wn = w % WGN;
    const int nbm = (M + BM - 1) / BM;
    const int nblk = int(gridDim.x);
    const int xcd = int(blockIdx.x) & 7, idx = int(blockIdx.x) >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    const int logical = xcd * per + min(xcd, rem) + idx;
    const int bm = logical % nbm, bn = logical / nbm;
    const int s0 = bm * BM, i0 = bn * BNC;

    doublex4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            accr[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};
            acci[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};
        }

    double2 ra[NA];
    BT rb[NB];   // raw storage type: converted when written to LDS, so the loads stay in flight
    auto gload = [&](int j0) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q, r = e / KC, c = e % KC;
            const int srow = s0 + r, j = j0 + c;
            ra[q] = (srow < M && j < n) ? A[size_t(arow ? arow[srow] : srow) * lda + j] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q, r = e / KC, c = e % KC;
            const int i = i0 + r, j = j0 + c;
            rb[q] = (i < n && j < n) ? B[size_t(i) * n + j] : BT{0, 0};
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q, r = e / KC, c = e % KC;
            As[buf][r * AS + c] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q, r = e / KC, c = e % KC;
            Bs[buf][r * AS + c] = to_d2(rb[q]);
        }
    };

    const int kq = lane >> 4, l16 = lane & 15;
    const int nch = (n + KC - 1) / KC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) gload((ch + 1) * KC);
        const double2* A_ = As[buf] + (wm * WM + l16) * AS + kq;
        const double2* B_ = Bs[buf] + (wn * WN + l16) * AS + kq;
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            double2 xa[TM], zb[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) xa[a] = A_[a * 16 * AS + kk];
#pragma unroll
            for (int b = 0; b < TN; ++b) zb[b] = B_[b * 16 * AS + kk];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a].x, zb[b].x, accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a].x, zb[b].y, acci[a][b], 0, 0, 0);
                }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xa[a].y, zb[b].y, accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a].y, zb[b].x, acci[a][b], 0, 0, 0);
                }
        }
        if (ch + 1 < nch) lstore(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int col = i0 + wn * WN + b * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = s0 + wm * WM + a * 16 + kq + 4 * r;
                if (row < M && col < n)
                    C[size_t(crow ? crow[row] : row) * ldc + col] = make_double2(accr[a][b][r], acci[a][b][r]);
            }
        }
}

template <int BM, int BNC, int KC, int WGM, typename BT>
static void launch_zgemm_tile(const double2* A, const BT* B, double2* C, int M, int n, int lda, int ldc,
                              const int* arow, const int* crow, hipStream_t s) {
    const size_t nblk = size_t((M + BM - 1) / BM) * size_t((n + BNC - 1) / BNC);
    EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "zgemm: problem too large");
    hipLaunchKernelGGL((zgemm_mfma_kernel<BM, BNC, KC, WGM, BT>), dim3(unsigned(nblk)), dim3(256), 0, s, A, B, C, M,
                       n, lda, ldc, arow, crow);
}

template <typename BT>
static void launch_zgemm_mfma(const double2* A, const BT* B, double2* C, int M, int n, int lda, int ldc,
                              const int* arow, const int* crow, hipStream_t s) {
    if (M <= 16)
        launch_zgemm_tile<16, 64, 16, 1>(A, B, C, M, n, lda, ldc, arow, crow, s);
    else if (M <= 64)
        launch_zgemm_tile<32, 64, 16, 1>(A, B, C, M, n, lda, ldc, arow, crow, s);
    else
        launch_zgemm_tile<64, 64, 16, 2>(A, B, C, M, n, lda, ldc, arow, crow, s);
}

void zgemm_nt(const void* A, int adt, const void* B, int bdt, void* C, int cdt, int M, int Nc, int K, int lda,
              int ldb, int ldc, double alr, double ali, bool accumulate, hipStream_t s, const int* arow,
              const int* crow) {
    dim3 grid((Nc + GT - 1) / GT, (M + GT - 1) / GT), blk(256);
    EFIE_REQUIRE(grid.y <= 65535, EFIE_ERR_ARG, "zgemm: too many rows");
    prof_begin(PROF_ZGEMM, s);
    // the operator products (B square, K = n, plain product): FP64 matrix cores
    if (adt == EFIE_C128 && cdt == EFIE_C128 && (bdt == EFIE_C128 || bdt == EFIE_C64) && Nc == K && ldb == K &&
        alr == 1.0 && ali == 0.0 && !accumulate && M >= 9) {
        if (bdt == EFIE_C128)
            launch_zgemm_mfma(static_cast<const double2*>(A), static_cast<const double2*>(B), static_cast<double2*>(C), M,
                              K, lda, ldc, arow, crow, s);
        else
            launch_zgemm_mfma(static_cast<const double2*>(A), static_cast<const float2*>(B), static_cast<double2*>(C), M,
                              K, lda, ldc, arow, crow, s);
        prof_end(PROF_ZGEMM, s, 8.0 * M * double(Nc) * K);
        return;
    }
#define ZG(ATy, BTy, CTy2)                                                                                     \
    hipLaunchKernelGGL((zgemm_nt_kernel<ATy, BTy, CTy2>), grid, blk, 0, s, static_cast<const ATy*>(A),         \
                       static_cast<const BTy*>(B), static_cast<CTy2*>(C), M, Nc, K, lda, ldb, ldc, alr, ali, \
                       int(accumulate), arow, crow)
    if (adt == EFIE_C128 && bdt == EFIE_C128 && cdt == EFIE_C128) ZG(double2, double2, double2);
    else if (adt == EFIE_C128 && bdt == EFIE_C64 && cdt == EFIE_C128) ZG(double2, float2, double2);
    else if (adt == EFIE_C64 && bdt == EFIE_C64 && cdt == EFIE_C64) ZG(float2, float2, float2);
    else throw Error{EFIE_ERR_ARG, "zgemm: unsupported dtype combination"};
    prof_end(PROF_ZGEMM, s, 8.0 * M * double(Nc) * K);
#undef ZG
}

}  // namespace efie

extern "C" int efie_convert(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t count, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(src && dst && count >= 0, EFIE_ERR_ARG, "convert: bad argument");
        EFIE_REQUIRE((src_dtype == EFIE_C128 || src_dtype == EFIE_C64) && (dst_dtype == EFIE_C128 || dst_dtype == EFIE_C64),
                     EFIE_ERR_ARG, "convert: bad dtype");
        const size_t n = size_t(count);
        if (src_dtype == dst_dtype) {
            EFIE_HIP_CHECK(hipMemcpyAsync(dst, src, n * (src_dtype == EFIE_C128 ? 16 : 8), hipMemcpyDeviceToDevice,
                                          stream));
        } else if (src_dtype == EFIE_C128) {
            efie::cast_c128_to_c64(src, dst, n, stream);
        } else {
            efie::cast_c64_to_c128(src, dst, n, stream);
        }
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

// FP64 matrix-core GEMM of the 2-D path: C = alpha A op(B) (+ C), complex128,
// op(B) = B^T (NT), B (NN) or the circulant matrix of a vector (CIRC).
//
// Same planar-complex scheme as the operator products of the 3-D solver: K chunks
// of A and of op(B) sit in LDS as complex rows (one 16-byte read gives a lane its
// operand), each 16 x 16 complex output block takes four v_mfma_f64_16x16x4f64
// per 4 complex K (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br).  Operand layouts of
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator register r of lane l holds D[l/16 + 4r][l%16].  Four wavefronts
// per block (WGM along the rows of C, 4/WGM along its columns), K chunks of KC
// complex values double-buffered in LDS with register prefetch, blocks dealt to
// the 8 XCDs in contiguous runs.
//
// The operand loader is what differs between the three forms: NT reads B along
// its rows (k contiguous), NN along its columns (i contiguous, so the threads of
// a wavefront read consecutive elements of a row of B), CIRC gathers
// c[(i - k) mod K] from a vector that stays in cache (a Toeplitz tile: consecutive
// k of one output column are consecutive elements of c, read backwards).
#include <algorithm>

#include "bie2d.h"

namespace efie {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int BM, int BNC, int KC, int WGM, int OP>
__global__ __launch_bounds__(256) void gemm2d_kernel(const double2* __restrict__ A, int lda, int conja,
                                                     const double2* __restrict__ B, int ldb, int conjb,
                                                     double2* __restrict__ C, int ldc, int M, int Nc, int K,
                                                     double2 alpha, int accumulate, int klen, size_t cstride) {
    constexpr int AS = KC + 1;
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
    const double sa = conja ? -1.0 : 1.0, sb = conjb ? -1.0 : 1.0;
    // split K: blockIdx.y takes the contraction range [kbeg, kend) and writes its own
    // partial product at C + blockIdx.y * cstride
    const int kbeg = int(blockIdx.y) * klen, kend = min(K, kbeg + klen);
    C += size_t(blockIdx.y) * cstride;

    doublex4 accr[TM][TN], acci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            accr[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};
            acci[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};
        }

    double2 ra[NA], rb[NB];
    auto bpos = [&](int q, int& r, int& c) {
        const int e = tid + 256 * q;
        if (OP == G2D_NN) {
            r = e % BNC;
            c = e / BNC;
        } else {
            r = e / KC;
            c = e % KC;
        }
    };
    auto gload = [&](int j0) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q, r = e / KC, c = e % KC;
            const int srow = s0 + r, j = j0 + c;
            double2 v = (srow < M && j < kend) ? A[size_t(srow) * lda + j] : make_double2(0.0, 0.0);
            v.y *= sa;
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            int r, c;
            bpos(q, r, c);
            const int i = i0 + r, j = j0 + c;
            double2 v = make_double2(0.0, 0.0);
            if (i < Nc && j < kend) {
                if (OP == G2D_NT) v = B[size_t(i) * ldb + j];
                else if (OP == G2D_NN) v = B[size_t(j) * ldb + i];
                else {
                    int m = i - j;
                    if (m < 0) m += K;
                    v = B[m];
                }
            }
            v.y *= sb;
            rb[q] = v;
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
            int r, c;
            bpos(q, r, c);
            Bs[buf][r * AS + c] = rb[q];
        }
    };

    const int kq = lane >> 4, l16 = lane & 15;
    const int nch = (kend - kbeg + KC - 1) / KC;
    gload(kbeg);
    lstore(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) gload(kbeg + (ch + 1) * KC);
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
                if (row < M && col < Nc) {
                    const double pr = accr[a][b][r], pi = acci[a][b][r];
                    double2 v = make_double2(alpha.x * pr - alpha.y * pi, alpha.x * pi + alpha.y * pr);
                    double2* dst = C + size_t(row) * ldc + col;
                    if (accumulate) {
                        const double2 o = *dst;
                        v.x += o.x;
                        v.y += o.y;
                    }
                    *dst = v;
                }
            }
        }
}

// sum of the split-K partial products: C = alpha sum_y part[y] (+ C)
__global__ void splitk_reduce_kernel(const double2* __restrict__ part, int nsplit, size_t cstride, int M, int Nc,
                                     double2* __restrict__ C, int ldc, double2 alpha, int accumulate) {
    const size_t tot = size_t(M) * Nc;
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int y = 0; y < nsplit; ++y) {
            const double2 v = part[size_t(y) * cstride + e];
            acc.x += v.x;
            acc.y += v.y;
        }
        double2 v = make_double2(alpha.x * acc.x - alpha.y * acc.y, alpha.x * acc.y + alpha.y * acc.x);
        const size_t row = e / Nc, col = e - row * Nc;
        double2* dst = C + row * ldc + col;
        if (accumulate) {
            v.x += dst->x;
            v.y += dst->y;
        }
        *dst = v;
    }
}

template <int BM, int BNC, int KC, int WGM, int OP>
void launch_tile(const double2* A, int lda, bool conja, const double2* B, int ldb, bool conjb, double2* C, int ldc,
                 int M, int Nc, int K, double2 alpha, bool acc, double2* scratch, size_t scratch_elems,
                 hipStream_t s) {
    const size_t nblk = size_t((M + BM - 1) / BM) * size_t((Nc + BNC - 1) / BNC);
    EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "gemm2d: problem too large");
    // few output tiles over a long contraction (the range finder's projections and
    // Gram products): split K over more workgroups into scratch, then reduce
    int nsplit = 1;
    if (scratch && nblk < 128 && K >= 2048) {
        nsplit = int(std::min<size_t>(std::min<size_t>(256 / nblk, size_t(K) / 1024), 64));
        while (nsplit > 1 && size_t(nsplit) * M * Nc > scratch_elems) --nsplit;
    }
    if (nsplit <= 1) {
        hipLaunchKernelGGL((gemm2d_kernel<BM, BNC, KC, WGM, OP>), dim3(unsigned(nblk), 1), dim3(256), 0, s, A, lda,
                           int(conja), B, ldb, int(conjb), C, ldc, M, Nc, K, alpha, int(acc), K, size_t(0));
        return;
    }
    const int klen = ((K + nsplit - 1) / nsplit + KC - 1) / KC * KC;
    nsplit = (K + klen - 1) / klen;
    const size_t cstride = size_t(M) * Nc;
    hipLaunchKernelGGL((gemm2d_kernel<BM, BNC, KC, WGM, OP>), dim3(unsigned(nblk), unsigned(nsplit)), dim3(256), 0, s,
                       A, lda, int(conja), B, ldb, int(conjb), scratch, Nc, M, Nc, K, make_double2(1.0, 0.0), 0, klen,
                       cstride);
    const size_t tot = size_t(M) * Nc;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(unsigned(std::min<size_t>((tot + 255) / 256, 65536))), dim3(256), 0,
                       s, scratch, nsplit, cstride, M, Nc, C, ldc, alpha, int(acc));
}

template <int OP>
void launch_op(const double2* A, int lda, bool conja, const double2* B, int ldb, bool conjb, double2* C, int ldc,
               int M, int Nc, int K, double2 alpha, bool acc, double2* scratch, size_t scratch_elems, hipStream_t s) {
    if (M <= 16)
        launch_tile<16, 64, 16, 1, OP>(A, lda, conja, B, ldb, conjb, C, ldc, M, Nc, K, alpha, acc, scratch,
                                       scratch_elems, s);
    else if (M <= 48)
        launch_tile<32, 64, 16, 1, OP>(A, lda, conja, B, ldb, conjb, C, ldc, M, Nc, K, alpha, acc, scratch,
                                       scratch_elems, s);
    else
        launch_tile<64, 64, 16, 2, OP>(A, lda, conja, B, ldb, conjb, C, ldc, M, Nc, K, alpha, acc, scratch,
                                       scratch_elems, s);
}

}  // namespace

void gemm2d(int op, const double2* A, int lda, bool conja, const double2* B, int ldb, bool conjb, double2* C,
            int ldc, int M, int Nc, int K, double2 alpha, bool accumulate, hipStream_t s, double2* scratch,
            size_t scratch_elems) {
    if (M <= 0 || Nc <= 0) return;
    EFIE_REQUIRE(K >= 1, EFIE_ERR_ARG, "gemm2d: empty contraction");
    prof_begin(PROF_ZGEMM, s);
    if (op == G2D_NT)
        launch_op<G2D_NT>(A, lda, conja, B, ldb, conjb, C, ldc, M, Nc, K, alpha, accumulate, scratch, scratch_elems, s);
    else if (op == G2D_NN)
        launch_op<G2D_NN>(A, lda, conja, B, ldb, conjb, C, ldc, M, Nc, K, alpha, accumulate, scratch, scratch_elems, s);
    else if (op == G2D_CIRC) {
        EFIE_REQUIRE(Nc == K, EFIE_ERR_ARG, "gemm2d: a circulant operand is square");
        launch_op<G2D_CIRC>(A, lda, conja, B, ldb, conjb, C, ldc, M, Nc, K, alpha, accumulate, scratch, scratch_elems,
                            s);
    } else throw Error{EFIE_ERR_ARG, "gemm2d: bad operand form"};
    prof_end(PROF_ZGEMM, s, 8.0 * M * double(Nc) * K);
    EFIE_HIP_CHECK(hipGetLastError());
}

}  // namespace efie

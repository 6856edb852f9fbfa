// Internal dense linear-algebra dispatchers (see linalg.hip, gemm_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace efie {

// y = Z x (single right-hand side); dtypes EFIE_C128 / EFIE_C64 per operand.
void gemv(const void* Z, int zdt, int n, const void* x, int xdt, void* y, int ydt, hipStream_t s);

// C[crow[r]][c] (+)= alpha * sum_k A[arow[r]][k] B[c][k], FP64 accumulation
// (arow / crow may be null: identity).
void zgemm_nt(const void* A, int adt, const void* B, int bdt, void* C, int cdt, int M, int Nc, int K, int lda,
              int ldb, int ldc, double alr, double ali, bool accumulate, hipStream_t s, const int* arow = nullptr,
              const int* crow = nullptr);

// Y[idx[c]] = Z X[idx[c]] for c < m <= 8 FP64 vectors (device idx), FP64 accumulation.
// part: FP64 partial sums of the K-split product, gemv_multi_part_bytes(n) bytes
// (nullptr: no split)
void gemv_multi(const void* Z, int zdt, int n, const double2* X, const int* idx, int m, double2* Y, hipStream_t s,
                double2* part);
size_t gemv_multi_part_bytes(int n);

// complex64 staging of selected FP64 rows and the way back
void gather_cast(const double2* X, const int* idx, int m, int n, float2* out, hipStream_t s);
void scatter_cast(const float2* in, const int* idx, int m, int n, double2* Y, hipStream_t s);

// Y (M x n, complex64) = X (M x n, complex64) * Z^T (Z n x n complex64) on FP32 matrix cores.
// mcap: rows of X that may be read (>= M; the rows past M are computed and dropped).
void cgemm_mfma(const void* X, const void* Z, void* Y, int M, int n, hipStream_t s, int mcap = 0);
bool cgemm_mfma_supported(int M, int n);
// Y[yrow[r]] (complex128) = sum_j X[r][j] Z[i][j]: same product with the FP32 matrix-core
// partial sums flushed into FP64 accumulators every two K chunks.  mcap: rows of X
// that may be read (>= M; the rows past M are computed and dropped); small_tile:
// M <= 32 takes the 32-row tile instead of the selected one.
void cgemm_mfma_acc64(const void* X, const void* Z, double2* Y, const int* yrow, int M, int n, hipStream_t s,
                      int mcap = 0, bool small_tile = false);

void cast_c128_to_c64(const void* a, void* b, size_t n, hipStream_t s);
void cast_c64_to_c128(const void* a, void* b, size_t n, hipStream_t s);

void fill_zero_bytes(void* p, size_t bytes, hipStream_t s);

// Y = Z X with the library's product choice (GEMV for one right-hand side,
// matrix cores for complex64, FP64 GEMM for complex128).  X, Y of dtype xdt.
void zx_product(const void* Z, int zdt, int n, const void* X, int xdt, void* Y, int nrhs, hipStream_t s);

}  // namespace efie

// Internal dense linear-algebra dispatchers (see linalg.hip, gemm_mfma.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace efie {

// y = Z x (single right-hand side); dtypes EFIE_C128 / EFIE_C64 per operand.
void gemv(const void* Z, int zdt, int n, const void* x, int xdt, void* y, int ydt, hipStream_t s);

// C[M][Nc] (+)= alpha * sum_k A[M][k] B[Nc][k], FP64 accumulation.
void zgemm_nt(const void* A, int adt, const void* B, int bdt, void* C, int cdt, int M, int Nc, int K, int lda,
              int ldb, int ldc, double alr, double ali, bool accumulate, hipStream_t s);

// Y (M x n, complex64) = X (M x n, complex64) * Z^T (Z n x n complex64) on FP32 matrix cores.
void cgemm_mfma(const void* X, const void* Z, void* Y, int M, int n, hipStream_t s);
bool cgemm_mfma_supported(int M, int n);

void cast_c128_to_c64(const void* a, void* b, size_t n, hipStream_t s);
void cast_c64_to_c128(const void* a, void* b, size_t n, hipStream_t s);

void fill_zero_bytes(void* p, size_t bytes, hipStream_t s);

// Y = Z X with the library's product choice (GEMV for one right-hand side,
// matrix cores for complex64, FP64 GEMM for complex128).  X, Y of dtype xdt.
void zx_product(const void* Z, int zdt, int n, const void* X, int xdt, void* Y, int nrhs, hipStream_t s);

}  // namespace efie

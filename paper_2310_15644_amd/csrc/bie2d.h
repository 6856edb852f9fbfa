// Internal declarations of the 2-D path (the paper's own method on a closed
// curve): geometry tables, the FP64 matrix-core GEMM with NT / NN / circulant
// operands, and the small dense factorizations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "efie_internal.h"

namespace efie {

// Structure-of-arrays tables of one closed polygon (device pointers into the
// caller's blob).  Segment a runs from node a to node a+1 (mod n).
struct DevContour {
    int32_t n;            // nodes = segments
    int32_t q;            // Gauss points per segment of the regular rule
    const double *ax, *ay, *bx, *by;   // segment start / end
    const double *len, *nx, *ny;       // length, outward unit normal
    const double *gx, *gw;             // q-point Gauss-Legendre rule on [0, 1]
    const double *hx, *hw;             // 8-point rule of the near-pair rules
};

enum Gemm2dOp { G2D_NT = 0, G2D_NN = 1, G2D_CIRC = 2 };

// C (M x Nc, ldc) = alpha * A op(B) (+ C if accumulate), FP64 matrix cores.
//   A: M x K row-major (lda), conjugated if conja.
//   NT:   B is Nc x K (ldb):  C[s][i] = sum_k A[s][k] B[i][k]
//   NN:   B is K x Nc (ldb):  C[s][i] = sum_k A[s][k] B[k][i]
//   CIRC: B is a vector c of length K = Nc: C[s][i] = sum_k A[s][k] c[(i - k) mod K]
//   B conjugated if conjb.
// With scratch (scratch_elems complex values), products with few output tiles and
// a long contraction are split along K into partial products reduced in a second
// pass (deterministic; no atomics).
void gemm2d(int op, const double2* A, int lda, bool conja, const double2* B, int ldb, bool conjb, double2* C,
            int ldc, int M, int Nc, int K, double2 alpha, bool accumulate, hipStream_t s, double2* scratch = nullptr,
            size_t scratch_elems = 0);

}  // namespace efie

// Krylov solves of Z J = V for many right-hand sides (columns), x0 = 0.
//
// Only active (unconverged) columns enter the Z-products: a compaction kernel
// lists them after every step, up to 8 columns use a multi-column GEMV (Z read
// once, FP64 accumulation) and more use the GEMM on the gathered columns.
//
// The paper names CG and CGS but states neither; the readings implemented are
//   COCG (van der Vorst and Melissen 1990): CG with the unconjugated bilinear
//        form a^T b, valid because Z = Z^T; one product Z p per iteration;
//   CGS  (Sonneveld 1989): conjugated inner products, shadow residual r~ = r0;
//        two products per iteration.
// Stopping rule: ||r_k||_2 <= tol ||b||_2 on the recurrence residual.
//
// Structure.  The host drives the iteration.  Each iteration launches the
// Z-products for all columns at once (GEMV for one column, GEMM otherwise) and
// one fused kernel per algorithm step in which one thread block owns one column:
// it reduces the inner products (FP64, fixed order, hence deterministic),
// forms the scalars and updates the vectors, and clears the column's active flag
// on convergence, breakdown or NaN.  The host reads the number of active
// columns after each iteration (one 4-byte copy).
//
// Mixed precision (complex64 Z).  COCG: one Krylov solve whose Z-products run on
// FP32 matrix cores, with reliable updates (Sleijpen and van der Vorst,
// Computing 56, 1996): whenever a column's recursive residual has dropped by a
// factor 10 since its last replacement, or claims convergence, it is replaced by
// the true residual V - Z J accumulated in FP64 from the stored complex64 Z, and
// only the true residual may declare convergence.  This keeps the FP32
// accumulation error of the products (~1e-5 ||Z|| ||p||, amplified along
// near-resonant directions) out of the recurrence.  CGS: an outer refinement
// loop around inner CGS solves.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "efie_internal.h"
#include "linalg.h"

namespace efie {

struct Col {
    double rho_r, rho_i;    // current rho (COCG: r^T r, CGS: r~^H r)
    double alpha_r, alpha_i;
    double bn2;             // ||b||^2
    double rn2;             // ||r||^2 (recurrence)
    double tol2;            // tol^2 ||b||^2
    double rn2_ref;         // ||r||^2 at the last true-residual replacement (reliable updates)
    int active, iters, status, upd;   // upd: true residual requested (mixed-precision COCG)
    int since;              // iterations since the last replacement
    int rst;                // restart the search direction at the next replacement
    int pad2[2];
};

constexpr int KB = 512;   // threads per column block

struct C2 {
    double r, i;
};
__device__ __forceinline__ C2 cmul(C2 a, C2 b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ C2 cdiv(C2 a, C2 b) {
    double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

// Block-wide sum of NV doubles; every thread gets the totals.
template <int NV>
__device__ void block_sum(double (&v)[NV], double* sh) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int u = 0; u < KB / 64; ++u) s += sh[u * NV + k];
        v[k] = s;
    }
}

__device__ __forceinline__ void finish_check(Col& c, double rn2) {
    c.rn2 = rn2;
    if (!(rn2 == rn2) || rn2 > 1e300) {
        c.status = EFIE_ERR_NAN;
        c.active = 0;
    } else if (rn2 <= c.tol2) {
        c.status = EFIE_OK;
        c.active = 0;
    }
}

// ------------------------------------------------------------------ COCG
// init: x = 0, r = b, p = r, rho = r^T r
__global__ __launch_bounds__(KB) void cocg_init(const double2* b, double2* x, double2* r, double2* p, Col* cols,
                                                int n, double tol) {
    __shared__ double sh[KB / 64 * 4];
    const int s = blockIdx.x;
    const double2* bs = b + size_t(s) * n;
    double v[4] = {0, 0, 0, 0};   // rho_r, rho_i, ||b||^2
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 e = bs[k];
        x[size_t(s) * n + k] = make_double2(0, 0);
        r[size_t(s) * n + k] = e;
        p[size_t(s) * n + k] = e;
        v[0] += e.x * e.x - e.y * e.y;
        v[1] += 2.0 * e.x * e.y;
        v[2] += e.x * e.x + e.y * e.y;
    }
    block_sum<4>(v, sh);
    if (threadIdx.x == 0) {
        Col c{};
        c.rho_r = v[0];
        c.rho_i = v[1];
        c.bn2 = v[2];
        c.tol2 = tol * tol * v[2];
        c.rn2_ref = v[2];
        c.active = 1;
        c.status = EFIE_NOT_CONVERGED;
        c.iters = 0;
        c.upd = 0;
        c.since = 0;
        c.rst = 0;
        finish_check(c, v[2]);
        if (v[2] == 0.0) c.status = EFIE_OK;
        cols[s] = c;
    }
}

// one COCG step after q = Z p:  mu = p^T q, alpha = rho/mu, x += alpha p,
// r -= alpha q, rho' = r^T r, beta = rho'/rho, p = r + beta p.
__global__ __launch_bounds__(KB) void cocg_step(double2* x, double2* r, double2* p, const double2* q, Col* cols,
                                                int n, int* counters, int reliable) {
    __shared__ double sh[KB / 64 * 4];
    __shared__ int go;
    const int s = blockIdx.x;
    if (threadIdx.x == 0) go = cols[s].active;
    __syncthreads();
    if (!go) return;
    const size_t o = size_t(s) * n;
    double v[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 pp = p[o + k], qq = q[o + k];
        v[0] += pp.x * qq.x - pp.y * qq.y;
        v[1] += pp.x * qq.y + pp.y * qq.x;
    }
    block_sum<4>(v, sh);
    Col c = cols[s];
    const C2 mu{v[0], v[1]};
    if (mu.r == 0.0 && mu.i == 0.0) {
        if (threadIdx.x == 0) {
            cols[s].status = EFIE_ERR_BREAKDOWN;
            cols[s].active = 0;
        }
        return;
    }
    const C2 alpha = cdiv(C2{c.rho_r, c.rho_i}, mu);
    double w[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 pp = p[o + k], qq = q[o + k], xx = x[o + k], rr = r[o + k];
        xx.x += alpha.r * pp.x - alpha.i * pp.y;
        xx.y += alpha.r * pp.y + alpha.i * pp.x;
        rr.x -= alpha.r * qq.x - alpha.i * qq.y;
        rr.y -= alpha.r * qq.y + alpha.i * qq.x;
        x[o + k] = xx;
        r[o + k] = rr;
        w[0] += rr.x * rr.x - rr.y * rr.y;
        w[1] += 2.0 * rr.x * rr.y;
        w[2] += rr.x * rr.x + rr.y * rr.y;
    }
    block_sum<4>(w, sh);
    const C2 rho_new{w[0], w[1]};
    if (rho_new.r == 0.0 && rho_new.i == 0.0 && w[2] > c.tol2) {
        if (threadIdx.x == 0) {
            cols[s].status = EFIE_ERR_BREAKDOWN;
            cols[s].active = 0;
            cols[s].rn2 = w[2];
            cols[s].iters = c.iters + 1;
        }
        return;
    }
    const C2 beta = cdiv(rho_new, C2{c.rho_r, c.rho_i});
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 pp = p[o + k], rr = r[o + k];
        double2 np;
        np.x = rr.x + beta.r * pp.x - beta.i * pp.y;
        np.y = rr.y + beta.r * pp.y + beta.i * pp.x;
        p[o + k] = np;
    }
    if (threadIdx.x == 0) {
        c.rho_r = rho_new.r;
        c.rho_i = rho_new.i;
        c.iters += 1;
        if (reliable) {
            // the recursive residual only requests a true one; it never converges alone.
            // Replacement after a tenfold drop, on a convergence claim, or after
            // 100 iterations without one (bounds the drift of a stalled column).
            c.rn2 = w[2];
            c.since += 1;
            if (!(w[2] == w[2]) || w[2] > 1e300) {
                c.status = EFIE_ERR_NAN;
                c.active = 0;
            } else if (w[2] <= c.tol2 || w[2] < 0.01 * c.rn2_ref || c.since >= 100) {
                c.upd = 1;
                atomicAdd(counters + 1, 1);
            }
        } else {
            finish_check(c, w[2]);
        }
        cols[s] = c;
        if (c.active) atomicAdd(counters, 1);
    }
}

// Reliable update of the flagged columns: r = b - y (y = Z x with FP64
// accumulation), rho = r^T r, and convergence decided on the true residual.
// If the true residual norm exceeds the recursive one by more than sqrt(10), the
// recurrence has lost track of it (or a restart was requested): the search
// direction restarts, p = r.
__global__ __launch_bounds__(KB) void cocg_replace(const double2* b, double2* r, double2* p, const double2* y,
                                                   Col* cols, int n, const int* idx, int* counters) {
    __shared__ double sh[KB / 64 * 4];
    const int s = idx[blockIdx.x];
    const size_t o = size_t(s) * n;
    const double rec = cols[s].rn2;   // read before block_sum's barriers; thread 0 rewrites cols[s] after them
    const int rst = cols[s].rst;
    double a[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        const double2 bb = b[o + k], yy = y[o + k];
        const double2 d = make_double2(bb.x - yy.x, bb.y - yy.y);
        r[o + k] = d;
        a[0] += d.x * d.x - d.y * d.y;
        a[1] += 2.0 * d.x * d.y;
        a[2] += d.x * d.x + d.y * d.y;
    }
    block_sum<4>(a, sh);
    if (a[2] > 10.0 * rec || rst)
        for (int k = threadIdx.x; k < n; k += KB) p[o + k] = r[o + k];
    if (threadIdx.x == 0) {
        Col c = cols[s];
        c.rho_r = a[0];
        c.rho_i = a[1];
        c.rn2_ref = a[2];
        c.upd = 0;
        c.since = 0;
        c.rst = 0;
        finish_check(c, a[2]);
        cols[s] = c;
        if (!c.active) atomicSub(counters, 1);
    }
}

// ------------------------------------------------------------------- CGS
// vectors: r, rt (shadow), u, p, q, v (also holds t), w
__global__ __launch_bounds__(KB) void cgs_init(const double2* b, double2* x, double2* r, double2* rt, double2* u,
                                               double2* p, Col* cols, int n, double tol) {
    __shared__ double sh[KB / 64 * 4];
    const int s = blockIdx.x;
    const size_t o = size_t(s) * n;
    double v[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 e = b[o + k];
        x[o + k] = make_double2(0, 0);
        r[o + k] = e;
        rt[o + k] = e;
        u[o + k] = e;
        p[o + k] = e;
        v[0] += e.x * e.x + e.y * e.y;
    }
    block_sum<4>(v, sh);
    if (threadIdx.x == 0) {
        Col c{};
        c.rho_r = v[0];   // r~^H r = ||r0||^2
        c.rho_i = 0.0;
        c.bn2 = v[0];
        c.tol2 = tol * tol * v[0];
        c.active = 1;
        c.status = EFIE_NOT_CONVERGED;
        finish_check(c, v[0]);
        if (v[0] == 0.0) c.status = EFIE_OK;
        cols[s] = c;
    }
}

// after v = Z p: sigma = r~^H v, alpha = rho/sigma, q = u - alpha v, w = u + q, x += alpha w
__global__ __launch_bounds__(KB) void cgs_step1(double2* x, const double2* rt, const double2* u, const double2* v,
                                                double2* q, double2* w, Col* cols, int n) {
    __shared__ double sh[KB / 64 * 4];
    __shared__ int go;
    const int s = blockIdx.x;
    if (threadIdx.x == 0) go = cols[s].active;
    __syncthreads();
    if (!go) return;
    const size_t o = size_t(s) * n;
    double a[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 t = rt[o + k], vv = v[o + k];
        a[0] += t.x * vv.x + t.y * vv.y;    // conj(rt) v
        a[1] += t.x * vv.y - t.y * vv.x;
    }
    block_sum<4>(a, sh);
    const C2 sigma{a[0], a[1]};
    Col c = cols[s];
    if (sigma.r == 0.0 && sigma.i == 0.0) {
        if (threadIdx.x == 0) {
            cols[s].status = EFIE_ERR_BREAKDOWN;
            cols[s].active = 0;
        }
        return;
    }
    const C2 alpha = cdiv(C2{c.rho_r, c.rho_i}, sigma);
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 uu = u[o + k], vv = v[o + k], xx = x[o + k];
        double2 qq, ww;
        qq.x = uu.x - (alpha.r * vv.x - alpha.i * vv.y);
        qq.y = uu.y - (alpha.r * vv.y + alpha.i * vv.x);
        ww.x = uu.x + qq.x;
        ww.y = uu.y + qq.y;
        xx.x += alpha.r * ww.x - alpha.i * ww.y;
        xx.y += alpha.r * ww.y + alpha.i * ww.x;
        q[o + k] = qq;
        w[o + k] = ww;
        x[o + k] = xx;
    }
    if (threadIdx.x == 0) {
        cols[s].alpha_r = alpha.r;
        cols[s].alpha_i = alpha.i;
    }
}

// after t = Z w: r -= alpha t, rho' = r~^H r, beta = rho'/rho, u = r + beta q,
// p = u + beta (q + beta p)
__global__ __launch_bounds__(KB) void cgs_step2(double2* r, const double2* rt, double2* u, double2* p,
                                                const double2* q, const double2* t, Col* cols, int n, int* counters) {
    __shared__ double sh[KB / 64 * 4];
    __shared__ int go;
    const int s = blockIdx.x;
    if (threadIdx.x == 0) go = cols[s].active;
    __syncthreads();
    if (!go) return;
    const size_t o = size_t(s) * n;
    Col c = cols[s];
    const C2 alpha{c.alpha_r, c.alpha_i};
    double a[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 rr = r[o + k], tt = t[o + k], sh_ = rt[o + k];
        rr.x -= alpha.r * tt.x - alpha.i * tt.y;
        rr.y -= alpha.r * tt.y + alpha.i * tt.x;
        r[o + k] = rr;
        a[0] += sh_.x * rr.x + sh_.y * rr.y;
        a[1] += sh_.x * rr.y - sh_.y * rr.x;
        a[2] += rr.x * rr.x + rr.y * rr.y;
    }
    block_sum<4>(a, sh);
    const C2 rho_new{a[0], a[1]};
    if (rho_new.r == 0.0 && rho_new.i == 0.0 && a[2] > c.tol2) {
        if (threadIdx.x == 0) {
            cols[s].status = EFIE_ERR_BREAKDOWN;
            cols[s].active = 0;
            cols[s].rn2 = a[2];
            cols[s].iters = c.iters + 1;
        }
        return;
    }
    const C2 beta = cdiv(rho_new, C2{c.rho_r, c.rho_i});
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 rr = r[o + k], qq = q[o + k], pp = p[o + k];
        double2 uu, np, tq;
        uu.x = rr.x + beta.r * qq.x - beta.i * qq.y;
        uu.y = rr.y + beta.r * qq.y + beta.i * qq.x;
        tq.x = qq.x + beta.r * pp.x - beta.i * pp.y;
        tq.y = qq.y + beta.r * pp.y + beta.i * pp.x;
        np.x = uu.x + beta.r * tq.x - beta.i * tq.y;
        np.y = uu.y + beta.r * tq.y + beta.i * tq.x;
        u[o + k] = uu;
        p[o + k] = np;
    }
    if (threadIdx.x == 0) {
        c.rho_r = rho_new.r;
        c.rho_i = rho_new.i;
        c.iters += 1;
        finish_check(c, a[2]);
        cols[s] = c;
        if (c.active) atomicAdd(counters, 1);
    }
}

// ----------------------------------------------------------- helper kernels
// List the columns whose flag (active, or upd) is set, in increasing order; one block.
__global__ __launch_bounds__(1024) void compact_kernel(const Col* cols, int S, int which, int* idx, int* count) {
    __shared__ int wsum[16];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int s0 = 0; s0 < S; s0 += 1024) {
        const int s = s0 + threadIdx.x;
        const int f = s < S ? (which == 0 ? cols[s].active : cols[s].upd) : 0;
        // inclusive scan inside the wavefront
        int v = f;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(v, o, 64);
            if (lane >= o) v += t;
        }
        if (lane == 63) wsum[w] = v;
        __syncthreads();
        int off = base;
        for (int u = 0; u < w; ++u) off += wsum[u];
        if (f) idx[off + v - 1] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int u = 0; u < 16; ++u) tot += wsum[u];
            base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// out = b - y, and per-column ||out||^2 into nrm[s], for the columns s = idx[block]
// (idx == nullptr: s = block)
__global__ __launch_bounds__(KB) void residual_kernel(const double2* b, const double2* y, double2* out, double* nrm,
                                                      double* bnrm, int n, const int* __restrict__ idx) {
    __shared__ double sh[KB / 64 * 4];
    const int s = idx ? idx[blockIdx.x] : int(blockIdx.x);
    const size_t o = size_t(s) * n;
    double a[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += KB) {
        double2 bb = b[o + k], yy = y[o + k];
        double2 d = make_double2(bb.x - yy.x, bb.y - yy.y);
        if (out) out[o + k] = d;
        a[0] += d.x * d.x + d.y * d.y;
        a[1] += bb.x * bb.x + bb.y * bb.y;
    }
    block_sum<4>(a, sh);
    if (threadIdx.x == 0) {
        nrm[s] = a[0];
        bnrm[s] = a[1];
    }
}

__global__ void axpy_inplace_kernel(double2* x, const double2* d, size_t n) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        double2 a = x[i], b = d[i];
        x[i] = make_double2(a.x + b.x, a.y + b.y);
    }
}

// flag every active column for a replacement with restart
__global__ void force_replace_kernel(Col* cols, int S, int* counters) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x)
        if (cols[s].active) {
            cols[s].upd = 1;
            cols[s].rst = 1;
            atomicAdd(counters + 1, 1);
        }
}

// Y[idx[c]] += X[idx[c]] for the m listed rows (n elements each)
__global__ void add_rows_kernel(double2* __restrict__ Y, const double2* __restrict__ X, const int* __restrict__ idx,
                                int n) {
    const size_t o = size_t(idx[blockIdx.y]) * n;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const double2 a = Y[o + k], b = X[o + k];
        Y[o + k] = make_double2(a.x + b.x, a.y + b.y);
    }
}

__global__ void iota_kernel(int* idx, int S) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) idx[i] = i;
}

// EFIE_VERBOSE=1 prints solver and Calderon-build progress to stderr (iteration counts, active columns, time)
bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("EFIE_VERBOSE");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}
double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

namespace {

struct Ws {
    double2 *r, *rt, *u, *p, *q, *v, *w;   // Krylov vectors (S x n each)
    double2 *res, *dlt;                     // outer refinement (CGS, mixed): residual and correction
    float2* x32;                            // complex64 staging of the product input
    int x32_rows;                           // its rows (S rounded up to 128)
    float2* y32;                            // complex64 product output (FP32 accumulation)
    bool acc64;                             // FP64 flush of the matrix-core partial sums
    double2* part;                          // partial sums of the K-split product of <= 8 columns
    Col* cols;
    double *nrm, *bnrm;
    int* counters;                          // [0] active, [1] flagged for a true residual, [2] count
    int *idx_a, *idx_u, *idx_all;           // column lists: active, flagged, all
    int* idx_ref;                           // columns still refined (preconditioned solve)
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
int64_t x32_rows(int64_t S) { return (S + 127) / 128 * 128; }


size_t layout(int64_t n, int64_t S, int dtype, Ws* ws, char* base) {
    const size_t vec = align256(size_t(n) * size_t(S) * 16);
    // the complex64 staging of the product input holds S rounded up to 128 rows, so
    // that every tile of the matrix-core product reads whole tiles (the rows past
    // the active columns are computed and dropped)
    const size_t vec32 = dtype == EFIE_C64 && S > 1 ? align256(size_t(n) * size_t(x32_rows(S)) * 8) : 0;
    const size_t outer = dtype == EFIE_C64 ? vec : 0;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    Ws w{};
    w.x32_rows = int(x32_rows(S));
    w.r = (double2*)take(vec); w.rt = (double2*)take(vec); w.u = (double2*)take(vec); w.p = (double2*)take(vec);
    w.q = (double2*)take(vec); w.v = (double2*)take(vec); w.w = (double2*)take(vec);
    w.res = (double2*)take(outer); w.dlt = (double2*)take(outer);
    w.x32 = (float2*)take(vec32);
    w.y32 = (float2*)take(vec32);
    w.part = (double2*)take(gemv_multi_part_bytes(int(n)));
    w.cols = (Col*)take(sizeof(Col) * size_t(S));
    w.nrm = (double*)take(sizeof(double) * size_t(S));
    w.bnrm = (double*)take(sizeof(double) * size_t(S));
    w.counters = (int*)take(sizeof(int) * 4);
    w.idx_a = (int*)take(sizeof(int) * size_t(S));
    w.idx_u = (int*)take(sizeof(int) * size_t(S));
    w.idx_all = (int*)take(sizeof(int) * size_t(S));
    w.idx_ref = (int*)take(sizeof(int) * size_t(S));
    if (ws) *ws = w;
    return off;
}

// Y[idx[c]] = Z X[idx[c]] for the m listed columns.  exact64: FP64 accumulation
// for every m (true residuals); otherwise complex64 Z with m > 8 uses the FP32
// matrix cores on complex64 copies of the columns, accumulating in FP32 (the
// complex64 result is then widened into the rows) or, with w.acc64, flushing the
// partial sums of every K chunk into FP64 accumulators.
void product(const void* Z, int zdt, int n, const double2* X, double2* Y, const int* idx, int m, bool exact64,
             const Ws& w, hipStream_t st) {
    if (m <= 0) return;
    if (m <= 8) {
        gemv_multi(Z, zdt, n, X, idx, m, Y, st, w.part);
    } else if (zdt == EFIE_C64 && !exact64) {
        gather_cast(X, idx, m, n, w.x32, st);
        if (w.acc64) {
            cgemm_mfma_acc64(w.x32, Z, Y, idx, m, n, st, w.x32_rows, true);
        } else {
            cgemm_mfma(w.x32, Z, w.y32, m, n, st, w.x32_rows);
            scatter_cast(w.y32, idx, m, n, Y, st);
        }
    } else {
        zgemm_nt(X, EFIE_C128, Z, zdt, Y, EFIE_C128, m, n, n, n, n, n, 1.0, 0.0, false, st, idx, idx);
    }
}

// The operator of a solve: Z, or P Z with a dense FP64 left factor P (the
// Calderon product), or P Z + Q M (the Calderon-stabilized CFIE, every factor
// complex128); tmp holds Z X for the rows in flight, tmp2 and tmp3 M X and Q M X.
struct Op {
    const void* Z;
    int zdt;
    const void* P;   // optional left factor (dtype pdt)
    double2* tmp;
    int pdt = EFIE_C128;
    const void* M = nullptr;   // optional second term Q M (complex128)
    const void* Q = nullptr;
    double2* tmp2 = nullptr;
    double2* tmp3 = nullptr;
};

void op_product(const Op& op, int n, const double2* X, double2* Y, const int* idx, int m, bool exact64, const Ws& w,
                hipStream_t st) {
    if (!op.P) {
        product(op.Z, op.zdt, n, X, Y, idx, m, exact64, w, st);
        return;
    }
    product(op.Z, op.zdt, n, X, op.tmp, idx, m, exact64, w, st);
    product(op.P, op.pdt, n, op.tmp, Y, idx, m, exact64 || op.pdt == EFIE_C128, w, st);
    if (op.M && m > 0) {
        product(op.M, EFIE_C128, n, X, op.tmp2, idx, m, true, w, st);
        product(op.Q, EFIE_C128, n, op.tmp2, op.tmp3, idx, m, true, w, st);
        hipLaunchKernelGGL(add_rows_kernel, dim3(unsigned(std::min(64, (n + 255) / 256)), unsigned(m)), dim3(256), 0,
                           st, Y, op.tmp3, idx, n);
    }
}

int compact(const Ws& w, int S, int which, int* idx, hipStream_t st) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, st, w.cols, S, which, idx, w.counters + 2);
    int h = 0;
    EFIE_HIP_CHECK(hipMemcpyAsync(&h, w.counters + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    EFIE_HIP_CHECK(hipStreamSynchronize(st));
    return h;
}

// FP64-accumulated residual out = b - Z x (Z of either dtype) for the m columns
// listed in idx; their norms into w.nrm / w.bnrm (other columns untouched).
void true_residual(const void* Z, int zdt, int n, const double2* b, const double2* x, double2* out,
                   const int* idx, int m, const Ws& w, hipStream_t st) {
    if (m <= 0) return;
    double2* y = w.q;   // scratch
    product(Z, zdt, n, x, y, idx, m, true, w, st);
    hipLaunchKernelGGL(residual_kernel, dim3(m), dim3(KB), 0, st, b, y, out, w.nrm, w.bnrm, n, idx);
}

// One Krylov solve of Z x = b for S columns.  Returns per-column Col states in host memory.
void krylov(const Op& op, int n, const double2* b, double2* x, int S, int solver, double tol, int maxit,
            bool reliable, const Ws& w, std::vector<Col>& out, hipStream_t st) {
    int h[2] = {0, 0};
    if (solver == EFIE_COCG) {
        hipLaunchKernelGGL(cocg_init, dim3(S), dim3(KB), 0, st, b, x, w.r, w.p, w.cols, n, tol);
        int m = compact(w, S, 0, w.idx_a, st);
        // products are FP64-accurate once at most 8 columns remain: on entering that
        // regime every remaining column restarts from its true residual
        bool exact_regime = !reliable || m <= 8;
        for (int it = 0; it < maxit && m > 0; ++it) {
            op_product(op, n, w.p, w.q, w.idx_a, m, false, w, st);
            fill_zero_bytes(w.counters, 2 * sizeof(int), st);
            hipLaunchKernelGGL(cocg_step, dim3(S), dim3(KB), 0, st, x, w.r, w.p, w.q, w.cols, n, w.counters,
                               int(reliable));
            if (!exact_regime && m <= 8) {
                exact_regime = true;
                hipLaunchKernelGGL(force_replace_kernel, dim3((S + 255) / 256), dim3(256), 0, st, w.cols, S,
                                   w.counters);
            }
            EFIE_HIP_CHECK(hipMemcpyAsync(h, w.counters, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
            EFIE_HIP_CHECK(hipStreamSynchronize(st));
            if (reliable && h[1] > 0) {
                const int mu = compact(w, S, 1, w.idx_u, st);
                op_product(op, n, x, w.v, w.idx_u, mu, true, w, st);
                hipLaunchKernelGGL(cocg_replace, dim3(mu), dim3(KB), 0, st, b, w.r, w.p, w.v, w.cols, n, w.idx_u,
                                   w.counters);
            }
            m = compact(w, S, 0, w.idx_a, st);
            if (verbose() && (it % 50 == 0 || m == 0))
                std::fprintf(stderr, "[efie] cocg it %d active %d/%d replaced %d t=%.3f\n", it, m, S,
                             reliable ? h[1] : 0, now_s()),
                    std::fflush(stderr);
        }
    } else {
        hipLaunchKernelGGL(cgs_init, dim3(S), dim3(KB), 0, st, b, x, w.r, w.rt, w.u, w.p, w.cols, n, tol);
        int m = compact(w, S, 0, w.idx_a, st);
        for (int it = 0; it < maxit && m > 0; ++it) {
            op_product(op, n, w.p, w.v, w.idx_a, m, false, w, st);
            hipLaunchKernelGGL(cgs_step1, dim3(S), dim3(KB), 0, st, x, w.rt, w.u, w.v, w.q, w.w, w.cols, n);
            op_product(op, n, w.w, w.v, w.idx_a, m, false, w, st);
            fill_zero_bytes(w.counters, 2 * sizeof(int), st);
            hipLaunchKernelGGL(cgs_step2, dim3(S), dim3(KB), 0, st, w.r, w.rt, w.u, w.p, w.q, w.v, w.cols, n,
                               w.counters);
            m = compact(w, S, 0, w.idx_a, st);
            if (verbose() && (it % 50 == 0 || m == 0))
                std::fprintf(stderr, "[efie] cgs it %d active %d/%d t=%.3f\n", it, m, S, now_s()), std::fflush(stderr);
        }
    }
    EFIE_HIP_CHECK(hipGetLastError());
    out.resize(S);
    EFIE_HIP_CHECK(hipMemcpyAsync(out.data(), w.cols, sizeof(Col) * S, hipMemcpyDeviceToHost, st));
    EFIE_HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace
}  // namespace efie

extern "C" int efie_solve_workspace_size(int64_t n, int64_t nrhs, int dtype, size_t* bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(bytes && n >= 1 && nrhs >= 1, EFIE_ERR_ARG, "solve_workspace_size: bad argument");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "solve_workspace_size: bad dtype");
        *bytes = efie::layout(n, nrhs, dtype, nullptr, nullptr);
        return int(EFIE_OK);
    });
}

extern "C" int efie_solve(const void* Z, int dtype, int64_t n, const void* V, void* J, int64_t nrhs,
                          const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE(Z && V && J && opts && ws, EFIE_ERR_ARG, "solve: null argument");
        EFIE_REQUIRE(dtype == EFIE_C128 || dtype == EFIE_C64, EFIE_ERR_ARG, "solve: bad dtype");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && nrhs >= 1 && nrhs <= 65535, EFIE_ERR_ARG,
                     "solve: bad sizes");
        EFIE_REQUIRE(opts->solver == EFIE_COCG || opts->solver == EFIE_CGS, EFIE_ERR_ARG, "solve: bad solver");
        EFIE_REQUIRE(opts->maxit >= 1 && opts->tol > 0.0, EFIE_ERR_ARG, "solve: need maxit >= 1 and tol > 0");
        const size_t need = layout(n, nrhs, dtype, nullptr, nullptr);
        EFIE_REQUIRE(ws_bytes >= need, EFIE_ERR_ARG, "solve: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "solve: workspace not 256-aligned");
        Ws w;
        layout(n, nrhs, dtype, &w, static_cast<char*>(ws));
        w.acc64 = opts->fp32_acc == 0;
        const int S = int(nrhs), nn = int(n);
        hipLaunchKernelGGL(iota_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, w.idx_all, S);
        const double2* b = static_cast<const double2*>(V);
        double2* x = static_cast<double2*>(J);
        std::vector<Col> cols;
        std::vector<int> iters(S, 0);
        std::vector<double> recur(S, 0.0);
        if (dtype == EFIE_C128 || opts->solver == EFIE_COCG) {
            // FP64 operator, or mixed precision with reliable updates
            krylov(Op{Z, dtype, nullptr, nullptr}, nn, b, x, S, opts->solver, opts->tol, opts->maxit, dtype == EFIE_C64, w,
                   cols, stream);
            for (int s = 0; s < S; ++s) {
                iters[s] = cols[s].iters;
                recur[s] = cols[s].bn2 > 0 ? std::sqrt(cols[s].rn2 / cols[s].bn2) : 0.0;
            }
        } else {
            EFIE_REQUIRE(opts->max_refine >= 1 && opts->inner_tol > 0.0, EFIE_ERR_ARG,
                         "solve: mixed precision needs max_refine >= 1 and inner_tol > 0");
            fill_zero_bytes(x, size_t(nn) * S * 16, stream);
            std::vector<double> h_nrm(S), h_bn(S);
            for (int outer = 0; outer < opts->max_refine; ++outer) {
                if (outer > 0) {
                    true_residual(Z, dtype, nn, b, x, w.res, w.idx_all, S, w, stream);
                    EFIE_HIP_CHECK(hipMemcpyAsync(h_nrm.data(), w.nrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
                    EFIE_HIP_CHECK(hipMemcpyAsync(h_bn.data(), w.bnrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
                    EFIE_HIP_CHECK(hipStreamSynchronize(stream));
                    bool done = true;
                    double worst = 0.0;
                    for (int s = 0; s < S; ++s) {
                        if (h_nrm[s] > opts->tol * opts->tol * h_bn[s]) done = false;
                        worst = std::max(worst, h_bn[s] > 0 ? std::sqrt(h_nrm[s] / h_bn[s]) : 0.0);
                    }
                    if (verbose())
                        std::fprintf(stderr, "[efie] refine %d worst relres %.3e t=%.3f\n", outer, worst, now_s()),
                            std::fflush(stderr);
                    if (done) break;
                } else {
                    EFIE_HIP_CHECK(hipMemcpyAsync(w.res, b, size_t(nn) * S * 16, hipMemcpyDeviceToDevice, stream));
                }
                // inner solve Z d = res to inner_tol (columns already converged have a
                // residual below tol; the inner solve then stops at once or adds little)
                krylov(Op{Z, dtype, nullptr, nullptr}, nn, w.res, w.dlt, S, opts->solver, opts->inner_tol, opts->maxit,
                       false, w, cols, stream);
                const size_t tot = size_t(nn) * S;
                hipLaunchKernelGGL(axpy_inplace_kernel, dim3(int(std::min<size_t>((tot + 255) / 256, 16384))),
                                   dim3(256), 0, stream, x, w.dlt, tot);
                for (int s = 0; s < S; ++s) {
                    iters[s] += cols[s].iters;
                    recur[s] = cols[s].bn2 > 0 ? std::sqrt(cols[s].rn2 / cols[s].bn2) : 0.0;
                }
            }
        }
        // true residual at exit (FP64 accumulation)
        true_residual(Z, dtype, nn, b, x, nullptr, w.idx_all, S, w, stream);
        std::vector<double> h_nrm(S), h_bn(S);
        EFIE_HIP_CHECK(hipMemcpyAsync(h_nrm.data(), w.nrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(h_bn.data(), w.bnrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        int ret = EFIE_OK;
        for (int s = 0; s < S; ++s) {
            const double rel = h_bn[s] > 0 ? std::sqrt(h_nrm[s] / h_bn[s]) : 0.0;
            // FP64 operator: the recurrence stopping rule decides; mixed precision:
            // the FP64-accumulated true residual of the outer loop decides.
            int st = cols[s].status;
            if (dtype == EFIE_C64 && st >= 0) st = rel <= opts->tol ? EFIE_OK : EFIE_NOT_CONVERGED;
            if (!(rel == rel)) st = EFIE_ERR_NAN;
            if (stats) {
                stats[s].iters = iters[s];
                stats[s].status = st;
                stats[s].relres_recur = recur[s];
                stats[s].relres_true = rel;
            }
            // per-column breakdown / NaN is reported in stats; the call returns a warning
            if (st != EFIE_OK) ret = EFIE_NOT_CONVERGED;
        }
        return ret;
    });
}

extern "C" int efie_solve_precond_workspace_size(int64_t n, int64_t nrhs, size_t* bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(bytes && n >= 1 && nrhs >= 1, EFIE_ERR_ARG, "solve_precond_workspace_size: bad argument");
        const size_t vec = efie::align256(size_t(n) * size_t(nrhs) * 16);
        // the complex64 staging of the mixed form is included, so one size serves both
        *bytes = efie::layout(n, nrhs, EFIE_C64, nullptr, nullptr) + 4 * vec;
        return int(EFIE_OK);
    });
}

extern "C" int efie_solve_precond_ex(const void* Z, int zdt, const void* P, int pdt, int64_t n, const void* V,
                                     void* J, int64_t nrhs, const efie_solve_opts* opts, efie_rhs_stats* stats,
                                     void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE((zdt == EFIE_C128 || zdt == EFIE_C64) && (pdt == EFIE_C128 || pdt == EFIE_C64), EFIE_ERR_ARG,
                     "solve_precond: bad dtype");
        const bool mixed = zdt == EFIE_C64 || pdt == EFIE_C64;
        EFIE_REQUIRE(Z && P && V && J && opts && ws, EFIE_ERR_ARG, "solve_precond: null argument");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && nrhs >= 1 && nrhs <= 65535, EFIE_ERR_ARG,
                     "solve_precond: bad sizes");
        EFIE_REQUIRE(opts->solver == EFIE_CGS, EFIE_ERR_ARG,
                     "solve_precond: the preconditioned operator is not symmetric; use EFIE_CGS");
        EFIE_REQUIRE(opts->maxit >= 1 && opts->tol > 0.0, EFIE_ERR_ARG, "solve_precond: need maxit >= 1 and tol > 0");
        const size_t base = layout(n, nrhs, EFIE_C64, nullptr, nullptr);
        const size_t vec = align256(size_t(n) * size_t(nrhs) * 16);
        EFIE_REQUIRE(ws_bytes >= base + 4 * vec, EFIE_ERR_ARG, "solve_precond: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "solve_precond: ws not aligned");
        Ws w;
        layout(n, nrhs, EFIE_C64, &w, static_cast<char*>(ws));
        w.acc64 = opts->fp32_acc == 0;
        double2* tmp = reinterpret_cast<double2*>(static_cast<char*>(ws) + base);
        double2* pb = reinterpret_cast<double2*>(static_cast<char*>(ws) + base + vec);
        double2* rt = reinterpret_cast<double2*>(static_cast<char*>(ws) + base + 2 * vec);   // true residual
        double2* dl = reinterpret_cast<double2*>(static_cast<char*>(ws) + base + 3 * vec);   // correction
        const int S = int(nrhs), nn = int(n);
        hipLaunchKernelGGL(iota_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, w.idx_all, S);
        const double2* b = static_cast<const double2*>(V);
        double2* x = static_cast<double2*>(J);
        // CGS on P Z J = P V stops on the preconditioned residual; the true residual
        // V - Z J can be larger by the conditioning of P.  Outer refinement on the
        // FP64 true residual: solve P Z d = P r for the columns still above tol, with
        // a tolerance scaled by the observed ratio of true to preconditioned
        // reduction, and add d, up to max_refine passes.
        const Op op{Z, zdt, P, tmp, pdt};
        std::vector<Col> cols;
        std::vector<int> iters(S, 0);
        std::vector<double> recur(S, 0.0), ratio(S, 1.0), rel(S, 0.0), h_nrm(S), h_bn(S);
        const size_t tot = size_t(nn) * S;
        const int passes = std::max(1, opts->max_refine);
        // first pass a little below tol (the true residual is usually a few times the
        // preconditioned one); the mixed form never asks the FP32 products for more than
        // inner_tol per pass
        const double floor_tau = mixed ? std::max(opts->inner_tol, 1e-13) : 1e-13;
        double tau = std::max(0.25 * opts->tol, floor_tau);
        // the right-hand side P r of a pass only has to be as accurate as the pass
        // (its tolerance >= inner_tol): the solver's own product forms it; the true
        // residual that decides convergence stays FP64-accumulated.  After the first
        // pass only the columns still above tol (listed in idx_ref) are refined: the
        // others keep x and their residual norms, and get a zero right-hand side.
        std::vector<int> h_ref(S);
        for (int s = 0; s < S; ++s) h_ref[s] = s;
        int m_ref = S;
        for (int pass = 0; pass < passes; ++pass) {
            const double2* rhs = pass == 0 ? b : rt;
            const int* ref = pass == 0 ? w.idx_all : w.idx_ref;
            if (pass > 0) fill_zero_bytes(pb, tot * sizeof(double2), stream);
            product(P, pdt, nn, rhs, pb, ref, m_ref, false, w, stream);
            double2* dst = pass == 0 ? x : dl;
            krylov(op, nn, pb, dst, S, EFIE_CGS, tau, opts->maxit, false, w, cols, stream);
            if (pass > 0)
                hipLaunchKernelGGL(axpy_inplace_kernel, dim3(int(std::min<size_t>((tot + 255) / 256, 16384))),
                                   dim3(256), 0, stream, x, dl, tot);
            true_residual(Z, zdt, nn, b, x, rt, ref, m_ref, w, stream);
            EFIE_HIP_CHECK(hipMemcpyAsync(h_nrm.data(), w.nrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipMemcpyAsync(h_bn.data(), w.bnrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipStreamSynchronize(stream));
            double need = 0.5;   // next pass tolerance (relative to its right-hand side)
            bool done = true;
            for (int s = 0; s < S; ++s) {
                iters[s] += cols[s].iters;
                const double r_in = pass == 0 ? 1.0 : rel[s];   // rhs norm of this pass / ||b||
                const double now = h_bn[s] > 0 ? std::sqrt(h_nrm[s] / h_bn[s]) : 0.0;
                const double pre = cols[s].bn2 > 0 ? std::sqrt(cols[s].rn2 / cols[s].bn2) : 0.0;
                if (r_in > 0 && pre > 0) ratio[s] = std::max(1.0, (now / r_in) / pre);
                recur[s] = pre;
                rel[s] = now;
                if (now > opts->tol) {
                    done = false;
                    need = std::min(need, 0.5 * opts->tol / (now * ratio[s]));
                }
            }
            if (verbose())
                std::fprintf(stderr, "[efie] precond pass %d worst true relres %.3e\n", pass,
                             *std::max_element(rel.begin(), rel.end())),
                    std::fflush(stderr);
            if (done) break;
            tau = std::max(need, floor_tau);
            m_ref = 0;
            for (int s = 0; s < S; ++s)
                if (rel[s] > opts->tol) h_ref[m_ref++] = s;
            EFIE_HIP_CHECK(hipMemcpyAsync(w.idx_ref, h_ref.data(), sizeof(int) * m_ref, hipMemcpyHostToDevice, stream));
        }
        int ret = EFIE_OK;
        for (int s = 0; s < S; ++s) {
            int st = cols[s].status;
            if (st >= 0) st = rel[s] <= opts->tol ? EFIE_OK : EFIE_NOT_CONVERGED;
            if (!(rel[s] == rel[s])) st = EFIE_ERR_NAN;
            if (stats) {
                stats[s].iters = iters[s];
                stats[s].status = st;
                stats[s].relres_recur = recur[s];
                stats[s].relres_true = rel[s];
            }
            if (st != EFIE_OK) ret = EFIE_NOT_CONVERGED;
        }
        return ret;
    });
}

extern "C" int efie_solve_precond(const void* Z, const void* P, int64_t n, const void* V, void* J, int64_t nrhs,
                                  const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
    return efie_solve_precond_ex(Z, EFIE_C128, P, EFIE_C128, n, V, J, nrhs, opts, stats, ws, ws_bytes, stream);
}

extern "C" int efie_solve_cfie_workspace_size(int64_t n, int64_t nrhs, size_t* bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(bytes && n >= 1 && nrhs >= 1, EFIE_ERR_ARG, "solve_cfie_workspace_size: bad argument");
        const size_t vec = efie::align256(size_t(n) * size_t(nrhs) * 16);
        *bytes = efie::layout(n, nrhs, EFIE_C128, nullptr, nullptr) + 5 * vec;
        return int(EFIE_OK);
    });
}

extern "C" int efie_solve_cfie(const void* Z, const void* P, const void* M, const void* Q, int64_t n, const void* V,
                               const void* H, void* J, int64_t nrhs, const efie_solve_opts* opts,
                               efie_rhs_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE(Z && P && M && Q && V && H && J && opts && ws, EFIE_ERR_ARG, "solve_cfie: null argument");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && nrhs >= 1 && nrhs <= 65535, EFIE_ERR_ARG,
                     "solve_cfie: bad sizes");
        EFIE_REQUIRE(opts->solver == EFIE_CGS, EFIE_ERR_ARG, "solve_cfie: the operator is not symmetric; use EFIE_CGS");
        EFIE_REQUIRE(opts->maxit >= 1 && opts->tol > 0.0, EFIE_ERR_ARG, "solve_cfie: need maxit >= 1 and tol > 0");
        const size_t base = layout(n, nrhs, EFIE_C128, nullptr, nullptr);
        const size_t vec = align256(size_t(n) * size_t(nrhs) * 16);
        EFIE_REQUIRE(ws_bytes >= base + 5 * vec, EFIE_ERR_ARG, "solve_cfie: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "solve_cfie: ws not aligned");
        Ws w;
        layout(n, nrhs, EFIE_C128, &w, static_cast<char*>(ws));
        w.acc64 = true;
        char* b0 = static_cast<char*>(ws) + base;
        Op op{Z, EFIE_C128, P, reinterpret_cast<double2*>(b0), EFIE_C128};
        op.M = M;
        op.Q = Q;
        op.tmp2 = reinterpret_cast<double2*>(b0 + vec);
        op.tmp3 = reinterpret_cast<double2*>(b0 + 2 * vec);
        double2* pb = reinterpret_cast<double2*>(b0 + 3 * vec);   // b = P V + Q H
        double2* y = reinterpret_cast<double2*>(b0 + 4 * vec);    // C x for the true residual
        const int S = int(nrhs), nn = int(n);
        hipLaunchKernelGGL(iota_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, w.idx_all, S);
        product(P, EFIE_C128, nn, static_cast<const double2*>(V), pb, w.idx_all, S, true, w, stream);
        product(Q, EFIE_C128, nn, static_cast<const double2*>(H), op.tmp3, w.idx_all, S, true, w, stream);
        hipLaunchKernelGGL(add_rows_kernel, dim3(unsigned(std::min(64, (nn + 255) / 256)), unsigned(S)), dim3(256), 0,
                           stream, pb, op.tmp3, w.idx_all, nn);
        double2* x = static_cast<double2*>(J);
        std::vector<Col> cols;
        krylov(op, nn, pb, x, S, EFIE_CGS, opts->tol, opts->maxit, false, w, cols, stream);
        // FP64 true residual of the stabilized system
        op_product(op, nn, x, y, w.idx_all, S, true, w, stream);
        hipLaunchKernelGGL(residual_kernel, dim3(S), dim3(KB), 0, stream, pb, y, nullptr, w.nrm, w.bnrm, nn,
                           w.idx_all);
        std::vector<double> h_nrm(S), h_bn(S);
        EFIE_HIP_CHECK(hipMemcpyAsync(h_nrm.data(), w.nrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(h_bn.data(), w.bnrm, sizeof(double) * S, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        int ret = EFIE_OK;
        for (int s = 0; s < S; ++s) {
            const double rel = h_bn[s] > 0 ? std::sqrt(h_nrm[s] / h_bn[s]) : 0.0;
            int st = cols[s].status;
            if (st >= 0) st = rel <= opts->tol ? EFIE_OK : EFIE_NOT_CONVERGED;
            if (!(rel == rel)) st = EFIE_ERR_NAN;
            if (stats) {
                stats[s].iters = cols[s].iters;
                stats[s].status = st;
                stats[s].relres_recur = cols[s].bn2 > 0 ? std::sqrt(cols[s].rn2 / cols[s].bn2) : 0.0;
                stats[s].relres_true = rel;
            }
            if (st != EFIE_OK) ret = EFIE_NOT_CONVERGED;
        }
        return ret;
    });
}

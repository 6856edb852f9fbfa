// Device side of the Calderon preconditioner (structure of the paper's Sec. III,
// eq. 16: second operator at k~, times a Gram inverse, times the first operator).
//
//   T_bary(k~)   dense EFIE matrix on the barycentric RWGs (the assembly kernels)
//   Y = T_bary R           one thread per output, gathers along a row of T_bary
//   T_BC = R^T Y           one thread per output, coalesced rows of Y
//   P = T_BC G_mix^{-1}    row s of P solves G_mix^T p_s = row s of T_BC; block CGNR
//                          (CG on the normal equations, one thread block per row,
//                          FP64), G_mix well conditioned so a few tens of steps.
// The preconditioned operator P Z is then applied as two dense products.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>

#include "calderon.h"
#include "linalg.h"

namespace efie {

void assemble_into(const DevMesh& m, double kr, double ki, double eta, int dtype, void* Z, void* Z2, int parts,
                   hipStream_t s);

struct DevCald {
    int N, Nb;
    const int32_t *r_ptr, *r_idx;   // CSC of R by BC function
    const double* r_val;
    const int32_t *g_ptr, *g_idx, *gt_ptr, *gt_idx;
    const double *g_val, *gt_val;
};

// Y[i][n] = sum_k Tb[i][r_idx[k]] r_val[k], k over column n of R
__global__ __launch_bounds__(256) void bc_right_kernel(DevCald c, const double2* __restrict__ Tb,
                                                       double2* __restrict__ Y) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y;
    if (n >= c.N) return;
    const double2* row = Tb + size_t(i) * c.Nb;
    double ar = 0, ai = 0;
    for (int k = c.r_ptr[n]; k < c.r_ptr[n + 1]; ++k) {
        const double2 t = row[c.r_idx[k]];
        ar += t.x * c.r_val[k];
        ai += t.y * c.r_val[k];
    }
    Y[size_t(i) * c.N + n] = make_double2(ar, ai);
}

// Tbc[m][n] = sum_k r_val[k] Y[r_idx[k]][n], k over column m of R
__global__ __launch_bounds__(256) void bc_left_kernel(DevCald c, const double2* __restrict__ Y,
                                                      double2* __restrict__ Tbc) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int m = blockIdx.y;
    if (n >= c.N) return;
    double ar = 0, ai = 0;
    for (int k = c.r_ptr[m]; k < c.r_ptr[m + 1]; ++k) {
        const double2 y = Y[size_t(c.r_idx[k]) * c.N + n];
        ar += c.r_val[k] * y.x;
        ai += c.r_val[k] * y.y;
    }
    Tbc[size_t(m) * c.N + n] = make_double2(ar, ai);
}

// Out[s][j] = sum_k val[k] X[s][idx[k]], k over row j of a real CSR matrix
__global__ __launch_bounds__(256) void spmm_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                                   const double* __restrict__ val, const double2* __restrict__ X,
                                                   double2* __restrict__ Out, int N) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= N) return;
    const double2* x = X + size_t(s) * N;
    double ar = 0, ai = 0;
    for (int k = ptr[j]; k < ptr[j + 1]; ++k) {
        const double2 v = x[idx[k]];
        ar += val[k] * v.x;
        ai += val[k] * v.y;
    }
    Out[size_t(s) * N + j] = make_double2(ar, ai);
}

// ------------------------------------------------------------- block CGNR
struct CgnrCol {
    double gamma, bn2, rn2, tol2;
    int active, iters, pad[2];
};
constexpr int CB = 256;

__device__ void csum(double (&v)[2], double* sh) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[2 * w] = v[0];
        sh[2 * w + 1] = v[1];
    }
    __syncthreads();
    v[0] = v[1] = 0.0;
    for (int u = 0; u < CB / 64; ++u) {
        v[0] += sh[2 * u];
        v[1] += sh[2 * u + 1];
    }
}

// w = 0, r = b, ||b||^2
__global__ __launch_bounds__(CB) void cgnr_init(const double2* b, double2* w, double2* r, CgnrCol* cols, int N,
                                                double tol) {
    __shared__ double sh[2 * CB / 64];
    const int s = blockIdx.x;
    const size_t o = size_t(s) * N;
    double v[2] = {0, 0};
    for (int k = threadIdx.x; k < N; k += CB) {
        const double2 x = b[o + k];
        w[o + k] = make_double2(0, 0);
        r[o + k] = x;
        v[0] += x.x * x.x + x.y * x.y;
    }
    csum(v, sh);
    if (threadIdx.x == 0) {
        CgnrCol c{};
        c.bn2 = v[0];
        c.rn2 = v[0];
        c.tol2 = tol * tol * v[0];
        c.active = v[0] > 0.0;
        cols[s] = c;
    }
}

// after z = G r (first time): p = z, gamma = ||z||^2
__global__ __launch_bounds__(CB) void cgnr_start(const double2* z, double2* p, CgnrCol* cols, int N) {
    __shared__ double sh[2 * CB / 64];
    const int s = blockIdx.x;
    const size_t o = size_t(s) * N;
    double v[2] = {0, 0};
    for (int k = threadIdx.x; k < N; k += CB) {
        const double2 x = z[o + k];
        p[o + k] = x;
        v[0] += x.x * x.x + x.y * x.y;
    }
    csum(v, sh);
    if (threadIdx.x == 0) cols[s].gamma = v[0];
}

// after t = G^T p: alpha = gamma / ||t||^2, w += alpha p, r -= alpha t
__global__ __launch_bounds__(CB) void cgnr_step1(double2* w, double2* r, const double2* p, const double2* t,
                                                 CgnrCol* cols, int N, int* nactive) {
    __shared__ double sh[2 * CB / 64];
    __shared__ int go;
    const int s = blockIdx.x;
    if (threadIdx.x == 0) go = cols[s].active;
    __syncthreads();
    if (!go) return;
    const size_t o = size_t(s) * N;
    double v[2] = {0, 0};
    for (int k = threadIdx.x; k < N; k += CB) {
        const double2 x = t[o + k];
        v[0] += x.x * x.x + x.y * x.y;
    }
    csum(v, sh);
    const double gamma = cols[s].gamma;
    const double alpha = v[0] > 0.0 ? gamma / v[0] : 0.0;
    double u[2] = {0, 0};
    for (int k = threadIdx.x; k < N; k += CB) {
        double2 ww = w[o + k], rr = r[o + k];
        const double2 pp = p[o + k], tt = t[o + k];
        ww.x += alpha * pp.x;
        ww.y += alpha * pp.y;
        rr.x -= alpha * tt.x;
        rr.y -= alpha * tt.y;
        w[o + k] = ww;
        r[o + k] = rr;
        u[0] += rr.x * rr.x + rr.y * rr.y;
    }
    csum(u, sh);
    if (threadIdx.x == 0) {
        CgnrCol c = cols[s];
        c.rn2 = u[0];
        c.iters += 1;
        if (u[0] <= c.tol2 || !(u[0] == u[0]) || v[0] == 0.0) c.active = 0;
        cols[s] = c;
        if (c.active) atomicAdd(nactive, 1);
    }
}

// after z = G r: beta = ||z||^2 / gamma, p = z + beta p
__global__ __launch_bounds__(CB) void cgnr_step2(const double2* z, double2* p, CgnrCol* cols, int N) {
    __shared__ double sh[2 * CB / 64];
    __shared__ int go;
    const int s = blockIdx.x;
    // read before the barriers below: thread 0 rewrites gamma at the end
    const double gamma = cols[s].gamma;
    if (threadIdx.x == 0) go = cols[s].active;
    __syncthreads();
    if (!go) return;
    const size_t o = size_t(s) * N;
    double v[2] = {0, 0};
    for (int k = threadIdx.x; k < N; k += CB) {
        const double2 x = z[o + k];
        v[0] += x.x * x.x + x.y * x.y;
    }
    csum(v, sh);
    const double beta = v[0] / gamma;
    for (int k = threadIdx.x; k < N; k += CB) {
        double2 pp = p[o + k];
        const double2 zz = z[o + k];
        pp.x = zz.x + beta * pp.x;
        pp.y = zz.y + beta * pp.y;
        p[o + k] = pp;
    }
    if (threadIdx.x == 0) cols[s].gamma = v[0];
}

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

struct CaldWs {
    double2 *Tb, *Y, *Tbc, *r, *z, *p, *t;
    CgnrCol* cols;
    int* counter;
};

size_t cald_layout(int64_t N, int64_t Nb, CaldWs* w, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += a256(bytes);
        return p;
    };
    CaldWs x{};
    const size_t nn = size_t(N) * size_t(N) * 16;
    x.Tb = (double2*)take(size_t(Nb) * size_t(Nb) * 16);
    x.Y = (double2*)take(size_t(Nb) * size_t(N) * 16);
    x.Tbc = (double2*)take(nn);
    x.r = (double2*)take(nn);
    x.z = (double2*)take(nn);
    x.p = (double2*)take(nn);
    x.t = (double2*)take(nn);
    x.cols = (CgnrCol*)take(sizeof(CgnrCol) * size_t(N));
    x.counter = (int*)take(16);
    if (w) *w = x;
    return off;
}

DevCald dev_cald(const efie_calderon_s& C) {
    const char* b = static_cast<const char*>(C.dev);
    const auto& o = C.offs;
    DevCald d{};
    d.N = int(C.N);
    d.Nb = int(C.bary.N);
    d.r_ptr = reinterpret_cast<const int32_t*>(b + o[0]);
    d.r_idx = reinterpret_cast<const int32_t*>(b + o[1]);
    d.r_val = reinterpret_cast<const double*>(b + o[2]);
    d.g_ptr = reinterpret_cast<const int32_t*>(b + o[3]);
    d.g_idx = reinterpret_cast<const int32_t*>(b + o[4]);
    d.g_val = reinterpret_cast<const double*>(b + o[5]);
    d.gt_ptr = reinterpret_cast<const int32_t*>(b + o[6]);
    d.gt_idx = reinterpret_cast<const int32_t*>(b + o[7]);
    d.gt_val = reinterpret_cast<const double*>(b + o[8]);
    return d;
}

template <class T>
size_t put(std::vector<char>& blob, std::vector<size_t>& offs, const std::vector<T>& v) {
    size_t off = a256(blob.size());
    blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    offs.push_back(off);
    return off;
}

}  // namespace
}  // namespace efie

extern "C" {

int efie_calderon_create(efie_mesh mesh, efie_calderon* out) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh && out, EFIE_ERR_ARG, "calderon_create: null argument");
        auto* C = new efie_calderon_s();
        try {
            C->primal = mesh;
            efie::build_calderon(*C, *mesh);
            // sparse arrays after the barycentric tables
            std::vector<char> blob;
            std::vector<size_t> offs;
            efie::put(blob, offs, C->r_ptr);
            efie::put(blob, offs, C->r_idx);
            efie::put(blob, offs, C->r_val);
            efie::put(blob, offs, C->g_ptr);
            efie::put(blob, offs, C->g_idx);
            efie::put(blob, offs, C->g_val);
            efie::put(blob, offs, C->gt_ptr);
            efie::put(blob, offs, C->gt_idx);
            efie::put(blob, offs, C->gt_val);
            blob.resize(efie::a256(blob.size()));
            C->host_blob.swap(blob);
            C->offs.swap(offs);
            C->bary_bytes = C->bary.host_blob.size();
        } catch (...) {
            delete C;
            throw;
        }
        *out = C;
        return int(EFIE_OK);
    });
}

void efie_calderon_destroy(efie_calderon c) { delete c; }

int efie_calderon_sizes(efie_calderon c, int64_t* n_bary_rwg, int64_t* n_bary_tri, size_t* table_bytes,
                        size_t* ws_bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c != nullptr, EFIE_ERR_ARG, "calderon_sizes: null");
        if (n_bary_rwg) *n_bary_rwg = c->bary.N;
        if (n_bary_tri) *n_bary_tri = c->bary.T;
        if (table_bytes) *table_bytes = efie::a256(c->bary_bytes) + c->host_blob.size();
        if (ws_bytes) *ws_bytes = efie::cald_layout(c->N, c->bary.N, nullptr, nullptr);
        return int(EFIE_OK);
    });
}

int efie_calderon_upload(efie_calderon c, void* dev, size_t bytes, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c && dev, EFIE_ERR_ARG, "calderon_upload: null argument");
        const size_t off = efie::a256(c->bary_bytes);
        EFIE_REQUIRE(bytes >= off + c->host_blob.size(), EFIE_ERR_ARG, "calderon_upload: buffer too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(dev) & 255) == 0, EFIE_ERR_ARG, "calderon_upload: not 256-aligned");
        char* d = static_cast<char*>(dev);
        EFIE_HIP_CHECK(hipMemcpyAsync(d, c->bary.host_blob.data(), c->bary_bytes, hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipMemcpyAsync(d + off, c->host_blob.data(), c->host_blob.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        efie::bind_tables(c->bary, d);
        c->dev = d + off;
        return int(EFIE_OK);
    });
}

int efie_calderon_host_matrices(efie_calderon c, double* R, double* G) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(c != nullptr, EFIE_ERR_ARG, "calderon_host_matrices: null");
        const size_t N = size_t(c->N), Nb = size_t(c->bary.N);
        if (R) {
            std::memset(R, 0, sizeof(double) * Nb * N);
            for (size_t n = 0; n < N; ++n)
                for (int32_t k = c->r_ptr[n]; k < c->r_ptr[n + 1]; ++k) R[size_t(c->r_idx[size_t(k)]) * N + n] = c->r_val[size_t(k)];
        }
        if (G) {
            std::memset(G, 0, sizeof(double) * N * N);
            for (size_t m = 0; m < N; ++m)
                for (int32_t k = c->g_ptr[m]; k < c->g_ptr[m + 1]; ++k) G[m * N + size_t(c->g_idx[size_t(k)])] = c->g_val[size_t(k)];
        }
        return int(EFIE_OK);
    });
}

int efie_calderon_assemble(efie_calderon c, double kt_re, double kt_im, double eta, void* P, void* Tbc_out,
                           double tol, int32_t maxit, double* relres, void* ws, size_t ws_bytes, hipStream_t stream) {
    using namespace efie;
    return guarded([&]() {
        EFIE_REQUIRE(c && P && ws, EFIE_ERR_ARG, "calderon_assemble: null argument");
        EFIE_REQUIRE(c->dev != nullptr, EFIE_ERR_STATE, "calderon_assemble: tables not uploaded");
        EFIE_REQUIRE(kt_im <= 0.0 && (kt_re != 0.0 || kt_im != 0.0), EFIE_ERR_ARG, "calderon_assemble: bad k~");
        EFIE_REQUIRE(tol > 0.0 && maxit >= 1, EFIE_ERR_ARG, "calderon_assemble: bad tol/maxit");
        const int64_t N = c->N, Nb = c->bary.N;
        EFIE_REQUIRE(N <= 65535 && Nb <= 65535, EFIE_ERR_ARG,
                     "calderon_assemble: at most 65535 primal and barycentric RWGs (one grid row per RWG)");
        const size_t need = cald_layout(N, Nb, nullptr, nullptr);
        EFIE_REQUIRE(ws_bytes >= need, EFIE_ERR_ARG, "calderon_assemble: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "calderon_assemble: ws not aligned");
        CaldWs w;
        cald_layout(N, Nb, &w, static_cast<char*>(ws));
        const DevCald d = dev_cald(*c);
        // second operator on the barycentric RWGs at k~
        assemble_into(c->bary.dm, kt_re, kt_im, eta, EFIE_C128, w.Tb, nullptr, 0, stream);
        dim3 g1(unsigned((N + 255) / 256), unsigned(Nb)), g2(unsigned((N + 255) / 256), unsigned(N));
        hipLaunchKernelGGL(bc_right_kernel, g1, dim3(256), 0, stream, d, w.Tb, w.Y);
        hipLaunchKernelGGL(bc_left_kernel, g2, dim3(256), 0, stream, d, w.Y, w.Tbc);
        if (Tbc_out)
            EFIE_HIP_CHECK(hipMemcpyAsync(Tbc_out, w.Tbc, size_t(N) * size_t(N) * 16, hipMemcpyDeviceToDevice, stream));
        // P: rows p_s solve G^T p_s = Tbc_s by CGNR (CG on G G^T y = G b)
        double2* X = static_cast<double2*>(P);
        const int S = int(N);
        dim3 gs(unsigned((N + 255) / 256), unsigned(S));
        hipLaunchKernelGGL(cgnr_init, dim3(S), dim3(CB), 0, stream, w.Tbc, X, w.r, w.cols, int(N), tol);
        hipLaunchKernelGGL(spmm_kernel, gs, dim3(256), 0, stream, d.g_ptr, d.g_idx, d.g_val, w.r, w.z, int(N));
        hipLaunchKernelGGL(cgnr_start, dim3(S), dim3(CB), 0, stream, w.z, w.p, w.cols, int(N));
        int h_active = S;
        int it = 0;
        for (; it < maxit && h_active > 0; ++it) {
            hipLaunchKernelGGL(spmm_kernel, gs, dim3(256), 0, stream, d.gt_ptr, d.gt_idx, d.gt_val, w.p, w.t, int(N));
            EFIE_HIP_CHECK(hipMemsetAsync(w.counter, 0, sizeof(int), stream));
            hipLaunchKernelGGL(cgnr_step1, dim3(S), dim3(CB), 0, stream, X, w.r, w.p, w.t, w.cols, int(N), w.counter);
            hipLaunchKernelGGL(spmm_kernel, gs, dim3(256), 0, stream, d.g_ptr, d.g_idx, d.g_val, w.r, w.z, int(N));
            hipLaunchKernelGGL(cgnr_step2, dim3(S), dim3(CB), 0, stream, w.z, w.p, w.cols, int(N));
            EFIE_HIP_CHECK(hipMemcpyAsync(&h_active, w.counter, sizeof(int), hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        }
        std::vector<CgnrCol> cols(static_cast<size_t>(S));
        EFIE_HIP_CHECK(hipMemcpyAsync(cols.data(), w.cols, sizeof(CgnrCol) * size_t(S), hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        double worst = 0.0;
        for (const auto& cc : cols) worst = std::max(worst, cc.bn2 > 0 ? std::sqrt(cc.rn2 / cc.bn2) : 0.0);
        if (relres) *relres = worst;
        EFIE_HIP_CHECK(hipGetLastError());
        return worst <= tol ? int(EFIE_OK) : int(EFIE_NOT_CONVERGED);
    });
}

}  // extern "C"

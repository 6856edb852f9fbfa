// Plane-wave excitation and far-field radiation on gfx950.
//
//   V[s][m] = int f_m . E0 pol_s exp(-j k khat_s . r) dS            (7-point rule)
//   F[s][d] = -(j k eta / 4 pi) (I - rhat rhat) . sum_n J[s][n] a_n(rhat_d),
//   a_n(rhat) = int f_n(r') exp(j k rhat . r') dS'                  (7-point rule)
// The far field is formed in two steps: a radiation matrix whose row 2d+c holds
// the (theta, phi)[c] component of -(j k eta/4 pi) a_n(rhat_d) for every n, then
// F = J R^T with the tiled complex GEMM (FP64), so F comes out as (nrhs, ndir, 2).
#include <hip/hip_runtime.h>

#include <cmath>

#include "efie_internal.h"
#include "linalg.h"

namespace efie {

// one thread per (right-hand side s, RWG m): sums its two triangles
__global__ __launch_bounds__(256) void excite_kernel(DevMesh m, double k, const double* khat, const double* pol,
                                                     int nrhs, double e0, double2* V) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = m.N, T = m.T;
    if (idx >= N * nrhs) return;
    const int s = idx / N, n = idx - s * N;
    const double kx = khat[3 * s], ky = khat[3 * s + 1], kz = khat[3 * s + 2];
    const double px = pol[3 * s], py = pol[3 * s + 1], pz = pol[3 * s + 2];
    double vr = 0, vi = 0;
    for (int h = 0; h < 2; ++h) {
        const int t = m.et[h * N + n], l = m.el[h * N + n];
        const double c = m.cf[l * T + t];
        const double ux = m.vx[l * T + t], uy = m.vy[l * T + t], uz = m.vz[l * T + t];
        const double ph0 = kx * m.cx[t] + ky * m.cy[t] + kz * m.cz[t];
        for (int a = 0; a < NQ; ++a) {
            const double dx = m.qx[a * T + t], dy = m.qy[a * T + t], dz = m.qz[a * T + t];
            const double fp = c * ((dx - ux) * px + (dy - uy) * py + (dz - uz) * pz);
            double sn, cs;
            sincos(-k * (ph0 + kx * dx + ky * dy + kz * dz), &sn, &cs);
            const double w = m.qw[a * T + t] * fp;
            vr += w * cs;
            vi += w * sn;
        }
    }
    V[size_t(s) * N + n] = make_double2(e0 * vr, e0 * vi);
}

// radiation matrix R[2d + c][n] = -(j k eta / 4 pi) e_c(rhat_d) . a_n(rhat_d)
__global__ __launch_bounds__(256) void radiation_kernel(DevMesh m, double k, double eta, const double* dirs,
                                                        int ndir, double2* Rm) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = m.N, T = m.T;
    if (idx >= N * ndir) return;
    const int d = idx / N, n = idx - d * N;
    const double rx = dirs[3 * d], ry = dirs[3 * d + 1], rz = dirs[3 * d + 2];
    // spherical unit vectors of rhat
    const double th = acos(fmin(1.0, fmax(-1.0, rz)));
    const double phv = atan2(ry, rx);
    double st, ct, sp, cp;
    sincos(th, &st, &ct);
    sincos(phv, &sp, &cp);
    const double tx = ct * cp, ty = ct * sp, tz = -st;
    const double qx_ = -sp, qy_ = cp, qz_ = 0.0;
    double ar[3] = {0, 0, 0}, ai[3] = {0, 0, 0};
    for (int h = 0; h < 2; ++h) {
        const int t = m.et[h * N + n], l = m.el[h * N + n];
        const double c = m.cf[l * T + t];
        const double ux = m.vx[l * T + t], uy = m.vy[l * T + t], uz = m.vz[l * T + t];
        const double ph0 = rx * m.cx[t] + ry * m.cy[t] + rz * m.cz[t];
        for (int a = 0; a < NQ; ++a) {
            const double dx = m.qx[a * T + t], dy = m.qy[a * T + t], dz = m.qz[a * T + t];
            double sn, cs;
            sincos(k * (ph0 + rx * dx + ry * dy + rz * dz), &sn, &cs);
            const double w = m.qw[a * T + t] * c;
            const double f[3] = {dx - ux, dy - uy, dz - uz};
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                ar[x] += w * f[x] * cs;
                ai[x] += w * f[x] * sn;
            }
        }
    }
    const double at_r = tx * ar[0] + ty * ar[1] + tz * ar[2], at_i = tx * ai[0] + ty * ai[1] + tz * ai[2];
    const double ap_r = qx_ * ar[0] + qy_ * ar[1] + qz_ * ar[2], ap_i = qx_ * ai[0] + qy_ * ai[1] + qz_ * ai[2];
    // times -(j k eta / 4 pi): (a_r + j a_i) * (-j c) = c a_i - j c a_r
    const double cc = k * eta / (4.0 * 3.14159265358979323846);
    Rm[size_t(2 * d) * N + n] = make_double2(cc * at_i, -cc * at_r);
    Rm[size_t(2 * d + 1) * N + n] = make_double2(cc * ap_i, -cc * ap_r);
}

// adjoint source of the far field: G[s][n] = sum_e W[s][e] R[e][n], R the
// radiation matrix (2 ndir x N, row 2d + c) that forms F = J R^T
__global__ __launch_bounds__(256) void radiation_adjoint_kernel(const double2* __restrict__ Rm,
                                                                const double2* __restrict__ W, int ne, int N, int nrhs,
                                                                double2* __restrict__ G) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (n >= N || s >= nrhs) return;
    double gr = 0.0, gi = 0.0;
    for (int e = 0; e < ne; ++e) {
        const double2 r = Rm[size_t(e) * N + n], w = W[size_t(s) * ne + e];
        gr += r.x * w.x - r.y * w.y;
        gi += r.x * w.y + r.y * w.x;
    }
    G[size_t(s) * N + n] = make_double2(gr, gi);
}

// J = sum_i |F_i|^2 over count far-field values, and W = conj(F) (its derivative
// with respect to F, the weight of the adjoint source).  One block: each thread
// sums a fixed stride of the values, then a fixed tree over the block, so the sum
// is the same on every call.
__global__ __launch_bounds__(256) void farfield_objective_kernel(const double2* __restrict__ F, int64_t count,
                                                                 double* __restrict__ J, double2* __restrict__ W) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) {
        const double2 f = F[i];
        a += f.x * f.x + f.y * f.y;
        if (W) W[i] = make_double2(f.x, -f.y);
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *J = sh[0];
}

}  // namespace efie

extern "C" int efie_excite_planewave(efie_mesh mesh, double k, const double* khat, const double* pol, int64_t nrhs,
                                     double e0, void* V, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh && khat && pol && V, EFIE_ERR_ARG, "excite: null argument");
        EFIE_REQUIRE(mesh->dev != nullptr, EFIE_ERR_STATE, "excite: mesh tables not uploaded");
        EFIE_REQUIRE(nrhs >= 1 && nrhs * mesh->N < (int64_t(1) << 31), EFIE_ERR_ARG, "excite: bad nrhs");
        const int tot = int(nrhs * mesh->N);
        efie::prof_begin(efie::PROF_EXCITE, stream);
        hipLaunchKernelGGL(efie::excite_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, mesh->dm, k, khat, pol,
                           int(nrhs), e0, static_cast<double2*>(V));
        efie::prof_end(efie::PROF_EXCITE, stream);
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

extern "C" int efie_farfield_workspace_size(efie_mesh mesh, int64_t ndir, size_t* bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh && bytes && ndir >= 1, EFIE_ERR_ARG, "farfield_workspace_size: bad argument");
        *bytes = size_t(2 * ndir) * size_t(mesh->N) * 16;
        return int(EFIE_OK);
    });
}

extern "C" int efie_farfield(efie_mesh mesh, double k, double eta, const void* J, int64_t nrhs, const double* dirs,
                             int64_t ndir, void* F, void* ws, size_t ws_bytes, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh && J && dirs && F && ws, EFIE_ERR_ARG, "farfield: null argument");
        EFIE_REQUIRE(mesh->dev != nullptr, EFIE_ERR_STATE, "farfield: mesh tables not uploaded");
        EFIE_REQUIRE(nrhs >= 1 && ndir >= 1 && nrhs < 65536 && 2 * ndir * mesh->N < (int64_t(1) << 31),
                     EFIE_ERR_ARG, "farfield: bad sizes");
        EFIE_REQUIRE(ws_bytes >= size_t(2 * ndir) * size_t(mesh->N) * 16, EFIE_ERR_ARG, "farfield: workspace too small");
        const int N = int(mesh->N);
        const int tot = int(ndir) * N;
        efie::prof_begin(efie::PROF_FARFIELD, stream);
        hipLaunchKernelGGL(efie::radiation_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, mesh->dm, k, eta,
                           dirs, int(ndir), static_cast<double2*>(ws));
        efie::prof_end(efie::PROF_FARFIELD, stream);
        // F[s][e] = sum_n J[s][n] R[e][n]
        efie::zgemm_nt(J, EFIE_C128, ws, EFIE_C128, F, EFIE_C128, int(nrhs), int(2 * ndir), N, N, N, int(2 * ndir),
                       1.0, 0.0, false, stream);
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

extern "C" int efie_farfield_adjoint(efie_mesh mesh, double k, double eta, const void* W, int64_t nrhs,
                                     const double* dirs, int64_t ndir, void* G, void* ws, size_t ws_bytes,
                                     hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(mesh && W && dirs && G && ws, EFIE_ERR_ARG, "farfield_adjoint: null argument");
        EFIE_REQUIRE(mesh->dev != nullptr, EFIE_ERR_STATE, "farfield_adjoint: mesh tables not uploaded");
        EFIE_REQUIRE(nrhs >= 1 && ndir >= 1 && nrhs < 65536 && 2 * ndir * mesh->N < (int64_t(1) << 31),
                     EFIE_ERR_ARG, "farfield_adjoint: bad sizes");
        EFIE_REQUIRE(ws_bytes >= size_t(2 * ndir) * size_t(mesh->N) * 16, EFIE_ERR_ARG,
                     "farfield_adjoint: workspace too small");
        const int N = int(mesh->N);
        const int tot = int(ndir) * N;
        hipLaunchKernelGGL(efie::radiation_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, mesh->dm, k, eta,
                           dirs, int(ndir), static_cast<double2*>(ws));
        hipLaunchKernelGGL(efie::radiation_adjoint_kernel, dim3((N + 255) / 256, unsigned(nrhs)), dim3(256), 0, stream,
                           static_cast<const double2*>(ws), static_cast<const double2*>(W), int(2 * ndir), N, int(nrhs),
                           static_cast<double2*>(G));
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

extern "C" int efie_farfield_objective(const void* F, int64_t count, void* J, void* W, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(F && J, EFIE_ERR_ARG, "farfield_objective: null argument");
        EFIE_REQUIRE(count >= 1, EFIE_ERR_ARG, "farfield_objective: need count >= 1");
        EFIE_REQUIRE(W != F, EFIE_ERR_ARG, "farfield_objective: W must not alias F");
        hipLaunchKernelGGL(efie::farfield_objective_kernel, dim3(1), dim3(256), 0, stream,
                           static_cast<const double2*>(F), count, static_cast<double*>(J), static_cast<double2*>(W));
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

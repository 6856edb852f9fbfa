// Device code of the magnetic (MFIE) operator K on a barycentric test triangle
// and a primal source triangle, for the Calderon-stabilized CFIE (the 3-D
// reading of the paper's Sec. III, eq. 16: the second term of C_p is the
// Calderon product of the MFIE operator).
//
//   K_mix[e][n] = int f_e(r) . int grad G_k(r, r') x f_n(r') dS' dS,
//   grad G = (r - r') g(R),   g(R) = -(1 + j k R) exp(-j k R) / (4 pi R^3),
// f_e an RWG function of the barycentric refinement (test triangle b inside the
// primal triangle t = b / 6), f_n a primal RWG function (source triangle q).
// With f_n = c_j (r' - v_j) on q, (r - r') x f_n(r') = c_j (r - r') x (r - v_j),
// so for the test points r_a (weights w_a) and the inner integrals
//   A_a = int (r_a - r') g(R) dS'      (a complex vector per test point)
// the nine values of the pair are
//   c_i c_j sum_a w_a (a - u_i) . (A_a x (X_a - v_j))
//     = c_i c_j [ M1 - u_i . M2 - v_j . (M3 - u_i x M4) ],
//   M1 = sum w a . (A x X),  M2 = sum w A x X,  M3 = sum w a x A,  M4 = sum w A,
// with a, u_i the test point and vertex offsets from b's centroid, X_a the test
// point and v_j the source vertex offsets from q's centroid.
//   * q = t (coplanar, the test triangle's own primal triangle): zero (principal
//     value: the integrand is normal to the plane, the test function tangential);
//   * (t, q) near (the EFIE near rule of the primal mesh): A_a = 7-point rule of
//     g_s (r_a - r') with g_s = g + 1/(4 pi R^3), minus J(r_a) / (4 pi),
//     J(r) = int (r - r')/|r - r'|^3 dS' in closed form (Wilton et al., IEEE TAP
//     32(3), 1984: the gradient of their potential integral), the normal part
//     taken as zero within 1e-12 of the longest edge of the plane;
//   * otherwise the 7 x 7 product rule of g.
// (1 + x) exp(-x) - 1 (x = j k R) is summed as its Taylor series
// sum_{m>=2} (-1)^(m+1) (m - 1) x^m / m! (m up to 23) for |x| < 1/2 and evaluated
// directly above.
#pragma once

#include <hip/hip_runtime.h>

#include "efie_internal.h"
#include "pair_kernels.h"

namespace efie {

struct Cx {
    double r, i;
};
__device__ __forceinline__ Cx cxmul(Cx a, Cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

// (1 + x) exp(-x) for x = j k R, k = kr + j ki (CK: ki != 0)
template <bool CK>
__device__ __forceinline__ Cx mfie_full(double kr, double ki, double R) {
    double s, c;
    sincos(kr * R, &s, &c);
    const double e = CK ? exp(ki * R) : 1.0;
    // (1 - ki R + j kr R) e^{ki R} (cos(kr R) - j sin(kr R))
    const double ar = 1.0 - ki * R, ai = kr * R;
    return {e * (ar * c + ai * s), e * (ai * c - ar * s)};
}

// (1 + x) exp(-x) - 1, x = j k R: the Taylor series for |x| < 1/2
__device__ inline Cx mfie_num(double kr, double ki, double R) {
    const Cx x = {-ki * R, kr * R};
    if (x.r * x.r + x.i * x.i < 0.25) {
        // term_m = x^m / m!, sum (-1)^(m+1) (m - 1) term_m
        Cx term = x, acc = {0.0, 0.0};
#pragma unroll
        for (int m = 2; m < 24; ++m) {
            term = cxmul(term, x);
            term.r *= 1.0 / double(m);
            term.i *= 1.0 / double(m);
            const double c = (m & 1) ? double(m - 1) : -double(m - 1);
            acc.r += c * term.r;
            acc.i += c * term.i;
        }
        return acc;
    }
    Cx v = mfie_full<true>(kr, ki, R);
    v.r -= 1.0;
    return v;
}

// J(r) = int_q (r - r')/|r - r'|^3 dS' for r = (px, py, pz) relative to q's
// centroid (vertex offsets v[3][3], unit normal n, longest edge h)
__device__ inline void grad_potential(double px, double py, double pz, const double (&v)[3][3], const double (&n)[3],
                                      double h, double (&J)[3]) {
    const double d = n[0] * (px - v[0][0]) + n[1] * (py - v[0][1]) + n[2] * (pz - v[0][2]);
    const double ad = fabs(d);
    const double rho[3] = {px - d * n[0], py - d * n[1], pz - d * n[2]};
    double beta = 0.0;
    J[0] = J[1] = J[2] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double* rm = v[i];
        const double* rp = v[(i + 1) % 3];
        double lt[3] = {rp[0] - rm[0], rp[1] - rm[1], rp[2] - rm[2]};
        const double ll = sqrt(lt[0] * lt[0] + lt[1] * lt[1] + lt[2] * lt[2]);
        lt[0] /= ll;
        lt[1] /= ll;
        lt[2] /= ll;
        const double u[3] = {lt[1] * n[2] - lt[2] * n[1], lt[2] * n[0] - lt[0] * n[2], lt[0] * n[1] - lt[1] * n[0]};
        const double lp = (rp[0] - rho[0]) * lt[0] + (rp[1] - rho[1]) * lt[1] + (rp[2] - rho[2]) * lt[2];
        const double lm = (rm[0] - rho[0]) * lt[0] + (rm[1] - rho[1]) * lt[1] + (rm[2] - rho[2]) * lt[2];
        const double P0 = (rm[0] - rho[0]) * u[0] + (rm[1] - rho[1]) * u[1] + (rm[2] - rho[2]) * u[2];
        const double R02 = P0 * P0 + d * d;
        const double Rp = sqrt((px - rp[0]) * (px - rp[0]) + (py - rp[1]) * (py - rp[1]) + (pz - rp[2]) * (pz - rp[2]));
        const double Rm = sqrt((px - rm[0]) * (px - rm[0]) + (py - rm[1]) * (py - rm[1]) + (pz - rm[2]) * (pz - rm[2]));
        if (sqrt(R02) < 1e-12 * h) continue;   // on the line of the edge: both terms vanish
        const double sp = lp >= 0.0 ? Rp + lp : R02 / (Rp - lp);
        const double sm = lm >= 0.0 ? Rm + lm : R02 / (Rm - lm);
        const double lg = log(sp / sm);
        beta += atan(P0 * lp / (R02 + ad * Rp)) - atan(P0 * lm / (R02 + ad * Rm));
        J[0] += lg * u[0];
        J[1] += lg * u[1];
        J[2] += lg * u[2];
    }
    const double sd = ad <= 1e-12 * h ? 0.0 : (d > 0.0 ? 1.0 : -1.0);
    J[0] += sd * beta * n[0];
    J[1] += sd * beta * n[1];
    J[2] += sd * beta * n[2];
}

// The nine K_mix values of test triangle p of the refinement mb against source
// triangle q of the primal mesh m: emit(i, j, re, im)
template <bool CK, typename Emit>
__device__ inline void mfie_pair(const DevMesh& mb, const DevMesh& m, int p, int q, double kr, double ki, bool near,
                                 Emit emit) {
    const int Tb = mb.T, T = m.T;
    const double Dx = mb.cx[p] - m.cx[q], Dy = mb.cy[p] - m.cy[q], Dz = mb.cz[p] - m.cz[q];
    double sx[NQ], sy[NQ], sz[NQ], sw[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
        sx[c] = m.qx[c * T + q];
        sy[c] = m.qy[c * T + q];
        sz[c] = m.qz[c * T + q];
        sw[c] = m.qw[c * T + q];
    }
    double vq[3][3], nq[3] = {m.nx[q], m.ny[q], m.nz[q]};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        vq[j][0] = m.vx[j * T + q];
        vq[j][1] = m.vy[j * T + q];
        vq[j][2] = m.vz[j * T + q];
    }
    const double hq = m.hm[q];
    constexpr double F = 1.0 / (4.0 * PI);
    Cx M1 = {0.0, 0.0}, M2[3] = {}, M3[3] = {}, M4[3] = {};
#pragma unroll 1
    for (int a = 0; a < NQ; ++a) {
        const double ax = mb.qx[a * Tb + p], ay = mb.qy[a * Tb + p], az = mb.qz[a * Tb + p], wa = mb.qw[a * Tb + p];
        const double X[3] = {Dx + ax, Dy + ay, Dz + az};
        Cx A[3] = {};
        if (!near) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                const double dx = X[0] - sx[c], dy = X[1] - sy[c], dz = X[2] - sz[c];
                const double R2 = dx * dx + dy * dy + dz * dz;
                const double rinv = rsqrt(R2);
                const Cx num = mfie_full<CK>(kr, ki, R2 * rinv);
                const double s = -sw[c] * F * (rinv * rinv * rinv);
                const double gr = s * num.r, gi = s * num.i;
                A[0].r += gr * dx; A[0].i += gi * dx;
                A[1].r += gr * dy; A[1].i += gi * dy;
                A[2].r += gr * dz; A[2].i += gi * dz;
            }
        } else {
#pragma unroll 1
            for (int c = 0; c < NQ; ++c) {
                const double dx = X[0] - sx[c], dy = X[1] - sy[c], dz = X[2] - sz[c];
                const double R = sqrt(dx * dx + dy * dy + dz * dz);
                const Cx num = mfie_num(kr, ki, R);
                const double s = -sw[c] * F / (R * R * R);
                const double gr = s * num.r, gi = s * num.i;
                A[0].r += gr * dx; A[0].i += gi * dx;
                A[1].r += gr * dy; A[1].i += gi * dy;
                A[2].r += gr * dz; A[2].i += gi * dz;
            }
            double J[3];
            grad_potential(X[0], X[1], X[2], vq, nq, hq, J);
            A[0].r -= F * J[0];
            A[1].r -= F * J[1];
            A[2].r -= F * J[2];
        }
        // P = A x X, then the moments
        const Cx P[3] = {{A[1].r * X[2] - A[2].r * X[1], A[1].i * X[2] - A[2].i * X[1]},
                         {A[2].r * X[0] - A[0].r * X[2], A[2].i * X[0] - A[0].i * X[2]},
                         {A[0].r * X[1] - A[1].r * X[0], A[0].i * X[1] - A[1].i * X[0]}};
        const double av[3] = {ax, ay, az};
        M1.r += wa * (ax * P[0].r + ay * P[1].r + az * P[2].r);
        M1.i += wa * (ax * P[0].i + ay * P[1].i + az * P[2].i);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            M2[d].r += wa * P[d].r;
            M2[d].i += wa * P[d].i;
            M4[d].r += wa * A[d].r;
            M4[d].i += wa * A[d].i;
        }
        // a x A
        M3[0].r += wa * (av[1] * A[2].r - av[2] * A[1].r);
        M3[0].i += wa * (av[1] * A[2].i - av[2] * A[1].i);
        M3[1].r += wa * (av[2] * A[0].r - av[0] * A[2].r);
        M3[1].i += wa * (av[2] * A[0].i - av[0] * A[2].i);
        M3[2].r += wa * (av[0] * A[1].r - av[1] * A[0].r);
        M3[2].i += wa * (av[0] * A[1].i - av[1] * A[0].i);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double u[3] = {mb.vx[i * Tb + p], mb.vy[i * Tb + p], mb.vz[i * Tb + p]};
        const double ci = mb.cf[i * Tb + p];
        // e = M1 - u . M2,  Wv = M3 - u x M4
        const Cx e = {M1.r - (u[0] * M2[0].r + u[1] * M2[1].r + u[2] * M2[2].r),
                      M1.i - (u[0] * M2[0].i + u[1] * M2[1].i + u[2] * M2[2].i)};
        const Cx Wv[3] = {{M3[0].r - (u[1] * M4[2].r - u[2] * M4[1].r), M3[0].i - (u[1] * M4[2].i - u[2] * M4[1].i)},
                          {M3[1].r - (u[2] * M4[0].r - u[0] * M4[2].r), M3[1].i - (u[2] * M4[0].i - u[0] * M4[2].i)},
                          {M3[2].r - (u[0] * M4[1].r - u[1] * M4[0].r), M3[2].i - (u[0] * M4[1].i - u[1] * M4[0].i)}};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double cc = ci * m.cf[j * T + q];
            const double vr = e.r - (vq[j][0] * Wv[0].r + vq[j][1] * Wv[1].r + vq[j][2] * Wv[2].r);
            const double vi = e.i - (vq[j][0] * Wv[0].i + vq[j][1] * Wv[1].i + vq[j][2] * Wv[2].i);
            emit(i, j, cc * vr, cc * vi);
        }
    }
}

}  // namespace efie

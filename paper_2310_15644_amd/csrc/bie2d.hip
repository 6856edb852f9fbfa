// The paper's own 2-D method on the GPU: Hankel-kernel boundary integral
// operators on a closed polygon (Sec. II, eqs. 1-5), the TM CFIE of a PEC
// cylinder (Sec. III, eq. 7, first row), its Calderon-stabilized form
//   C_p = N_k~ G^-1 S_k + (G/2 - D*_k~) G^-1 (G/2 + D*_k)          (eq. 16)
// with k~ = k - 0.4 j k^(1/3) a^(-2/3), the circular counterpart C_p,c (C_p on the
// circle of the same perimeter and node count: circulant), a randomized skeleton
// of C_p - C_p,c and the inverse of C_p by the Woodbury identity (eqs. 17-18).
//
// Discretization (readings; the paper names no rule):
//  * Galerkin with piecewise-linear functions lambda_i on the polygon through the
//    nodes: segment a runs from node a to node a+1 (mod n), x in [0, 1] its local
//    parameter, lambda_a = 1 - x and lambda_{a+1} = x on it;
//  * G_k(R) = -(j/4) H0^(2)(k R); D* differentiates along the outward normal of
//    the test point; N through the Maue identity
//      (lambda_i, N lambda_j) = int int G [lambda_i' lambda_j' - k^2 (n . n') lambda_i lambda_j];
//  * segment pairs that share no node: q x q Gauss-Legendre; adjacent pairs: both
//    segments parametrized from the shared node, the unit square split along the
//    diagonal into two triangles, each mapped by (s, t) -> (s, s t) (Duffy) with
//    s = sigma^2, 8 x 8 Gauss-Legendre in (sigma, t); the segment with itself: D*
//    vanishes (straight segment), G = -(1/2 pi) ln R + G_reg with the log part in
//    closed form (int int ln|x - y| over the unit square: -3/2, with weight x:
//    -3/4, x y: -7/16) and G_reg by 8 x 8 Gauss-Legendre;
//  * TM excitation E_z = exp(-j k khat . r): e_i = (lambda_i, E_z),
//    h_i = (lambda_i, H_t) with H_t = -(khat . n) E_z / eta; the right-hand side of
//    the stabilized system b_p = N_k~ G^-1 e/(j k eta) + (G/2 - D*_k~) G^-1 h.
//
// Hankel functions of complex argument (Im z <= 0), FP64, own implementation:
// for |z| >= 17 the Hankel asymptotic expansion H_nu^(2)(z) ~ (2/(pi z))^(1/2)
// exp(-j(z - nu pi/2 - pi/4)) sum_k (-j)^k a_k(nu) / z^k, a_k(nu) =
// prod_{m<=k} (4 nu^2 - (2m-1)^2) / (k! 8^k), summed up to its smallest term or
// until the terms fall below 1e-17 of the sum (error below 4e-15 for |z| >= 17); below, J_n(z) by Miller's backward recurrence from
// n = 2 floor(|z|/2) + 30, normalized by J_0 + 2 sum J_2k = 1, and
// Y_0 = (2/pi)(ln(z/2) + gamma) J_0 - (4/pi) sum_k (-1)^k J_2k / k,
// Y_1 = -Y_0' = (2/pi)[(ln(z/2) + gamma) J_1 - J_0 / z] + (2/pi) sum_k (-1)^k (J_2k-1 - J_2k+1) / k
// (Neumann series; Abramowitz and Stegun 9.1.88, 9.1.27).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bie2d.h"
#include "linalg.h"

namespace efie {
namespace {

constexpr double PI2D = 3.14159265358979323846;
constexpr double EULER = 0.57721566490153286061;
constexpr int NQN = 8;          // points of the near-pair rules
constexpr int TILE = 15;        // entries per side of an assembly tile (16 x 16 segment pairs)

// ------------------------------------------------------------ complex helpers
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 crcp(double2 a) {
    // 1/a with scaling (Smith's method)
    if (fabs(a.x) >= fabs(a.y)) {
        const double r = a.y / a.x, d = a.x + a.y * r;
        return make_double2(1.0 / d, -r / d);
    }
    const double r = a.x / a.y, d = a.y + a.x * r;
    return make_double2(r / d, -1.0 / d);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) { return cmul(a, crcp(b)); }
__device__ __forceinline__ double2 cexp_(double2 a) {
    double s, c;
    sincos(a.y, &s, &c);
    const double e = exp(a.x);
    return make_double2(e * c, e * s);
}
__device__ __forceinline__ double2 clog_(double2 a) { return make_double2(log(hypot(a.x, a.y)), atan2(a.y, a.x)); }
__device__ __forceinline__ double2 csqrt_(double2 a) {
    const double r = hypot(a.x, a.y);
    if (r == 0.0) return make_double2(0.0, 0.0);
    if (a.x >= 0.0) {
        const double t = sqrt(0.5 * (r + a.x));
        return make_double2(t, 0.5 * a.y / t);
    }
    const double t = sqrt(0.5 * (r - a.x));
    return make_double2(0.5 * fabs(a.y) / t, a.y >= 0.0 ? t : -t);
}
__device__ __forceinline__ double cabs_(double2 a) { return hypot(a.x, a.y); }

struct H01 {
    double2 h0, h1;
};

// Miller's backward recurrence: the normalized J_0, J_1 and the Neumann sums
// (Y-parts without the logarithmic terms), z not 0.
struct Jsums {
    double2 j0, j1, ysum0, ysum1;   // ysum0 = -(4/pi) sum (-1)^k J_2k/k, ysum1 = (2/pi) sum (-1)^k (J_2k-1 - J_2k+1)/k
};

__device__ Jsums bessel_small(double2 z) {
    const double az = cabs_(z);
    const int M = 2 * (int(0.5 * az) + 15);
    const double2 iz = crcp(z);
    double2 jn1 = make_double2(0.0, 0.0);           // J_{m+1}
    double2 jn = make_double2(1e-30, 0.0);          // J_m, unnormalized
    double2 norm = make_double2(0.0, 0.0), s0 = norm, s1 = norm, j1 = norm, j0 = norm;
    for (int m = M; m >= 0; --m) {
        // contributions of J_m
        if (m == 0) {
            norm = cadd(norm, jn);
            j0 = jn;
        } else if ((m & 1) == 0) {
            const int k = m >> 1;
            norm = cadd(norm, cscale(jn, 2.0));
            s0 = cadd(s0, cscale(jn, ((k & 1) ? -1.0 : 1.0) / k));
        } else {
            // odd m: + (-1)^((m+1)/2) / ((m+1)/2) from J_{2k-1}, - (-1)^((m-1)/2) / ((m-1)/2) from J_{2k+1}
            const int ka = (m + 1) >> 1;
            double c = ((ka & 1) ? -1.0 : 1.0) / ka;
            if (m >= 3) {
                const int kb = (m - 1) >> 1;
                c -= ((kb & 1) ? -1.0 : 1.0) / kb;
            }
            s1 = cadd(s1, cscale(jn, c));
            if (m == 1) j1 = jn;
        }
        if (m == 0) break;
        // J_{m-1} = (2m / z) J_m - J_{m+1}
        const double2 jm = csub(cscale(cmul(iz, jn), 2.0 * m), jn1);
        jn1 = jn;
        jn = jm;
        // keep the unnormalized sequence in range (every accumulated quantity is linear in it)
        const double mag = fabs(jn.x) + fabs(jn.y);
        if (mag > 1e200) {
            const double f = 1e-200;
            jn = cscale(jn, f);
            jn1 = cscale(jn1, f);
            norm = cscale(norm, f);
            s0 = cscale(s0, f);
            s1 = cscale(s1, f);
            j1 = cscale(j1, f);
        }
    }
    const double2 inv = crcp(norm);
    Jsums r;
    r.j0 = cmul(j0, inv);
    r.j1 = cmul(j1, inv);
    r.ysum0 = cscale(cmul(s0, inv), -4.0 / PI2D);
    r.ysum1 = cscale(cmul(s1, inv), 2.0 / PI2D);
    return r;
}

// H0^(2)(z) and H1^(2)(z), Re z > 0, Im z <= 0
__device__ H01 hankel2_01(double2 z) {
    const double az = cabs_(z);
    H01 h;
    if (az >= 17.0) {
        const double2 m = cmul(make_double2(0.0, -1.0), crcp(z));   // -j / z
        double2 s0 = make_double2(1.0, 0.0), s1 = s0, t0 = s0, t1 = s0;
        double prev = 2.0;
        for (int k = 1; k <= 60; ++k) {
            // an asymptotic series: summed up to its smallest term (or to 1e-17 of the sum)
            const double f = double(2 * k - 1) * double(2 * k - 1);
            const double2 n0 = cscale(cmul(t0, m), (0.0 - f) / (8.0 * k));
            const double2 n1 = cscale(cmul(t1, m), (4.0 - f) / (8.0 * k));
            const double mag = cabs_(n0) + cabs_(n1);
            if (mag > prev) break;
            t0 = n0;
            t1 = n1;
            prev = mag;
            s0 = cadd(s0, t0);
            s1 = cadd(s1, t1);
            if (mag < 1e-17 * cabs_(s0)) break;
        }
        // (2/(pi z))^(1/2) exp(-j (z - pi/4)); the order-1 phase adds exp(j pi/2) = j
        const double2 pre = cmul(csqrt_(cscale(crcp(z), 2.0 / PI2D)),
                                 cexp_(make_double2(z.y, -(z.x - 0.25 * PI2D))));
        h.h0 = cmul(pre, s0);
        h.h1 = cmul(cmul(pre, make_double2(0.0, 1.0)), s1);
        return h;
    }
    const Jsums b = bessel_small(z);
    const double2 lg = cadd(clog_(cscale(z, 0.5)), make_double2(EULER, 0.0));
    const double2 y0 = cadd(cscale(cmul(lg, b.j0), 2.0 / PI2D), b.ysum0);
    const double2 y1 = cadd(cscale(csub(cmul(lg, b.j1), cmul(b.j0, crcp(z))), 2.0 / PI2D), b.ysum1);
    h.h0 = make_double2(b.j0.x + y0.y, b.j0.y - y0.x);          // J0 - j Y0
    h.h1 = make_double2(b.j1.x + y1.y, b.j1.y - y1.x);
    return h;
}

// G_reg(R) = G(R) + ln(R) / (2 pi) for the self pair (|kappa R| small), from the
// series without cancellation: G = -(j/4) J0 - (1/(2 pi))(ln(kappa R/2) + gamma) J0 - ysum0/4
__device__ double2 green_reg(double2 kap, double R) {
    const double2 lk = cadd(clog_(cscale(kap, 0.5)), make_double2(EULER, 0.0));   // ln(kappa/2) + gamma
    if (R == 0.0) {
        return make_double2(-lk.x / (2.0 * PI2D), -0.25 - lk.y / (2.0 * PI2D));
    }
    const Jsums b = bessel_small(cscale(kap, R));
    const double lr = log(R);
    // -(j/4) J0 - (1/2pi) [lk J0 + ln R (J0 - 1)] - ysum0 / 4
    double2 g = make_double2(0.25 * b.j0.y, -0.25 * b.j0.x);
    const double2 t = cadd(cmul(lk, b.j0), cscale(make_double2(b.j0.x - 1.0, b.j0.y), lr));
    g = csub(g, cscale(t, 1.0 / (2.0 * PI2D)));
    g = csub(g, cscale(b.ysum0, 0.25));
    return g;
}

// moments of one segment pair: mS[alpha][beta] = int int G phi_alpha phi_beta dx dy,
// mD likewise with dG/dn_test, m0 = int int G (no segment lengths)
struct PairMom {
    double2 s[2][2], d[2][2], m0;
};

__device__ __forceinline__ void accum(PairMom& pm, double2 kap, double rx, double ry, double px, double py,
                                      double nx, double ny, double xa, double yb, double w) {
    const double dx = rx - px, dy = ry - py;
    const double R = sqrt(dx * dx + dy * dy);
    const H01 h = hankel2_01(cscale(kap, R));
    // G = -(j/4) H0, dG/dR = (j kappa / 4) H1
    const double2 G = make_double2(0.25 * h.h0.y, -0.25 * h.h0.x);
    const double2 jk = make_double2(-0.25 * kap.y, 0.25 * kap.x);
    const double2 dG = cscale(cmul(jk, h.h1), (dx * nx + dy * ny) / R);
    const double pa[2] = {1.0 - xa, xa}, pb[2] = {1.0 - yb, yb};
    const double2 Gw = cscale(G, w), dGw = cscale(dG, w);
#pragma unroll
    for (int al = 0; al < 2; ++al)
#pragma unroll
        for (int be = 0; be < 2; ++be) {
            const double f = pa[al] * pb[be];
            pm.s[al][be] = cadd(pm.s[al][be], cscale(Gw, f));
            pm.d[al][be] = cadd(pm.d[al][be], cscale(dGw, f));
        }
    pm.m0 = cadd(pm.m0, Gw);
}

template <int Q>
__device__ PairMom pair_moments(const DevContour& c, double2 kap, int a, int b) {
    PairMom pm;
#pragma unroll
    for (int al = 0; al < 2; ++al)
#pragma unroll
        for (int be = 0; be < 2; ++be) pm.s[al][be] = pm.d[al][be] = make_double2(0.0, 0.0);
    pm.m0 = make_double2(0.0, 0.0);
    const int n = c.n;
    const double nxa = c.nx[a], nya = c.ny[a];
    if (a == b) {
        const double L = c.len[a];
#pragma unroll 1
        for (int p = 0; p < NQN; ++p)
#pragma unroll 1
            for (int q = 0; q < NQN; ++q) {
                const double xp = c.hx[p], xq = c.hx[q], w = c.hw[p] * c.hw[q];
                const double2 g = cscale(green_reg(kap, L * fabs(xp - xq)), w);
                const double pa[2] = {1.0 - xp, xp}, pb[2] = {1.0 - xq, xq};
                for (int al = 0; al < 2; ++al)
                    for (int be = 0; be < 2; ++be) pm.s[al][be] = cadd(pm.s[al][be], cscale(g, pa[al] * pb[be]));
                pm.m0 = cadd(pm.m0, g);
            }
        // -(1/2 pi) [ln L int int phi phi + int int phi phi ln|x - y|]
        const double lnL = log(L), f = -1.0 / (2.0 * PI2D);
        const double lm[2][2] = {{-7.0 / 16.0, -5.0 / 16.0}, {-5.0 / 16.0, -7.0 / 16.0}};
        for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) pm.s[al][be].x += f * (0.25 * lnL + lm[al][be]);
        pm.m0.x += f * (lnL - 1.5);
        return pm;
    }
    const bool next = b == (a + 1) % n, prev = b == (a + n - 1) % n;
    if (next || prev) {
        // V shared node; Pa, Pb the other ends of a and b
        double vx, vy, pax, pay, pbx, pby;
        if (next) {
            vx = c.bx[a]; vy = c.by[a]; pax = c.ax[a]; pay = c.ay[a]; pbx = c.bx[b]; pby = c.by[b];
        } else {
            vx = c.ax[a]; vy = c.ay[a]; pax = c.bx[a]; pay = c.by[a]; pbx = c.ax[b]; pby = c.ay[b];
        }
#pragma unroll 1
        for (int p = 0; p < NQN; ++p)
#pragma unroll 1
            for (int q = 0; q < NQN; ++q) {
                const double sg = c.hx[p], t = c.hx[q];
                const double w = c.hw[p] * c.hw[q] * 2.0 * sg * sg * sg;
                const double s = sg * sg;
#pragma unroll 1
                for (int tri = 0; tri < 2; ++tri) {
                    const double u = tri == 0 ? s : s * t, v = tri == 0 ? s * t : s;
                    const double rx = vx + u * (pax - vx), ry = vy + u * (pay - vy);
                    const double px = vx + v * (pbx - vx), py = vy + v * (pby - vy);
                    const double xa = next ? 1.0 - u : u, yb = next ? v : 1.0 - v;
                    accum(pm, kap, rx, ry, px, py, nxa, nya, xa, yb, w);
                }
            }
        return pm;
    }
    const double ax = c.ax[a], ay = c.ay[a], bx = c.bx[a] - ax, by = c.by[a] - ay;
    const double qx = c.ax[b], qy = c.ay[b], sx = c.bx[b] - qx, sy = c.by[b] - qy;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const double xp = c.gx[p];
        const double rx = ax + xp * bx, ry = ay + xp * by;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double yq = c.gx[q];
            accum(pm, kap, rx, ry, qx + yq * sx, qy + yq * sy, nxa, nya, xp, yq, c.gw[p] * c.gw[q]);
        }
    }
    return pm;
}

// One block: entries (i, j), i in [i0, i0 + TILE), j in [j0, j0 + TILE) of the
// requested window; its 16 x 16 segment pairs (a in i0-1 .. i0+14, b in j0-1 ..
// j0+14, mod n) are evaluated once, one per thread, into LDS and each entry adds
// its four.  Out: S, Dm, Nm (any may be null) at [(i - row0) * ld + (j - col0)].
template <int Q>
__global__ __launch_bounds__(256) void assemble2d_kernel(DevContour c, double kr, double ki, int row0, int nrows,
                                                         int col0, int ncols, int ld, double2* __restrict__ S,
                                                         double2* __restrict__ Dm, double2* __restrict__ Nm) {
    __shared__ PairMom pm[16 * 16];
    const int n = c.n;
    const int tcols = (ncols + TILE - 1) / TILE;
    const int ti = int(blockIdx.x) / tcols, tj = int(blockIdx.x) - ti * tcols;
    const int i0 = row0 + ti * TILE, j0 = col0 + tj * TILE;
    const double2 kap = make_double2(kr, ki);
    {
        const int t = threadIdx.x;
        const int a = (i0 - 1 + t / 16 + n) % n, b = (j0 - 1 + t % 16 + n) % n;
        pm[t] = pair_moments<Q>(c, kap, a, b);
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= TILE * TILE) return;
    const int li = t / TILE, lj = t - li * TILE;
    const int i = i0 + li, j = j0 + lj;
    if (i >= row0 + nrows || j >= col0 + ncols) return;
    const double2 k2 = make_double2(kr * kr - ki * ki, 2.0 * kr * ki);
    double2 vs = make_double2(0.0, 0.0), vd = vs, vn = vs;
    for (int da = 0; da < 2; ++da) {
        // da = 0: segment i-1 (node i is its end, alpha = 1); da = 1: segment i (alpha = 0)
        const int a = (i - 1 + da + n) % n, al = 1 - da;
        for (int db = 0; db < 2; ++db) {
            const int b = (j - 1 + db + n) % n, be = 1 - db;
            const PairMom& m = pm[(li + da) * 16 + (lj + db)];
            const double LL = c.len[a] * c.len[b];
            const double2 sv = cscale(m.s[al][be], LL);
            vs = cadd(vs, sv);
            vd = cadd(vd, cscale(m.d[al][be], LL));
            const double sig = (al == be) ? 1.0 : -1.0;          // lambda' = -1/L (start), +1/L (end)
            const double nn = c.nx[a] * c.nx[b] + c.ny[a] * c.ny[b];
            vn = cadd(vn, csub(cscale(m.m0, sig), cscale(cmul(k2, sv), nn)));
        }
    }
    const size_t o = size_t(i - row0) * ld + (j - col0);
    if (S) S[o] = vs;
    if (Dm) Dm[o] = vd;
    if (Nm) Nm[o] = vn;
}

// e (and h) for plane waves exp(-j k khat . r), khat = (cos phi, sin phi): one
// thread per (right-hand side, node)
// TM (te = 0): e = (lambda, E_z), h = (lambda, H_t), H_t = -(khat . n) E_z / eta;
// TE (te = 1): e = (lambda, E_t), E_t = eta (khat . n) H_z, h = (lambda, H_z);
// the incident field exp(-j k khat . r) is E_z (TM) or H_z (TE)
__global__ void excite2d_kernel(DevContour c, double k, double eta, const double* __restrict__ phis, int nrhs,
                                double2* __restrict__ e, double2* __restrict__ h, int te) {
    const int n = c.n;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nrhs) return;
    const int s = idx / n, i = idx - s * n;
    double sp, cp;
    sincos(phis[s], &sp, &cp);
    double2 ev = make_double2(0.0, 0.0), hv = ev;
    for (int da = 0; da < 2; ++da) {
        const int a = (i - 1 + da + n) % n;
        const int al = 1 - da;
        const double L = c.len[a];
        const double kn = cp * c.nx[a] + sp * c.ny[a];
        for (int p = 0; p < c.q; ++p) {
            const double x = c.gx[p];
            const double rx = c.ax[a] + x * (c.bx[a] - c.ax[a]), ry = c.ay[a] + x * (c.by[a] - c.ay[a]);
            double s_, c_;
            sincos(-k * (cp * rx + sp * ry), &s_, &c_);
            const double wphi = L * c.gw[p] * (al == 0 ? 1.0 - x : x);
            if (te) {
                ev.x += wphi * eta * kn * c_;
                ev.y += wphi * eta * kn * s_;
                hv.x += wphi * c_;
                hv.y += wphi * s_;
            } else {
                ev.x += wphi * c_;
                ev.y += wphi * s_;
                hv.x -= wphi * kn * c_ / eta;
                hv.y -= wphi * kn * s_ / eta;
            }
        }
    }
    e[idx] = ev;
    if (h) h[idx] = hv;
}

// F[s][d] = sum_i J[s][i] int w lambda_i exp(j k rhat_d . r) dS: one thread per (s, d);
// w = 1 (TM) or rhat_d . n (TE, constant on each segment)
__global__ void farfield2d_kernel(DevContour c, double k, const double2* __restrict__ J, int nrhs,
                                  const double* __restrict__ phis, int nphi, double2* __restrict__ F, int te) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrhs * nphi) return;
    const int s = idx / nphi, d = idx - s * nphi;
    const int n = c.n;
    double sp, cp;
    sincos(phis[d], &sp, &cp);
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < n; ++a) {
        const double2 ja = J[size_t(s) * n + a], jb = J[size_t(s) * n + (a + 1) % n];
        double2 m0 = make_double2(0.0, 0.0), m1 = m0;
        for (int p = 0; p < c.q; ++p) {
            const double x = c.gx[p];
            const double rx = c.ax[a] + x * (c.bx[a] - c.ax[a]), ry = c.ay[a] + x * (c.by[a] - c.ay[a]);
            double s_, c_;
            sincos(k * (cp * rx + sp * ry), &s_, &c_);
            const double w = c.len[a] * c.gw[p] * (te ? cp * c.nx[a] + sp * c.ny[a] : 1.0);
            m0.x += w * (1.0 - x) * c_;
            m0.y += w * (1.0 - x) * s_;
            m1.x += w * x * c_;
            m1.y += w * x * s_;
        }
        acc = cadd(acc, cadd(cmul(ja, m0), cmul(jb, m1)));
    }
    F[idx] = acc;
}

// Y = alpha G X (+ beta Y): the Gram matrix (cyclic tridiagonal: (L_{i-1} + L_i)/3
// on the diagonal, L/6 beside it) applied to rows of X
__global__ void gram_apply_kernel(DevContour c, const double2* __restrict__ X, double2* __restrict__ Y, int nvec,
                                  double alpha, double beta) {
    const int n = c.n;
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(n) * nvec) return;
    const int s = int(idx / n), i = int(idx - size_t(s) * n);
    const int im = (i + n - 1) % n, ip = (i + 1) % n;
    const double2* x = X + size_t(s) * n;
    const double lm = c.len[im], li = c.len[i];
    const double dre = (lm + li) / 3.0;
    double2 v = make_double2(dre * x[i].x + lm / 6.0 * x[im].x + li / 6.0 * x[ip].x,
                             dre * x[i].y + lm / 6.0 * x[im].y + li / 6.0 * x[ip].y);
    v = cscale(v, alpha);
    if (beta != 0.0) v = cadd(v, cscale(Y[idx], beta));
    Y[idx] = v;
}

// Y = G^-1 X by Jacobi sweeps y <- D^-1 (x - O y) (O the off-diagonal part):
// every row's off-diagonal sum is half its diagonal, so each sweep contracts the
// error at least twofold and JAC sweeps give 2^-JAC.  A block owns JW nodes of one
// vector and iterates in LDS on a window with JAC nodes of halo on each side
// (the halo's values go stale from the edge inwards, one node per sweep).
constexpr int JAC = 56, JW = 1024, JH = JW + 2 * JAC;
__global__ __launch_bounds__(256) void gram_solve_kernel(DevContour c, const double2* __restrict__ X,
                                                         double2* __restrict__ Y, int nvec) {
    __shared__ double2 xs[JH], ya[JH], yb[JH];
    __shared__ double lin[JH + 1];
    const int n = c.n;
    const int nblk = (n + JW - 1) / JW;
    const int s = int(blockIdx.x) / nblk, bw = int(blockIdx.x) - s * nblk;
    const int i0 = bw * JW - JAC;
    const double2* x = X + size_t(s) * n;
    for (int t = threadIdx.x; t < JH; t += blockDim.x) {
        const int i = ((i0 + t) % n + n) % n;
        xs[t] = x[i];
        lin[t] = c.len[(i + n - 1) % n];          // L_{i-1}
        if (t == JH - 1) lin[JH] = c.len[i];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < JH; t += blockDim.x) {
        const double d = (lin[t] + lin[t + 1]) / 3.0;
        ya[t] = cscale(xs[t], 1.0 / d);
    }
    __syncthreads();
    double2* cur = ya;
    double2* nxt = yb;
    for (int it = 0; it < JAC; ++it) {
        for (int t = threadIdx.x; t < JH; t += blockDim.x) {
            if (t == 0 || t == JH - 1) {
                nxt[t] = cur[t];
                continue;
            }
            const double lm = lin[t], li = lin[t + 1];
            const double d = (lm + li) / 3.0;
            const double2 r = csub(xs[t], cadd(cscale(cur[t - 1], lm / 6.0), cscale(cur[t + 1], li / 6.0)));
            nxt[t] = cscale(r, 1.0 / d);
        }
        __syncthreads();
        double2* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    for (int t = threadIdx.x; t < JW; t += blockDim.x) {
        const int i = bw * JW + t;
        if (i < n) Y[size_t(s) * n + i] = cur[JAC + t];
    }
}

// X[m] = sum_i x[i] exp(sign 2 pi j (m i mod n) / n) (scale applied): direct DFT
__global__ void dft_kernel(const double2* __restrict__ x, double2* __restrict__ X, int n, double sign, double scale) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int i = 0; i < n; ++i) {
        const long long q = (long long)m * i % n;
        double s_, c_;
        sincos(sign * 2.0 * PI2D * double(q) / double(n), &s_, &c_);
        acc = cadd(acc, cmul(x[i], make_double2(c_, s_)));
    }
    X[m] = cscale(acc, scale);
}

// eigenvalues of the counterpart C_c and of its inverse from those of its factors
// TM: lC = lN lS / lG + (lG/2 - lDt)(lG/2 + lD) / lG  (lN at k~, lS at k, lD at k, lDt at k~);
// TE: lC = lS lN / lG + (lG/2 + lDt)(lG/2 - lD) / lG  (lS at k~, lN at k, lD, lDt the
//     spectra of the double layer D = D*^T at k and k~)
__global__ void circ_combine_kernel(const double2* __restrict__ lS, const double2* __restrict__ lD,
                                    const double2* __restrict__ lN, const double2* __restrict__ lDt,
                                    const double2* __restrict__ lG, double2* __restrict__ lC, double2* __restrict__ lCi,
                                    int n, int te) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double2 g = lG[m], ig = crcp(g);
    const double2 hg = cscale(g, 0.5);
    const double2 t1 = cmul(cmul(lN[m], lS[m]), ig);
    const double2 t2 = te ? cmul(cmul(cadd(hg, lDt[m]), csub(hg, lD[m])), ig)
                          : cmul(cmul(csub(hg, lDt[m]), cadd(hg, lD[m])), ig);
    const double2 v = cadd(t1, t2);
    lC[m] = v;
    lCi[m] = crcp(v);
}

// first column of the transpose of a circulant: ct[m] = c[(n - m) mod n]
__global__ void circ_transpose_kernel(const double2* __restrict__ c, double2* __restrict__ ct, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) ct[m] = c[(n - m) % n];
}

// first column of the circle's Gram matrix
__global__ void gram_column_kernel(DevContour c, double2* __restrict__ g) {
    const int n = c.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    if (i == 0) v = (c.len[n - 1] + c.len[0]) / 3.0;
    else if (i == 1) v = c.len[0] / 6.0;
    if (i == n - 1) v += c.len[n - 1] / 6.0;
    g[i] = make_double2(v, 0.0);
}

// Y = conj(X)
__global__ void conj_kernel(const double2* __restrict__ X, double2* __restrict__ Y, size_t count) {
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += size_t(gridDim.x) * blockDim.x)
        Y[e] = make_double2(X[e].x, -X[e].y);
}

// norms of the rows of X (nvec x n): one block per row
__global__ __launch_bounds__(256) void row_norm_kernel(const double2* __restrict__ X, int n, double* __restrict__ out) {
    __shared__ double red[256];
    const double2* x = X + size_t(blockIdx.x) * n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += x[i].x * x[i].x + x[i].y * x[i].y;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0]);
}

// Cholesky of the Hermitian b x b Gram matrix Gm (row-major, b <= 64) with shift
// added to its diagonal, Gm = R^H R (R upper); writes (R^-1)^T into T (b x b) and
// info = 0, or info = column + 1 of a non-positive pivot.  One block, LDS.
__global__ __launch_bounds__(256) void chol_inv_kernel(const double2* __restrict__ Gm, int b, double shift,
                                                       double2* __restrict__ T, int* __restrict__ info) {
    __shared__ double2 R[64][65];
    __shared__ double2 Ri[64][65];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    for (int e = tid; e < b * b; e += 256) {
        const int r = e / b, c = e % b;
        double2 v = Gm[e];
        if (r == c) v = make_double2(v.x + shift, 0.0);
        R[r][c] = v;
        Ri[r][c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    // right-looking: row k of R from the updated trailing matrix
    for (int k = 0; k < b; ++k) {
        if (tid == 0) {
            const double d = R[k][k].x;
            if (!(d > 0.0) && !bad) bad = k + 1;
            R[k][k] = make_double2(d > 0.0 ? sqrt(d) : 1.0, 0.0);
        }
        __syncthreads();
        const double rkk = R[k][k].x;
        for (int c = k + 1 + tid; c < b; c += 256) R[k][c] = cscale(R[k][c], 1.0 / rkk);
        __syncthreads();
        for (int e = tid; e < (b - k - 1) * (b - k - 1); e += 256) {
            const int r = k + 1 + e / (b - k - 1), c = k + 1 + e % (b - k - 1);
            if (c >= r) {
                // A[r][c] -= conj(R[k][r]) R[k][c]
                const double2 x = R[k][r], y = R[k][c];
                R[r][c] = csub(R[r][c], make_double2(x.x * y.x + x.y * y.y, x.x * y.y - x.y * y.x));
            }
        }
        __syncthreads();
    }
    // inverse of the upper triangular R, column by column (thread per column)
    for (int c = tid; c < b; c += 256) {
        Ri[c][c] = make_double2(1.0 / R[c][c].x, 0.0);
        for (int r = c - 1; r >= 0; --r) {
            double2 acc = make_double2(0.0, 0.0);
            for (int m = r + 1; m <= c; ++m) acc = cadd(acc, cmul(R[r][m], Ri[m][c]));
            Ri[r][c] = cscale(acc, -1.0 / R[r][r].x);
        }
    }
    __syncthreads();
    for (int e = tid; e < b * b; e += 256) {
        const int r = e / b, c = e % b;
        T[e] = (c <= r) ? Ri[c][r] : make_double2(0.0, 0.0);       // T = (R^-1)^T
    }
    if (tid == 0) *info = bad;
}

// Blocked right-looking LU with partial pivoting of the r x r matrix M (row-major,
// in place; the same factors and pivot order as the unblocked elimination): for
// each panel of LU_NB columns, the panel is factored in one workgroup (pivot search
// over its column below the diagonal, row swap within the panel, scaling, rank-1
// update of the panel), its row swaps are applied to the columns outside the panel,
// the block row to its right is solved against the panel's unit lower triangle, and
// the trailing matrix takes the update A22 -= L21 U12 on the matrix cores.
constexpr int LU_NB = 64;

__global__ __launch_bounds__(1024) void lu_panel_kernel(double2* __restrict__ M, int r, int k0, int kb,
                                                        int* __restrict__ piv, int* __restrict__ info) {
    __shared__ double vmax[1024];
    __shared__ int imax[1024];
    const int tid = threadIdx.x;
    for (int j = k0; j < k0 + kb; ++j) {
        double best = -1.0;
        int bi = j;
        for (int i = j + tid; i < r; i += 1024) {
            const double v = cabs_(M[size_t(i) * r + j]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        vmax[tid] = best;
        imax[tid] = bi;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
            if (tid < o && (vmax[tid + o] > vmax[tid] || (vmax[tid + o] == vmax[tid] && imax[tid + o] < imax[tid]))) {
                vmax[tid] = vmax[tid + o];
                imax[tid] = imax[tid + o];
            }
            __syncthreads();
        }
        const int p = imax[0];
        const double pv = vmax[0];
        __syncthreads();
        if (tid == 0) {
            piv[j] = p;
            if (!(pv > 0.0) && *info == 0) *info = j + 1;
        }
        if (p != j)
            for (int c = k0 + tid; c < k0 + kb; c += 1024) {
                const double2 t = M[size_t(j) * r + c];
                M[size_t(j) * r + c] = M[size_t(p) * r + c];
                M[size_t(p) * r + c] = t;
            }
        __syncthreads();
        const double2 inv = pv > 0.0 ? crcp(M[size_t(j) * r + j]) : make_double2(0.0, 0.0);
        for (int i = j + 1 + tid; i < r; i += 1024) M[size_t(i) * r + j] = cmul(M[size_t(i) * r + j], inv);
        __syncthreads();
        const int w = k0 + kb - j - 1;
        if (w > 0)
            for (size_t e = tid; e < size_t(r - j - 1) * w; e += 1024) {
                const int i = j + 1 + int(e / w), c = j + 1 + int(e % w);
                M[size_t(i) * r + c] = csub(M[size_t(i) * r + c], cmul(M[size_t(i) * r + j], M[size_t(j) * r + c]));
            }
        __syncthreads();
    }
}

// the panel's row swaps (in pivot order) on the columns outside [k0, k0 + kb): a thread per column
__global__ void lu_swap_kernel(double2* __restrict__ M, int r, int k0, int kb, const int* __restrict__ piv) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = t < k0 ? t : t + kb;          // skip the panel's columns
    if (t >= r - kb) return;
    for (int j = k0; j < k0 + kb; ++j) {
        const int p = piv[j];
        if (p != j) {
            const double2 x = M[size_t(j) * r + c];
            M[size_t(j) * r + c] = M[size_t(p) * r + c];
            M[size_t(p) * r + c] = x;
        }
    }
}

// U12 = L11^-1 A12 for the block row [k0, k0 + kb) right of the panel: a thread per column
__global__ void lu_trsm_kernel(double2* __restrict__ M, int r, int k0, int kb) {
    const int c = k0 + kb + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= r) return;
    for (int i = 1; i < kb; ++i) {
        double2 acc = M[size_t(k0 + i) * r + c];
        for (int t = 0; t < i; ++t) acc = csub(acc, cmul(M[size_t(k0 + i) * r + k0 + t], M[size_t(k0 + t) * r + c]));
        M[size_t(k0 + i) * r + c] = acc;
    }
}

// sum over the block of 256 threads (four wavefronts)
__device__ double2 block_sum(double2 v, double2* red) {
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_down(v.x, o);
        v.y += __shfl_down(v.y, o);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return cadd(cadd(red[0], red[1]), cadd(red[2], red[3]));
}

// row s of X (r values) overwritten by M^-1 X[s] from the LU factors: a block per
// row, the substitutions row by row, each row's dot product over the block
__global__ __launch_bounds__(256) void lu_solve_kernel(const double2* __restrict__ LU, const int* __restrict__ piv,
                                                       int r, double2* __restrict__ X, int nrhs) {
    __shared__ double2 red[4];
    const int s = blockIdx.x;
    if (s >= nrhs) return;
    double2* x = X + size_t(s) * r;
    if (threadIdx.x == 0)
        for (int k = 0; k < r; ++k) {
            const int p = piv[k];
            if (p != k) {
                const double2 t = x[k];
                x[k] = x[p];
                x[p] = t;
            }
        }
    __syncthreads();
    for (int i = 1; i < r; ++i) {           // L (unit diagonal)
        double2 acc = make_double2(0.0, 0.0);
        for (int m = threadIdx.x; m < i; m += 256) acc = cadd(acc, cmul(LU[size_t(i) * r + m], x[m]));
        const double2 t = block_sum(acc, red);
        if (threadIdx.x == 0) x[i] = csub(x[i], t);
        __syncthreads();
    }
    for (int i = r - 1; i >= 0; --i) {      // U
        double2 acc = make_double2(0.0, 0.0);
        for (int m = i + 1 + threadIdx.x; m < r; m += 256) acc = cadd(acc, cmul(LU[size_t(i) * r + m], x[m]));
        const double2 t = block_sum(acc, red);
        if (threadIdx.x == 0) x[i] = cdiv(csub(x[i], t), LU[size_t(i) * r + i]);
        __syncthreads();
    }
}

__global__ void identity_add_kernel(double2* __restrict__ M, int r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < r) M[size_t(i) * r + i].x += 1.0;
}

unsigned grid_of(size_t count) { return unsigned(std::min<size_t>((count + 255) / 256, size_t(1) << 20)); }

}  // namespace
}  // namespace efie

// ===================================================================== host side
namespace {

using efie::DevContour;

// Gauss-Legendre rule on [0, 1] by Newton's iteration on P_q (Golub-Welsch would
// do as well); nodes ascending
void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < q; ++i) {
        double t = std::cos(3.14159265358979323846 * (i + 0.75) / (q + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (q == 1) {
                p1 = t;
                p0 = 1.0;
            }
            dp = q * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= q; ++k) {
            const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = q * (t * p1 - p0) / (t * t - 1.0);
        x[q - 1 - i] = 0.5 * (t + 1.0);
        w[q - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);      // 2/((1-t^2) P'^2) halved for [0, 1]
    }
}

struct HostContour {
    std::vector<double> ax, ay, bx, by, len, nx, ny;
    double perimeter = 0.0;
};

HostContour make_contour(const double* nodes, int64_t n) {
    HostContour h;
    h.ax.resize(n); h.ay.resize(n); h.bx.resize(n); h.by.resize(n);
    h.len.resize(n); h.nx.resize(n); h.ny.resize(n);
    for (int64_t a = 0; a < n; ++a) {
        const int64_t b = (a + 1) % n;
        EFIE_REQUIRE(std::isfinite(nodes[2 * a]) && std::isfinite(nodes[2 * a + 1]), EFIE_ERR_ARG,
                     "bie2d: non-finite node");
        h.ax[a] = nodes[2 * a];
        h.ay[a] = nodes[2 * a + 1];
        h.bx[a] = nodes[2 * b];
        h.by[a] = nodes[2 * b + 1];
        const double dx = h.bx[a] - h.ax[a], dy = h.by[a] - h.ay[a];
        const double L = std::sqrt(dx * dx + dy * dy);
        EFIE_REQUIRE(L > 0.0, EFIE_ERR_DEGENERATE, "bie2d: zero-length segment");
        h.len[a] = L;
        h.nx[a] = dy / L;      // outward for a counter-clockwise contour
        h.ny[a] = -dx / L;
        h.perimeter += L;
    }
    double area = 0.0;
    for (int64_t a = 0; a < n; ++a) area += h.ax[a] * h.by[a] - h.bx[a] * h.ay[a];
    EFIE_REQUIRE(area > 0.0, EFIE_ERR_MESH_ORIENT, "bie2d: contour must run counter-clockwise");
    return h;
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct efie_bie2d_s {
    int64_t n = 0;
    int q = 4;
    HostContour curve[2];          // 0: the scatterer, 1: its circular counterpart
    std::vector<char> blob;        // packed device tables of both contours
    std::vector<size_t> offs;
    void* dev = nullptr;
    DevContour dc[2]{};
    // state of the last setup (device pointers into the caller's workspace)
    double k = 0.0, kt_re = 0.0, kt_im = 0.0;
    int pol = 0;                   // 0 TM, 1 TE
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t rmax = 0, block = 0, nvec = 0;
    // TM: S_k, D*_k, N_k~, D*_k~;  TE: S_k~, D*_k, N_k, D*_k~ (S / N at the wavenumber their term uses)
    double2 *S = nullptr, *Dst = nullptr, *Nt = nullptr, *Dtt = nullptr;
    double2 *cC = nullptr, *cCT = nullptr, *cI = nullptr, *cIT = nullptr;    // counterpart, inverse (+ transposes)
    double2 *T1 = nullptr, *T2 = nullptr, *T3 = nullptr;                       // nvec x n temporaries
    double2 *Qm = nullptr, *Bm = nullptr, *Wm = nullptr, *Mm = nullptr;        // skeleton and Woodbury factors
    double2 *Gb = nullptr, *Tb = nullptr;                                      // block x block
    double2* split = nullptr;                                                  // split-K partial products
    size_t split_n = 0;
    double* nrm = nullptr;
    int* piv = nullptr;
    int* info = nullptr;
    int64_t rank = -1;
    bool ready = false;
};

namespace {

using efie::gemm2d;

struct Layout {
    size_t S, Dst, Nt, Dtt, cC, cCT, cI, cIT, eig, T1, T2, T3, Qm, Bm, Wm, Mm, Gb, Tb, nrm, piv, info, split, total;
};

// scratch of the split-K products (the range finder's projections onto the basis
// and its Gram matrices): up to 64 partial products of 64 x max(rmax, 64)
size_t split_elems(int64_t rmax) { return size_t(64) * 64 * size_t(std::max<int64_t>(rmax, 64)); }

Layout layout(int64_t n, int64_t rmax, int64_t block, int64_t nvec) {
    Layout L{};
    size_t o = 0;
    const size_t nn = size_t(n) * size_t(n) * 16, v = size_t(n) * 16;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += a256(bytes);
        return at;
    };
    L.S = take(nn); L.Dst = take(nn); L.Nt = take(nn); L.Dtt = take(nn);
    L.cC = take(v); L.cCT = take(v); L.cI = take(v); L.cIT = take(v);
    L.eig = take(12 * v);       // 5 first columns, 5 spectra, 2 combined spectra
    L.T1 = take(size_t(nvec) * v); L.T2 = take(size_t(nvec) * v); L.T3 = take(size_t(nvec) * v);
    L.Qm = take(size_t(rmax) * v); L.Bm = take(size_t(rmax) * v); L.Wm = take(size_t(rmax) * v);
    L.Mm = take(size_t(rmax) * size_t(rmax) * 16);
    L.Gb = take(size_t(block) * size_t(block) * 16); L.Tb = take(size_t(block) * size_t(block) * 16);
    L.nrm = take(size_t(std::max(nvec, block)) * 8);
    L.piv = take(size_t(rmax) * 4);
    L.info = take(64);
    L.split = take(split_elems(rmax) * 16);
    L.total = o;
    return L;
}

void launch_assemble(const DevContour& c, double kr, double ki, int row0, int nrows, int col0, int ncols, int ld,
                     double2* S, double2* D, double2* N, int q, hipStream_t s) {
    const int tr = (nrows + efie::TILE - 1) / efie::TILE, tc = (ncols + efie::TILE - 1) / efie::TILE;
    const size_t nblk = size_t(tr) * size_t(tc);
    EFIE_REQUIRE(nblk < (size_t(1) << 31), EFIE_ERR_ARG, "bie2d_assemble: window too large");
    efie::prof_begin(efie::PROF_FAR, s);
#define B2D_Q(QQ)                                                                                                 \
    case QQ:                                                                                                      \
        hipLaunchKernelGGL((efie::assemble2d_kernel<QQ>), dim3(unsigned(nblk)), dim3(256), 0, s, c, kr, ki, row0, \
                           nrows, col0, ncols, ld, S, D, N);                                                      \
        break
    switch (q) {
        B2D_Q(2); B2D_Q(3); B2D_Q(4); B2D_Q(5); B2D_Q(6); B2D_Q(8);
        default: throw efie::Error{EFIE_ERR_ARG, "bie2d: q must be 2..6 or 8"};
    }
#undef B2D_Q
    efie::prof_end(efie::PROF_FAR, s, double(nrows) * double(ncols));
    EFIE_HIP_CHECK(hipGetLastError());
}

void gram_solve(const efie_bie2d_s& h, int which, const double2* X, double2* Y, int nvec, hipStream_t s) {
    const int nb = int((h.n + efie::JW - 1) / efie::JW);
    hipLaunchKernelGGL(efie::gram_solve_kernel, dim3(unsigned(nb * nvec)), dim3(256), 0, s, h.dc[which], X, Y, nvec);
}
void gram_apply(const efie_bie2d_s& h, int which, const double2* X, double2* Y, int nvec, double alpha, double beta,
                hipStream_t s) {
    hipLaunchKernelGGL(efie::gram_apply_kernel, dim3(efie::grid_of(size_t(h.n) * nvec)), dim3(256), 0, s,
                       h.dc[which], X, Y, nvec, alpha, beta);
}

const double2 ONE = {1.0, 0.0}, MONE = {-1.0, 0.0};

// Y = C_p X (trans = 0) or C_p^T X (trans = 1) for nvec rows X (nvec <= h.nvec);
// with sub_c also minus the counterpart (the skeleton's operator A = C_p - C_c).
// Rows are vectors: a "product with M" is C[s][i] = sum_k X[s][k] M[i][k] (NT) for
// M x, and sum_k X[s][k] M[k][i] (NN) for M^T x.
void apply_cp(efie_bie2d_s& h, const double2* X, double2* Y, int nvec, bool trans, bool sub_c, hipStream_t s) {
    const int n = int(h.n);
    if (h.pol == 1) {
        // TE: C_p = S~ G^-1 N + (G/2 + D~) G^-1 (G/2 - D), D = D*^T;
        //     C_p^T = N G^-1 S~ + (G/2 - D*) G^-1 (G/2 + D*~)
        if (!trans) {
            gemm2d(efie::G2D_NT, X, n, false, h.Nt, n, false, h.T1, n, nvec, n, n, ONE, false, s);
            gram_solve(h, 0, h.T1, h.T2, nvec, s);
            gemm2d(efie::G2D_NT, h.T2, n, false, h.S, n, false, Y, n, nvec, n, n, ONE, false, s);
            gemm2d(efie::G2D_NN, X, n, false, h.Dst, n, false, h.T1, n, nvec, n, n, MONE, false, s);
            gram_apply(h, 0, X, h.T1, nvec, 0.5, 1.0, s);
            gram_solve(h, 0, h.T1, h.T2, nvec, s);
            gemm2d(efie::G2D_NN, h.T2, n, false, h.Dtt, n, false, Y, n, nvec, n, n, ONE, true, s);
            gram_apply(h, 0, h.T2, Y, nvec, 0.5, 1.0, s);
            if (sub_c) gemm2d(efie::G2D_CIRC, X, n, false, h.cC, 0, false, Y, n, nvec, n, n, MONE, true, s);
        } else {
            gemm2d(efie::G2D_NT, X, n, false, h.S, n, false, h.T1, n, nvec, n, n, ONE, false, s);
            gram_solve(h, 0, h.T1, h.T2, nvec, s);
            gemm2d(efie::G2D_NT, h.T2, n, false, h.Nt, n, false, Y, n, nvec, n, n, ONE, false, s);
            gemm2d(efie::G2D_NT, X, n, false, h.Dtt, n, false, h.T1, n, nvec, n, n, ONE, false, s);
            gram_apply(h, 0, X, h.T1, nvec, 0.5, 1.0, s);
            gram_solve(h, 0, h.T1, h.T2, nvec, s);
            gemm2d(efie::G2D_NT, h.T2, n, false, h.Dst, n, false, Y, n, nvec, n, n, MONE, true, s);
            gram_apply(h, 0, h.T2, Y, nvec, 0.5, 1.0, s);
            if (sub_c) gemm2d(efie::G2D_CIRC, X, n, false, h.cCT, 0, false, Y, n, nvec, n, n, MONE, true, s);
        }
        return;
    }
    if (!trans) {
        // first term: N~ G^-1 S X
        gemm2d(efie::G2D_NT, X, n, false, h.S, n, false, h.T1, n, nvec, n, n, ONE, false, s);
        gram_solve(h, 0, h.T1, h.T2, nvec, s);
        gemm2d(efie::G2D_NT, h.T2, n, false, h.Nt, n, false, Y, n, nvec, n, n, ONE, false, s);
        // second term: (G/2 - D*~) G^-1 (G/2 + D*) X
        gemm2d(efie::G2D_NT, X, n, false, h.Dst, n, false, h.T1, n, nvec, n, n, ONE, false, s);
        gram_apply(h, 0, X, h.T1, nvec, 0.5, 1.0, s);
        gram_solve(h, 0, h.T1, h.T2, nvec, s);
        gemm2d(efie::G2D_NT, h.T2, n, false, h.Dtt, n, false, Y, n, nvec, n, n, MONE, true, s);
        gram_apply(h, 0, h.T2, Y, nvec, 0.5, 1.0, s);
        if (sub_c) gemm2d(efie::G2D_CIRC, X, n, false, h.cC, 0, false, Y, n, nvec, n, n, MONE, true, s);
    } else {
        // C_p^T = S G^-1 N~ + (G/2 + D) G^-1 (G/2 - D~), D = D*^T (S, N~ and G symmetric)
        gemm2d(efie::G2D_NT, X, n, false, h.Nt, n, false, h.T1, n, nvec, n, n, ONE, false, s);
        gram_solve(h, 0, h.T1, h.T2, nvec, s);
        gemm2d(efie::G2D_NT, h.T2, n, false, h.S, n, false, Y, n, nvec, n, n, ONE, false, s);
        gemm2d(efie::G2D_NN, X, n, false, h.Dtt, n, false, h.T1, n, nvec, n, n, MONE, false, s);
        gram_apply(h, 0, X, h.T1, nvec, 0.5, 1.0, s);
        gram_solve(h, 0, h.T1, h.T2, nvec, s);
        gemm2d(efie::G2D_NN, h.T2, n, false, h.Dst, n, false, Y, n, nvec, n, n, ONE, true, s);
        gram_apply(h, 0, h.T2, Y, nvec, 0.5, 1.0, s);
        if (sub_c) gemm2d(efie::G2D_CIRC, X, n, false, h.cCT, 0, false, Y, n, nvec, n, n, MONE, true, s);
    }
}

void require_setup(const efie_bie2d_s* h, const char* who) {
    EFIE_REQUIRE(h != nullptr, EFIE_ERR_ARG, std::string(who) + ": null handle");
    EFIE_REQUIRE(h->dev != nullptr, EFIE_ERR_STATE, std::string(who) + ": tables not uploaded");
    EFIE_REQUIRE(h->ready, EFIE_ERR_STATE, std::string(who) + ": efie_bie2d_setup not called");
}

}  // namespace

extern "C" {

int efie_bie2d_create(const double* nodes, const double* circle_nodes, int64_t n, int q, efie_bie2d* out) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(nodes && circle_nodes && out, EFIE_ERR_ARG, "bie2d_create: null argument");
        EFIE_REQUIRE(n >= 8 && n < (int64_t(1) << 28), EFIE_ERR_ARG, "bie2d_create: need 8 <= n < 2^28");
        EFIE_REQUIRE(q >= 2 && q <= 8 && q != 7, EFIE_ERR_ARG, "bie2d_create: q must be 2..6 or 8");
        auto* h = new efie_bie2d_s();
        try {
            h->n = n;
            h->q = q;
            h->curve[0] = make_contour(nodes, n);
            h->curve[1] = make_contour(circle_nodes, n);
            std::vector<double> gx, gw, hx, hw;
            gauss_legendre01(q, gx, gw);
            gauss_legendre01(efie::NQN, hx, hw);
            auto add = [&](const std::vector<double>& v) {
                const size_t off = a256(h->blob.size());
                h->blob.resize(off + v.size() * 8);
                std::memcpy(h->blob.data() + off, v.data(), v.size() * 8);
                h->offs.push_back(off);
            };
            for (int c = 0; c < 2; ++c) {
                const HostContour& hc = h->curve[c];
                add(hc.ax); add(hc.ay); add(hc.bx); add(hc.by); add(hc.len); add(hc.nx); add(hc.ny);
                add(gx); add(gw); add(hx); add(hw);
            }
            h->blob.resize(a256(h->blob.size()));
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return int(EFIE_OK);
    });
}

void efie_bie2d_destroy(efie_bie2d h) { delete h; }

int efie_bie2d_sizes(efie_bie2d h, int64_t rmax, int64_t block, int64_t nvec, size_t* table_bytes,
                     size_t* ws_bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(h && table_bytes && ws_bytes, EFIE_ERR_ARG, "bie2d_sizes: null argument");
        EFIE_REQUIRE(block >= 1 && block <= 64 && rmax >= 0 && rmax <= h->n && nvec >= block, EFIE_ERR_ARG,
                     "bie2d_sizes: need 1 <= block <= 64, 0 <= rmax <= n, nvec >= block");
        *table_bytes = h->blob.size();
        *ws_bytes = layout(h->n, rmax, block, nvec).total;
        return int(EFIE_OK);
    });
}

int efie_bie2d_upload(efie_bie2d h, void* dev, size_t bytes, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(h && dev, EFIE_ERR_ARG, "bie2d_upload: null argument");
        EFIE_REQUIRE(bytes >= h->blob.size(), EFIE_ERR_ARG, "bie2d_upload: buffer too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(dev) & 255) == 0, EFIE_ERR_ARG, "bie2d_upload: not 256-aligned");
        EFIE_HIP_CHECK(hipMemcpyAsync(dev, h->blob.data(), h->blob.size(), hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        const char* b = static_cast<const char*>(dev);
        for (int c = 0; c < 2; ++c) {
            auto D = [&](int i) { return reinterpret_cast<const double*>(b + h->offs[size_t(11 * c + i)]); };
            DevContour& d = h->dc[c];
            d.n = int32_t(h->n);
            d.q = h->q;
            d.ax = D(0); d.ay = D(1); d.bx = D(2); d.by = D(3); d.len = D(4); d.nx = D(5); d.ny = D(6);
            d.gx = D(7); d.gw = D(8); d.hx = D(9); d.hw = D(10);
        }
        h->dev = dev;
        return int(EFIE_OK);
    });
}

int efie_bie2d_perimeter(efie_bie2d h, int which, double* perimeter) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(h && perimeter && (which == 0 || which == 1), EFIE_ERR_ARG, "bie2d_perimeter: bad argument");
        *perimeter = h->curve[which].perimeter;
        return int(EFIE_OK);
    });
}

int efie_bie2d_assemble(efie_bie2d h, int which, double k_re, double k_im, void* S, void* Dstar, void* Nm,
                        int64_t row0, int64_t nrows, int64_t col0, int64_t ncols, int64_t ld, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(h && (which == 0 || which == 1), EFIE_ERR_ARG, "bie2d_assemble: bad handle or contour");
        EFIE_REQUIRE(h->dev != nullptr, EFIE_ERR_STATE, "bie2d_assemble: tables not uploaded");
        EFIE_REQUIRE(S || Dstar || Nm, EFIE_ERR_ARG, "bie2d_assemble: no output");
        EFIE_REQUIRE(std::isfinite(k_re) && std::isfinite(k_im) && k_re > 0.0 && k_im <= 0.0, EFIE_ERR_ARG,
                     "bie2d_assemble: need Re k > 0, Im k <= 0");
        EFIE_REQUIRE(row0 >= 0 && col0 >= 0 && nrows >= 1 && ncols >= 1 && row0 + nrows <= h->n &&
                         col0 + ncols <= h->n && ld >= ncols,
                     EFIE_ERR_ARG, "bie2d_assemble: bad window");
        launch_assemble(h->dc[which], k_re, k_im, int(row0), int(nrows), int(col0), int(ncols), int(ld),
                        static_cast<double2*>(S), static_cast<double2*>(Dstar), static_cast<double2*>(Nm), h->q,
                        stream);
        return int(EFIE_OK);
    });
}

int efie_bie2d_setup(efie_bie2d h, int pol, double k, double kt_re, double kt_im, int64_t rmax, int64_t block,
                     int64_t nvec, void* ws, size_t ws_bytes, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(h && ws, EFIE_ERR_ARG, "bie2d_setup: null argument");
        EFIE_REQUIRE(h->dev != nullptr, EFIE_ERR_STATE, "bie2d_setup: tables not uploaded");
        EFIE_REQUIRE(std::isfinite(k) && k > 0.0 && std::isfinite(kt_re) && kt_re > 0.0 && kt_im <= 0.0,
                     EFIE_ERR_ARG, "bie2d_setup: need k > 0, Re k~ > 0, Im k~ <= 0");
        EFIE_REQUIRE(block >= 1 && block <= 64 && rmax >= 0 && rmax <= h->n && nvec >= block, EFIE_ERR_ARG,
                     "bie2d_setup: need 1 <= block <= 64, 0 <= rmax <= n, nvec >= block");
        EFIE_REQUIRE(pol == 0 || pol == 1, EFIE_ERR_ARG, "bie2d_setup: pol must be 0 (TM) or 1 (TE)");
        const Layout L = layout(h->n, rmax, block, nvec);
        EFIE_REQUIRE(ws_bytes >= L.total, EFIE_ERR_ARG, "bie2d_setup: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG, "bie2d_setup: ws not 256-aligned");
        char* w = static_cast<char*>(ws);
        auto P = [&](size_t o) { return reinterpret_cast<double2*>(w + o); };
        h->ws = w;
        h->ws_bytes = ws_bytes;
        h->rmax = rmax;
        h->block = block;
        h->nvec = nvec;
        h->k = k;
        h->kt_re = kt_re;
        h->kt_im = kt_im;
        h->pol = pol;
        h->S = P(L.S); h->Dst = P(L.Dst); h->Nt = P(L.Nt); h->Dtt = P(L.Dtt);
        h->cC = P(L.cC); h->cCT = P(L.cCT); h->cI = P(L.cI); h->cIT = P(L.cIT);
        h->T1 = P(L.T1); h->T2 = P(L.T2); h->T3 = P(L.T3);
        h->Qm = P(L.Qm); h->Bm = P(L.Bm); h->Wm = P(L.Wm); h->Mm = P(L.Mm);
        h->Gb = P(L.Gb); h->Tb = P(L.Tb);
        h->nrm = reinterpret_cast<double*>(w + L.nrm);
        h->piv = reinterpret_cast<int*>(w + L.piv);
        h->info = reinterpret_cast<int*>(w + L.info);
        h->split = P(L.split);
        h->split_n = split_elems(rmax);
        h->rank = -1;
        const int n = int(h->n);
        // the four operators of C_p on the scatterer (TM: S and D* at k, N and D* at k~;
        // TE: N and D* at k, S and D* at k~)
        const bool te = pol == 1;
        launch_assemble(h->dc[0], k, 0.0, 0, n, 0, n, n, te ? nullptr : h->S, h->Dst, te ? h->Nt : nullptr, h->q,
                        stream);
        launch_assemble(h->dc[0], kt_re, kt_im, 0, n, 0, n, n, te ? h->S : nullptr, h->Dtt, te ? nullptr : h->Nt, h->q,
                        stream);
        // the counterpart: first columns of its factors on the circle, their spectra
        // (direct DFT), the spectrum of C_c and of its inverse, back to first columns
        double2* e = P(L.eig);
        double2 *cS = e, *cD = e + n, *cN = e + 2 * n, *cDt = e + 3 * n, *cG = e + 4 * n, *l1 = e + 5 * n,
                *l2 = e + 6 * n;
        launch_assemble(h->dc[1], k, 0.0, 0, n, 0, 1, 1, te ? nullptr : cS, cD, te ? cN : nullptr, h->q, stream);
        launch_assemble(h->dc[1], kt_re, kt_im, 0, n, 0, 1, 1, te ? cS : nullptr, cDt, te ? nullptr : cN, h->q, stream);
        hipLaunchKernelGGL(efie::gram_column_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, h->dc[1], cG);
        double2* lam[5] = {e + 7 * n, e + 8 * n, e + 9 * n, e + 10 * n, e + 11 * n};
        const double2* cols[5] = {cS, cD, cN, cDt, cG};
        if (te) {
            // the double layer D = D*^T: first columns of the transposes (scratch l1, l2)
            hipLaunchKernelGGL(efie::circ_transpose_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, cD, l1, n);
            hipLaunchKernelGGL(efie::circ_transpose_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, cDt, l2, n);
            cols[1] = l1;
            cols[3] = l2;
        }
        for (int i = 0; i < 5; ++i)
            hipLaunchKernelGGL(efie::dft_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, cols[i], lam[i], n, -1.0,
                               1.0);
        hipLaunchKernelGGL(efie::circ_combine_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, lam[0], lam[1],
                           lam[2], lam[3], lam[4], l1, l2, n, int(te));
        hipLaunchKernelGGL(efie::dft_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, l1, h->cC, n, 1.0, 1.0 / n);
        hipLaunchKernelGGL(efie::dft_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, l2, h->cI, n, 1.0, 1.0 / n);
        hipLaunchKernelGGL(efie::circ_transpose_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, h->cC, h->cCT, n);
        hipLaunchKernelGGL(efie::circ_transpose_kernel, dim3(efie::grid_of(n)), dim3(256), 0, stream, h->cI, h->cIT, n);
        EFIE_HIP_CHECK(hipGetLastError());
        h->ready = true;
        return int(EFIE_OK);
    });
}

int efie_bie2d_apply(efie_bie2d h, int op, const void* X, void* Y, int64_t nvec, hipStream_t stream) {
    return efie::guarded([&]() {
        require_setup(h, "bie2d_apply");
        EFIE_REQUIRE(X && Y && X != Y, EFIE_ERR_ARG, "bie2d_apply: null or aliased vectors");
        EFIE_REQUIRE(nvec >= 1 && nvec <= h->nvec, EFIE_ERR_ARG, "bie2d_apply: nvec beyond the setup's");
        const int n = int(h->n), nv = int(nvec);
        const auto* x = static_cast<const double2*>(X);
        auto* y = static_cast<double2*>(Y);
        switch (op) {
            case 0: apply_cp(*h, x, y, nv, false, false, stream); break;
            case 1: apply_cp(*h, x, y, nv, true, false, stream); break;
            case 2: gemm2d(efie::G2D_CIRC, x, n, false, h->cC, 0, false, y, n, nv, n, n, ONE, false, stream); break;
            case 3: gemm2d(efie::G2D_CIRC, x, n, false, h->cI, 0, false, y, n, nv, n, n, ONE, false, stream); break;
            case 4: gram_solve(*h, 0, x, y, nv, stream); break;
            case 5: apply_cp(*h, x, y, nv, false, true, stream); break;
            default: throw efie::Error{EFIE_ERR_ARG, "bie2d_apply: bad operator"};
        }
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

int efie_bie2d_rhs(efie_bie2d h, const double* phis, int64_t nrhs, double eta, void* e, void* hv, void* bp,
                   hipStream_t stream) {
    return efie::guarded([&]() {
        require_setup(h, "bie2d_rhs");
        EFIE_REQUIRE(phis && e && hv && nrhs >= 1, EFIE_ERR_ARG, "bie2d_rhs: bad argument");
        EFIE_REQUIRE(!bp || nrhs <= h->nvec, EFIE_ERR_ARG, "bie2d_rhs: nrhs beyond the setup's nvec");
        const int n = int(h->n), nr = int(nrhs);
        // the angles go to the device through the last temporary (nrhs doubles)
        double* dphi = reinterpret_cast<double*>(h->T3);
        EFIE_REQUIRE(size_t(nr) * 8 <= size_t(h->nvec) * size_t(n) * 16, EFIE_ERR_ARG, "bie2d_rhs: too many angles");
        EFIE_HIP_CHECK(hipMemcpyAsync(dphi, phis, size_t(nr) * 8, hipMemcpyHostToDevice, stream));
        auto* ed = static_cast<double2*>(e);
        auto* hd = static_cast<double2*>(hv);
        hipLaunchKernelGGL(efie::excite2d_kernel, dim3(efie::grid_of(size_t(n) * nr)), dim3(256), 0, stream,
                           h->dc[0], h->k, eta, dphi, nr, ed, hd, h->pol);
        if (bp && h->pol == 1) {
            // TE: b_p = S~ G^-1 (j k/eta) e_t - (G/2 + D~) G^-1 h_z, D~ = D*~^T
            auto* b = static_cast<double2*>(bp);
            const double2 f = {0.0, h->k / eta};
            gram_solve(*h, 0, ed, h->T1, nr, stream);
            gemm2d(efie::G2D_NT, h->T1, n, false, h->S, n, false, b, n, nr, n, n, f, false, stream);
            gram_solve(*h, 0, hd, h->T2, nr, stream);
            gemm2d(efie::G2D_NN, h->T2, n, false, h->Dtt, n, false, b, n, nr, n, n, MONE, true, stream);
            gram_apply(*h, 0, h->T2, b, nr, -0.5, 1.0, stream);
        } else if (bp) {
            // b_p = N~ G^-1 e/(j k eta) + (G/2 - D*~) G^-1 h
            auto* b = static_cast<double2*>(bp);
            const double2 f = {0.0, -1.0 / (h->k * eta)};              // 1/(j k eta)
            gram_solve(*h, 0, ed, h->T1, nr, stream);
            gemm2d(efie::G2D_NT, h->T1, n, false, h->Nt, n, false, b, n, nr, n, n, f, false, stream);
            gram_solve(*h, 0, hd, h->T2, nr, stream);
            gemm2d(efie::G2D_NT, h->T2, n, false, h->Dtt, n, false, b, n, nr, n, n, MONE, true, stream);
            gram_apply(*h, 0, h->T2, b, nr, 0.5, 1.0, stream);
        }
        EFIE_HIP_CHECK(hipGetLastError());
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));   // the angles' staging is reused by later calls
        return int(EFIE_OK);
    });
}

int efie_bie2d_skeleton(efie_bie2d h, const void* omega, int64_t ncols, double tol, int64_t* rank, double* est,
                        double* ref, hipStream_t stream) {
    return efie::guarded([&]() {
        require_setup(h, "bie2d_skeleton");
        EFIE_REQUIRE(omega && rank && tol > 0.0, EFIE_ERR_ARG, "bie2d_skeleton: bad argument");
        const int n = int(h->n), b = int(h->block);
        EFIE_REQUIRE(ncols >= b, EFIE_ERR_ARG, "bie2d_skeleton: the test matrix holds less than one block");
        const auto* om = static_cast<const double2*>(omega);   // rows: ncols x n
        std::vector<double> nr(static_cast<size_t>(b), 0.0);
        // reference scale: the largest column norm of C_p Omega_0
        apply_cp(*h, om, h->T3, b, false, false, stream);
        hipLaunchKernelGGL(efie::row_norm_kernel, dim3(b), dim3(256), 0, stream, h->T3, n, h->nrm);
        EFIE_HIP_CHECK(hipMemcpyAsync(nr.data(), h->nrm, size_t(b) * 8, hipMemcpyDeviceToHost, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        const double refv = *std::max_element(nr.begin(), nr.end());
        int r = 0;
        double estv = 0.0;
        bool done = false;
        for (int64_t c0 = 0; c0 < ncols && !done; c0 += b) {
            const int mb = int(std::min<int64_t>(b, ncols - c0));    // the last block may be partial
            // Y = (C_p - C_c) Omega_b, projected twice against Q
            apply_cp(*h, om + size_t(c0) * n, h->T3, mb, false, true, stream);
            for (int pass = 0; pass < 2 && r > 0; ++pass) {
                // P (mb x r) = Y Q^H rows: P[s][t] = sum_k Y[s][k] conj(Q[t][k]); Y -= P Q
                gemm2d(efie::G2D_NT, h->T3, n, false, h->Qm, n, true, h->T1, r, mb, r, n, ONE, false, stream,
                       h->split, h->split_n);
                gemm2d(efie::G2D_NN, h->T1, r, false, h->Qm, n, false, h->T3, n, mb, n, r, MONE, true, stream);
            }
            hipLaunchKernelGGL(efie::row_norm_kernel, dim3(mb), dim3(256), 0, stream, h->T3, n, h->nrm);
            EFIE_HIP_CHECK(hipMemcpyAsync(nr.data(), h->nrm, size_t(mb) * 8, hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipStreamSynchronize(stream));
            estv = *std::max_element(nr.begin(), nr.begin() + mb);
            if (estv <= tol * refv) {
                done = true;
                break;
            }
            const int take = std::min(mb, n - r);
            EFIE_REQUIRE(r + take <= h->rmax, EFIE_ERR_ARG,
                         "bie2d_skeleton: the rank exceeds rmax of the setup (raise rmax or tol)");
            // orthonormal basis of the block: shifted Cholesky QR, then two plain passes
            for (int pass = 0; pass < 3; ++pass) {
                gemm2d(efie::G2D_NT, h->T3, n, true, h->T3, n, false, h->Gb, mb, mb, mb, n, ONE, false, stream,
                       h->split, h->split_n);
                double shift = 0.0;
                if (pass == 0) {
                    double mx = 0.0;
                    for (int i = 0; i < mb; ++i) mx = std::max(mx, nr[size_t(i)]);
                    shift = 11.0 * (double(n) * mb + double(mb) * (mb + 1)) * 1.1102230246251565e-16 * mx * mx * mb;
                }
                hipLaunchKernelGGL(efie::chol_inv_kernel, dim3(1), dim3(256), 0, stream, h->Gb, mb, shift, h->Tb,
                                   h->info);
                int info = 0;
                EFIE_HIP_CHECK(hipMemcpyAsync(&info, h->info, 4, hipMemcpyDeviceToHost, stream));
                // Y <- T Y (T = (R^-1)^T): the new rows
                gemm2d(efie::G2D_NN, h->Tb, mb, false, h->T3, n, false, h->T1, n, mb, n, mb, ONE, false, stream);
                EFIE_HIP_CHECK(hipMemcpyAsync(h->T3, h->T1, size_t(mb) * n * 16, hipMemcpyDeviceToDevice, stream));
                EFIE_HIP_CHECK(hipStreamSynchronize(stream));
                EFIE_REQUIRE(info == 0, EFIE_ERR_BREAKDOWN, "bie2d_skeleton: Cholesky QR broke down");
                if (pass == 0 && r > 0) {
                    // the projection again after the shifted pass (round-off of the first)
                    gemm2d(efie::G2D_NT, h->T3, n, false, h->Qm, n, true, h->T1, r, mb, r, n, ONE, false, stream,
                           h->split, h->split_n);
                    gemm2d(efie::G2D_NN, h->T1, r, false, h->Qm, n, false, h->T3, n, mb, n, r, MONE, true, stream);
                }
            }
            EFIE_HIP_CHECK(hipMemcpyAsync(h->Qm + size_t(r) * n, h->T3, size_t(take) * n * 16,
                                          hipMemcpyDeviceToDevice, stream));
            r += take;
            if (r == n) {
                estv = 0.0;
                done = true;
            }
        }
        EFIE_REQUIRE(done, EFIE_ERR_ARG, "bie2d_skeleton: test matrix exhausted before the tolerance was met");
        // V^T = Q^H (C_p - C_c): row t is (C_p - C_c)^T conj(q_t), a block of rows at a
        // time (the conjugated rows staged in T3, which apply_cp does not use as scratch)
        for (int t0 = 0; t0 < r; t0 += b) {
            const int m = std::min(b, r - t0);
            hipLaunchKernelGGL(efie::conj_kernel, dim3(efie::grid_of(size_t(m) * n)), dim3(256), 0, stream,
                               h->Qm + size_t(t0) * n, h->T3, size_t(m) * n);
            apply_cp(*h, h->T3, h->Bm + size_t(t0) * n, m, true, true, stream);
        }
        if (r > 0) {
            // W = C_c^-1 Q (rows), M = I + V^T W: M[t][u] = sum_k V^T[t][k] W[u][k]; LU
            gemm2d(efie::G2D_CIRC, h->Qm, n, false, h->cI, 0, false, h->Wm, n, r, n, n, ONE, false, stream);
            gemm2d(efie::G2D_NT, h->Bm, n, false, h->Wm, n, false, h->Mm, r, r, r, n, ONE, false, stream);
            hipLaunchKernelGGL(efie::identity_add_kernel, dim3(efie::grid_of(r)), dim3(256), 0, stream, h->Mm, r);
            efie::fill_zero_bytes(h->info, 8, stream);   // the failure flag (a fill kernel, no memset node)
            for (int k0 = 0; k0 < r; k0 += efie::LU_NB) {
                const int kb = std::min(efie::LU_NB, r - k0);
                hipLaunchKernelGGL(efie::lu_panel_kernel, dim3(1), dim3(1024), 0, stream, h->Mm, r, k0, kb, h->piv,
                                   h->info);
                if (r - kb > 0)
                    hipLaunchKernelGGL(efie::lu_swap_kernel, dim3(efie::grid_of(r - kb)), dim3(256), 0, stream, h->Mm, r,
                                       k0, kb, h->piv);
                const int rest = r - k0 - kb;
                if (rest > 0) {
                    hipLaunchKernelGGL(efie::lu_trsm_kernel, dim3(efie::grid_of(rest)), dim3(256), 0, stream, h->Mm, r,
                                       k0, kb);
                    // A22 -= L21 U12
                    gemm2d(efie::G2D_NN, h->Mm + size_t(k0 + kb) * r + k0, r, false, h->Mm + size_t(k0) * r + k0 + kb, r,
                           false, h->Mm + size_t(k0 + kb) * r + k0 + kb, r, rest, rest, kb, MONE, true, stream);
                }
            }
            int info = 0;
            EFIE_HIP_CHECK(hipMemcpyAsync(&info, h->info, 4, hipMemcpyDeviceToHost, stream));
            EFIE_HIP_CHECK(hipStreamSynchronize(stream));
            EFIE_REQUIRE(info == 0, EFIE_ERR_BREAKDOWN, "bie2d_skeleton: I + V^T C_c^-1 U is singular");
        }
        EFIE_HIP_CHECK(hipGetLastError());
        *rank = r;
        if (est) *est = estv;
        if (ref) *ref = refv;
        h->rank = r;
        return int(EFIE_OK);
    });
}

int efie_bie2d_solve(efie_bie2d h, const void* B, void* X, int64_t nrhs, hipStream_t stream) {
    return efie::guarded([&]() {
        require_setup(h, "bie2d_solve");
        EFIE_REQUIRE(h->rank >= 0, EFIE_ERR_STATE, "bie2d_solve: efie_bie2d_skeleton not called");
        EFIE_REQUIRE(B && X && B != X, EFIE_ERR_ARG, "bie2d_solve: null or aliased vectors");
        EFIE_REQUIRE(nrhs >= 1 && nrhs <= h->nvec, EFIE_ERR_ARG, "bie2d_solve: nrhs beyond the setup's nvec");
        const int n = int(h->n), r = int(h->rank), nr = int(nrhs);
        auto* x = static_cast<double2*>(X);
        // x = y - W M^-1 (V^T y), y = C_c^-1 b
        gemm2d(efie::G2D_CIRC, static_cast<const double2*>(B), n, false, h->cI, 0, false, x, n, nr, n, n, ONE, false,
               stream);
        if (r > 0) {
            EFIE_REQUIRE(size_t(nr) * r <= size_t(h->nvec) * n, EFIE_ERR_ARG, "bie2d_solve: too many right-hand sides");
            gemm2d(efie::G2D_NT, x, n, false, h->Bm, n, false, h->T1, r, nr, r, n, ONE, false, stream, h->split,
                   h->split_n);
            hipLaunchKernelGGL(efie::lu_solve_kernel, dim3(nr), dim3(256), 0, stream, h->Mm, h->piv, r, h->T1, nr);
            gemm2d(efie::G2D_NN, h->T1, r, false, h->Wm, n, false, x, n, nr, n, r, MONE, true, stream);
        }
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

int efie_bie2d_factors(efie_bie2d h, void* U, void* Vt, hipStream_t stream) {
    return efie::guarded([&]() {
        require_setup(h, "bie2d_factors");
        EFIE_REQUIRE(h->rank >= 0, EFIE_ERR_STATE, "bie2d_factors: efie_bie2d_skeleton not called");
        const size_t bytes = size_t(h->rank) * size_t(h->n) * 16;
        if (U && bytes) EFIE_HIP_CHECK(hipMemcpyAsync(U, h->Qm, bytes, hipMemcpyDeviceToDevice, stream));
        if (Vt && bytes) EFIE_HIP_CHECK(hipMemcpyAsync(Vt, h->Bm, bytes, hipMemcpyDeviceToDevice, stream));
        return int(EFIE_OK);
    });
}

int efie_bie2d_counterpart(efie_bie2d h, void* col, void* col_inv, hipStream_t stream) {
    return efie::guarded([&]() {
        require_setup(h, "bie2d_counterpart");
        const size_t bytes = size_t(h->n) * 16;
        if (col) EFIE_HIP_CHECK(hipMemcpyAsync(col, h->cC, bytes, hipMemcpyDeviceToDevice, stream));
        if (col_inv) EFIE_HIP_CHECK(hipMemcpyAsync(col_inv, h->cI, bytes, hipMemcpyDeviceToDevice, stream));
        return int(EFIE_OK);
    });
}

int efie_bie2d_farfield(efie_bie2d h, int pol, double k, const void* J, int64_t nrhs, const double* phis,
                        int64_t nphi, void* F, hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(h && J && phis && F && nrhs >= 1 && nphi >= 1, EFIE_ERR_ARG, "bie2d_farfield: bad argument");
        EFIE_REQUIRE(pol == 0 || pol == 1, EFIE_ERR_ARG, "bie2d_farfield: pol must be 0 (TM) or 1 (TE)");
        EFIE_REQUIRE(h->dev != nullptr, EFIE_ERR_STATE, "bie2d_farfield: tables not uploaded");
        EFIE_REQUIRE(std::isfinite(k) && k > 0.0, EFIE_ERR_ARG, "bie2d_farfield: need k > 0");
        hipLaunchKernelGGL(efie::farfield2d_kernel, dim3(efie::grid_of(size_t(nrhs) * nphi)), dim3(256), 0, stream,
                           h->dc[0], k, static_cast<const double2*>(J), int(nrhs), phis, int(nphi),
                           static_cast<double2*>(F), pol);
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

}  // extern "C"

// Adjoint vertex gradient of a far-field objective.
//
// For J = sum_{d,c} |F_dc|^2 with F = R(x) j, Z(x) j = V(x) and the adjoint
// Z lambda = R^T conj(F) (Z = Z^T), the gradient with respect to the vertex
// positions x is
//   dJ/dx = 2 Re[ sum_dc w_dc (dR_dc/dx) j + lambda^T dV/dx - lambda^T (dZ/dx) j ],
// w = conj(F).  This file evaluates the three terms for given j, lambda, w:
//
//  * operator term: lambda^T Z j = sum_{p,q} lambda_p^T B_pq j_q over triangle-pair
//    blocks B_pq, and B_pq(x) = B_qp(x)^T as functions of all vertex positions
//    (the pair integral is symmetric; near blocks are symmetrised).  Hence the
//    derivative with respect to the vertices of triangle t is the sum over q of
//    the derivatives of  lambda_t^T B_tq j_q + j_t^T B_tq lambda_q  taken with
//    respect to t's vertices only (t as test triangle).  One block owns one test
//    triangle t and 256 source triangles: its lanes' derivatives reduce to the 9
//    coordinates of t, added with 9 atomics.
//      far pairs: analytic chain rule through G(R) = exp(-jkR)/R, the quadrature
//      points r_a = sum_k l^a_k P_k and the edge lengths in the RWG coefficients;
//      near pairs: forward-mode dual numbers (value + one directional derivative)
//      through the smooth part and the closed-form singular integrals, one pass
//      per test coordinate.
//  * excitation and radiation terms: per triangle, same chain rule.
// Per-triangle-vertex accumulators (T x 3 x 3) are finally scattered to vertices.
#include <hip/hip_runtime.h>

#include <cmath>

#include "efie_internal.h"
#include "linalg.h"
#include "pair_kernels.h"

namespace efie {

struct Rule {
    double bary[7][3];   // Radon degree-5 rule: barycentric coordinates and weights (sum 1)
    double w[7];
};

struct C {
    double r, i;
};
__device__ __forceinline__ C cm(C a, C b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ C cs(C a, double s) { return {a.r * s, a.i * s}; }
__device__ __forceinline__ C ca(C a, C b) { return {a.r + b.r, a.i + b.i}; }

// ------------------------------------------------------------ dual numbers
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double b, Dual a) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double b, Dual a) { return {b - a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double b, Dual a) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dual operator/(double a, Dual b) {
    const double q = a / b.v;
    return {q, -q * b.d / b.v};
}
__device__ __forceinline__ double val(Dual a) { return a.v; }
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ Dual dsqrt(Dual a) {
    const double s = sqrt(a.v);
    return {s, a.d / (2.0 * s)};
}
__device__ __forceinline__ Dual dlog(Dual a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ Dual datan(Dual a) { return {atan(a.v), a.d / (1.0 + a.v * a.v)}; }
__device__ __forceinline__ Dual dabs(Dual a) { return a.v >= 0.0 ? a : -a; }
__device__ __forceinline__ void dsincos(Dual a, Dual& s, Dual& c) {
    double sv, cv;
    sincos(a.v, &sv, &cv);
    s = {sv, cv * a.d};
    c = {cv, -sv * a.d};
}
__device__ __forceinline__ Dual dexpm1(Dual a) { return {expm1(a.v), exp(a.v) * a.d}; }

struct CD {   // complex dual
    Dual r, i;
};

// 3-vectors of duals
struct D3 {
    Dual x, y, z;
};
__device__ __forceinline__ D3 sub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Dual dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 crs(D3 a, D3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 scl(D3 a, Dual s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ D3 add(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ Dual nrm(D3 a) { return dsqrt(dot(a, a)); }
__device__ __forceinline__ D3 mk(double x, double y, double z) { return {{x, 0}, {y, 0}, {z, 0}}; }

// Closed-form I0, I1 (Wilton et al. 1984) with dual arithmetic: source triangle u[3]
// (counter-clockwise, positions relative to any common origin), observation point r.
__device__ void potentials_d(const D3& r, const D3 u[3], double h, Dual& I0, D3& I1) {
    const D3 e1 = sub(u[1], u[0]), e2 = sub(u[2], u[0]);
    D3 n = crs(e1, e2);
    const Dual nn = nrm(n);
    n = {n.x / nn, n.y / nn, n.z / nn};
    const Dual d = dot(sub(r, u[0]), n);
    const Dual ad = dabs(d);
    const D3 rho = sub(r, scl(n, d));
    I0 = {0, 0};
    I1 = mk(0, 0, 0);
#pragma unroll 1
    for (int e = 0; e < 3; ++e) {
        const D3 rm = u[e], rp = u[(e + 1) % 3];
        D3 lt = sub(rp, rm);
        const Dual len = nrm(lt);
        lt = {lt.x / len, lt.y / len, lt.z / len};
        const D3 uu = crs(lt, n);
        const Dual lp = dot(sub(rp, rho), lt), lm = dot(sub(rm, rho), lt);
        const Dual P0 = dot(sub(rm, rho), uu);
        const Dual R02 = P0 * P0 + d * d;
        const Dual Rp = nrm(sub(r, rp)), Rm = nrm(sub(r, rm));
        Dual lg = {0, 0}, at = {0, 0};
        if (sqrt(R02.v) >= 1e-12 * h) {
            const Dual fp = lp.v >= 0.0 ? Rp + lp : R02 / (Rp - lp);
            const Dual fm = lm.v >= 0.0 ? Rm + lm : R02 / (Rm - lm);
            lg = dlog(fp / fm);
            at = datan(P0 * lp / (R02 + ad * Rp)) - datan(P0 * lm / (R02 + ad * Rm));
        }
        I0 = I0 + P0 * lg - ad * at;
        const Dual c1 = 0.5 * (R02 * lg + lp * Rp - lm * Rm);
        I1 = add(I1, scl(uu, c1));
    }
}

// sum_ij a_i b_j B_near(i,j) for the near pair (test t with vertices Pt, source q with
// vertices Pq), B_near = Scale.A * T_A + Scale.P * T_Phi with T_A, T_Phi the smooth
// (7x7 rule) plus symmetrised singular parts; a_i = alpha_i (complex, excluding the
// edge length), b_j likewise; edge lengths and all geometry from the vertices.
__device__ CD near_contract(const D3 Pt[3], const D3 Pq[3], const double st[3], const double sq[3], C a[3], C b[3],
                            double kr, const Scale& sc, const Rule& rule, double ht, double hq) {
    // RWG coefficients: f_i = s_i l_i / (2 A) (r - P_i), div = s_i l_i / A
    Dual lt_[3], lq_[3];
    for (int i = 0; i < 3; ++i) {
        lt_[i] = nrm(sub(Pt[(i + 1) % 3], Pt[(i + 2) % 3]));
        lq_[i] = nrm(sub(Pq[(i + 1) % 3], Pq[(i + 2) % 3]));
    }
    const Dual At = 0.5 * nrm(crs(sub(Pt[1], Pt[0]), sub(Pt[2], Pt[0])));
    const Dual Aq = 0.5 * nrm(crs(sub(Pq[1], Pq[0]), sub(Pq[2], Pq[0])));
    D3 rt[7], rq[7];
    for (int k = 0; k < 7; ++k) {
        rt[k] = add(add(scl(Pt[0], {rule.bary[k][0], 0}), scl(Pt[1], {rule.bary[k][1], 0})), scl(Pt[2], {rule.bary[k][2], 0}));
        rq[k] = add(add(scl(Pq[0], {rule.bary[k][0], 0}), scl(Pq[1], {rule.bary[k][1], 0})), scl(Pq[2], {rule.bary[k][2], 0}));
    }
    // complex weights: alpha_i = a_i s_i l_i, beta_j = b_j s_j l_j
    CD al[3], be[3];
    for (int i = 0; i < 3; ++i) {
        al[i] = {lt_[i] * (a[i].r * st[i]), lt_[i] * (a[i].i * st[i])};
        be[i] = {lq_[i] * (b[i].r * sq[i]), lq_[i] * (b[i].i * sq[i])};
    }
    CD A0 = {{0, 0}, {0, 0}}, B0 = {{0, 0}, {0, 0}};
    for (int i = 0; i < 3; ++i) {
        A0 = {A0.r + al[i].r, A0.i + al[i].i};
        B0 = {B0.r + be[i].r, B0.i + be[i].i};
    }
    // smooth part:  (1/4) sum_ab w w Gs U_a . U'_b   and   A0 B0 sum_ab w w Gs
    CD TA = {{0, 0}, {0, 0}}, TP = {{0, 0}, {0, 0}};
#pragma unroll 1
    for (int ia = 0; ia < 7; ++ia) {
        // U_a = sum_i alpha_i (r_a - P_i) (complex vector: real and imaginary parts)
        D3 Ur = mk(0, 0, 0), Ui = mk(0, 0, 0);
        for (int i = 0; i < 3; ++i) {
            const D3 dv = sub(rt[ia], Pt[i]);
            Ur = add(Ur, scl(dv, al[i].r));
            Ui = add(Ui, scl(dv, al[i].i));
        }
#pragma unroll 1
        for (int ib = 0; ib < 7; ++ib) {
            D3 Vr = mk(0, 0, 0), Vi = mk(0, 0, 0);
            for (int j = 0; j < 3; ++j) {
                const D3 dv = sub(rq[ib], Pq[j]);
                Vr = add(Vr, scl(dv, be[j].r));
                Vi = add(Vi, scl(dv, be[j].i));
            }
            const D3 dd = sub(rt[ia], rq[ib]);
            const Dual R2 = dot(dd, dd);
            CD g;   // (exp(-jkR) - 1)/R, -jk at R = 0
            if (R2.v == 0.0) {
                g = {{0, 0}, {-kr, 0}};
            } else {
                const Dual R = dsqrt(R2);
                Dual s2, c2;
                dsincos(-0.5 * kr * R, s2, c2);
                g = {(-2.0 * s2 * s2) / R, (2.0 * s2 * c2) / R};
            }
            const double ww = rule.w[ia] * rule.w[ib];
            const Dual uvr = dot(Ur, Vr) - dot(Ui, Vi), uvi = dot(Ur, Vi) + dot(Ui, Vr);
            TA.r = TA.r + ww * 0.25 * (g.r * uvr - g.i * uvi);
            TA.i = TA.i + ww * 0.25 * (g.r * uvi + g.i * uvr);
            TP.r = TP.r + ww * g.r;
            TP.i = TP.i + ww * g.i;
        }
    }
    // TP currently holds sum w w g; times A0 B0
    {
        const Dual abr = A0.r * B0.r - A0.i * B0.i, abi = A0.r * B0.i + A0.i * B0.r;
        const Dual tr = TP.r * abr - TP.i * abi, ti = TP.r * abi + TP.i * abr;
        TP = {tr, ti};
    }
    // singular part: 1/2 [X_tq + X_qt^T], both contracted with (a, b):
    //  X_tq contracted = sum_a w_a A_t/(A_t) ... written with the area-free weights:
    //   sum_ij alpha_i beta_j [ sum_a w_a (1/2)(r_a - P_i) . (1/(2 A_q)) int_q (r' - Q_j)/R ]
    //   and the scalar part sum_ij alpha_i beta_j (1/A_q) sum_a w_a int_q 1/R.
    for (int side = 0; side < 2; ++side) {
        const D3* Po = side == 0 ? Pt : Pq;          // outer (test) triangle of this block
        const D3* Pi = side == 0 ? Pq : Pt;          // inner (analytic) triangle
        const D3* ro = side == 0 ? rt : rq;
        const CD* co = side == 0 ? al : be;          // weights on the outer triangle
        const CD* ci = side == 0 ? be : al;
        const Dual Ai = side == 0 ? Aq : At;
        const double hi = side == 0 ? hq : ht;
        CD s1 = {{0, 0}, {0, 0}}, s0 = {{0, 0}, {0, 0}};
#pragma unroll 1
        for (int ia = 0; ia < 7; ++ia) {
            Dual I0;
            D3 I1;
            potentials_d(ro[ia], Pi, hi, I0, I1);
            const D3 e1 = sub(Pi[1], Pi[0]), e2 = sub(Pi[2], Pi[0]);
            D3 n = crs(e1, e2);
            const Dual nn = nrm(n);
            n = {n.x / nn, n.y / nn, n.z / nn};
            const Dual d = dot(sub(ro[ia], Pi[0]), n);
            const D3 rho = sub(ro[ia], scl(n, d));
            // U_o = sum_i co_i (r_a - Po_i);  inner W = sum_j ci_j (I1 + (rho - Pi_j) I0)
            D3 Ur = mk(0, 0, 0), Ui = mk(0, 0, 0), Wr = mk(0, 0, 0), Wi = mk(0, 0, 0);
            for (int i = 0; i < 3; ++i) {
                const D3 dv = sub(ro[ia], Po[i]);
                Ur = add(Ur, scl(dv, co[i].r));
                Ui = add(Ui, scl(dv, co[i].i));
                const D3 iv = add(I1, scl(sub(rho, Pi[i]), I0));
                Wr = add(Wr, scl(iv, ci[i].r));
                Wi = add(Wi, scl(iv, ci[i].i));
            }
            const double wa = rule.w[ia];
            // (1/2)(1/(2 A_i)) U . W
            const Dual f = wa * 0.25 / Ai;
            s1.r = s1.r + f * (dot(Ur, Wr) - dot(Ui, Wi));
            s1.i = s1.i + f * (dot(Ur, Wi) + dot(Ui, Wr));
            s0.r = s0.r + (wa / Ai) * I0;
        }
        // scalar part: (sum co)(sum ci) s0
        CD So = {{0, 0}, {0, 0}}, Si = {{0, 0}, {0, 0}};
        for (int i = 0; i < 3; ++i) {
            So = {So.r + co[i].r, So.i + co[i].i};
            Si = {Si.r + ci[i].r, Si.i + ci[i].i};
        }
        const Dual pr = So.r * Si.r - So.i * Si.i, pi = So.r * Si.i + So.i * Si.r;
        TA.r = TA.r + 0.5 * s1.r;
        TA.i = TA.i + 0.5 * s1.i;
        TP.r = TP.r + 0.5 * pr * s0.r;
        TP.i = TP.i + 0.5 * pi * s0.r;
    }
    // Z = A T_A + P T_Phi (complex constants; the 1/(4 pi) is in the Scale)
    CD out;
    out.r = sc.ar * TA.r - sc.ai * TA.i + sc.pr * TP.r - sc.pi * TP.i;
    out.i = sc.ar * TA.i + sc.ai * TA.r + sc.pr * TP.i + sc.pi * TP.r;
    return out;
}

// ---------------------------------------------------------- operator term
// acc[t][k][x] += -2 Re d/dP_k^x (lambda_t^T B_tq j_q + j_t^T B_tq lambda_q), far pairs.
__global__ __launch_bounds__(256) void grad_far_kernel(DevMesh m, double kr, Scale sc, Rule rule,
                                                       const double2* __restrict__ lam, const double2* __restrict__ jv,
                                                       double* __restrict__ acc, int nqblk) {
    __shared__ double red[4][9];
    const int T = m.T;
    const int t = blockIdx.x / nqblk;
    const int q = (blockIdx.x - t * nqblk) * 256 + threadIdx.x;
    double out[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = 0.0;
    const bool live = q < T && !is_near(m, t, q);
    if (live) {
        // test triangle (uniform): vertex offsets u, point offsets d, coefficients
        double ut[3][3], e[3][3], lt[3];
        C aL[3], aJ[3];   // alpha with lambda / with j on the test triangle
        for (int i = 0; i < 3; ++i) {
            ut[i][0] = m.vx[i * T + t];
            ut[i][1] = m.vy[i * T + t];
            ut[i][2] = m.vz[i * T + t];
        }
        for (int i = 0; i < 3; ++i) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
            double ev[3] = {ut[i1][0] - ut[i2][0], ut[i1][1] - ut[i2][1], ut[i1][2] - ut[i2][2]};
            lt[i] = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
            for (int x = 0; x < 3; ++x) e[i][x] = ev[x] / lt[i];
            const double s = m.cf[i * T + t] > 0.0 ? 1.0 : -1.0;
            const double2 l = lam[m.te[i * T + t]], jj = jv[m.te[i * T + t]];
            aL[i] = {l.x * s * lt[i], l.y * s * lt[i]};
            aJ[i] = {jj.x * s * lt[i], jj.y * s * lt[i]};
        }
        // source triangle
        double uq[3][3], dq[7][3];
        C bJ[3], bL[3];
        for (int j = 0; j < 3; ++j) {
            uq[j][0] = m.vx[j * T + q];
            uq[j][1] = m.vy[j * T + q];
            uq[j][2] = m.vz[j * T + q];
        }
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const double dx = uq[j1][0] - uq[j2][0], dy = uq[j1][1] - uq[j2][1], dz = uq[j1][2] - uq[j2][2];
            const double l = sqrt(dx * dx + dy * dy + dz * dz);
            const double s = m.cf[j * T + q] > 0.0 ? 1.0 : -1.0;
            const double2 lj = lam[m.te[j * T + q]], jj = jv[m.te[j * T + q]];
            bJ[j] = {jj.x * s * l, jj.y * s * l};
            bL[j] = {lj.x * s * l, lj.y * s * l};
        }
        for (int b = 0; b < 7; ++b) {
            dq[b][0] = m.qx[b * T + q];
            dq[b][1] = m.qy[b * T + q];
            dq[b][2] = m.qz[b * T + q];
        }
        const double D[3] = {m.cx[t] - m.cx[q], m.cy[t] - m.cy[q], m.cz[t] - m.cz[q]};
        const C A0L = ca(ca(aL[0], aL[1]), aL[2]), A0J = ca(ca(aJ[0], aJ[1]), aJ[2]);
        const C B0J = ca(ca(bJ[0], bJ[1]), bJ[2]), B0L = ca(ca(bL[0], bL[1]), bL[2]);
        const C c1 = {0.25 * sc.ar, 0.25 * sc.ai}, c2 = {sc.pr, sc.pi};
        const C AB1 = cm(c2, cm(A0L, B0J)), AB2 = cm(c2, cm(A0J, B0L));
        // accumulators
        C part1[3][3];        // sum_a w_a l^a_k Gvec_a          [k][x]
        C KL1[3][3], KL2[3][3];   // sum_a w_a l^a_k K_a           [k][x]
        C Kw1[3], Kw2[3];     // sum_a w_a K_a
        C Y1[3], Y2[3];       // sum_a w_a (d_a - u_i) . K_a     [i]
        C M0 = {0, 0};
        for (int k = 0; k < 3; ++k) {
            for (int x = 0; x < 3; ++x) part1[k][x] = KL1[k][x] = KL2[k][x] = {0, 0};
            Kw1[k] = Kw2[k] = Y1[k] = Y2[k] = {0, 0};
        }
#pragma unroll 1
        for (int a = 0; a < 7; ++a) {
            const double da[3] = {m.qx[a * T + t], m.qy[a * T + t], m.qz[a * T + t]};
            const double wa = rule.w[a];
            C UL[3], UJ[3];   // U_a with lambda / j weights
            for (int x = 0; x < 3; ++x) {
                UL[x] = {0, 0};
                UJ[x] = {0, 0};
                for (int i = 0; i < 3; ++i) {
                    UL[x] = ca(UL[x], cs(aL[i], da[x] - ut[i][x]));
                    UJ[x] = ca(UJ[x], cs(aJ[i], da[x] - ut[i][x]));
                }
            }
            C Gv[3] = {{0, 0}, {0, 0}, {0, 0}}, K1[3] = {{0, 0}, {0, 0}, {0, 0}}, K2[3] = {{0, 0}, {0, 0}, {0, 0}};
            C S0 = {0, 0};
#pragma unroll 1
            for (int b = 0; b < 7; ++b) {
                const double wb = rule.w[b];
                const double dl[3] = {D[0] + da[0] - dq[b][0], D[1] + da[1] - dq[b][1], D[2] + da[2] - dq[b][2]};
                const double R2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
                const double Ri = rsqrt(R2);
                const double R = R2 * Ri;
                double sn, csn;
                sincos(kr * R, &sn, &csn);
                const C G = {csn * Ri, -sn * Ri};                 // exp(-jkR)/R
                // dG/dR / R = -G (jk + 1/R) / R
                const C Gp = cs(cm(G, C{Ri, kr}), -Ri);
                C VJ[3], VL[3];
                for (int x = 0; x < 3; ++x) {
                    VJ[x] = {0, 0};
                    VL[x] = {0, 0};
                    for (int j = 0; j < 3; ++j) {
                        VJ[x] = ca(VJ[x], cs(bJ[j], dq[b][x] - uq[j][x]));
                        VL[x] = ca(VL[x], cs(bL[j], dq[b][x] - uq[j][x]));
                    }
                }
                C u1 = {0, 0}, u2 = {0, 0};
                for (int x = 0; x < 3; ++x) {
                    u1 = ca(u1, cm(UL[x], VJ[x]));
                    u2 = ca(u2, cm(UJ[x], VL[x]));
                }
                const C Phi = ca(ca(cm(c1, u1), AB1), ca(cm(c1, u2), AB2));
                const C gp = cs(cm(Gp, Phi), wb);
                const C gw = cs(G, wb);
                for (int x = 0; x < 3; ++x) {
                    Gv[x] = ca(Gv[x], cs(gp, dl[x]));
                    K1[x] = ca(K1[x], cm(gw, VJ[x]));
                    K2[x] = ca(K2[x], cm(gw, VL[x]));
                }
                S0 = ca(S0, gw);
            }
            M0 = ca(M0, cs(S0, wa));
            for (int k = 0; k < 3; ++k) {
                const double lk = rule.bary[a][k] * wa;
                for (int x = 0; x < 3; ++x) {
                    part1[k][x] = ca(part1[k][x], cs(Gv[x], lk));
                    KL1[k][x] = ca(KL1[k][x], cs(K1[x], lk));
                    KL2[k][x] = ca(KL2[k][x], cs(K2[x], lk));
                }
            }
            for (int x = 0; x < 3; ++x) {
                Kw1[x] = ca(Kw1[x], cs(K1[x], wa));
                Kw2[x] = ca(Kw2[x], cs(K2[x], wa));
            }
            for (int i = 0; i < 3; ++i)
                for (int x = 0; x < 3; ++x) {
                    Y1[i] = ca(Y1[i], cs(K1[x], wa * (da[x] - ut[i][x])));
                    Y2[i] = ca(Y2[i], cs(K2[x], wa * (da[x] - ut[i][x])));
                }
        }
        // assemble dS/dP_k^x
        for (int k = 0; k < 3; ++k) {
            for (int x = 0; x < 3; ++x) {
                C g = part1[k][x];
                g = ca(g, cm(c1, ca(cm(A0L, KL1[k][x]), cs(cm(aL[k], Kw1[x]), -1.0))));
                g = ca(g, cm(c1, ca(cm(A0J, KL2[k][x]), cs(cm(aJ[k], Kw2[x]), -1.0))));
                // edge-length derivatives: l_i depends on P_{i+1} (+e_i) and P_{i+2} (-e_i)
                for (int i = 0; i < 3; ++i) {
                    double dl = 0.0;
                    if (k == (i + 1) % 3) dl = e[i][x];
                    else if (k == (i + 2) % 3) dl = -e[i][x];
                    if (dl == 0.0) continue;
                    // d alpha_i / dP = (alpha_i / l_i) dl
                    const C dL = cs(aL[i], dl / lt[i]), dJ = cs(aJ[i], dl / lt[i]);
                    g = ca(g, cm(c1, ca(cm(Y1[i], dL), cm(Y2[i], dJ))));
                    g = ca(g, cm(c2, cm(M0, ca(cm(B0J, dL), cm(B0L, dJ)))));
                }
                out[3 * k + x] = -2.0 * g.r;
            }
        }
    }
    // reduce over the block: 9 values for triangle t
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) out[k] += __shfl_xor(out[k], o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 9; ++k) red[w][k] = out[k];
    __syncthreads();
    if (threadIdx.x < 9) {
        const double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        atomicAdd(&acc[size_t(t) * 9 + threadIdx.x], s);
    }
}

// near pairs: one thread per ordered near pair (t, q), 9 dual passes
__global__ __launch_bounds__(128) void grad_near_kernel(DevMesh m, double kr, Scale sc, Rule rule,
                                                        const double2* __restrict__ lam, const double2* __restrict__ jv,
                                                        double* __restrict__ acc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.n_near) return;
    const int T = m.T;
    const int t = m.near_p[e], q = m.near_q[e];
    // positions relative to the centroid of q
    const double D[3] = {m.cx[t] - m.cx[q], m.cy[t] - m.cy[q], m.cz[t] - m.cz[q]};
    double pt[3][3], pq[3][3], st[3], sq[3];
    C aL[3], aJ[3], bJ[3], bL[3];
    for (int i = 0; i < 3; ++i) {
        pt[i][0] = D[0] + m.vx[i * T + t];
        pt[i][1] = D[1] + m.vy[i * T + t];
        pt[i][2] = D[2] + m.vz[i * T + t];
        pq[i][0] = m.vx[i * T + q];
        pq[i][1] = m.vy[i * T + q];
        pq[i][2] = m.vz[i * T + q];
        st[i] = m.cf[i * T + t] > 0.0 ? 1.0 : -1.0;
        sq[i] = m.cf[i * T + q] > 0.0 ? 1.0 : -1.0;
        const double2 lt_ = lam[m.te[i * T + t]], jt = jv[m.te[i * T + t]];
        const double2 lq_ = lam[m.te[i * T + q]], jq = jv[m.te[i * T + q]];
        aL[i] = {lt_.x, lt_.y};
        aJ[i] = {jt.x, jt.y};
        bJ[i] = {jq.x, jq.y};
        bL[i] = {lq_.x, lq_.y};
    }
    D3 Pq[3];
    for (int i = 0; i < 3; ++i) Pq[i] = mk(pq[i][0], pq[i][1], pq[i][2]);
    const double ht = m.hm[t], hq = m.hm[q];
#pragma unroll 1
    for (int c = 0; c < 9; ++c) {
        const int k = c / 3, x = c % 3;
        D3 Pt[3];
        for (int i = 0; i < 3; ++i) {
            Pt[i] = mk(pt[i][0], pt[i][1], pt[i][2]);
            if (i == k) {
                if (x == 0) Pt[i].x.d = 1.0;
                else if (x == 1) Pt[i].y.d = 1.0;
                else Pt[i].z.d = 1.0;
            }
        }
        const CD s1 = near_contract(Pt, Pq, st, sq, aL, bJ, kr, sc, rule, ht, hq);
        const CD s2 = near_contract(Pt, Pq, st, sq, aJ, bL, kr, sc, rule, ht, hq);
        atomicAdd(&acc[size_t(t) * 9 + c], -2.0 * (s1.r.d + s2.r.d));
    }
}

// ------------------------------------------------ excitation and radiation terms
// per triangle t:  S_V = (e0/2) sum_a w_a (U^lambda_a . pol) exp(-j k khat . r_a)
//                  S_R = (1/2) sum_a w_a U^j_a . E(r_a),  E(r) = sum_dc W_dc rho e_dc exp(j k rhat_d . r)
// acc[t][k][x] += 2 Re dS/dP_k^x
__global__ __launch_bounds__(128) void grad_tri_kernel(DevMesh m, double kr, double eta, Rule rule,
                                                       const double2* __restrict__ lam, const double2* __restrict__ jv,
                                                       const double2* __restrict__ W, const double* __restrict__ dirs,
                                                       int ndir, double kx, double ky, double kz, double px, double py,
                                                       double pz, double e0, double* __restrict__ acc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.T) return;
    const int T = m.T;
    double u[3][3], e[3][3], l[3];
    C aL[3], aJ[3];
    for (int i = 0; i < 3; ++i) {
        u[i][0] = m.vx[i * T + t];
        u[i][1] = m.vy[i * T + t];
        u[i][2] = m.vz[i * T + t];
    }
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
        const double ev[3] = {u[i1][0] - u[i2][0], u[i1][1] - u[i2][1], u[i1][2] - u[i2][2]};
        l[i] = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        for (int x = 0; x < 3; ++x) e[i][x] = ev[x] / l[i];
        const double s = m.cf[i * T + t] > 0.0 ? 1.0 : -1.0;
        const double2 a = lam[m.te[i * T + t]], b = jv[m.te[i * T + t]];
        aL[i] = {a.x * s * l[i], a.y * s * l[i]};
        aJ[i] = {b.x * s * l[i], b.y * s * l[i]};
    }
    const double c0[3] = {m.cx[t], m.cy[t], m.cz[t]};
    const C AL = ca(ca(aL[0], aL[1]), aL[2]), AJ = ca(ca(aJ[0], aJ[1]), aJ[2]);
    const double rho = kr * eta / (4.0 * 3.14159265358979323846);   // E carries -j rho
    C g[3][3];
    for (int k = 0; k < 3; ++k)
        for (int x = 0; x < 3; ++x) g[k][x] = {0, 0};
    C YL[3] = {{0, 0}, {0, 0}, {0, 0}}, YJ[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int a = 0; a < 7; ++a) {
        const double da[3] = {m.qx[a * T + t], m.qy[a * T + t], m.qz[a * T + t]};
        const double wa = 0.5 * rule.w[a];
        C UL[3], UJ[3];
        for (int x = 0; x < 3; ++x) {
            UL[x] = UJ[x] = {0, 0};
            for (int i = 0; i < 3; ++i) {
                UL[x] = ca(UL[x], cs(aL[i], da[x] - u[i][x]));
                UJ[x] = ca(UJ[x], cs(aJ[i], da[x] - u[i][x]));
            }
        }
        // excitation field H_V = e0 pol exp(-j k khat . r) and grad_r (U.H_V)
        double sn, csn;
        sincos(-kr * (kx * (c0[0] + da[0]) + ky * (c0[1] + da[1]) + kz * (c0[2] + da[2])), &sn, &csn);
        const C ph = {e0 * csn, e0 * sn};
        C H[3] = {cs(ph, px), cs(ph, py), cs(ph, pz)};
        C UH = ca(ca(cm(UL[0], H[0]), cm(UL[1], H[1])), cm(UL[2], H[2]));
        C gradUH[3];
        const C mjk = {0.0, -kr};
        for (int x = 0; x < 3; ++x) gradUH[x] = cs(cm(UH, mjk), x == 0 ? kx : (x == 1 ? ky : kz));
        // radiation field E(r) = sum_dc W_dc (-j rho) e_dc exp(j k rhat . r): with U = U^j
        C Ef[3] = {{0, 0}, {0, 0}, {0, 0}};
        C gradUE[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int d = 0; d < ndir; ++d) {
            const double rx = dirs[3 * d], ry = dirs[3 * d + 1], rz = dirs[3 * d + 2];
            const double th = acos(fmin(1.0, fmax(-1.0, rz)));
            const double phv = atan2(ry, rx);
            double sth, cth, sph, cph;
            sincos(th, &sth, &cth);
            sincos(phv, &sph, &cph);
            const double et[3] = {cth * cph, cth * sph, -sth}, ep[3] = {-sph, cph, 0.0};
            double s2, c2;
            sincos(kr * (rx * (c0[0] + da[0]) + ry * (c0[1] + da[1]) + rz * (c0[2] + da[2])), &s2, &c2);
            // coefficient W_dc * (-j rho) * exp(j phase)
            const C ex = cm(C{c2, s2}, C{0.0, -rho});
            const double2 w0 = W[2 * d], w1 = W[2 * d + 1];
            const C wt = cm(C{w0.x, w0.y}, ex), wp = cm(C{w1.x, w1.y}, ex);
            C f[3];
            for (int x = 0; x < 3; ++x) f[x] = ca(cs(wt, et[x]), cs(wp, ep[x]));
            const C UE = ca(ca(cm(UJ[0], f[0]), cm(UJ[1], f[1])), cm(UJ[2], f[2]));
            for (int x = 0; x < 3; ++x) Ef[x] = ca(Ef[x], f[x]);
            const C jkU = cm(UE, C{0.0, kr});
            gradUE[0] = ca(gradUE[0], cs(jkU, rx));
            gradUE[1] = ca(gradUE[1], cs(jkU, ry));
            gradUE[2] = ca(gradUE[2], cs(jkU, rz));
        }
        for (int k = 0; k < 3; ++k) {
            const double lk = rule.bary[a][k];
            for (int x = 0; x < 3; ++x) {
                // (A0 l^a_k - alpha_k) H + l^a_k grad(U.H)
                C t1 = cs(cm(ca(cs(AL, lk), cs(aL[k], -1.0)), H[x]), wa);
                C t2 = cs(gradUH[x], wa * lk);
                C t3 = cs(cm(ca(cs(AJ, lk), cs(aJ[k], -1.0)), Ef[x]), wa);
                C t4 = cs(gradUE[x], wa * lk);
                g[k][x] = ca(g[k][x], ca(ca(t1, t2), ca(t3, t4)));
            }
        }
        for (int i = 0; i < 3; ++i)
            for (int x = 0; x < 3; ++x) {
                YL[i] = ca(YL[i], cs(H[x], wa * (da[x] - u[i][x])));
                YJ[i] = ca(YJ[i], cs(Ef[x], wa * (da[x] - u[i][x])));
            }
    }
    for (int k = 0; k < 3; ++k)
        for (int x = 0; x < 3; ++x) {
            C gg = g[k][x];
            for (int i = 0; i < 3; ++i) {
                double dl = 0.0;
                if (k == (i + 1) % 3) dl = e[i][x];
                else if (k == (i + 2) % 3) dl = -e[i][x];
                if (dl == 0.0) continue;
                gg = ca(gg, cm(YL[i], cs(aL[i], dl / l[i])));
                gg = ca(gg, cm(YJ[i], cs(aJ[i], dl / l[i])));
            }
            atomicAdd(&acc[size_t(t) * 9 + 3 * k + x], 2.0 * gg.r);
        }
}

__global__ void grad_scatter_kernel(DevMesh m, const double* __restrict__ acc, double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.T) return;
    for (int k = 0; k < 3; ++k) {
        const int v = m.tv[k * m.T + t];
        for (int x = 0; x < 3; ++x) atomicAdd(&out[3 * size_t(v) + x], acc[size_t(t) * 9 + 3 * k + x]);
    }
}

Rule radon_rule() {
    Rule r{};
    radon7(r.bary, r.w);
    return r;
}

}  // namespace efie

using namespace efie;

extern "C" int efie_vertex_grad_workspace_size(efie_mesh mesh, size_t* bytes) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh && bytes, EFIE_ERR_ARG, "vertex_grad_workspace_size: null");
        *bytes = size_t(mesh->T) * 9 * sizeof(double);
        return int(EFIE_OK);
    });
}

extern "C" int efie_vertex_grad(efie_mesh mesh, double k, double eta, const void* J, const void* lambda,
                                const void* W, const double* dirs, int64_t ndir, const double* khat, const double* pol,
                                double e0, double* dxyz, void* ws, size_t ws_bytes, hipStream_t stream) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh && J && lambda && W && dirs && khat && pol && dxyz && ws, EFIE_ERR_ARG,
                     "vertex_grad: null argument");
        EFIE_REQUIRE(mesh->dev != nullptr, EFIE_ERR_STATE, "vertex_grad: mesh tables not uploaded");
        EFIE_REQUIRE(mesh->far3 == 0.0, EFIE_ERR_ARG, "vertex_grad: differentiates the 7x7 rule only (far rule on)");
        EFIE_REQUIRE(k > 0.0 && std::isfinite(k) && ndir >= 1 && ndir < (int64_t(1) << 20), EFIE_ERR_ARG,
                     "vertex_grad: bad k or ndir");
        EFIE_REQUIRE(ws_bytes >= size_t(mesh->T) * 9 * sizeof(double), EFIE_ERR_ARG, "vertex_grad: ws too small");
        const DevMesh& m = mesh->dm;
        double* acc = static_cast<double*>(ws);
        fill_zero_bytes(acc, size_t(m.T) * 9 * sizeof(double), stream);
        fill_zero_bytes(dxyz, size_t(mesh->nv) * 3 * sizeof(double), stream);
        const Rule rule = radon_rule();
        const double f = eta / (4.0 * 3.14159265358979323846);
        Scale sc{};
        sc.ar = 0.0;
        sc.ai = f * k;
        sc.pr = 0.0;
        sc.pi = -f / k;
        const double2* lam = static_cast<const double2*>(lambda);
        const double2* jv = static_cast<const double2*>(J);
        const int nqblk = (m.T + 255) / 256;
        EFIE_REQUIRE(size_t(m.T) * nqblk < (size_t(1) << 31), EFIE_ERR_ARG, "vertex_grad: mesh too large");
        const double tpairs = double(m.T) * double(m.T) - double(m.n_near);
        prof_begin(PROF_GRAD_FAR, stream);
        hipLaunchKernelGGL(grad_far_kernel, dim3(unsigned(size_t(m.T) * nqblk)), dim3(256), 0, stream, m, k, sc, rule,
                           lam, jv, acc, nqblk);
        prof_end(PROF_GRAD_FAR, stream, tpairs);
        if (m.n_near) {
            prof_begin(PROF_GRAD_NEAR, stream);
            hipLaunchKernelGGL(grad_near_kernel, dim3((m.n_near + 127) / 128), dim3(128), 0, stream, m, k, sc, rule,
                               lam, jv, acc);
            prof_end(PROF_GRAD_NEAR, stream, double(m.n_near));
        }
        prof_begin(PROF_GRAD_TRI, stream);
        hipLaunchKernelGGL(grad_tri_kernel, dim3((m.T + 127) / 128), dim3(128), 0, stream, m, k, eta, rule, lam, jv,
                           static_cast<const double2*>(W), dirs, int(ndir), khat[0], khat[1], khat[2], pol[0], pol[1],
                           pol[2], e0, acc);
        prof_end(PROF_GRAD_TRI, stream, double(m.T));
        hipLaunchKernelGGL(grad_scatter_kernel, dim3((m.T + 127) / 128), dim3(128), 0, stream, m, acc, dxyz);
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

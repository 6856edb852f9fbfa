// Device code shared by the single-mesh and the batched assembly kernels:
// Green's function evaluations, the far-pair moment accumulation, the
// closed-form potentials of the singular part and the near-pair blocks.
// (Formulas and readings are described in assemble.hip.)
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "efie_internal.h"

namespace efie {

constexpr double PI = 3.14159265358979323846;
constexpr int FAR_BLOCK = 256;
constexpr int FAR_PB = 4;   // test triangles per block of the row-building far kernel

struct Scale {          // Z contribution = A * T_A + P * T_Phi (complex), or parts mode
    double ar, ai, pr, pi;
};

template <typename R>
struct Tables {
    const R *qx, *qy, *qz, *qw, *vx, *vy, *vz, *cf, *dv;
    const R *q3x, *q3y, *q3z, *q3w;   // 3-point rule of the adaptive far rule (null: not used)
};

// Whether the far pair (p, q) takes the 3x3 rule: D^2 >= (far3 h)^2 with h the
// larger longest edge of the two triangles, all in FP64 without contraction (the
// same decision as the oracle's)
__device__ __forceinline__ bool far3_pair(const DevMesh& m, int p, int q) {
    const double dx = __dsub_rn(m.cx[q], m.cx[p]);
    const double dy = __dsub_rn(m.cy[q], m.cy[p]);
    const double dz = __dsub_rn(m.cz[q], m.cz[p]);
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const double lim = __dmul_rn(m.far3, fmax(m.hm[p], m.hm[q]));
    return d2 >= __dmul_rn(lim, lim);
}

// Whether the pair (p, q) is near: the triangles share a vertex, or their
// centroids are closer than near_factor times the larger longest edge (decided
// as on the host, so that the device agrees with the ordered near-pair list).
__device__ __forceinline__ bool is_near(const DevMesh& m, int p, int q) {
    const int T = m.T;
    const int a0 = m.tv[p], a1 = m.tv[T + p], a2 = m.tv[2 * T + p];
    const int b0 = m.tv[q], b1 = m.tv[T + q], b2 = m.tv[2 * T + q];
    const bool share = (a0 == b0) | (a0 == b1) | (a0 == b2) | (a1 == b0) | (a1 == b1) | (a1 == b2) | (a2 == b0) |
                       (a2 == b1) | (a2 == b2);
    return share || near_by_distance(m.cx[p], m.cy[p], m.cz[p], m.cx[q], m.cy[q], m.cz[q], m.hm[p], m.hm[q], m.nf);
}

// ------------------------------------------------------------------ helpers
template <typename R>
__device__ __forceinline__ void atomic_add_c(void* Z, size_t idx, R re, R im);

template <>
__device__ __forceinline__ void atomic_add_c<double>(void* Z, size_t idx, double re, double im) {
    double* z = static_cast<double*>(Z) + 2 * idx;
    atomicAdd(z, re);
    atomicAdd(z + 1, im);
}
template <>
__device__ __forceinline__ void atomic_add_c<float>(void* Z, size_t idx, float re, float im) {
    float* z = static_cast<float*>(Z) + 2 * idx;
    atomicAdd(z, re);
    atomicAdd(z + 1, im);
}

// exp(-j k R) / R for k = kr + j ki.  FP64: library sincos/exp.
__device__ __forceinline__ void green_far(double kr, double ki, bool ck, double R2, double& gr, double& gi) {
    double rinv = rsqrt(R2);
    double R = R2 * rinv;
    double s, c;
    sincos(kr * R, &s, &c);
    double e = ck ? exp(ki * R) * rinv : rinv;
    gr = c * e;
    gi = -s * e;
}
// FP32: the phase is passed in revolutions (k / 2 pi) and evaluated with the
// hardware sine/cosine, whose input is in revolutions (valid for |x| < 256).
__device__ __forceinline__ void green_far(float krev, float ki, bool ck, float R2, float& gr, float& gi) {
    float rinv = __builtin_amdgcn_rsqf(R2);
    float R = R2 * rinv;
    float x = krev * R;
    float s = __builtin_amdgcn_sinf(x);
    float c = __builtin_amdgcn_cosf(x);
    float e = ck ? __expf(ki * R) * rinv : rinv;
    gr = c * e;
    gi = -s * e;
}

// -------------------------------------------------------- far-pair kernel
// The pair (p, q) of one mesh (not near): the 7 x 7 Green's function moments and
// the nine half-function products.  emit(i, j, zr, zi) receives the Z
// contribution of test edge i of p and source edge j of q (PARTS: zr, zi are the
// T_A part and emit2 gets the T_Phi part).
// The product rule of NP points per triangle, point offsets and weights from the
// tables (qx, qy, qz, qw), [NP][T].
// PRE: the source triangle's points and weights come from pre[4][NP] (x, y, z, w)
// already in registers instead of the tables
template <int NP, typename R, bool CK, bool PARTS, bool PRE = false, typename Emit, typename Emit2>
__device__ __forceinline__ void far_pair_rule(const DevMesh& m, const Tables<R>& tb, const R* __restrict__ qx,
                                              const R* __restrict__ qy, const R* __restrict__ qz,
                                              const R* __restrict__ qw, int p, int q, R kphase, R ki,
                                              const Scale& sc, Emit emit, Emit2 emit2,
                                              const R (*pre)[NP] = nullptr) {
    const int T = m.T;
    const R Dx = R(m.cx[p] - m.cx[q]);
    const R Dy = R(m.cy[p] - m.cy[q]);
    const R Dz = R(m.cz[p] - m.cz[q]);
    R sx[NP], sy[NP], sz[NP], sw[NP];
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        sx[b] = PRE ? pre[0][b] : qx[b * T + q];
        sy[b] = PRE ? pre[1][b] : qy[b * T + q];
        sz[b] = PRE ? pre[2][b] : qz[b * T + q];
        sw[b] = PRE ? pre[3][b] : qw[b * T + q];
    }
    R m0r = 0, m0i = 0;
    R mdr[3] = {0, 0, 0}, mdi[3] = {0, 0, 0};     // sum W W G d_a
    R mpr[3] = {0, 0, 0}, mpi[3] = {0, 0, 0};     // sum W W G d'_b
    R mmr = 0, mmi = 0;                             // sum W W G d_a . d'_b
#pragma unroll 1
    for (int a = 0; a < NP; ++a) {
        const R ax = qx[a * T + p], ay = qy[a * T + p], az = qz[a * T + p], wa = qw[a * T + p];
        const R ox = Dx + ax, oy = Dy + ay, oz = Dz + az;
        R s0r = 0, s0i = 0, s1r[3] = {0, 0, 0}, s1i[3] = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const R dx = ox - sx[b], dy = oy - sy[b], dz = oz - sz[b];
            const R R2 = dx * dx + dy * dy + dz * dz;
            R gr, gi;
            green_far(kphase, ki, CK, R2, gr, gi);
            gr *= sw[b];
            gi *= sw[b];
            s0r += gr;
            s0i += gi;
            s1r[0] += gr * sx[b]; s1i[0] += gi * sx[b];
            s1r[1] += gr * sy[b]; s1i[1] += gi * sy[b];
            s1r[2] += gr * sz[b]; s1i[2] += gi * sz[b];
        }
        m0r += wa * s0r;
        m0i += wa * s0i;
        const R av[3] = {ax, ay, az};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            mdr[d] += wa * av[d] * s0r;
            mdi[d] += wa * av[d] * s0i;
            mpr[d] += wa * s1r[d];
            mpi[d] += wa * s1i[d];
        }
        mmr += wa * (ax * s1r[0] + ay * s1r[1] + az * s1r[2]);
        mmi += wa * (ax * s1i[0] + ay * s1i[1] + az * s1i[2]);
    }
    // nine half-function products
    R uq[3][3], cq[3], gq[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        uq[j][0] = tb.vx[j * T + q];
        uq[j][1] = tb.vy[j * T + q];
        uq[j][2] = tb.vz[j * T + q];
        cq[j] = tb.cf[j * T + q];
        gq[j] = tb.dv[j * T + q];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const R ux = tb.vx[i * T + p], uy = tb.vy[i * T + p], uz = tb.vz[i * T + p];
        const R ci = tb.cf[i * T + p], gi_ = tb.dv[i * T + p];
        // terms that depend on i only
        const R bir = mmr - (ux * mpr[0] + uy * mpr[1] + uz * mpr[2]);
        const R bii = mmi - (ux * mpi[0] + uy * mpi[1] + uz * mpi[2]);
        const R er[3] = {mdr[0] - ux * m0r, mdr[1] - uy * m0r, mdr[2] - uz * m0r};
        const R ei[3] = {mdi[0] - ux * m0i, mdi[1] - uy * m0i, mdi[2] - uz * m0i};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // Mdd' - u_i.Md' - u'_j.(Md - u_i M0)
            const R tar = ci * cq[j] * (bir - (uq[j][0] * er[0] + uq[j][1] * er[1] + uq[j][2] * er[2]));
            const R tai = ci * cq[j] * (bii - (uq[j][0] * ei[0] + uq[j][1] * ei[1] + uq[j][2] * ei[2]));
            const R gg = gi_ * gq[j];
            const R tpr = gg * m0r, tpi = gg * m0i;
            if (PARTS) {
                emit(i, j, tar * R(sc.ar), tai * R(sc.ar));
                emit2(i, j, tpr * R(sc.ar), tpi * R(sc.ar));
            } else {
                const R zr = R(sc.ar) * tar - R(sc.ai) * tai + R(sc.pr) * tpr - R(sc.pi) * tpi;
                const R zi = R(sc.ar) * tai + R(sc.ai) * tar + R(sc.pr) * tpi + R(sc.pi) * tpr;
                emit(i, j, zr, zi);
            }
        }
    }
}

// The far pair (p, q) by the 7x7 rule, or by the 3x3 rule where the adaptive far
// rule is on (m.far3 > 0) and the pair is far enough.
template <typename R, bool CK, bool PARTS, typename Emit, typename Emit2>
__device__ __forceinline__ void far_pair_emit(const DevMesh& m, const Tables<R>& tb, int p, int q, R kphase, R ki,
                                              const Scale& sc, Emit emit, Emit2 emit2) {
    if (m.far3 > 0.0 && far3_pair(m, p, q))
        far_pair_rule<3, R, CK, PARTS>(m, tb, tb.q3x, tb.q3y, tb.q3z, tb.q3w, p, q, kphase, ki, sc, emit, emit2);
    else
        far_pair_rule<NQ, R, CK, PARTS>(m, tb, tb.qx, tb.qy, tb.qz, tb.qw, p, q, kphase, ki, sc, emit, emit2);
}

// The pair (p, q) added to Z (and Z2 in parts mode) with atomics; near pairs skipped.
template <typename R, bool CK, bool PARTS>
__device__ __forceinline__ void far_pair(const DevMesh& m, const Tables<R>& tb, int p, int q, R kphase, R ki,
                                         const Scale& sc, void* Z, void* Z2) {
    const int T = m.T;
    if (is_near(m, p, q)) return;
    const size_t N = size_t(m.N);
    auto at = [&](void* dst) {
        return [=, &m](int i, int j, R re, R im) {
            atomic_add_c<R>(dst, size_t(m.te[i * T + p]) * N + size_t(m.te[j * T + q]), re, im);
        };
    };
    far_pair_emit<R, CK, PARTS>(m, tb, p, q, kphase, ki, sc, at(Z), at(Z2));
}

// ----------------------------------------------------- closed-form potentials
// I0 = int 1/|r - r'| dS' and I1 = int (rho' - rho)/|r - r'| dS' over the flat
// triangle with vertex positions u[0..2] (counter-clockwise about the unit normal
// n); r, u relative to the same origin.  Edge-sum formulas of Wilton et al. 1984.
static __device__ void potentials(const double r[3], const double u[3][3], const double n[3], double h, double& I0,
                           double I1[3]) {
    const double d = n[0] * (r[0] - u[0][0]) + n[1] * (r[1] - u[0][1]) + n[2] * (r[2] - u[0][2]);
    const double ad = fabs(d);
    const double rho[3] = {r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2]};
    I0 = 0.0;
    I1[0] = I1[1] = I1[2] = 0.0;
#pragma unroll 1
    for (int e = 0; e < 3; ++e) {
        const double* rm = u[e];
        const double* rp = u[(e + 1) % 3];
        double lt[3] = {rp[0] - rm[0], rp[1] - rm[1], rp[2] - rm[2]};
        const double len = sqrt(lt[0] * lt[0] + lt[1] * lt[1] + lt[2] * lt[2]);
        lt[0] /= len; lt[1] /= len; lt[2] /= len;
        const double uu[3] = {lt[1] * n[2] - lt[2] * n[1], lt[2] * n[0] - lt[0] * n[2], lt[0] * n[1] - lt[1] * n[0]};
        const double lp = (rp[0] - rho[0]) * lt[0] + (rp[1] - rho[1]) * lt[1] + (rp[2] - rho[2]) * lt[2];
        const double lm = (rm[0] - rho[0]) * lt[0] + (rm[1] - rho[1]) * lt[1] + (rm[2] - rho[2]) * lt[2];
        const double P0 = (rm[0] - rho[0]) * uu[0] + (rm[1] - rho[1]) * uu[1] + (rm[2] - rho[2]) * uu[2];
        const double R02 = P0 * P0 + d * d;
        const double Rp = sqrt((r[0] - rp[0]) * (r[0] - rp[0]) + (r[1] - rp[1]) * (r[1] - rp[1]) +
                               (r[2] - rp[2]) * (r[2] - rp[2]));
        const double Rm = sqrt((r[0] - rm[0]) * (r[0] - rm[0]) + (r[1] - rm[1]) * (r[1] - rm[1]) +
                               (r[2] - rm[2]) * (r[2] - rm[2]));
        double lg = 0.0, at = 0.0;
        if (sqrt(R02) >= 1e-12 * h) {
            // R + l, written as R0^2 / (R - l) for l < 0 (same value, no cancellation)
            const double fp = lp >= 0.0 ? Rp + lp : R02 / (Rp - lp);
            const double fm = lm >= 0.0 ? Rm + lm : R02 / (Rm - lm);
            lg = log(fp / fm);
            at = atan(P0 * lp / (R02 + ad * Rp)) - atan(P0 * lm / (R02 + ad * Rm));
        }
        I0 += P0 * lg - ad * at;
        const double c1 = 0.5 * (R02 * lg + lp * Rp - lm * Rm);
        I1[0] += c1 * uu[0];
        I1[1] += c1 * uu[1];
        I1[2] += c1 * uu[2];
    }
}

// Test point a of the singular block X(i,j) = sum_a W_a f_i(r_a) . int_s f_j(r')/R dS'
// and of the scalar s0 = sum_a W_a int_s 1/R dS' (test triangle t, source triangle
// s): w times that point's terms added to Y[i][j] (TR: to Y[j][i]) and to s0.
static __device__ void singular_point(const DevMesh& m, int t, int s, int a, double w, bool TR, double Y[3][3],
                                      double& s0) {
    const int T = m.T;
    // everything relative to the source centroid
    const double D[3] = {m.cx[t] - m.cx[s], m.cy[t] - m.cy[s], m.cz[t] - m.cz[s]};
    double us[3][3];
    for (int k = 0; k < 3; ++k) {
        us[k][0] = m.vx[k * T + s]; us[k][1] = m.vy[k * T + s]; us[k][2] = m.vz[k * T + s];
    }
    const double n[3] = {m.nx[s], m.ny[s], m.nz[s]};
    const double da[3] = {m.qx[a * T + t], m.qy[a * T + t], m.qz[a * T + t]};
    const double wa = w * m.qw[a * T + t];
    const double r[3] = {D[0] + da[0], D[1] + da[1], D[2] + da[2]};
    double I0, I1[3];
    potentials(r, us, n, m.hm[s], I0, I1);
    const double dd = n[0] * (r[0] - us[0][0]) + n[1] * (r[1] - us[0][1]) + n[2] * (r[2] - us[0][2]);
    const double rho[3] = {r[0] - dd * n[0], r[1] - dd * n[1], r[2] - dd * n[2]};
    s0 += wa * I0;
    double inner[3][3];
    for (int j = 0; j < 3; ++j) {
        const double cs = m.cf[j * T + s];
        for (int x = 0; x < 3; ++x) inner[j][x] = cs * (I1[x] + (rho[x] - us[j][x]) * I0);
    }
    for (int i = 0; i < 3; ++i) {
        const double ct = m.cf[i * T + t];
        const double f[3] = {ct * (da[0] - m.vx[i * T + t]), ct * (da[1] - m.vy[i * T + t]),
                             ct * (da[2] - m.vz[i * T + t])};
        for (int j = 0; j < 3; ++j) {
            const double v = wa * (f[0] * inner[j][0] + f[1] * inner[j][1] + f[2] * inner[j][2]);
            if (TR) Y[j][i] += v;
            else Y[i][j] += v;
        }
    }
}

// (exp(-jkR) - 1)/R with exp(z) - 1 = expm1(x) cos y - 2 sin^2(y/2) + j exp(x) sin y,
// z = -j k R = x + j y; value -j k at R = 0.
static __device__ __forceinline__ void green_smooth(double kr, double ki, double R2, double& gr, double& gi) {
    if (R2 == 0.0) {
        gr = ki;
        gi = -kr;
        return;
    }
    const double R = sqrt(R2);
    const double x = ki * R, y = -kr * R;
    double s2, c2;
    sincos(0.5 * y, &s2, &c2);
    const double siny = 2.0 * s2 * c2;
    const double cosy = 1.0 - 2.0 * s2 * s2;
    const double nr = expm1(x) * cosy - 2.0 * s2 * s2;
    const double ni = exp(x) * siny;
    gr = nr / R;
    gi = ni / R;
}

// Near pair e of the ordered list, computed by a group of NEAR_G = 8 consecutive
// lanes (g = 0..7 its lane in the group; every lane of the group calls this with
// the same valid e): lane g < 7 takes test point a = g of p, i.e. the smooth part's
// row a of the 7 x 7 rule and the two singular blocks' terms at test point a (of p
// against q, and of q against p), so all lanes of a wave run the same code.  The
// moments are summed over the group with a butterfly of lane exchanges (a fixed
// order: deterministic), then lane g emits entries 3 i + j = g, g + 8:
// emit(i, j, zr, zi) receives the FP64 Z contribution of test edge i and source
// edge j (PARTS: T_A part; emit2: T_Phi).
constexpr int NEAR_G = 8;

template <bool PARTS, typename Emit, typename Emit2>
__device__ void near_pair_group(const DevMesh& m, int e, int g, double kr, double ki, const Scale& sc, Emit emit,
                                Emit2 emit2) {
    const int p = m.near_p[e], q = m.near_q[e];
    const int T = m.T;
    // v: the smooth part's moments as in the far kernel (offsets from the centroids)
    //   [0,1] M0, [2..7] Md (re, im per axis), [8..13] Md', [14,15] Mdd';
    // Y = (X_pq + X_qp^T) / 2 of the singular part, and s0 its scalar
    double v[16];
    for (int x = 0; x < 16; ++x) v[x] = 0.0;
    double Y[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double s0 = 0.0;
    if (g < NQ) {
        const int a = g;
        const double D[3] = {m.cx[p] - m.cx[q], m.cy[p] - m.cy[q], m.cz[p] - m.cz[q]};
        const double ax = m.qx[a * T + p], ay = m.qy[a * T + p], az = m.qz[a * T + p], wa = m.qw[a * T + p];
        double s0r = 0, s0i = 0, s1r[3] = {0, 0, 0}, s1i[3] = {0, 0, 0};
#pragma unroll 1
        for (int b = 0; b < NQ; ++b) {
            const double bx = m.qx[b * T + q], by = m.qy[b * T + q], bz = m.qz[b * T + q], wb = m.qw[b * T + q];
            const double dx = D[0] + ax - bx, dy = D[1] + ay - by, dz = D[2] + az - bz;
            double gr, gi;
            green_smooth(kr, ki, dx * dx + dy * dy + dz * dz, gr, gi);
            gr *= wb;
            gi *= wb;
            s0r += gr; s0i += gi;
            s1r[0] += gr * bx; s1i[0] += gi * bx;
            s1r[1] += gr * by; s1i[1] += gi * by;
            s1r[2] += gr * bz; s1i[2] += gi * bz;
        }
        const double av[3] = {ax, ay, az};
        v[0] = wa * s0r;
        v[1] = wa * s0i;
        for (int d = 0; d < 3; ++d) {
            v[2 + 2 * d] = wa * av[d] * s0r;
            v[3 + 2 * d] = wa * av[d] * s0i;
            v[8 + 2 * d] = wa * s1r[d];
            v[9 + 2 * d] = wa * s1i[d];
        }
        v[14] = wa * (ax * s1r[0] + ay * s1r[1] + az * s1r[2]);
        v[15] = wa * (ax * s1i[0] + ay * s1i[1] + az * s1i[2]);
        // singular part, symmetrised: (X_pq + X_qp^T) / 2
        singular_point(m, p, q, a, 0.5, false, Y, s0);
        singular_point(m, q, p, a, 0.5, true, Y, s0);
    }
#pragma unroll
    for (int o = 1; o < NEAR_G; o <<= 1) {
#pragma unroll
        for (int x = 0; x < 16; ++x) v[x] += __shfl_xor(v[x], o, NEAR_G);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Y[i][j] += __shfl_xor(Y[i][j], o, NEAR_G);
        s0 += __shfl_xor(s0, o, NEAR_G);
    }
    const double m0r = v[0], m0i = v[1];
    for (int idx = g; idx < 9; idx += NEAR_G) {
        const int i = idx / 3, j = idx - 3 * (idx / 3);
        const double ux = m.vx[i * T + p], uy = m.vy[i * T + p], uz = m.vz[i * T + p];
        const double ci = m.cf[i * T + p], gi_ = m.dv[i * T + p];
        const double vx = m.vx[j * T + q], vy = m.vy[j * T + q], vz = m.vz[j * T + q];
        const double cj = m.cf[j * T + q], gj = m.dv[j * T + q];
        const double br = v[14] - (ux * v[8] + uy * v[10] + uz * v[12]) -
                          (vx * (v[2] - ux * m0r) + vy * (v[4] - uy * m0r) + vz * (v[6] - uz * m0r));
        const double bi = v[15] - (ux * v[9] + uy * v[11] + uz * v[13]) -
                          (vx * (v[3] - ux * m0i) + vy * (v[5] - uy * m0i) + vz * (v[7] - uz * m0i));
        const double tar = ci * cj * br + Y[i][j];
        const double tai = ci * cj * bi;
        const double gg = gi_ * gj;
        const double tpr = gg * (m0r + s0), tpi = gg * m0i;
        if (PARTS) {
            emit(i, j, tar * sc.ar, tai * sc.ar);
            emit2(i, j, tpr * sc.ar, tpi * sc.ar);
        } else {
            const double zr = sc.ar * tar - sc.ai * tai + sc.pr * tpr - sc.pi * tpi;
            const double zi = sc.ar * tai + sc.ai * tar + sc.pr * tpi + sc.pi * tpr;
            emit(i, j, zr, zi);
        }
    }
}

// near pair e added to Z (and Z2 in parts mode) with atomics, in ZT precision (by
// the group of 8 lanes, lane g)
template <typename ZT, bool PARTS>
__device__ void near_pair(const DevMesh& m, int e, int g, double kr, double ki, const Scale& sc, void* Z, void* Z2) {
    const int p = m.near_p[e], q = m.near_q[e];
    const int T = m.T;
    const size_t N = size_t(m.N);
    auto at = [&](void* dst) {
        return [=, &m](int i, int j, double re, double im) {
            atomic_add_c<ZT>(dst, size_t(m.te[i * T + p]) * N + size_t(m.te[j * T + q]), ZT(re), ZT(im));
        };
    };
    near_pair_group<PARTS>(m, e, g, kr, ki, sc, at(Z), at(Z2));
}

}  // namespace efie

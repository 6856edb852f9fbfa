// Host side of the Calderon preconditioner: barycentric refinement, the
// Buffa-Christiansen coefficient matrix R (g_n = sum_e R[e][n] f_e over the
// barycentric RWGs f_e) and the sparse mixed Gram matrix
// (G_mix)_mn = int (n x f_m) . g_n dS.
//
// Construction (readings; the paper fixes only the multiplicative structure and
// k~ of its Sec. III):
//  * each triangle (v0,v1,v2) with centroid c and edge midpoints m01, m12, m20
//    becomes (v0,m01,c), (m01,v1,c), (v1,m12,c), (m12,v2,c), (v2,m20,c), (m20,v0,c);
//    barycentric vertex ids: original, then midpoints in RWG order, then centroids;
//  * g_n (primal edge n = (a, b), a < b) flows from the dual cell of a to the dual
//    cell of b through the two halves of the dual edge (flux 1/2 each), puts equal
//    charge +1/N_a (-1/N_b) on each barycentric triangle of cell(a) (cell(b)) and
//    no flux across the two halves of edge n (Buffa-Christiansen 2007; Andriulli
//    et al. 2008 for the multiplicative Calderon use);
//  * G_mix by the 7-point rule on every barycentric triangle (exact: the integrand
//    is quadratic there).
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cmath>
#include <map>

#include "calderon.h"

namespace efie {

namespace {
struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// value of the RWG half-function carried by local edge i of triangle t at r
V3 rwg_value(const efie_mesh_s& m, int64_t t, int i, V3 r) {
    const int32_t e = m.tri_edge[3 * t + i];
    const double c = m.tri_sign[3 * t + i] * m.edge_len[e] / (2.0 * m.area[t]);
    const int32_t v = m.tri[3 * t + i];
    const V3 p{m.xyz[3 * v], m.xyz[3 * v + 1], m.xyz[3 * v + 2]};
    const V3 d = sub(r, p);
    return {c * d.x, c * d.y, c * d.z};
}
}  // namespace

namespace {
uint64_t spread21(uint64_t x) {   // 21 bits -> every third bit
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}
// Morton code of p in the box [lo, hi] (21 bits per axis)
uint64_t morton(const double* p, const double* lo, const double* hi) {
    uint64_t code = 0;
    for (int d = 0; d < 3; ++d) {
        const double u = hi[d] > lo[d] ? (p[d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
        code |= spread21(uint64_t(std::min(2097151.0, std::max(0.0, u * 2097151.0)))) << d;
    }
    return code;
}
}  // namespace

void build_calderon(efie_calderon_s& C, const efie_mesh_s& m) {
    const int64_t V = m.nv, N = m.N, T = m.T;
    // ---------------------------------------------------- barycentric refinement
    // Refinement vertices in canonical order: the primal vertices, the edge
    // midpoints (V + n), the triangle centroids (V + N + t).  The barycentric mesh
    // is built on them renumbered by Morton code (vid[canonical] = internal id), so
    // that its lexicographic edge numbering is spatially coherent: the barycentric
    // RWGs in the support of neighbouring BC functions get neighbouring indices.
    std::vector<double> xyz(3 * size_t(V + N + T));
    for (int64_t i = 0; i < 3 * V; ++i) xyz[i] = m.xyz[i];
    for (int64_t n = 0; n < N; ++n)
        for (int d = 0; d < 3; ++d)
            xyz[3 * (V + n) + d] = 0.5 * (m.xyz[3 * size_t(m.edge_v[2 * n]) + d] + m.xyz[3 * size_t(m.edge_v[2 * n + 1]) + d]);
    for (int64_t t = 0; t < T; ++t)
        for (int d = 0; d < 3; ++d)
            xyz[3 * (V + N + t) + d] = (m.xyz[3 * size_t(m.tri[3 * t]) + d] + m.xyz[3 * size_t(m.tri[3 * t + 1]) + d] +
                                        m.xyz[3 * size_t(m.tri[3 * t + 2]) + d]) / 3.0;
    std::vector<int32_t> tri(18 * size_t(T));
    for (int64_t t = 0; t < T; ++t) {
        const int32_t v0 = m.tri[3 * t], v1 = m.tri[3 * t + 1], v2 = m.tri[3 * t + 2];
        const int32_t m12 = int32_t(V + m.tri_edge[3 * t]), m20 = int32_t(V + m.tri_edge[3 * t + 1]),
                      m01 = int32_t(V + m.tri_edge[3 * t + 2]);
        const int32_t c = int32_t(V + N + t);
        const int32_t sub6[6][3] = {{v0, m01, c}, {m01, v1, c}, {v1, m12, c}, {m12, v2, c}, {v2, m20, c}, {m20, v0, c}};
        for (int k = 0; k < 6; ++k)
            for (int j = 0; j < 3; ++j) tri[18 * t + 3 * k + j] = sub6[k][j];
    }
    const int64_t VB = V + N + T;
    std::vector<int32_t> vid(static_cast<size_t>(VB));
    {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < VB; ++v)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], xyz[3 * size_t(v) + d]);
                hi[d] = std::max(hi[d], xyz[3 * size_t(v) + d]);
            }
        std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(VB));
        for (int64_t v = 0; v < VB; ++v) key[size_t(v)] = {morton(&xyz[3 * size_t(v)], lo, hi), int32_t(v)};
        std::sort(key.begin(), key.end());
        for (int64_t i = 0; i < VB; ++i) vid[size_t(key[size_t(i)].second)] = int32_t(i);
        std::vector<double> x2(xyz.size());
        for (int64_t v = 0; v < VB; ++v)
            for (int d = 0; d < 3; ++d) x2[3 * size_t(vid[size_t(v)]) + d] = xyz[3 * size_t(v) + d];
        xyz.swap(x2);
        for (auto& t : tri) t = vid[size_t(t)];
    }
    build_mesh(C.bary, xyz.data(), VB, tri.data(), 6 * T, m.near_factor);
    pack_tables(C.bary);
    const efie_mesh_s& b = C.bary;
    // canonical index of every barycentric RWG: its rank among the edges of the
    // refinement sorted by canonical (lower, higher) vertex id; where the internal
    // (lower, higher) order of its vertices is the reverse of the canonical one,
    // T+ and T- swap and the canonical RWG is the negative of the internal one
    {
        std::vector<int32_t> inv(static_cast<size_t>(VB));
        for (int64_t v = 0; v < VB; ++v) inv[size_t(vid[size_t(v)])] = int32_t(v);
        std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> ce(static_cast<size_t>(b.N));
        for (int64_t e = 0; e < b.N; ++e) {
            const int32_t a = inv[size_t(b.edge_v[2 * e])], c = inv[size_t(b.edge_v[2 * e + 1])];
            ce[size_t(e)] = {{std::min(a, c), std::max(a, c)}, int32_t(e)};
        }
        std::sort(ce.begin(), ce.end());
        C.bary_canon.resize(static_cast<size_t>(b.N));
        C.bary_flip.resize(static_cast<size_t>(b.N));
        for (int64_t i = 0; i < b.N; ++i) C.bary_canon[size_t(ce[size_t(i)].second)] = int32_t(i);
        for (int64_t e = 0; e < b.N; ++e)
            C.bary_flip[size_t(e)] = inv[size_t(b.edge_v[2 * e])] > inv[size_t(b.edge_v[2 * e + 1])] ? 1 : 0;
    }

    // --------------------------------------------------- Buffa-Christiansen R
    std::map<std::pair<int32_t, int32_t>, int32_t> bedge;
    for (int64_t e = 0; e < b.N; ++e) bedge[{b.edge_v[2 * e], b.edge_v[2 * e + 1]}] = int32_t(e);
    auto edge_of = [&](int32_t p, int32_t q) { return bedge.at({std::min(p, q), std::max(p, q)}); };
    // triangles around each barycentric vertex, rotated to start there: (tri, X, Y)
    struct Corner {
        int32_t t, X, Y;
    };
    std::vector<std::vector<Corner>> around(static_cast<size_t>(b.nv));
    for (int64_t t = 0; t < b.T; ++t) {
        const int32_t p = b.tri[3 * t], q = b.tri[3 * t + 1], r = b.tri[3 * t + 2];
        around[size_t(p)].push_back({int32_t(t), q, r});
        around[size_t(q)].push_back({int32_t(t), r, p});
        around[size_t(r)].push_back({int32_t(t), p, q});
    }
    auto from_plus = [&](int32_t t, int32_t e) { return b.edge_t[2 * e] == t ? 1.0 : -1.0; };
    std::vector<std::map<int32_t, double>> cols(static_cast<size_t>(N));
    for (int64_t n = 0; n < N; ++n) {
        const int32_t mid = vid[size_t(V + n)];
        for (int side = 0; side < 2; ++side) {
            const int32_t c = vid[size_t(m.edge_v[2 * n + side])];
            const double sigma = side == 0 ? 1.0 : -1.0;
            const auto& ring = around[size_t(c)];
            const int Nc = int(ring.size());
            // counter-clockwise order starting with the triangle (c, mid, *)
            std::vector<Corner> order;
            order.reserve(Nc);
            auto find_X = [&](int32_t X) {
                for (const auto& k : ring)
                    if (k.X == X) return k;
                throw Error{EFIE_ERR_MESH_ORIENT, "calderon: broken vertex ring"};
            };
            order.push_back(find_X(mid));
            while (int(order.size()) < Nc) order.push_back(find_X(order.back().Y));
            double x = 0.0;
            for (int i = 0; i < Nc; ++i) {
                const Corner& k = order[size_t(i)];
                const double o = (k.X == mid || k.Y == mid) ? sigma / 2.0 : 0.0;
                x += sigma / Nc - o;   // flux from t_i into t_{i+1}
                if (i < Nc - 1) {
                    const int32_t e = edge_of(c, k.Y);
                    cols[size_t(n)][e] += from_plus(k.t, e) * x / b.edge_len[e];
                }
            }
            if (side == 0) {
                for (const Corner* k : {&order.front(), &order.back()}) {
                    const int32_t e = edge_of(k->X, k->Y);
                    cols[size_t(n)][e] += from_plus(k->t, e) * 0.5 / b.edge_len[e];
                }
            }
        }
    }
    C.r_ptr.assign(size_t(N) + 1, 0);
    C.r_idx.clear();
    C.r_val.clear();
    for (int64_t n = 0; n < N; ++n) {
        for (const auto& kv : cols[size_t(n)]) {
            if (kv.second == 0.0) continue;
            C.r_idx.push_back(kv.first);
            C.r_val.push_back(kv.second);
        }
        C.r_ptr[size_t(n) + 1] = int32_t(C.r_idx.size());
    }
    // the same coefficients by barycentric edge (rows of R)
    C.re_ptr.assign(size_t(b.N) + 1, 0);
    for (int32_t e : C.r_idx) C.re_ptr[size_t(e) + 1]++;
    for (int64_t e = 0; e < b.N; ++e) C.re_ptr[size_t(e) + 1] += C.re_ptr[size_t(e)];
    C.re_idx.assign(C.r_idx.size(), 0);
    C.re_val.assign(C.r_val.size(), 0.0);
    {
        std::vector<int32_t> fill(C.re_ptr.begin(), C.re_ptr.end() - 1);
        for (int64_t n = 0; n < N; ++n)
            for (int32_t k = C.r_ptr[size_t(n)]; k < C.r_ptr[size_t(n) + 1]; ++k) {
                const int32_t e = C.r_idx[size_t(k)];
                C.re_idx[size_t(fill[size_t(e)])] = int32_t(n);
                C.re_val[size_t(fill[size_t(e)])] = C.r_val[size_t(k)];
                fill[size_t(e)]++;
            }
    }

    // ----------------------------------------------------------- mixed Gram
    double qb[7][3], qw[7];
    radon7(qb, qw);
    std::vector<std::map<int32_t, double>> grows(static_cast<size_t>(N));
    for (int64_t bt = 0; bt < b.T; ++bt) {
        const int64_t t = bt / 6;
        const V3 nrm{m.normal[3 * t], m.normal[3 * t + 1], m.normal[3 * t + 2]};
        V3 P[3];
        for (int j = 0; j < 3; ++j) {
            const int32_t v = b.tri[3 * bt + j];
            P[j] = {b.xyz[3 * v], b.xyz[3 * v + 1], b.xyz[3 * v + 2]};
        }
        double I[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // int (n x f_primal_i) . f_bary_j
        for (int a = 0; a < 7; ++a) {
            const V3 r{qb[a][0] * P[0].x + qb[a][1] * P[1].x + qb[a][2] * P[2].x,
                       qb[a][0] * P[0].y + qb[a][1] * P[1].y + qb[a][2] * P[2].y,
                       qb[a][0] * P[0].z + qb[a][1] * P[1].z + qb[a][2] * P[2].z};
            const double w = qw[a] * b.area[bt];
            for (int i = 0; i < 3; ++i) {
                const V3 nf = cross(nrm, rwg_value(m, t, i, r));
                for (int j = 0; j < 3; ++j) I[i][j] += w * dot(nf, rwg_value(b, bt, j, r));
            }
        }
        for (int i = 0; i < 3; ++i) {
            const int32_t row = m.tri_edge[3 * t + i];
            for (int j = 0; j < 3; ++j) {
                const int32_t e = b.tri_edge[3 * bt + j];
                // every BC function that uses barycentric RWG e
                for (int32_t k = C.re_ptr[size_t(e)]; k < C.re_ptr[size_t(e) + 1]; ++k)
                    grows[size_t(row)][C.re_idx[size_t(k)]] += I[i][j] * C.re_val[size_t(k)];
            }
        }
    }
    C.g_ptr.assign(size_t(N) + 1, 0);
    C.g_idx.clear();
    C.g_val.clear();
    for (int64_t r = 0; r < N; ++r) {
        for (const auto& kv : grows[size_t(r)]) {
            C.g_idx.push_back(kv.first);
            C.g_val.push_back(kv.second);
        }
        C.g_ptr[size_t(r) + 1] = int32_t(C.g_idx.size());
    }
    // transpose of G
    C.gt_ptr.assign(size_t(N) + 1, 0);
    for (int32_t c : C.g_idx) C.gt_ptr[size_t(c) + 1]++;
    for (int64_t r = 0; r < N; ++r) C.gt_ptr[size_t(r) + 1] += C.gt_ptr[size_t(r)];
    C.gt_idx.assign(C.g_idx.size(), 0);
    C.gt_val.assign(C.g_val.size(), 0.0);
    std::vector<int32_t> fill(C.gt_ptr.begin(), C.gt_ptr.end() - 1);
    for (int64_t r = 0; r < N; ++r)
        for (int32_t k = C.g_ptr[size_t(r)]; k < C.g_ptr[size_t(r) + 1]; ++k) {
            const int32_t c = C.g_idx[size_t(k)];
            C.gt_idx[size_t(fill[size_t(c)])] = int32_t(r);
            C.gt_val[size_t(fill[size_t(c)])] = C.g_val[size_t(k)];
            fill[size_t(c)]++;
        }
    // a spatially coherent order of the primal RWGs (Morton code of the edge midpoint
    // in the bounding box, 21 bits per axis): the device contractions walk BC
    // functions and Gram rows in this order so that neighbouring threads gather
    // neighbouring data
    {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < V; ++v)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], m.xyz[3 * size_t(v) + d]);
                hi[d] = std::max(hi[d], m.xyz[3 * size_t(v) + d]);
            }
        std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(N));
        for (int64_t n = 0; n < N; ++n) {
            double mid[3];
            for (int d = 0; d < 3; ++d)
                mid[d] = 0.5 * (m.xyz[3 * size_t(m.edge_v[2 * n]) + d] + m.xyz[3 * size_t(m.edge_v[2 * n + 1]) + d]);
            key[size_t(n)] = {morton(mid, lo, hi), int32_t(n)};
        }
        std::sort(key.begin(), key.end());
        C.n_order.resize(static_cast<size_t>(N));
        for (int64_t n = 0; n < N; ++n) C.n_order[size_t(n)] = key[size_t(n)].second;
    }
    // Runs of consecutive BC functions in n_order, each of at most BC_BLOCK functions
    // whose supports hold at most BC_UMAX distinct barycentric RWGs (a run closes
    // when the next function would break either bound): per run its first position
    // in n_order (run_t0), the sorted distinct RWGs it reads (u_ptr / u_idx), and
    // for every entry k of R's CSC the position of its RWG in the list of the run
    // holding its BC function (r_loc).  The source-side contraction gathers each
    // listed RWG once per run.
    {
        C.run_t0.assign(1, 0);
        C.u_ptr.assign(1, 0);
        C.u_idx.clear();
        C.r_loc.assign(C.r_idx.size(), 0);
        C.u_max = 0;
        std::vector<int32_t> mark(static_cast<size_t>(b.N), -1), fs;
        int32_t run = 0;
        auto close_run = [&](int64_t t_end) {
            std::sort(fs.begin(), fs.end());
            for (int64_t t = C.run_t0.back(); t < t_end; ++t) {
                const int32_t n = C.n_order[size_t(t)];
                for (int32_t k = C.r_ptr[size_t(n)]; k < C.r_ptr[size_t(n) + 1]; ++k)
                    C.r_loc[size_t(k)] =
                        int32_t(std::lower_bound(fs.begin(), fs.end(), C.r_idx[size_t(k)]) - fs.begin());
            }
            C.u_idx.insert(C.u_idx.end(), fs.begin(), fs.end());
            C.u_ptr.push_back(int32_t(C.u_idx.size()));
            C.u_max = std::max<int64_t>(C.u_max, int64_t(fs.size()));
            C.run_t0.push_back(int32_t(t_end));
            fs.clear();
            ++run;
        };
        for (int64_t t = 0; t < N; ++t) {
            const int32_t n = C.n_order[size_t(t)];
            int extra = 0;
            for (int32_t k = C.r_ptr[size_t(n)]; k < C.r_ptr[size_t(n) + 1]; ++k)
                extra += mark[size_t(C.r_idx[size_t(k)])] != run;   // entries of one column are distinct
            EFIE_REQUIRE(extra <= BC_UMAX, EFIE_ERR_ARG, "calderon: a BC function with too large a support");
            if (t > C.run_t0.back() && (t - C.run_t0.back() == BC_BLOCK || int64_t(fs.size()) + extra > BC_UMAX))
                close_run(t);
            for (int32_t k = C.r_ptr[size_t(n)]; k < C.r_ptr[size_t(n) + 1]; ++k) {
                const int32_t f = C.r_idx[size_t(k)];
                if (mark[size_t(f)] != run) {
                    mark[size_t(f)] = run;
                    fs.push_back(f);
                }
            }
        }
        if (N > 0) close_run(N);
        // what the device contraction relies on: every local position names its RWG
        for (int32_t r = 0; r < run; ++r) {
            EFIE_REQUIRE(C.u_ptr[size_t(r) + 1] - C.u_ptr[size_t(r)] <= BC_UMAX &&
                             C.run_t0[size_t(r) + 1] - C.run_t0[size_t(r)] <= BC_BLOCK,
                         EFIE_ERR_STATE, "calderon: BC run out of bounds");
            for (int32_t t = C.run_t0[size_t(r)]; t < C.run_t0[size_t(r) + 1]; ++t) {
                const int32_t n = C.n_order[size_t(t)];
                for (int32_t k = C.r_ptr[size_t(n)]; k < C.r_ptr[size_t(n) + 1]; ++k)
                    EFIE_REQUIRE(C.r_loc[size_t(k)] >= 0 &&
                                     C.r_loc[size_t(k)] < C.u_ptr[size_t(r) + 1] - C.u_ptr[size_t(r)] &&
                                     C.u_idx[size_t(C.u_ptr[size_t(r)] + C.r_loc[size_t(k)])] == C.r_idx[size_t(k)],
                                 EFIE_ERR_STATE, "calderon: BC run list inconsistent");
            }
        }
        if (verbose())
            std::fprintf(stderr, "[efie] calderon BC runs: %d, distinct barycentric RWGs per run mean %.0f max %lld, "
                         "total %.2f N_bary\n", run, double(C.u_idx.size()) / double(std::max(run, 1)),
                         (long long)C.u_max, double(C.u_idx.size()) / double(b.N));
    }
    C.N = N;
}

}  // namespace efie

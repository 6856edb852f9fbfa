// Host side of libefie: mesh validation, RWG topology, near-pair lists and the
// packing of the structure-of-arrays device tables.
//
// RWG functions: Rao, Wilton, Glisson, IEEE TAP 30(3), 1982.  For the interior
// edge (a, b), a < b, T+ is the triangle whose counter-clockwise boundary runs
// a -> b and T- the one running b -> a; f = l/(2A+) (r - v+) on T+ and
// l/(2A-) (v- - r) on T-.  Edges are numbered lexicographically by (a, b).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "efie_internal.h"

namespace efie {

namespace {

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

}  // namespace

// Radon's 7-point degree-5 rule on a triangle (Stroud T2:5-1), barycentric.
void radon7(double bary[7][3], double w[7]) {
    const double s = std::sqrt(15.0);
    const double a1 = (9.0 - 2.0 * s) / 21.0, b1 = (6.0 + s) / 21.0;
    const double a2 = (9.0 + 2.0 * s) / 21.0, b2 = (6.0 - s) / 21.0;
    const double w1 = (155.0 + s) / 1200.0, w2 = (155.0 - s) / 1200.0;
    const double B[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
                            {a1, b1, b1}, {b1, a1, b1}, {b1, b1, a1},
                            {a2, b2, b2}, {b2, a2, b2}, {b2, b2, a2}};
    const double W[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
    for (int i = 0; i < 7; ++i) {
        w[i] = W[i];
        for (int j = 0; j < 3; ++j) bary[i][j] = B[i][j];
    }
}


void build_mesh(efie_mesh_s& m, const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                double near_factor) {
    EFIE_REQUIRE(xyz && tri, EFIE_ERR_ARG, "mesh: null pointer");
    EFIE_REQUIRE(nv >= 4 && nt >= 4, EFIE_ERR_ARG, "mesh: need at least 4 vertices and 4 triangles");
    EFIE_REQUIRE(nt < (int64_t(1) << 30), EFIE_ERR_ARG, "mesh: too many triangles");
    EFIE_REQUIRE(near_factor > 0.0 && std::isfinite(near_factor), EFIE_ERR_ARG, "mesh: near_factor must be > 0");
    m.nv = nv;
    m.T = nt;
    m.near_factor = near_factor;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tri.assign(tri, tri + 3 * nt);
    for (int64_t i = 0; i < 3 * nt; ++i)
        EFIE_REQUIRE(tri[i] >= 0 && tri[i] < nv, EFIE_ERR_ARG, "mesh: vertex index out of range");
    for (int64_t i = 0; i < 3 * nv; ++i)
        EFIE_REQUIRE(std::isfinite(xyz[i]), EFIE_ERR_ARG, "mesh: non-finite vertex coordinate");

    auto P = [&](int64_t v) { return V3{xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2]}; };
    {
        double blo[3] = {xyz[0], xyz[1], xyz[2]}, bhi[3] = {xyz[0], xyz[1], xyz[2]};
        for (int64_t v = 0; v < nv; ++v)
            for (int d = 0; d < 3; ++d) {
                blo[d] = std::min(blo[d], xyz[3 * v + d]);
                bhi[d] = std::max(bhi[d], xyz[3 * v + d]);
            }
        m.diam = norm(V3{bhi[0] - blo[0], bhi[1] - blo[1], bhi[2] - blo[2]});
    }
    const int64_t T = nt;
    m.area.resize(T);
    m.normal.resize(3 * T);
    m.centroid.resize(3 * T);
    m.hmax.resize(T);
    for (int64_t t = 0; t < T; ++t) {
        V3 p0 = P(tri[3 * t]), p1 = P(tri[3 * t + 1]), p2 = P(tri[3 * t + 2]);
        V3 c = cross(sub(p1, p0), sub(p2, p0));
        double dbl = norm(c);
        EFIE_REQUIRE(dbl > 0.0, EFIE_ERR_DEGENERATE, "mesh: degenerate triangle " + std::to_string(t));
        m.area[t] = 0.5 * dbl;
        m.normal[3 * t] = c.x / dbl;
        m.normal[3 * t + 1] = c.y / dbl;
        m.normal[3 * t + 2] = c.z / dbl;
        m.centroid[3 * t] = (p0.x + p1.x + p2.x) / 3.0;
        m.centroid[3 * t + 1] = (p0.y + p1.y + p2.y) / 3.0;
        m.centroid[3 * t + 2] = (p0.z + p1.z + p2.z) / 3.0;
        m.hmax[t] = std::max({norm(sub(p1, p2)), norm(sub(p2, p0)), norm(sub(p0, p1))});
    }

    // Undirected edge -> the (triangle, local edge) uses in each direction.
    struct Use {
        int32_t t_ab = -1, i_ab = -1, t_ba = -1, i_ba = -1;
        int count = 0;
        bool dup_dir = false;
    };
    std::map<std::pair<int32_t, int32_t>, Use> edges;
    for (int64_t t = 0; t < T; ++t) {
        for (int i = 0; i < 3; ++i) {
            int32_t a = tri[3 * t + (i + 1) % 3], b = tri[3 * t + (i + 2) % 3];
            EFIE_REQUIRE(a != b, EFIE_ERR_DEGENERATE, "mesh: repeated vertex in a triangle");
            auto key = std::make_pair(std::min(a, b), std::max(a, b));
            Use& u = edges[key];
            u.count++;
            if (a < b) {
                if (u.t_ab >= 0) u.dup_dir = true;
                u.t_ab = int32_t(t);
                u.i_ab = i;
            } else {
                if (u.t_ba >= 0) u.dup_dir = true;
                u.t_ba = int32_t(t);
                u.i_ba = i;
            }
        }
    }
    for (auto& kv : edges) {
        const Use& u = kv.second;
        EFIE_REQUIRE(u.count <= 2, EFIE_ERR_MESH_NONMANIFOLD, "mesh: edge shared by more than two triangles");
        EFIE_REQUIRE(u.count == 2, EFIE_ERR_MESH_OPEN, "mesh: open edge");
        EFIE_REQUIRE(!u.dup_dir, EFIE_ERR_MESH_ORIENT, "mesh: inconsistent orientation");
    }
    const int64_t N = int64_t(edges.size());
    m.N = N;
    m.edge_v.resize(2 * N);
    m.edge_t.resize(2 * N);
    m.edge_l.resize(2 * N);
    m.edge_len.resize(N);
    m.tri_edge.assign(3 * T, -1);
    m.tri_sign.assign(3 * T, 0);
    int64_t n = 0;
    for (auto& kv : edges) {   // std::map iterates in lexicographic (a, b) order
        const Use& u = kv.second;
        m.edge_v[2 * n] = kv.first.first;
        m.edge_v[2 * n + 1] = kv.first.second;
        m.edge_t[2 * n] = u.t_ab;
        m.edge_t[2 * n + 1] = u.t_ba;
        m.edge_l[2 * n] = u.i_ab;
        m.edge_l[2 * n + 1] = u.i_ba;
        m.edge_len[n] = norm(sub(P(kv.first.second), P(kv.first.first)));
        m.tri_edge[3 * u.t_ab + u.i_ab] = int32_t(n);
        m.tri_sign[3 * u.t_ab + u.i_ab] = +1;
        m.tri_edge[3 * u.t_ba + u.i_ba] = int32_t(n);
        m.tri_sign[3 * u.t_ba + u.i_ba] = -1;
        ++n;
    }

    // Near pairs: sharing a vertex, or |c_p - c_q| < near_factor * max(h_p, h_q).
    double hglob = *std::max_element(m.hmax.begin(), m.hmax.end());
    double cell = near_factor * hglob;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t t = 0; t < T; ++t)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], m.centroid[3 * t + d]);
            hi[d] = std::max(hi[d], m.centroid[3 * t + d]);
        }
    int64_t dim[3];
    for (int d = 0; d < 3; ++d) dim[d] = std::max<int64_t>(1, int64_t((hi[d] - lo[d]) / cell) + 1);
    // bound the grid size for pathological inputs
    while (dim[0] * dim[1] * dim[2] > 8 * T + 64) {
        cell *= 1.5;
        for (int d = 0; d < 3; ++d) dim[d] = std::max<int64_t>(1, int64_t((hi[d] - lo[d]) / cell) + 1);
    }
    auto cell_of = [&](int64_t t, int d) {
        int64_t c = int64_t((m.centroid[3 * t + d] - lo[d]) / cell);
        return std::min<int64_t>(std::max<int64_t>(c, 0), dim[d] - 1);
    };
    std::vector<std::vector<int32_t>> grid(size_t(dim[0] * dim[1] * dim[2]));
    for (int64_t t = 0; t < T; ++t)
        grid[size_t((cell_of(t, 0) * dim[1] + cell_of(t, 1)) * dim[2] + cell_of(t, 2))].push_back(int32_t(t));
    std::vector<std::vector<int32_t>> vtri(static_cast<size_t>(nv));
    for (int64_t t = 0; t < T; ++t)
        for (int i = 0; i < 3; ++i) vtri[size_t(tri[3 * t + i])].push_back(int32_t(t));

    m.near_p.clear();
    m.near_q.clear();
    std::vector<int32_t> cand;
    for (int64_t p = 0; p < T; ++p) {
        cand.clear();
        int64_t c0 = cell_of(p, 0), c1 = cell_of(p, 1), c2 = cell_of(p, 2);
        const double* cp = &m.centroid[3 * p];
        for (int64_t i = std::max<int64_t>(c0 - 1, 0); i <= std::min(c0 + 1, dim[0] - 1); ++i)
            for (int64_t j = std::max<int64_t>(c1 - 1, 0); j <= std::min(c1 + 1, dim[1] - 1); ++j)
                for (int64_t k = std::max<int64_t>(c2 - 1, 0); k <= std::min(c2 + 1, dim[2] - 1); ++k)
                    for (int32_t q : grid[size_t((i * dim[1] + j) * dim[2] + k)]) {
                        const double* cq = &m.centroid[3 * size_t(q)];
                        if (near_by_distance(cp[0], cp[1], cp[2], cq[0], cq[1], cq[2], m.hmax[p], m.hmax[q],
                                             near_factor))
                            cand.push_back(q);
                    }
        for (int i = 0; i < 3; ++i)
            for (int32_t q : vtri[size_t(tri[3 * p + i])]) cand.push_back(q);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int32_t q : cand) {
            m.near_p.push_back(int32_t(p));
            m.near_q.push_back(q);
        }
    }
    // the pairs with q >= p (the kernels that use the symmetry compute only these)
    m.near_up.clear();
    for (size_t e = 0; e < m.near_p.size(); ++e)
        if (m.near_q[e] >= m.near_p[e]) m.near_up.push_back(int32_t(e));
}

namespace {
struct Packer {
    std::vector<char> blob;
    std::vector<size_t> offs;
    template <class T>
    size_t add(const std::vector<T>& v) {
        size_t off = (blob.size() + 255) & ~size_t(255);
        blob.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
        offs.push_back(off);
        return off;
    }
};
}  // namespace

void pack_tables(efie_mesh_s& m) {
    const int64_t T = m.T, N = m.N;
    double bary[7][3], w[7];
    radon7(bary, w);
    std::vector<double> cx(T), cy(T), cz(T), qx(7 * T), qy(7 * T), qz(7 * T), qw(7 * T);
    std::vector<double> vx(3 * T), vy(3 * T), vz(3 * T), cf(3 * T), dv(3 * T), nx(T), ny(T), nz(T), hm(T);
    std::vector<int32_t> te(3 * T), tv(3 * T), et(2 * N), el(2 * N);
    // interior 3-point rule of degree 2 (the distance-adaptive far rule):
    // barycentric (2/3, 1/6, 1/6) and permutations, weights 1/3
    const double b3[3][3] = {{2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0},
                             {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
    std::vector<double> q3x(3 * T), q3y(3 * T), q3z(3 * T), q3w(3 * T);
    for (int64_t t = 0; t < T; ++t) {
        // vertex offsets from the centroid; points r = sum_k lambda_k p_k become
        // sum_k lambda_k (p_k - c) since the barycentric weights sum to one
        double X[3][3];
        for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 3; ++d) X[i][d] = m.xyz[3 * size_t(m.tri[3 * t + i]) + d] - m.centroid[3 * t + d];
        cx[t] = m.centroid[3 * t];
        cy[t] = m.centroid[3 * t + 1];
        cz[t] = m.centroid[3 * t + 2];
        hm[t] = m.hmax[t];
        for (int a = 0; a < 7; ++a) {
            qx[a * T + t] = bary[a][0] * X[0][0] + bary[a][1] * X[1][0] + bary[a][2] * X[2][0];
            qy[a * T + t] = bary[a][0] * X[0][1] + bary[a][1] * X[1][1] + bary[a][2] * X[2][1];
            qz[a * T + t] = bary[a][0] * X[0][2] + bary[a][1] * X[1][2] + bary[a][2] * X[2][2];
            qw[a * T + t] = w[a] * m.area[t];
        }
        for (int a = 0; a < 3; ++a) {
            q3x[a * T + t] = b3[a][0] * X[0][0] + b3[a][1] * X[1][0] + b3[a][2] * X[2][0];
            q3y[a * T + t] = b3[a][0] * X[0][1] + b3[a][1] * X[1][1] + b3[a][2] * X[2][1];
            q3z[a * T + t] = b3[a][0] * X[0][2] + b3[a][1] * X[1][2] + b3[a][2] * X[2][2];
            q3w[a * T + t] = m.area[t] / 3.0;
        }
        for (int i = 0; i < 3; ++i) {
            vx[i * T + t] = X[i][0];
            vy[i * T + t] = X[i][1];
            vz[i * T + t] = X[i][2];
            int32_t e = m.tri_edge[3 * t + i];
            double s = m.tri_sign[3 * t + i];
            cf[i * T + t] = s * m.edge_len[e] / (2.0 * m.area[t]);
            dv[i * T + t] = s * m.edge_len[e] / m.area[t];
            te[i * T + t] = e;
            tv[i * T + t] = m.tri[3 * t + i];
        }
        nx[t] = m.normal[3 * t];
        ny[t] = m.normal[3 * t + 1];
        nz[t] = m.normal[3 * t + 2];
    }
    for (int64_t n = 0; n < N; ++n) {
        et[n] = m.edge_t[2 * n];
        et[N + n] = m.edge_t[2 * n + 1];
        el[n] = m.edge_l[2 * n];
        el[N + n] = m.edge_l[2 * n + 1];
    }
    auto f32 = [](const std::vector<double>& v) {
        std::vector<float> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = float(v[i]);
        return o;
    };
    Packer pk;
    pk.add(cx); pk.add(cy); pk.add(cz);
    pk.add(qx); pk.add(qy); pk.add(qz); pk.add(qw);
    pk.add(vx); pk.add(vy); pk.add(vz); pk.add(cf); pk.add(dv);
    pk.add(nx); pk.add(ny); pk.add(nz); pk.add(hm);
    pk.add(f32(qx)); pk.add(f32(qy)); pk.add(f32(qz)); pk.add(f32(qw));
    pk.add(f32(vx)); pk.add(f32(vy)); pk.add(f32(vz)); pk.add(f32(cf)); pk.add(f32(dv));
    pk.add(te);
    pk.add(tv);
    pk.add(m.near_p); pk.add(m.near_q);
    pk.add(et); pk.add(el);
    pk.add(q3x); pk.add(q3y); pk.add(q3z); pk.add(q3w);
    pk.add(f32(q3x)); pk.add(f32(q3y)); pk.add(f32(q3z)); pk.add(f32(q3w));
    pk.add(m.near_up);
    pk.blob.resize((pk.blob.size() + 255) & ~size_t(255));
    m.host_blob.swap(pk.blob);
    m.offs.swap(pk.offs);
}

// The tables pack_tables writes, in its order: the count each scales with
// ('T' triangles, 'N' RWGs, 'E' ordered near pairs, 'U' those with q >= p), how
// many elements per unit, and the element size.
namespace {
struct TableSpec {
    char kind;
    int per, esz;
};
const TableSpec kTables[] = {
    {'T', 1, 8}, {'T', 1, 8}, {'T', 1, 8},                                            // cx cy cz
    {'T', 7, 8}, {'T', 7, 8}, {'T', 7, 8}, {'T', 7, 8},                               // qx qy qz qw
    {'T', 3, 8}, {'T', 3, 8}, {'T', 3, 8}, {'T', 3, 8}, {'T', 3, 8},                  // vx vy vz cf dv
    {'T', 1, 8}, {'T', 1, 8}, {'T', 1, 8}, {'T', 1, 8},                               // nx ny nz hm
    {'T', 7, 4}, {'T', 7, 4}, {'T', 7, 4}, {'T', 7, 4},                               // FP32 q
    {'T', 3, 4}, {'T', 3, 4}, {'T', 3, 4}, {'T', 3, 4}, {'T', 3, 4},                  // FP32 v cf dv
    {'T', 3, 4}, {'T', 3, 4},                                                         // te tv
    {'E', 1, 4}, {'E', 1, 4},                                                         // near_p near_q
    {'N', 2, 4}, {'N', 2, 4},                                                         // et el
    {'T', 3, 8}, {'T', 3, 8}, {'T', 3, 8}, {'T', 3, 8},                               // q3 (FP64)
    {'T', 3, 4}, {'T', 3, 4}, {'T', 3, 4}, {'T', 3, 4},                               // q3 (FP32)
    {'U', 1, 4},                                                                      // near_up
};
}  // namespace

int table_count() { return int(sizeof(kTables) / sizeof(kTables[0])); }

size_t table_bytes_of(const efie_mesh_s& m, int t) {
    const TableSpec& s = kTables[t];
    const size_t units = s.kind == 'T'   ? size_t(m.T)
                         : s.kind == 'N' ? size_t(m.N)
                         : s.kind == 'E' ? m.near_p.size()
                                         : m.near_up.size();
    return units * size_t(s.per) * size_t(s.esz);
}

void bind_pointers(DevMesh& d, const void* base, const std::vector<size_t>& o) {
    const char* b = static_cast<const char*>(base);
    int i = 0;
    auto D = [&]() { return reinterpret_cast<const double*>(b + o[size_t(i++)]); };
    auto F = [&]() { return reinterpret_cast<const float*>(b + o[size_t(i++)]); };
    auto I = [&]() { return reinterpret_cast<const int32_t*>(b + o[size_t(i++)]); };
    d.cx = D(); d.cy = D(); d.cz = D();
    d.qx = D(); d.qy = D(); d.qz = D(); d.qw = D();
    d.vx = D(); d.vy = D(); d.vz = D(); d.cf = D(); d.dv = D();
    d.nx = D(); d.ny = D(); d.nz = D(); d.hm = D();
    d.qx32 = F(); d.qy32 = F(); d.qz32 = F(); d.qw32 = F();
    d.vx32 = F(); d.vy32 = F(); d.vz32 = F(); d.cf32 = F(); d.dv32 = F();
    d.te = I();
    d.tv = I();
    d.near_p = I(); d.near_q = I();
    d.et = I(); d.el = I();
    d.q3x = D(); d.q3y = D(); d.q3z = D(); d.q3w = D();
    d.q3x32 = F(); d.q3y32 = F(); d.q3z32 = F(); d.q3w32 = F();
    d.near_up = I();
}

void bind_tables(efie_mesh_s& m, void* dev) {
    DevMesh& d = m.dm;
    d.T = int32_t(m.T);
    d.N = int32_t(m.N);
    d.nf = m.near_factor;
    d.diam = m.diam;
    d.n_near = int32_t(m.near_p.size());
    d.n_up = int32_t(m.near_up.size());
    bind_pointers(d, dev, m.offs);
    d.far3 = m.far3;
    m.dev = dev;
}

}  // namespace efie

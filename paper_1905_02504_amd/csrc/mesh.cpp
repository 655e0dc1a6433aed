// Geodesic shell mesh (Section II.a, transposed to the cube): each of the six
// cube faces is a spherical quadrilateral whose vertex grid is refined level
// by level -- great-circle midpoints on edges, great-circle intersection of
// the two mid-lines at centres -- until N x N columns per face.  Columns are
// extruded radially into geometric shells (self-similar zones, Section V.b),
// which makes every radial column of zones a scaled copy of its first zone.
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "rg_internal.hpp"

namespace rg {

namespace {

struct V3 {
    double x, y, z;
};
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 crs(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dt3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 unit(V3 a)
{
    double n = std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
    return {a.x / n, a.y / n, a.z / n};
}

// point where the great circle through p1,p2 meets the one through q1,q2 (side of hint)
V3 gc_cross(V3 p1, V3 p2, V3 q1, V3 q2, V3 hint)
{
    V3 d = unit(crs(crs(p1, p2), crs(q1, q2)));
    if (dt3(d, hint) < 0) d = {-d.x, -d.y, -d.z};
    return d;
}

// cube faces: outward normal, tangents u, v (u x v = normal)
const double FACE[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},  {{-1, 0, 0}, {0, 0, 1}, {0, 1, 0}},
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 0}},  {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {1, 0, 0}, {0, 1, 0}},  {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

struct BitsHash {
    size_t operator()(const std::array<uint64_t, 3> &k) const
    {
        uint64_t h = k[0] * 0x9E3779B97F4A7C15ull;
        h ^= k[1] + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
        h ^= k[2] + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

}  // namespace

// point a fraction k/3 (k = 1, 2) of the great-circle arc from a to b, by
// spherical interpolation; third_point(b, a, 3 - k) gives the same bits, so
// patches that share a cube edge share its vertices exactly
V3 third_point(V3 a, V3 b, int k)
{
    const V3 c = crs(a, b);
    const double th = std::atan2(std::sqrt(dt3(c, c)), dt3(a, b)), st = std::sin(th);
    const double wa = std::sin((3 - k) * th / 3.0) / st, wb = std::sin(k * th / 3.0) / st;
    return unit({wa * a.x + wb * b.x, wa * a.y + wb * b.y, wa * a.z + wb * b.z});
}

bool build_mesh(const rg_mesh_desc &d, Mesh &m)
{
    int N = d.n_ang;
    // N = 2^levels (first grid: the patch corners) or 3 * 2^levels (first
    // grid: the patch split 3 x 3 by great circles through the thirds of its
    // edges), then levels bisections
    int base = N % 3 == 0 ? 3 : 1, levels = 0;
    while ((base << levels) < N) levels++;
    if (N < 2 || (base << levels) != N) {
        set_error("n_ang must be 2^k (k >= 1) or 3 * 2^k (k >= 0)");
        return false;
    }
    m.N = N;
    m.Nr = d.n_rad;
    m.g = d.n_ghost > 0 ? d.n_ghost : 3;
    m.K = m.Nr + 2 * m.g;
    m.map_order = d.map_order;
    m.r_in = d.r_in;
    m.r_out = d.r_out;
    m.q = std::pow(d.r_out / d.r_in, 1.0 / d.n_rad);
    m.radius.resize(m.K + 1);
    for (int kf = 0; kf <= m.K; kf++)
        m.radius[kf] = d.r_in * std::pow(d.r_out / d.r_in, double(kf - m.g) / d.n_rad);

    // vertex grid of every patch, refined level by level
    const int n1 = N + 1;
    std::vector<V3> grid(6 * n1 * n1);
    const double s = 1.0 / std::sqrt(3.0);
    for (int p = 0; p < 6; p++) {
        std::vector<V3> cur(4), nxt;
        int n = 1;
        for (int j = 0; j < 2; j++)
            for (int i = 0; i < 2; i++) {
                V3 c;
                c.x = s * (FACE[p][0][0] + (2 * i - 1) * FACE[p][1][0] + (2 * j - 1) * FACE[p][2][0]);
                c.y = s * (FACE[p][0][1] + (2 * i - 1) * FACE[p][1][1] + (2 * j - 1) * FACE[p][2][1]);
                c.z = s * (FACE[p][0][2] + (2 * i - 1) * FACE[p][1][2] + (2 * j - 1) * FACE[p][2][2]);
                cur[j * 2 + i] = c;
            }
        if (base == 3) {
            // edges split at their thirds, interior points where the great
            // circles joining opposite edges' thirds meet
            std::vector<V3> g3(16);
            auto G = [&](int i, int j) -> V3 & { return g3[j * 4 + i]; };
            G(0, 0) = cur[0];
            G(3, 0) = cur[1];
            G(0, 3) = cur[2];
            G(3, 3) = cur[3];
            for (int k = 1; k <= 2; k++) {
                G(k, 0) = third_point(G(0, 0), G(3, 0), k);
                G(k, 3) = third_point(G(0, 3), G(3, 3), k);
                G(0, k) = third_point(G(0, 0), G(0, 3), k);
                G(3, k) = third_point(G(3, 0), G(3, 3), k);
            }
            for (int j = 1; j <= 2; j++)
                for (int i = 1; i <= 2; i++) {
                    V3 hint = add(add(G(0, 0), G(3, 0)), add(G(0, 3), G(3, 3)));
                    G(i, j) = gc_cross(G(i, 0), G(i, 3), G(0, j), G(3, j), hint);
                }
            cur.swap(g3);
            n = 3;
        }
        for (int lev = 0; lev < levels; lev++) {
            int n2 = 2 * n;
            nxt.assign((n2 + 1) * (n2 + 1), V3{0, 0, 0});
            auto C = [&](int i, int j) -> V3 & { return cur[j * (n + 1) + i]; };
            auto X = [&](int i, int j) -> V3 & { return nxt[j * (n2 + 1) + i]; };
            for (int j = 0; j <= n; j++)
                for (int i = 0; i <= n; i++) X(2 * i, 2 * j) = C(i, j);
            for (int j = 0; j <= n; j++)
                for (int i = 0; i < n; i++) X(2 * i + 1, 2 * j) = unit(add(C(i, j), C(i + 1, j)));
            for (int j = 0; j < n; j++)
                for (int i = 0; i <= n; i++) X(2 * i, 2 * j + 1) = unit(add(C(i, j), C(i, j + 1)));
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    V3 hint = add(add(C(i, j), C(i + 1, j)), add(C(i + 1, j + 1), C(i, j + 1)));
                    X(2 * i + 1, 2 * j + 1) =
                        gc_cross(X(2 * i + 1, 2 * j), X(2 * i + 1, 2 * j + 2), X(2 * i, 2 * j + 1), X(2 * i + 2, 2 * j + 1), hint);
                }
            cur.swap(nxt);
            n = n2;
        }
        for (int k = 0; k < n1 * n1; k++) grid[p * n1 * n1 + k] = cur[k];
    }

    // global vertex ids: identical bit patterns on shared patch edges
    std::unordered_map<std::array<uint64_t, 3>, int, BitsHash> vid;
    std::vector<int> gid(6 * n1 * n1);
    m.vpos.clear();
    for (size_t k = 0; k < grid.size(); k++) {
        std::array<uint64_t, 3> key;
        std::memcpy(key.data(), &grid[k], 24);
        auto it = vid.find(key);
        if (it == vid.end()) {
            int id = (int)(m.vpos.size() / 3);
            vid.emplace(key, id);
            m.vpos.push_back(grid[k].x);
            m.vpos.push_back(grid[k].y);
            m.vpos.push_back(grid[k].z);
            gid[k] = id;
        } else {
            gid[k] = it->second;
        }
    }
    m.nv = (int)(m.vpos.size() / 3);
    if (m.nv != 6 * N * N + 2) {
        set_error("vertex de-duplication failed");
        return false;
    }
    m.ncol = 6 * N * N;
    m.col_v.resize(4 * m.ncol);
    for (int p = 0; p < 6; p++)
        for (int j = 0; j < N; j++)
            for (int i = 0; i < N; i++) {
                int c = (p * N + j) * N + i;
                const int *G = &gid[p * n1 * n1];
                m.col_v[4 * c + 0] = G[j * n1 + i];
                m.col_v[4 * c + 1] = G[j * n1 + i + 1];
                m.col_v[4 * c + 2] = G[(j + 1) * n1 + i + 1];
                m.col_v[4 * c + 3] = G[(j + 1) * n1 + i];
            }

    // angular edges; local faces xi- (v0 v3), xi+ (v1 v2), eta- (v0 v1), eta+ (v3 v2)
    const int LFV[4][2] = {{0, 3}, {1, 2}, {0, 1}, {3, 2}};
    std::map<std::pair<int, int>, int> emap;
    m.col_ae.resize(4 * m.ncol);
    m.ae_v.clear();
    m.ae_col.clear();
    m.ae_lf.clear();
    for (int c = 0; c < m.ncol; c++)
        for (int lf = 0; lf < 4; lf++) {
            int a = m.col_v[4 * c + LFV[lf][0]], b = m.col_v[4 * c + LFV[lf][1]];
            std::pair<int, int> key(std::min(a, b), std::max(a, b));
            auto it = emap.find(key);
            int e;
            if (it == emap.end()) {
                e = (int)(m.ae_v.size() / 2);
                emap.emplace(key, e);
                m.ae_v.push_back(key.first);
                m.ae_v.push_back(key.second);
                m.ae_col.push_back(c);
                m.ae_col.push_back(-1);
                m.ae_lf.push_back(lf);
                m.ae_lf.push_back(-1);
            } else {
                e = it->second;
                m.ae_col[2 * e + 1] = c;
                m.ae_lf[2 * e + 1] = lf;
            }
            m.col_ae[4 * c + lf] = e;
        }
    m.nae = (int)(m.ae_v.size() / 2);
    if (m.nae != 12 * N * N) {
        set_error("angular edge construction failed");
        return false;
    }

    // columns around each vertex, counter-clockwise about the outward radial
    m.v_ncol.assign(m.nv, 0);
    m.v_col.assign(4 * m.nv, -1);
    for (int c = 0; c < m.ncol; c++)
        for (int k = 0; k < 4; k++) {
            int v = m.col_v[4 * c + k];
            if (m.v_ncol[v] >= 4) {
                set_error("vertex valence above 4");
                return false;
            }
            m.v_col[4 * v + m.v_ncol[v]++] = c;
        }
    for (int v = 0; v < m.nv; v++) {
        V3 p{m.vpos[3 * v], m.vpos[3 * v + 1], m.vpos[3 * v + 2]};
        int n = m.v_ncol[v];
        double ang[4];
        V3 ea{0, 0, 0};
        for (int s = 0; s < n; s++) {
            int c = m.v_col[4 * v + s];
            V3 cc{0, 0, 0};
            for (int k = 0; k < 4; k++) {
                int w = m.col_v[4 * c + k];
                cc = add(cc, V3{m.vpos[3 * w], m.vpos[3 * w + 1], m.vpos[3 * w + 2]});
            }
            double pr = dt3(cc, p);
            V3 d{cc.x - pr * p.x, cc.y - pr * p.y, cc.z - pr * p.z};
            if (s == 0) ea = unit(d);
            V3 eb = crs(p, ea);
            ang[s] = std::atan2(dt3(d, eb), dt3(d, ea));
        }
        for (int i = 1; i < n; i++)
            for (int j = i; j > 0 && ang[j - 1] > ang[j]; j--) {
                std::swap(ang[j - 1], ang[j]);
                std::swap(m.v_col[4 * v + j - 1], m.v_col[4 * v + j]);
            }
    }
    m.nrf = (int64_t)m.ncol * (m.K + 1);
    m.nfaces = m.nrf + (int64_t)m.nae * m.K;
    m.nre = (int64_t)m.nv * m.K;
    m.nedges = m.nre + (int64_t)m.nae * (m.K + 1);
    m.nzones = (int64_t)m.ncol * m.K;
    return true;
}

}  // namespace rg

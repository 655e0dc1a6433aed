// Reference prism of the library (host, FP64): nodes of Fig. 7 in the
// numbering of Appendices B-D (unit edges, centroid at the origin), the
// monomials of eqs. (5.12)-(5.14) generated as triangle polynomials of degree
// <= p-1 times {1, zeta} plus zeta^k {1, xi, eta} for 2 <= k <= p-1, the nodal
// basis of eq. (5.3), nodal derivative matrices D_d, the time levels and the
// time matrix R of eqs. (5.15)-(5.17) and (B.9), (C.18), (D.28).
#include <cmath>
#include <vector>

#include "prism.hpp"
#include "rg_internal.hpp"

namespace rg {

namespace {

const double SQ3 = std::sqrt(3.0);

// (xi, eta) of triangle vertex k
void corner(int k, double *p)
{
    p[0] = k == 0 ? -0.5 : k == 1 ? 0.5 : 0.0;
    p[1] = k == 2 ? 1.0 / SQ3 : -0.5 / SQ3;
}

// One node kind per line of the printed numbering: vertices at zeta = 1/2
// then -1/2; the vertical-edge points; the triangle-edge points at the top
// then the bottom (each edge k from vertex k to vertex k+1, in order along
// it); the triangle centroids.
void prism_nodes(int p, std::vector<std::array<double, 3>> &nd)
{
    nd.clear();
    double c[2];
    auto verts = [&](double z) {
        for (int k = 0; k < 3; k++) { corner(k, c); nd.push_back({c[0], c[1], z}); }
    };
    auto edges = [&](double z) {
        for (int k = 0; k < 3; k++)
            for (int s = 1; s < p - 1; s++) {
                double a[2], b[2], t = double(s) / (p - 1);
                corner(k, a);
                corner((k + 1) % 3, b);
                nd.push_back({a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1]), z});
            }
    };
    verts(0.5);
    verts(-0.5);
    for (int s = 1; s < p - 1; s++) verts(0.5 - double(s) / (p - 1));
    edges(0.5);
    edges(-0.5);
    if (p == 4) {
        nd.push_back({0.0, 0.0, 0.5});
        nd.push_back({0.0, 0.0, -0.5});
    }
}

void prism_monomials(int p, std::vector<std::array<int, 3>> &mo)
{
    mo.clear();
    for (int deg = 0; deg <= p - 1; deg++)
        for (int a = deg; a >= 0; a--)
            for (int c = 0; c <= 1; c++) mo.push_back({a, deg - a, c});
    for (int k = 2; k <= p - 1; k++) {
        mo.push_back({0, 0, k});
        mo.push_back({1, 0, k});
        mo.push_back({0, 1, k});
    }
}

double mono_val(const std::array<int, 3> &e, const double *x)
{
    double v = 1.0;
    for (int d = 0; d < 3; d++)
        for (int k = 0; k < e[d]; k++) v *= x[d];
    return v;
}

double mono_der(const std::array<int, 3> &e, int dir, const double *x)
{
    if (e[dir] == 0) return 0.0;
    double v = e[dir];
    for (int d = 0; d < 3; d++)
        for (int k = 0; k < e[d] - (d == dir); k++) v *= x[d];
    return v;
}

// Face rules of Appendix A.  Triangle rules as orbits of barycentric points
// (weight, and the point's barycentric coordinates; every distinct
// permutation is a point): (A.1) one orbit (2/3, 1/6, 1/6); (A.3) (5/6,
// 1/12, 1/12) and (1/2, 1/4, 1/4); (A.5) (5/6, 1/12, 1/12), the six points
// (7/12, 1/3, 1/12) and the centroid.  Square rules on [0, 1]^2: (A.2) the
// three printed points, (A.4) 2 x 2 Gauss points, (A.6) 2 Gauss points in x
// by 3 in y.  A side face maps x along its triangle edge and y to zeta.
void face_points(PrismRef &r)
{
    struct Orbit { double w, l0, l1, l2; };
    std::vector<Orbit> orb;
    if (r.order == 2) orb = {{1.0 / 3, 2.0 / 3, 1.0 / 6, 1.0 / 6}};
    else if (r.order == 3) orb = {{1.0 / 8, 5.0 / 6, 1.0 / 12, 1.0 / 12}, {5.0 / 24, 0.5, 0.25, 0.25}};
    else orb = {{32.0 / 405, 5.0 / 6, 1.0 / 12, 1.0 / 12}, {14.0 / 135, 7.0 / 12, 1.0 / 3, 1.0 / 12},
                {19.0 / 135, 1.0 / 3, 1.0 / 3, 1.0 / 3}};
    double V[3][2];
    for (int k = 0; k < 3; k++) corner(k, V[k]);
    std::vector<std::array<double, 3>> tri;   // (xi, eta, weight)
    for (const Orbit &o : orb) {
        const double l[3] = {o.l0, o.l1, o.l2};
        const int perm[6][3] = {{0, 1, 2}, {1, 0, 2}, {1, 2, 0}, {0, 2, 1}, {2, 0, 1}, {2, 1, 0}};
        std::vector<std::array<double, 3>> seen;
        for (auto &pm : perm) {
            const std::array<double, 3> b = {l[pm[0]], l[pm[1]], l[pm[2]]};
            bool dup = false;
            for (auto &x : seen) dup |= x == b;
            if (dup) continue;
            seen.push_back(b);
            tri.push_back({b[0] * V[0][0] + b[1] * V[1][0] + b[2] * V[2][0],
                           b[0] * V[0][1] + b[1] * V[1][1] + b[2] * V[2][1], o.w});
        }
    }
    std::vector<std::array<double, 3>> sq;   // (x, y, weight)
    if (r.order == 2) {
        const double g = 0.5 / std::sqrt(3.0);
        sq = {{0.5 - g, 0.5 + g, 0.25}, {0.5 + g, 0.5 + g, 0.25}, {0.5, 0.5 - g, 0.5}};
    } else {
        double gx[3], gwx[3], gy[3], gwy[3];
        const int ny = r.order == 3 ? 2 : 3;
        gauss_legendre01(2, gx, gwx);
        gauss_legendre01(ny, gy, gwy);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < 2; i++) sq.push_back({gx[i], gy[j], gwx[i] * gwy[j]});
    }
    r.QT = (int)tri.size();
    r.QS = (int)sq.size();
    r.Q = 2 * r.QT + 3 * r.QS;
    r.fpt.clear();
    r.fw.clear();
    for (int f = 0; f < 2; f++)
        for (auto &t : tri) {
            r.fpt.push_back({t[0], t[1], f == 0 ? 0.5 : -0.5});
            r.fw.push_back(t[2]);
        }
    for (int k = 0; k < 3; k++)
        for (auto &s : sq) {
            const double *a = V[k], *b = V[(k + 1) % 3];
            r.fpt.push_back({a[0] + s[0] * (b[0] - a[0]), a[1] + s[0] * (b[1] - a[1]), s[1] - 0.5});
            r.fw.push_back(s[2]);
        }
}

}  // namespace

// inverse of the Vandermonde matrix V[i][k] = m_k(x_i), so that
// psi_l = sum_k C[k][l] m_k
bool lagrange_coefficients(const std::vector<std::array<double, 3>> &x, const std::vector<std::array<int, 3>> &mo,
                           std::vector<double> &C)
{
    const int n = (int)x.size();
    std::vector<double> V((size_t)n * n);
    for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) V[(size_t)i * n + k] = mono_val(mo[k], x[i].data());
    std::vector<int> piv;
    if (!lu_factor(n, V, piv)) return false;
    C.assign((size_t)n * n, 0.0);
    std::vector<double> col(n);
    for (int l = 0; l < n; l++) {
        std::fill(col.begin(), col.end(), 0.0);
        col[l] = 1.0;
        lu_solve(n, V, piv, col.data());
        for (int k = 0; k < n; k++) C[(size_t)k * n + l] = col[k];
    }
    return true;
}

// derivative matrices D[d][i][l] = sum_k d m_k / d xi_d (x_i) C[k][l]
void derivative_matrices(const std::vector<std::array<double, 3>> &x, const std::vector<std::array<int, 3>> &mo,
                         const std::vector<double> &C, std::vector<double> &D)
{
    const int n = (int)x.size();
    D.assign((size_t)3 * n * n, 0.0);
    for (int d = 0; d < 3; d++)
        for (int i = 0; i < n; i++)
            for (int k = 0; k < n; k++) {
                const double g = mono_der(mo[k], d, x[i].data());
                if (g == 0.0) continue;
                for (int l = 0; l < n; l++) D[((size_t)d * n + i) * n + l] += g * C[(size_t)k * n + l];
            }
}

// triangle lattice of degree mo: barycentric (i, j, k) / mo, i descending,
// then j descending
void lattice(int mo, std::vector<std::array<int, 3>> &bary, std::vector<std::array<double, 3>> &x)
{
    double V[3][2];
    for (int k = 0; k < 3; k++) corner(k, V[k]);
    bary.clear();
    x.clear();
    for (int i = mo; i >= 0; i--)
        for (int j = mo - i; j >= 0; j--) {
            const int k = mo - i - j;
            bary.push_back({i, j, k});
            const double l0 = double(i) / mo, l1 = double(j) / mo, l2 = double(k) / mo;
            x.push_back({l0 * V[0][0] + l1 * V[1][0] + l2 * V[2][0], l0 * V[0][1] + l1 * V[1][1] + l2 * V[2][1], 0.0});
        }
}

bool build_prism_ref(int order, PrismRef &r)
{
    if (order < 2 || order > 4) return false;
    r.order = order;
    prism_nodes(order, r.node);
    prism_monomials(order, r.mono);
    r.N = (int)r.node.size();
    if ((int)r.mono.size() != r.N) return false;
    if (!lagrange_coefficients(r.node, r.mono, r.coef)) return false;
    derivative_matrices(r.node, r.mono, r.coef, r.D);
    r.M = order;
    if (!time_galerkin(order, r.tau, r.wt, r.R)) return false;
    // lattice index of each node's (xi, eta): the map's triangle lattice has
    // degree p-1, whose points are exactly the nodes' (xi, eta)
    std::vector<std::array<int, 3>> bary;
    std::vector<std::array<double, 3>> lx;
    lattice(order - 1, bary, lx);
    r.lat.assign(r.N, -1);
    for (int i = 0; i < r.N; i++)
        for (int a = 0; a < (int)lx.size(); a++)
            if (std::fabs(lx[a][0] - r.node[i][0]) < 1e-12 && std::fabs(lx[a][1] - r.node[i][1]) < 1e-12) r.lat[i] = a;
    for (int i = 0; i < r.N; i++)
        if (r.lat[i] < 0) return false;
    face_points(r);
    // trace tables: the basis functions that do not vanish at each point
    r.fidx.assign((size_t)r.Q * TRACE_TERMS, 0);
    r.fval.assign((size_t)r.Q * TRACE_TERMS, 0.0);
    for (int q = 0; q < r.Q; q++) {
        int n = 0;
        for (int l = 0; l < r.N; l++) {
            const double v = r.psi(l, r.fpt[q].data());
            if (std::fabs(v) < 1e-14) continue;
            if (n == TRACE_TERMS) return false;
            r.fidx[(size_t)q * TRACE_TERMS + n] = l;
            r.fval[(size_t)q * TRACE_TERMS + n] = v;
            n++;
        }
    }
    return true;
}

double PrismRef::psi(int l, const double *xi) const
{
    double s = 0.0;
    for (int k = 0; k < N; k++) s += coef[(size_t)k * N + l] * mono_val(mono[k], xi);
    return s;
}

}  // namespace rg

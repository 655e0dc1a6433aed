// Geometry precompute (Section VI step 1), host FP64, one radial column at a
// time.  With geometric shells every zone of a column is the column's first
// (shell-0) zone scaled about the origin by q^k, so every reconstruction and
// predictor matrix below is built once per column and shared by its K zones
// (the amortisation of Sections IV.b step 7 and V.b).
//
// Per column:
//  - isoparametric map (eq. 5.2): tensor Lagrange surface of order map_order
//    through great-circle nodes, linear in the radial direction;
//  - Gauss cubature: volume, centroid, l0 = |V|^(1/3), moments (eqs. 3.2-3.3);
//  - WENO-AO: large-stencil least-squares rows by the parallel-axis
//    expansion of eq. (3.4) generalised to any degree, pseudo-inverses of the
//    large and of seven small (linear) stencils, quadratic forms of the
//    smoothness indicators;
//  - divergence-free B (Section IV.b steps 1-9): the KKT system with the
//    divergence identities (4.10), face-flux constraints (4.14), closeness
//    rows (4.3/4.6/4.9) and face nodal rows (4.15), inverted once and fused
//    with evaluation at the ADER nodes (step 10: the new zone mean);
//  - ADER nodes: Jacobian and flux metrics (eq. 5.11) in curl form, whose
//    discrete divergence vanishes so uniform states stay uniform;
//  - face quadrature (area vectors, eqs. 5.6-5.8) and edge Simpson points.
#include <cmath>
#include <cstring>

#include "rg_geom_host.hpp"

namespace rg {

namespace {

inline double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline void normalize(double *a)
{
    double n = std::sqrt(dot(a, a));
    a[0] /= n; a[1] /= n; a[2] /= n;
}

}  // namespace

// point at fraction t of the great-circle arc from unit vector a to unit
// vector b: a rotated by t times the arc's angle within the plane of a and b
void arc_point(const double *a, const double *b, double t, double *o)
{
    double u[3];
    const double ab = dot(a, b);
    for (int i = 0; i < 3; i++) u[i] = b[i] - ab * a[i];   // the in-plane direction orthogonal to a
    const double un = std::sqrt(dot(u, u));
    const double th = std::atan2(un, ab);
    const double ca = std::cos(t * th), sa = std::sin(t * th) / un;
    for (int i = 0; i < 3; i++) o[i] = ca * a[i] + sa * u[i];
}

namespace {

// where the great circle through p1, p2 meets the great circle through q1, q2:
// the unit vector in the plane of p1, p2 orthogonal to the second circle's
// normal, on the side of hint
void circles_meet(const double *p1, const double *p2, const double *q1, const double *q2, const double *hint,
                  double *o)
{
    double n2[3];
    cross(q1, q2, n2);
    const double s1 = dot(p1, n2), s2 = dot(p2, n2);
    for (int i = 0; i < 3; i++) o[i] = s2 * p1[i] - s1 * p2[i];
    normalize(o);
    if (dot(o, hint) < 0) { o[0] = -o[0]; o[1] = -o[1]; o[2] = -o[2]; }
}

// monomial coefficients of the 1-D Lagrange basis on mo + 1 equidistant nodes
// of [-1/2, 1/2]: basis a is sum_k coef[a][k] x^k, expanded from its product
// form once per order
struct LagrangePoly {
    double coef[4][4] = {};
    explicit LagrangePoly(int mo)
    {
        for (int a = 0; a <= mo; a++) {
            const double ta = -0.5 + double(a) / mo;
            double pc[4] = {1.0, 0.0, 0.0, 0.0};   // running product, degree 0
            int deg = 0;
            for (int b = 0; b <= mo; b++) {
                if (b == a) continue;
                const double tb = -0.5 + double(b) / mo, den = ta - tb;
                // multiply by (x - tb) / den
                double nx[4] = {0.0, 0.0, 0.0, 0.0};
                for (int k = 0; k <= deg; k++) {
                    nx[k + 1] += pc[k] / den;
                    nx[k] -= tb * pc[k] / den;
                }
                deg++;
                for (int k = 0; k <= deg; k++) pc[k] = nx[k];
            }
            for (int k = 0; k <= mo; k++) coef[a][k] = pc[k];
        }
    }
    // value and derivative of basis a at x (Horner)
    void eval(int mo, int a, double x, double &v, double &d) const
    {
        v = coef[a][mo];
        d = 0.0;
        for (int k = mo - 1; k >= 0; k--) {
            d = d * x + v;
            v = v * x + coef[a][k];
        }
    }
};

const LagrangePoly &lagrange(int mo)
{
    static const LagrangePoly q2(2), q3(3);
    return mo == 2 ? q2 : q3;
}

double det3(const double *j)
{
    return j[0] * (j[4] * j[8] - j[5] * j[7]) - j[1] * (j[3] * j[8] - j[5] * j[6]) + j[2] * (j[3] * j[7] - j[4] * j[6]);
}

double binom(int n, int k)
{
    double v = 1.0;
    for (int i = 0; i < k; i++) v = v * (n - i) / (i + 1);
    return v;
}

double falling(int a, int b)
{
    double v = 1.0;
    for (int i = 0; i < b; i++) v *= a - i;
    return v;
}

}  // namespace

// surface nodes of column c (node (a, b) at index a + (mo + 1) b): the four
// corners, points at equal arc fractions along the four edges, and inside
// the meeting points of the great circles joining opposite edges' points
void column_surface_nodes(const Mesh &m, int c, double *sn)
{
    const int mo = m.map_order, n1 = mo + 1;
    const double *v0 = &m.vpos[3 * m.col_v[4 * c]], *v1 = &m.vpos[3 * m.col_v[4 * c + 1]];
    const double *v2 = &m.vpos[3 * m.col_v[4 * c + 2]], *v3 = &m.vpos[3 * m.col_v[4 * c + 3]];
    auto node = [&](int a, int b) { return &sn[3 * (a + n1 * b)]; };
    // the boundary: edges v0 -> v1 (b = 0), v3 -> v2 (b = mo), v0 -> v3
    // (a = 0), v1 -> v2 (a = mo), corners included
    for (int j = 0; j <= mo; j++) {
        const double t = double(j) / mo;
        arc_point(v0, v1, t, node(j, 0));
        arc_point(v3, v2, t, node(j, mo));
        if (j > 0 && j < mo) {
            arc_point(v0, v3, t, node(0, j));
            arc_point(v1, v2, t, node(mo, j));
        }
    }
    for (int i = 0; i < 3; i++) {   // the end points exactly
        node(0, 0)[i] = v0[i]; node(mo, 0)[i] = v1[i]; node(mo, mo)[i] = v2[i]; node(0, mo)[i] = v3[i];
    }
    double hint[3];
    for (int i = 0; i < 3; i++) hint[i] = v0[i] + v1[i] + v2[i] + v3[i];
    for (int b = 1; b < mo; b++)
        for (int a = 1; a < mo; a++) circles_meet(node(a, 0), node(a, mo), node(0, b), node(mo, b), hint, node(a, b));
}

// map of a zone with surface nodes sn between radii r0 < r1, x = R(xi_2)
// S(xi_0, xi_1) with S the tensor Lagrange interpolant of the surface nodes
// and R linear in xi_2; jac[n*3+d] = dx_n/dxi_d.  S is evaluated curve by
// curve: first along xi_0 through each row b of nodes, then along xi_1
// through the rows' values.
void zone_map(int mo, const double *sn, double r0, double r1, const double *xi, double *x, double *jac)
{
    const int n1 = mo + 1;
    const LagrangePoly &L = lagrange(mo);
    double la[4], dla[4], lb[4], dlb[4];
    for (int a = 0; a <= mo; a++) {
        L.eval(mo, a, xi[0], la[a], dla[a]);
        L.eval(mo, a, xi[1], lb[a], dlb[a]);
    }
    double S[3] = {0, 0, 0}, Sa[3] = {0, 0, 0}, Sb[3] = {0, 0, 0};
    for (int b = 0; b <= mo; b++) {
        double row[3] = {0, 0, 0}, drow[3] = {0, 0, 0};   // the row curve at xi_0 and its xi_0 derivative
        for (int a = 0; a <= mo; a++)
            for (int i = 0; i < 3; i++) {
                row[i] += la[a] * sn[3 * (a + n1 * b) + i];
                drow[i] += dla[a] * sn[3 * (a + n1 * b) + i];
            }
        for (int i = 0; i < 3; i++) {
            S[i] += lb[b] * row[i];
            Sa[i] += lb[b] * drow[i];
            Sb[i] += dlb[b] * row[i];
        }
    }
    const double h = 0.5 + xi[2], R = r0 + h * (r1 - r0), dR = r1 - r0;
    for (int i = 0; i < 3; i++) {
        x[i] = R * S[i];
        if (jac) {
            jac[i * 3 + 0] = R * Sa[i];
            jac[i * 3 + 1] = R * Sb[i];
            jac[i * 3 + 2] = dR * S[i];
        }
    }
}

int moment_index(int a, int b, int c) { return a * 25 + b * 5 + c; }

// ---------------------------------------------------------------- pass 1
void column_pass1(const Mesh &m, const RefEl &r, int c, ColData &cd)
{
    const int mo = m.map_order, N = r.N, Q = r.Q;
    column_surface_nodes(m, c, cd.sn);
    const double r0 = m.radius[0], r1 = m.radius[1];
    const int na = (r.order == 3) ? 8 : 10, nr = 6;
    std::vector<double> ax(na), aw(na), rx(nr), rw(nr);
    gauss_legendre01(na, ax.data(), aw.data());
    gauss_legendre01(nr, rx.data(), rw.data());
    std::vector<double> px, pw;
    px.reserve(3 * na * na * nr);
    double vol = 0.0, cen[3] = {0, 0, 0};
    for (int k = 0; k < nr; k++)
        for (int j = 0; j < na; j++)
            for (int i = 0; i < na; i++) {
                double xi[3] = {ax[i] - 0.5, ax[j] - 0.5, rx[k] - 0.5}, x[3], jac[9];
                zone_map(mo, cd.sn, r0, r1, xi, x, jac);
                double w = aw[i] * aw[j] * rw[k] * det3(jac);
                vol += w;
                for (int d = 0; d < 3; d++) cen[d] += w * x[d];
                px.insert(px.end(), x, x + 3);
                pw.push_back(w);
            }
    for (int d = 0; d < 3; d++) cen[d] /= vol;
    cd.vol = vol;
    std::memcpy(cd.cen, cen, 24);
    cd.len = std::cbrt(vol);
    std::fill(cd.mom, cd.mom + 125, 0.0);
    for (size_t p = 0; p < pw.size(); p++) {
        double X[3];
        for (int d = 0; d < 3; d++) X[d] = (px[3 * p + d] - cen[d]) / cd.len;
        double pa[5], pb[5], pc[5];
        pa[0] = pb[0] = pc[0] = 1.0;
        for (int e = 1; e < 5; e++) { pa[e] = pa[e - 1] * X[0]; pb[e] = pb[e - 1] * X[1]; pc[e] = pc[e - 1] * X[2]; }
        for (int a = 0; a < 5; a++)
            for (int b = 0; a + b < 5; b++)
                for (int cc = 0; a + b + cc < 5; cc++) cd.mom[moment_index(a, b, cc)] += pw[p] * pa[a] * pb[b] * pc[cc];
    }
    for (int i = 0; i < 125; i++) cd.mom[i] /= vol;

    // faces of the shell-0 zone: points, outward unit normals, |dA|
    for (int lf = 0; lf < 6; lf++) {
        int axis = lf / 2, u = axis == 0 ? 1 : 0, v = axis == 2 ? 1 : 2;
        double sg = ((lf & 1) ? 1.0 : -1.0) * (axis == 1 ? -1.0 : 1.0);
        double A = 0.0, fc[3] = {0, 0, 0}, nb[3] = {0, 0, 0};
        for (int q = 0; q < Q; q++) {
            double xi[3], jac[9], hu[3], hv[3], dA[3];
            face_ref_point(r, lf, q, xi);
            zone_map(mo, cd.sn, r0, r1, xi, &cd.fx[lf][q][0], jac);
            for (int i = 0; i < 3; i++) { hu[i] = jac[i * 3 + u]; hv[i] = jac[i * 3 + v]; }
            cross(hu, hv, dA);
            double w = r.gw[q % r.Q1] * r.gw[q / r.Q1], a = std::sqrt(dot(dA, dA));
            for (int i = 0; i < 3; i++) cd.fn[lf][q][i] = sg * dA[i] / a;
            cd.fdA[lf][q] = w * a;
            A += w * a;
            for (int i = 0; i < 3; i++) { fc[i] += w * a * cd.fx[lf][q][i]; nb[i] += w * sg * dA[i]; }
        }
        cd.farea[lf] = A;
        for (int i = 0; i < 3; i++) cd.fcen[lf][i] = fc[i] / A;
        normalize(nb);
        std::memcpy(cd.fnbar[lf], nb, 24);
    }
    // in-sphere diameter: twice the least centroid-to-face-plane distance
    double dmin = 1e300;
    for (int lf = 0; lf < 6; lf++) {
        double d[3] = {cd.fcen[lf][0] - cen[0], cd.fcen[lf][1] - cen[1], cd.fcen[lf][2] - cen[2]};
        dmin = std::min(dmin, std::fabs(dot(d, cd.fnbar[lf])));
    }
    cd.dins = 2.0 * dmin;

    // ADER nodes: positions, Jacobians, curl-form metrics from the interpolated
    // products (x_l - c_l) grad_xi x_m
    cd.nx.resize(3 * N);
    cd.nJ.resize(N);
    cd.nM.resize(9 * N);
    std::vector<double> V(9 * N);
    for (int i = 0; i < N; i++) {
        double jac[9];
        zone_map(mo, cd.sn, r0, r1, r.node[i].data(), &cd.nx[3 * i], jac);
        cd.nJ[i] = det3(jac);
        for (int n = 0; n < 3; n++) {
            int mm = (n + 1) % 3, ll = (n + 2) % 3;
            for (int j = 0; j < 3; j++) V[i * 9 + n * 3 + j] = (cd.nx[3 * i + ll] - cen[ll]) * jac[mm * 3 + j];
        }
    }
    for (int i = 0; i < N; i++)
        for (int n = 0; n < 3; n++) {
            double g[3][3] = {{0}};  // g[j][d] = d/dxi_d of interpolated V_j
            for (int l = 0; l < N; l++)
                for (int d = 0; d < 3; d++) {
                    double Dv = r.D[((size_t)d * N + i) * N + l];
                    if (Dv == 0.0) continue;
                    for (int j = 0; j < 3; j++) g[j][d] += Dv * V[l * 9 + n * 3 + j];
                }
            cd.nM[i * 9 + 0 * 3 + n] = -(g[2][1] - g[1][2]);
            cd.nM[i * 9 + 1 * 3 + n] = -(g[0][2] - g[2][0]);
            cd.nM[i * 9 + 2 * 3 + n] = -(g[1][0] - g[0][1]);
        }
}

// Taylor-basis value X^e - C_e (constant 1 for e = 0)
static double tbasis(const double *mom, const std::array<int, 3> &e, const double *X)
{
    if (e[0] + e[1] + e[2] == 0) return 1.0;
    double v = 1.0;
    for (int d = 0; d < 3; d++)
        for (int k = 0; k < e[d]; k++) v *= X[d];
    return v - mom[moment_index(e[0], e[1], e[2])];
}

// least-squares pseudo-inverse of an n x m matrix A (n >= m, full column
// rank, row-major): P = R^-1 Q^T from a Householder QR factorisation, which
// keeps the conditioning of A itself (the normal equations would square it,
// and the stencils of thin shells are poorly conditioned).  P is m x n.
static bool pinv(int n, int m, const std::vector<double> &A, std::vector<double> &P)
{
    std::vector<double> R(A), Qt((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) Qt[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n);
    for (int j = 0; j < m; j++) {
        double nrm = 0.0;
        for (int i = j; i < n; i++) nrm += R[(size_t)i * m + j] * R[(size_t)i * m + j];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) return false;
        const double a = R[(size_t)j * m + j], alpha = a > 0 ? -nrm : nrm;
        double vn = 0.0;
        for (int i = j; i < n; i++) {
            v[i] = R[(size_t)i * m + j] - (i == j ? alpha : 0.0);
            vn += v[i] * v[i];
        }
        if (!(vn > 0.0)) continue;
        // apply H = I - 2 v v^T / (v^T v) to the remaining columns of R and to Q^T
        for (int k = j; k < m; k++) {
            double d = 0.0;
            for (int i = j; i < n; i++) d += v[i] * R[(size_t)i * m + k];
            d *= 2.0 / vn;
            for (int i = j; i < n; i++) R[(size_t)i * m + k] -= d * v[i];
        }
        for (int k = 0; k < n; k++) {
            double d = 0.0;
            for (int i = j; i < n; i++) d += v[i] * Qt[(size_t)i * n + k];
            d *= 2.0 / vn;
            for (int i = j; i < n; i++) Qt[(size_t)i * n + k] -= d * v[i];
        }
    }
    // rank check relative to the largest diagonal entry of R
    double dmax = 0.0;
    for (int j = 0; j < m; j++) dmax = std::max(dmax, std::abs(R[(size_t)j * m + j]));
    for (int j = 0; j < m; j++)
        if (!(std::abs(R[(size_t)j * m + j]) > 1e-14 * dmax)) return false;
    // back substitution R P = (Q^T)[0:m, :]
    P.assign((size_t)m * n, 0.0);
    for (int k = 0; k < n; k++)
        for (int i = m - 1; i >= 0; i--) {
            double s = Qt[(size_t)i * n + k];
            for (int l = i + 1; l < m; l++) s -= R[(size_t)i * m + l] * P[(size_t)l * n + k];
            P[(size_t)i * n + k] = s / R[(size_t)i * m + i];
        }
    return true;
}

// 2-norm condition number sigma_max / sigma_min of an n x m matrix (n >= m,
// row-major) by one-sided Jacobi rotations of its columns (Hestenes): the
// columns converge to mutually orthogonal vectors whose norms are the
// singular values, accurately also for the smallest ones.
static double cond2(int n, int m, const std::vector<double> &A)
{
    std::vector<double> W(A);
    for (int sweep = 0; sweep < 40; sweep++) {
        double off = 0.0;
        for (int j = 0; j < m - 1; j++)
            for (int k = j + 1; k < m; k++) {
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = 0; i < n; i++) {
                    const double x = W[(size_t)i * m + j], y = W[(size_t)i * m + k];
                    a += x * x;
                    b += y * y;
                    g += x * y;
                }
                if (g == 0.0 || std::abs(g) <= 1e-15 * std::sqrt(a * b)) continue;
                off = std::max(off, std::abs(g) / std::sqrt(a * b));
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < n; i++) {
                    const double x = W[(size_t)i * m + j], y = W[(size_t)i * m + k];
                    W[(size_t)i * m + j] = cs * x - sn * y;
                    W[(size_t)i * m + k] = sn * x + cs * y;
                }
            }
        if (off < 1e-15) break;
    }
    double smax = 0.0, smin = 1e300;
    for (int j = 0; j < m; j++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += W[(size_t)i * m + j] * W[(size_t)i * m + j];
        s = std::sqrt(s);
        smax = std::max(smax, s);
        smin = std::min(smin, s);
    }
    return smin > 0.0 ? smax / smin : INFINITY;
}

// 1-norm condition number ||K||_1 ||K^-1||_1 of a symmetric matrix from its
// LU factors, with ||K^-1||_1 estimated by Hager's method (a few solves with
// K and, K being symmetric, with K^T = K; the estimate is a lower bound that
// is exact in most cases).
static double cond1_symmetric(int n, const std::vector<double> &K, const std::vector<double> &LU,
                              const std::vector<int> &piv)
{
    double knorm = 0.0;
    for (int j = 0; j < n; j++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += std::abs(K[(size_t)i * n + j]);
        knorm = std::max(knorm, s);
    }
    std::vector<double> x(n, 1.0 / n), y(n), z(n);
    double est = 0.0;
    for (int it = 0; it < 5; it++) {
        y = x;
        lu_solve(n, LU, piv, y.data());
        double ny = 0.0;
        for (double v : y) ny += std::abs(v);
        if (it > 0 && ny <= est) break;
        est = ny;
        for (int i = 0; i < n; i++) z[i] = y[i] >= 0 ? 1.0 : -1.0;
        lu_solve(n, LU, piv, z.data());
        int jmax = 0;
        double zx = 0.0;
        for (int i = 0; i < n; i++) {
            zx += z[i] * x[i];
            if (std::abs(z[i]) > std::abs(z[jmax])) jmax = i;
        }
        if (std::abs(z[jmax]) <= zx) break;
        std::fill(x.begin(), x.end(), 0.0);
        x[jmax] = 1.0;
    }
    return knorm * est;
}

// ---------------------------------------------------------------- pass 2
bool column_pass2(const Mesh &m, const RefEl &r, const std::vector<ColData> &cols, int c, HostGeom &hg)
{
    const ColData &cd = cols[c];
    const int N = r.N, NC = r.NC, NS = r.NS, Q = r.Q, NB = r.NB, p = r.order;
    const double q = m.q;
    // ---- stencil: face neighbours first (local faces 0..5), then the rest
    std::vector<std::pair<int, int>> st;
    int fnb[4];
    for (int lf = 0; lf < 4; lf++) {
        int ae = m.col_ae[4 * c + lf];
        fnb[lf] = (m.ae_col[2 * ae] == c) ? m.ae_col[2 * ae + 1] : m.ae_col[2 * ae];
        st.push_back({fnb[lf], 0});
    }
    st.push_back({c, -1});
    st.push_back({c, +1});
    std::vector<int> vn;  // columns sharing a vertex with c (not c)
    for (int k = 0; k < 4; k++) {
        int v = m.col_v[4 * c + k];
        for (int s = 0; s < m.v_ncol[v]; s++) {
            int o = m.v_col[4 * v + s];
            if (o != c && std::find(vn.begin(), vn.end(), o) == vn.end()) vn.push_back(o);
        }
    }
    auto has = [&](int col, int dk) {
        for (auto &e : st)
            if (e.first == col && e.second == dk) return true;
        return false;
    };
    for (int o : vn)
        if (!has(o, 0)) st.push_back({o, 0});
    for (int dk : {-1, 1})
        for (int o : vn)
            if (!has(o, dk)) st.push_back({o, dk});
    if (p == 4) {
        for (int dk : {-2, 2}) st.push_back({c, dk});
        for (int lf = 0; lf < 4; lf++) {
            int c1 = fnb[lf], ae = m.col_ae[4 * c + lf];
            int lf1 = (m.ae_col[2 * ae] == c1) ? m.ae_lf[2 * ae] : m.ae_lf[2 * ae + 1];
            int ae2 = m.col_ae[4 * c1 + (lf1 ^ 1)];
            int c2 = (m.ae_col[2 * ae2] == c1) ? m.ae_col[2 * ae2 + 1] : m.ae_col[2 * ae2];
            if (c2 != c && !has(c2, 0)) st.push_back({c2, 0});
        }
    }
    const int ns = (int)st.size();
    if (ns > NS) { set_error("stencil larger than its slot count"); return false; }
    for (int j = 0; j < NS; j++)
        hg.stm[(size_t)c * NS + j] = (j < ns) ? st[j].first * 8 + (st[j].second + 3) : -1;
    hg.stn[c] = ns;

    // ---- large-stencil rows: average over zone j of zone 0's Taylor basis,
    // by the parallel-axis expansion with zone j's own moments
    std::vector<double> A((size_t)ns * NC);
    for (int j = 0; j < ns; j++) {
        const ColData &cj = cols[st[j].first];
        double sc = std::pow(q, st[j].second);
        double d[3], rho = sc * cj.len / cd.len;
        for (int i = 0; i < 3; i++) d[i] = (sc * cj.cen[i] - cd.cen[i]) / cd.len;
        for (int a = 0; a < NC; a++) {
            const auto &al = r.tex[a];
            double s = 0.0;
            for (int b0 = 0; b0 <= al[0]; b0++)
                for (int b1 = 0; b1 <= al[1]; b1++)
                    for (int b2 = 0; b2 <= al[2]; b2++) {
                        double t = binom(al[0], b0) * binom(al[1], b1) * binom(al[2], b2) *
                                   std::pow(d[0], al[0] - b0) * std::pow(d[1], al[1] - b1) * std::pow(d[2], al[2] - b2) *
                                   std::pow(rho, b0 + b1 + b2) * cj.mom[moment_index(b0, b1, b2)];
                        s += t;
                    }
            A[(size_t)j * NC + a] = s - cd.mom[moment_index(al[0], al[1], al[2])];
        }
    }
    std::vector<double> P;
    if (!pinv(ns, NC, A, P)) { set_error("singular large-stencil least squares"); return false; }
    hg.cond_lsq[c] = cond2(ns, NC, A);
    double *Pl = &hg.Pl[(size_t)c * NC * NS];
    for (int a = 0; a < NC; a++)
        for (int j = 0; j < NS; j++) Pl[a * NS + j] = (j < ns) ? P[(size_t)a * ns + j] : 0.0;

    // ---- small stencils on the six face neighbours: central, then one-sided
    double dface[6][3];
    for (int j = 0; j < 6; j++) {
        const ColData &cj = cols[st[j].first];
        double sc = std::pow(q, st[j].second);
        for (int i = 0; i < 3; i++) dface[j][i] = (sc * cj.cen[i] - cd.cen[i]) / cd.len;
    }
    double *Ps = &hg.Ps[(size_t)c * 7 * 18];
    for (int s = 0; s < 7; s++) {
        std::vector<int> mem;
        for (int j = 0; j < 6; j++)
            if (s == 0 || j != ((s - 1) ^ 1)) mem.push_back(j);
        std::vector<double> As(mem.size() * 3), Pss;
        for (size_t k = 0; k < mem.size(); k++)
            for (int i = 0; i < 3; i++) As[k * 3 + i] = dface[mem[k]][i];
        if (!pinv((int)mem.size(), 3, As, Pss)) { set_error("singular small-stencil least squares"); return false; }
        for (int i = 0; i < 18; i++) Ps[s * 18 + i] = 0.0;
        for (int i = 0; i < 3; i++)
            for (size_t k = 0; k < mem.size(); k++) Ps[s * 18 + i * 6 + mem[k]] = Pss[i * mem.size() + k];
    }

    // ---- smoothness quadratic form: sum over derivative multi-indices of the
    // zone average of products of derivatives of the Taylor basis
    double *Qs = &hg.Qs[(size_t)c * NC * NC];
    for (int a = 0; a < NC; a++)
        for (int b = 0; b < NC; b++) {
            const auto &ea = r.tex[a], &eb = r.tex[b];
            double s = 0.0;
            for (const auto &be : r.tex) {
                if (be[0] > ea[0] || be[1] > ea[1] || be[2] > ea[2]) continue;
                if (be[0] > eb[0] || be[1] > eb[1] || be[2] > eb[2]) continue;
                double f = 1.0;
                for (int d = 0; d < 3; d++) f *= falling(ea[d], be[d]) * falling(eb[d], be[d]);
                s += f * cd.mom[moment_index(ea[0] + eb[0] - 2 * be[0], ea[1] + eb[1] - 2 * be[1], ea[2] + eb[2] - 2 * be[2])];
            }
            Qs[a * NC + b] = s;
        }

    // ---- Taylor basis at the ADER nodes
    double *Ev = &hg.Ev[(size_t)c * N * NC];
    std::vector<double> Xn(3 * N);
    for (int i = 0; i < N; i++) {
        for (int d = 0; d < 3; d++) Xn[3 * i + d] = (cd.nx[3 * i + d] - cd.cen[d]) / cd.len;
        for (int a = 0; a < NC; a++) Ev[i * NC + a] = tbasis(cd.mom, r.tex[a], &Xn[3 * i]);
    }
    std::memcpy(&hg.nJ[(size_t)c * N], cd.nJ.data(), sizeof(double) * N);
    std::memcpy(&hg.nM[(size_t)c * N * 9], cd.nM.data(), sizeof(double) * N * 9);
    hg.dins[c] = cd.dins;

    // ---- radial faces: canonical data = bottom face of the shell-0 zone, normal +r
    for (int qq = 0; qq < Q; qq++) {
        for (int i = 0; i < 3; i++) hg.fnR[((size_t)c * Q + qq) * 3 + i] = -cd.fn[4][qq][i];
        hg.fwR[(size_t)c * Q + qq] = cd.fdA[4][qq] / cd.farea[4];
        double Xb[3], Xa[3];
        for (int d = 0; d < 3; d++) {
            Xa[d] = (cd.fx[4][qq][d] - cd.cen[d]) / cd.len;        // zone above (its bottom face)
            Xb[d] = (q * cd.fx[4][qq][d] - cd.cen[d]) / cd.len;    // zone below (its top face)
        }
        for (int a = 0; a < NC; a++) {
            hg.fevR[(((size_t)c * 2 + 0) * Q + qq) * NC + a] = tbasis(cd.mom, r.tex[a], Xb);
            hg.fevR[(((size_t)c * 2 + 1) * Q + qq) * NC + a] = tbasis(cd.mom, r.tex[a], Xa);
        }
    }

    // ---- face point order and orientation relative to the canonical faces
    int perm[6][9], sgn[6];
    for (int lf = 0; lf < 6; lf++)
        for (int qq = 0; qq < Q; qq++) perm[lf][qq] = qq;
    sgn[4] = -1;
    sgn[5] = +1;
    for (int lf = 0; lf < 4; lf++) {
        int ae = m.col_ae[4 * c + lf];
        int side = (m.ae_col[2 * ae] == c) ? 0 : 1;
        hg.col_ae[4 * c + lf] = ae;
        hg.col_side[4 * c + lf] = side;
        sgn[lf] = side == 0 ? 1 : -1;
        if (side == 1) {
            const ColData &c0 = cols[m.ae_col[2 * ae]];
            int lf0 = m.ae_lf[2 * ae];
            for (int qq = 0; qq < Q; qq++) {
                int best = -1;
                double bd = 1e300;
                for (int q0 = 0; q0 < Q; q0++) {
                    double dd = 0;
                    for (int i = 0; i < 3; i++) dd += (cd.fx[lf][qq][i] - c0.fx[lf0][q0][i]) * (cd.fx[lf][qq][i] - c0.fx[lf0][q0][i]);
                    if (dd < bd) { bd = dd; best = q0; }
                }
                perm[lf][qq] = best;
            }
        }
        for (int qq = 0; qq < Q; qq++) hg.col_perm[((size_t)c * 4 + lf) * Q + qq] = perm[lf][qq];
    }

    // ---- divergence-free B: KKT system, inverted for all inputs at once
    const int nu = 3 * NB, nrow = nu + 6 * Q, ndiv = NC, ncon = ndiv + 6, NIN = r.NIN;
    const int inB = 0, inF = 3 * (NC + 1), inM = 3 * (NC + 1) + 6 * Q;
    std::vector<double> Am((size_t)nrow * nu, 0.0), Sb((size_t)nrow * NIN, 0.0);
    std::vector<double> Cm((size_t)ncon * nu, 0.0), Sd((size_t)ncon * NIN, 0.0);
    for (int comp = 0; comp < 3; comp++)
        for (int k = 0; k < NB; k++) {
            int row = comp * NB + k;
            Am[(size_t)row * nu + row] = 1.0;
            const auto &e = r.bex[comp][k];
            int deg = e[0] + e[1] + e[2];
            if (deg == 0) Sb[(size_t)row * NIN + inB + comp * (NC + 1)] = 1.0;
            else if (deg <= p - 1) {
                int a = 0;
                while (r.tex[a] != e) a++;
                Sb[(size_t)row * NIN + inB + comp * (NC + 1) + 1 + a] = 1.0;
            }
        }
    for (int lf = 0; lf < 6; lf++)
        for (int qq = 0; qq < Q; qq++) {
            int row = nu + lf * Q + qq;
            double X[3], wq = cd.fdA[lf][qq] / cd.farea[lf];
            for (int d = 0; d < 3; d++) X[d] = (cd.fx[lf][qq][d] - cd.cen[d]) / cd.len;
            for (int comp = 0; comp < 3; comp++)
                for (int k = 0; k < NB; k++) {
                    double val = cd.fn[lf][qq][comp] * tbasis(cd.mom, r.bex[comp][k], X);
                    Am[(size_t)row * nu + comp * NB + k] = val;
                    Cm[(size_t)(ndiv + lf) * nu + comp * NB + k] += wq * val;
                }
            Sb[(size_t)row * NIN + inF + lf * Q + perm[lf][qq]] = sgn[lf];
        }
    for (int lf = 0; lf < 6; lf++) Sd[(size_t)(ndiv + lf) * NIN + inM + lf] = sgn[lf];
    for (int i = 0; i < ndiv; i++)
        for (int comp = 0; comp < 3; comp++) {
            std::array<int, 3> t = r.tex[i];
            t[comp] += 1;
            for (int k = 0; k < NB; k++)
                if (r.bex[comp][k] == t) Cm[(size_t)i * nu + comp * NB + k] += t[comp];
        }
    const int nk = nu + ncon;
    std::vector<double> K((size_t)nk * nk, 0.0), rhs((size_t)nk * NIN, 0.0);
    for (int i = 0; i < nu; i++)
        for (int j = 0; j < nu; j++) {
            double s = 0.0;
            for (int k = 0; k < nrow; k++) s += Am[(size_t)k * nu + i] * Am[(size_t)k * nu + j];
            K[(size_t)i * nk + j] = 2.0 * s;
        }
    for (int i = 0; i < ncon; i++)
        for (int j = 0; j < nu; j++) {
            K[(size_t)(nu + i) * nk + j] = Cm[(size_t)i * nu + j];
            K[(size_t)j * nk + nu + i] = Cm[(size_t)i * nu + j];
        }
    for (int i = 0; i < nu; i++)
        for (int j = 0; j < NIN; j++) {
            double s = 0.0;
            for (int k = 0; k < nrow; k++) s += Am[(size_t)k * nu + i] * Sb[(size_t)k * NIN + j];
            rhs[(size_t)i * NIN + j] = 2.0 * s;
        }
    for (int i = 0; i < ncon; i++)
        for (int j = 0; j < NIN; j++) rhs[(size_t)(nu + i) * NIN + j] = Sd[(size_t)i * NIN + j];
    std::vector<int> piv;
    const std::vector<double> Kfull(K);
    if (!lu_factor(nk, K, piv)) { set_error("singular divergence-free KKT system"); return false; }
    hg.cond_kkt[c] = cond1_symmetric(nk, Kfull, K, piv);
    std::vector<double> G((size_t)nu * NIN), col(nk);
    for (int j = 0; j < NIN; j++) {
        for (int i = 0; i < nk; i++) col[i] = rhs[(size_t)i * NIN + j];
        lu_solve(nk, K, piv, col.data());
        for (int i = 0; i < nu; i++) G[(size_t)i * NIN + j] = col[i];
    }
    // fused map: B at the ADER nodes, then the three new zone means
    double *Mb = &hg.Mb[(size_t)c * r.NOUTB * NIN];
    for (int comp = 0; comp < 3; comp++)
        for (int i = 0; i < N; i++) {
            double *row = &Mb[(size_t)(comp * N + i) * NIN];
            for (int j = 0; j < NIN; j++) row[j] = 0.0;
            for (int k = 0; k < NB; k++) {
                double b = tbasis(cd.mom, r.bex[comp][k], &Xn[3 * i]);
                const double *g = &G[(size_t)(comp * NB + k) * NIN];
                for (int j = 0; j < NIN; j++) row[j] += b * g[j];
            }
        }
    for (int comp = 0; comp < 3; comp++)
        std::memcpy(&Mb[(size_t)(3 * N + comp) * NIN], &G[(size_t)(comp * NB) * NIN], sizeof(double) * NIN);
    return true;
}

// ---------------------------------------------------------------- pass 3: angular edges, vertices
void symmetric_frame(const double *u0, const double *w0, const double *t, double *e1, double *e2)
{
    double u[3], w[3], b[3], bp[3];
    double pu = dot(u0, t), pw = dot(w0, t);
    for (int i = 0; i < 3; i++) { u[i] = u0[i] - pu * t[i]; w[i] = w0[i] - pw * t[i]; }
    normalize(u);
    normalize(w);
    for (int i = 0; i < 3; i++) b[i] = u[i] + w[i];
    normalize(b);
    cross(t, b, bp);
    const double h = std::sqrt(0.5);
    for (int i = 0; i < 3; i++) { e1[i] = h * (b[i] - bp[i]); e2[i] = h * (b[i] + bp[i]); }
}

// local face (0..3) -> local edge on the zeta- side, and its (from, to) corners
static const int LF_EDGE[4] = {4, 5, 0, 1};
static const int LF_FROMTO[4][2] = {{0, 3}, {1, 2}, {0, 1}, {3, 2}};

void angular_edge_pass(const Mesh &m, const RefEl &r, const std::vector<ColData> &cols, int ae, HostGeom &hg)
{
    const int Q = r.Q, NC = r.NC;
    const int c0 = m.ae_col[2 * ae], c1 = m.ae_col[2 * ae + 1], lf0 = m.ae_lf[2 * ae];
    const ColData &d0 = cols[c0], &d1 = cols[c1];
    // canonical face = local face lf0 of side 0, outward from side 0
    for (int qq = 0; qq < Q; qq++) {
        for (int i = 0; i < 3; i++) hg.fnA[((size_t)ae * Q + qq) * 3 + i] = d0.fn[lf0][qq][i];
        hg.fwA[(size_t)ae * Q + qq] = d0.fdA[lf0][qq] / d0.farea[lf0];
        double X0[3], X1[3];
        for (int d = 0; d < 3; d++) {
            X0[d] = (d0.fx[lf0][qq][d] - d0.cen[d]) / d0.len;
            X1[d] = (d0.fx[lf0][qq][d] - d1.cen[d]) / d1.len;
        }
        for (int a = 0; a < NC; a++) {
            hg.fevA[(((size_t)ae * 2 + 0) * Q + qq) * NC + a] = tbasis(d0.mom, r.tex[a], X0);
            hg.fevA[(((size_t)ae * 2 + 1) * Q + qq) * NC + a] = tbasis(d1.mom, r.tex[a], X1);
        }
    }
    // edge curve at interface 0 from side 0's map, canonical direction a -> b
    int le = LF_EDGE[lf0];
    int from = m.col_v[4 * c0 + LF_FROMTO[lf0][0]];
    bool rev = (from != m.ae_v[2 * ae]);
    const double simpson[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    double xm[3], tm[3];
    double pts[3][3], tan[3][3];
    for (int s = 0; s < 3; s++) {
        double xi[3], jac[9];
        edge_ref_point(le, rev ? 1.0 - 0.5 * s : 0.5 * s, xi);
        zone_map(m.map_order, d0.sn, m.radius[0], m.radius[1], xi, pts[s], jac);
        for (int i = 0; i < 3; i++) tan[s][i] = (rev ? -1.0 : 1.0) * jac[i * 3 + le / 4];
        double a = std::sqrt(dot(tan[s], tan[s]));
        hg.aeW[(size_t)ae * 3 + s] = simpson[s] * a;
        for (int i = 0; i < 3; i++) tan[s][i] /= a;
    }
    std::memcpy(xm, pts[1], 24);
    std::memcpy(tm, tan[1], 24);
    // which column lies to the right (t x r_hat)
    double rh[3] = {xm[0], xm[1], xm[2]}, mh[3];
    normalize(rh);
    cross(tm, rh, mh);
    double dc[3] = {d1.cen[0] - xm[0], d1.cen[1] - xm[1], d1.cen[2] - xm[2]};
    bool side1_right = dot(dc, mh) > 0;
    hg.ae_rs[ae] = side1_right ? 1 : -1;
    const ColData &L = side1_right ? d0 : d1, &Rr = side1_right ? d1 : d0;
    // zones about the edge at interface 1, counter-clockwise: (L,0) (L,1) (R,1) (R,0)
    const double q = m.q;
    double cz[4][3];
    for (int i = 0; i < 3; i++) {
        cz[0][i] = L.cen[i];
        cz[1][i] = q * L.cen[i];
        cz[2][i] = q * Rr.cen[i];
        cz[3][i] = Rr.cen[i];
    }
    double u[3], w[3];
    for (int i = 0; i < 3; i++) {
        u[i] = cz[1][i] + cz[2][i] - cz[0][i] - cz[3][i];
        w[i] = cz[2][i] + cz[3][i] - cz[0][i] - cz[1][i];
    }
    for (int s = 0; s < 3; s++) {
        double *F = &hg.aeF[((size_t)ae * 3 + s) * 9];
        symmetric_frame(u, w, tan[s], F, F + 3);
        std::memcpy(F + 6, tan[s], 24);
    }
    std::memcpy(&hg.emid_ae[(size_t)ae * 3], xm, 24);
    std::memcpy(&hg.etan_ae[(size_t)ae * 3], tm, 24);
    // face centre / normal of the canonical angular face at shell 0
    std::memcpy(&hg.fcen_ae[(size_t)ae * 3], d0.fcen[lf0], 24);
    std::memcpy(&hg.fnrm_ae[(size_t)ae * 3], d0.fnbar[lf0], 24);
    hg.farea_ae[ae] = d0.farea[lf0];
}

void vertex_pass(const Mesh &m, const RefEl &r, const std::vector<ColData> &cols, int v, HostGeom &hg)
{
    (void)r;
    const double *t = &m.vpos[3 * v];
    int n = m.v_ncol[v];
    double *F = &hg.vF[(size_t)v * 9];
    std::fill(F, F + 9, 0.0);
    std::memcpy(F + 6, t, 24);
    std::fill(&hg.vN3[(size_t)v * 9], &hg.vN3[(size_t)v * 9] + 9, 0.0);
    if (n == 4) {
        const double *c[4];
        for (int s = 0; s < 4; s++) c[s] = cols[m.v_col[4 * v + s]].cen;
        double u[3], w[3];
        for (int i = 0; i < 3; i++) {
            u[i] = c[1][i] + c[2][i] - c[0][i] - c[3][i];
            w[i] = c[2][i] + c[3][i] - c[0][i] - c[1][i];
        }
        symmetric_frame(u, w, t, F, F + 3);
    } else {
        // normals of the angular faces between consecutive columns, along the radial line
        for (int s = 0; s < n; s++) {
            int ca = m.v_col[4 * v + s], cb = m.v_col[4 * v + (s + 1) % n];
            int ae = -1, lfa = -1;
            for (int lf = 0; lf < 4; lf++) {
                int e = m.col_ae[4 * ca + lf];
                int other = (m.ae_col[2 * e] == ca) ? m.ae_col[2 * e + 1] : m.ae_col[2 * e];
                if (other == cb) { ae = e; lfa = lf; }
            }
            (void)ae;
            // tangent of that face's angular edge at the vertex, from column ca's map
            int le = LF_EDGE[lfa];
            int cf = m.col_v[4 * ca + LF_FROMTO[lfa][0]];
            double sv = (cf == v) ? 0.0 : 1.0, xi[3], x[3], jac[9], tg[3], nn[3];
            edge_ref_point(le, sv, xi);
            zone_map(m.map_order, cols[ca].sn, m.radius[0], m.radius[1], xi, x, jac);
            for (int i = 0; i < 3; i++) tg[i] = jac[i * 3 + le / 4];
            cross(tg, t, nn);
            normalize(nn);
            double dc[3];
            for (int i = 0; i < 3; i++) dc[i] = cols[cb].cen[i] - cols[ca].cen[i];
            if (dot(nn, dc) < 0)
                for (int i = 0; i < 3; i++) nn[i] = -nn[i];
            std::memcpy(&hg.vN3[(size_t)v * 9 + s * 3], nn, 24);
        }
    }
}

// per-column edge bookkeeping: local edge -> slot about the edge, reversal;
// circulation signs of the angular edges about +r
void column_pass4(const Mesh &m, const HostGeom &hg, int c, HostGeom &out)
{
    // local edges 0..7 are angular (on local faces eta-/eta+/xi-/xi+ at zeta-/zeta+)
    const int LE_FACE[8] = {2, 3, 2, 3, 0, 1, 0, 1};
    const int LE_ZUP[8] = {0, 0, 1, 1, 0, 0, 1, 1};
    for (int le = 0; le < 8; le++) {
        int lf = LE_FACE[le];
        int ae = m.col_ae[4 * c + lf];
        int from = m.col_v[4 * c + LF_FROMTO[lf][0]];
        int rev = (from != m.ae_v[2 * ae]);
        bool isRight = (hg.ae_rs[ae] > 0) == (m.ae_col[2 * ae + 1] == c);
        // zone above the interface for zeta- edges, below it for zeta+ edges
        int slot = LE_ZUP[le] == 0 ? (isRight ? 2 : 1) : (isRight ? 3 : 0);
        out.col_slot[(size_t)c * 12 + le] = slot;
        out.col_rev[(size_t)c * 12 + le] = rev;
    }
    const int LE_CORNER[4] = {0, 1, 3, 2};
    for (int k = 0; k < 4; k++) {
        int v = m.col_v[4 * c + LE_CORNER[k]];
        int slot = 0;
        for (int s = 0; s < m.v_ncol[v]; s++)
            if (m.v_col[4 * v + s] == c) slot = s;
        out.col_slot[(size_t)c * 12 + 8 + k] = slot;
        out.col_rev[(size_t)c * 12 + 8 + k] = 0;
    }
    // counter-clockwise traversal v0 -> v1 -> v2 -> v3 about +r
    const int TRAV[4][2] = {{3, 0}, {1, 2}, {0, 1}, {2, 3}};
    for (int lf = 0; lf < 4; lf++) {
        int ae = m.col_ae[4 * c + lf];
        int from = m.col_v[4 * c + TRAV[lf][0]];
        out.col_sgn[(size_t)c * 4 + lf] = (from == m.ae_v[2 * ae]) ? 1 : -1;
    }
    for (int k = 0; k < 4; k++) out.col_v[(size_t)c * 4 + k] = m.col_v[4 * c + k];
}

}  // namespace rg

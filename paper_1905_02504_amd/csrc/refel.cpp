// Reference element of the library (host, FP64):
//  - hexahedral serendipity element on [-1/2,1/2]^3 (Section V.b transposed to
//    hexahedra): vertices plus equidistant edge nodes, monomials of
//    superlinear degree <= p-1, nodal Lagrange basis by eq. (5.3);
//  - nodal derivative matrices D_d (the space is closed under
//    differentiation, so the space-time Galerkin system of eqs. (5.24)-(5.29)
//    factors into R (x) D, cf. eqs. (C.34)-(C.36) and (D.29)-(D.32));
//  - time levels tau = 0 plus Gauss points (eqs. 5.15-5.17) and the 1-D time
//    Galerkin matrix R = (K_tau^11)^-1 M^1. (printed as B.9, C.18, D.28);
//  - Taylor-basis multi-indices (eq. 3.1) and the divergence-free B basis of
//    eqs. (4.1)/(4.4)/(4.7) generalised to degree p (each component carries
//    all monomials of degree <= p-1 plus the degree-p monomials containing
//    its own coordinate);
//  - interpolation weights from nodal values to face quadrature points and
//    edge Simpson points.
#include <cmath>

#include "rg_internal.hpp"

namespace rg {

void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 200; it++) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dx = p1 / dp;
            t -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        x[i] = 0.5 * (1.0 - t);
        w[i] = 1.0 / ((1.0 - t * t) * dp * dp);
    }
}

bool lu_factor(int n, std::vector<double> &A, std::vector<int> &piv)
{
    piv.resize(n);
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = std::fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; i++)
            if (std::fabs(A[(size_t)i * n + k]) > best) { best = std::fabs(A[(size_t)i * n + k]); p = i; }
        if (best == 0.0) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; j++) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
        double inv = 1.0 / A[(size_t)k * n + k];
        for (int i = k + 1; i < n; i++) {
            double f = A[(size_t)i * n + k] * inv;
            A[(size_t)i * n + k] = f;
            if (f != 0.0)
                for (int j = k + 1; j < n; j++) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
        }
    }
    return true;
}

// the factorisation swapped whole rows, so apply every interchange first
void lu_solve(int n, const std::vector<double> &LU, const std::vector<int> &piv, double *b)
{
    for (int k = 0; k < n; k++) std::swap(b[k], b[piv[k]]);
    for (int i = 1; i < n; i++) {
        double s = b[i];
        for (int j = 0; j < i; j++) s -= LU[(size_t)i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < n; j++) s -= LU[(size_t)i * n + j] * b[j];
        b[i] = s / LU[(size_t)i * n + i];
    }
}

static double monomial(const std::array<int, 3> &e, const double *x)
{
    double v = 1.0;
    for (int d = 0; d < 3; d++) v *= std::pow(x[d], e[d]);
    return v;
}

static double monomial_d(const std::array<int, 3> &e, int dir, const double *x)
{
    if (e[dir] == 0) return 0.0;
    double v = e[dir];
    for (int d = 0; d < 3; d++) v *= std::pow(x[d], e[d] - (d == dir));
    return v;
}

double RefEl::psi(int l, const double *xi) const
{
    double s = 0.0;
    for (int k = 0; k < N; k++) s += coef[(size_t)k * N + l] * monomial(sexp[k], xi);
    return s;
}

double RefEl::dpsi(int l, int d, const double *xi) const
{
    double s = 0.0;
    for (int k = 0; k < N; k++) s += coef[(size_t)k * N + l] * monomial_d(sexp[k], d, xi);
    return s;
}

// local faces: 0 xi-, 1 xi+, 2 eta-, 3 eta+, 4 zeta-, 5 zeta+; face parameters
// (u, v) = (eta, zeta), (xi, zeta), (xi, eta); point q = qu + Q1 * qv
void face_ref_point(const RefEl &r, int lf, int q, double *xi)
{
    double u = r.gq[q % r.Q1] - 0.5, v = r.gq[q / r.Q1] - 0.5;
    double fix = (lf & 1) ? 0.5 : -0.5;
    int axis = lf / 2;
    if (axis == 0) { xi[0] = fix; xi[1] = u; xi[2] = v; }
    else if (axis == 1) { xi[0] = u; xi[1] = fix; xi[2] = v; }
    else { xi[0] = u; xi[1] = v; xi[2] = fix; }
}

// local edges: 0-3 along xi at (eta, zeta) = (-,-), (+,-), (-,+), (+,+);
// 4-7 along eta at (xi, zeta); 8-11 along zeta at (xi, eta); s in [0,1]
void edge_ref_point(int le, double s, double *xi)
{
    int axis = le / 4, c = le % 4;
    int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    xi[axis] = s - 0.5;
    xi[a1] = (c & 1) ? 0.5 : -0.5;
    xi[a2] = (c & 2) ? 0.5 : -0.5;
}

// time levels tau = 0 plus M-1 Gauss points (eqs. 5.15-5.17), their Gauss
// weights (wt[0] = 0) and the 1-D time Galerkin matrix R = (K_tau^11)^-1 M^1
// ((M-1) x M; printed as B.9, C.18, D.28)
bool time_galerkin(int M, std::vector<double> &tau, std::vector<double> &wt, std::vector<double> &R)
{
    const int p = M;
    tau.assign(p, 0.0);
    wt.assign(p, 0.0);
    gauss_legendre01(p - 1, &tau[1], &wt[1]);
    {
        const int nq = 8;
        double tx[8], tw[8];
        gauss_legendre01(nq, tx, tw);
        auto phi = [&](int j, double t) {
            double v = 1.0;
            for (int k = 0; k < M; k++)
                if (k != j) v *= (t - tau[k]) / (tau[j] - tau[k]);
            return v;
        };
        auto dphi = [&](int j, double t) {
            double s = 0.0;
            for (int k = 0; k < M; k++) {
                if (k == j) continue;
                double v = 1.0 / (tau[j] - tau[k]);
                for (int m = 0; m < M; m++)
                    if (m != j && m != k) v *= (t - tau[m]) / (tau[j] - tau[m]);
                s += v;
            }
            return s;
        };
        int E = M - 1;
        std::vector<double> K11((size_t)E * E, 0.0), M1((size_t)E * M, 0.0);
        for (int a = 0; a < nq; a++)
            for (int j = 1; j < M; j++) {
                for (int l = 1; l < M; l++) K11[(j - 1) * E + (l - 1)] += tw[a] * phi(j, tx[a]) * dphi(l, tx[a]);
                for (int l = 0; l < M; l++) M1[(j - 1) * M + l] += tw[a] * phi(j, tx[a]) * phi(l, tx[a]);
            }
        std::vector<int> pv;
        if (!lu_factor(E, K11, pv)) return false;
        R.assign((size_t)E * M, 0.0);
        for (int l = 0; l < M; l++) {
            std::vector<double> col(E);
            for (int j = 0; j < E; j++) col[j] = M1[j * M + l];
            lu_solve(E, K11, pv, col.data());
            for (int j = 0; j < E; j++) R[j * M + l] = col[j];
        }
    }
    return true;
}

bool build_refel(int order, RefEl &r)
{
    if (order != 3 && order != 4) return false;
    r.order = order;
    const int p = order;
    // nodes
    r.node.clear();
    for (int v = 0; v < 8; v++)
        r.node.push_back({(v & 1) ? 0.5 : -0.5, (v & 2) ? 0.5 : -0.5, (v & 4) ? 0.5 : -0.5});
    for (int axis = 0; axis < 3; axis++) {
        int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
        for (int c = 0; c < 4; c++)
            for (int k = 1; k <= p - 2; k++) {
                std::array<double, 3> x{};
                x[axis] = -0.5 + double(k) / (p - 1);
                x[a1] = (c & 1) ? 0.5 : -0.5;
                x[a2] = (c & 2) ? 0.5 : -0.5;
                r.node.push_back(x);
            }
    }
    r.N = (int)r.node.size();
    // serendipity monomials: superlinear degree <= p - 1
    r.sexp.clear();
    for (int a = 0; a <= p; a++)
        for (int b = 0; b <= p; b++)
            for (int c = 0; c <= p; c++) {
                int lin = (a == 1) + (b == 1) + (c == 1);
                if (a + b + c - lin <= p - 1) r.sexp.push_back({a, b, c});
            }
    if ((int)r.sexp.size() != r.N) return false;
    const int N = r.N;
    // Lagrange basis: coef = V^-1 with V[i][k] = m_k(node_i)
    std::vector<double> V((size_t)N * N);
    for (int i = 0; i < N; i++)
        for (int k = 0; k < N; k++) V[(size_t)i * N + k] = monomial(r.sexp[k], r.node[i].data());
    std::vector<int> piv;
    if (!lu_factor(N, V, piv)) return false;
    r.coef.assign((size_t)N * N, 0.0);
    for (int l = 0; l < N; l++) {
        std::vector<double> e(N, 0.0);
        e[l] = 1.0;
        lu_solve(N, V, piv, e.data());
        for (int k = 0; k < N; k++) r.coef[(size_t)k * N + l] = e[k];
    }
    r.D.assign((size_t)3 * N * N, 0.0);
    for (int d = 0; d < 3; d++)
        for (int i = 0; i < N; i++)
            for (int l = 0; l < N; l++) {
                // entries are exact multiples of 1/2; remove the rounding of the inversion
                double v = r.dpsi(l, d, r.node[i].data()), h = std::round(2.0 * v) / 2.0;
                r.D[((size_t)d * N + i) * N + l] = std::fabs(v - h) < 1e-9 ? h : v;
            }

    // time levels and the 1-D time Galerkin matrix
    r.M = p;
    if (!time_galerkin(p, r.tau, r.wt, r.R)) return false;

    // Taylor basis multi-indices of degree 1..p-1
    r.tex.clear();
    for (int d = 1; d <= p - 1; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) r.tex.push_back({a, b, d - a - b});
    r.NC = (int)r.tex.size();
    for (int c = 0; c < 3; c++) {
        r.bex[c].clear();
        r.bex[c].push_back({0, 0, 0});
        for (auto &e : r.tex) r.bex[c].push_back(e);
        for (int a = p; a >= 0; a--)
            for (int b = p - a; b >= 0; b--) {
                std::array<int, 3> e{a, b, p - a - b};
                if (e[c] >= 1) r.bex[c].push_back(e);
            }
    }
    r.NB = (int)r.bex[0].size();

    r.Q1 = p - 1;
    r.Q = r.Q1 * r.Q1;
    r.gq.resize(r.Q1);
    r.gw.resize(r.Q1);
    gauss_legendre01(r.Q1, r.gq.data(), r.gw.data());
    r.NS = (p == 3) ? 26 : 32;
    r.NIN = 3 * (r.NC + 1) + 6 * r.Q + 6;
    r.NOUTB = 3 * N + 3;

    // nodes on faces and edges, and interpolation weights
    r.NFN = 4 * (p - 1);
    r.NEN = p;
    r.fnode.assign(6 * r.NFN, -1);
    r.fint.assign((size_t)6 * r.Q * r.NFN, 0.0);
    // Face nodes are listed in one order for every face: by their position in
    // the face's two free coordinates (lower axis first), as found on face 0.
    // The weights at the face quadrature points are then the same for all six
    // faces (fintc), which the predictor relies on.
    for (int lf = 0; lf < 6; lf++) {
        int axis = lf / 2, ua = axis == 0 ? 1 : 0, va = axis == 2 ? 1 : 2;
        double fix = (lf & 1) ? 0.5 : -0.5;
        for (int k = 0; k < r.NFN; k++) {
            int n = 0;
            if (lf == 0) {
                for (int l = 0; l < N; l++)
                    if (r.node[l][0] == -0.5 && n++ == k) r.fnode[k] = l;
                continue;
            }
            const auto &ref = r.node[r.fnode[k]];
            for (int l = 0; l < N; l++)
                if (r.node[l][axis] == fix && r.node[l][ua] == ref[1] && r.node[l][va] == ref[2]) {
                    r.fnode[lf * r.NFN + k] = l;
                    n++;
                }
            if (n != 1) return false;
        }
        for (int k = 0; k < r.NFN; k++)
            if (r.fnode[lf * r.NFN + k] < 0) return false;
        for (int q = 0; q < r.Q; q++) {
            double xi[3];
            face_ref_point(r, lf, q, xi);
            for (int k = 0; k < r.NFN; k++) r.fint[((size_t)lf * r.Q + q) * r.NFN + k] = r.psi(r.fnode[lf * r.NFN + k], xi);
        }
    }
    r.fintc.assign((size_t)r.NFN * r.Q, 0.0);
    for (int k = 0; k < r.NFN; k++)
        for (int q = 0; q < r.Q; q++) r.fintc[(size_t)k * r.Q + q] = r.fint[(size_t)q * r.NFN + k];
    for (int lf = 1; lf < 6; lf++)
        for (int q = 0; q < r.Q; q++)
            for (int k = 0; k < r.NFN; k++)
                if (std::abs(r.fint[((size_t)lf * r.Q + q) * r.NFN + k] - r.fintc[(size_t)k * r.Q + q]) > 1e-13) return false;
    r.enode.assign(12 * r.NEN, -1);
    r.eint.assign((size_t)12 * 3 * r.NEN, 0.0);
    for (int le = 0; le < 12; le++) {
        int axis = le / 4, c = le % 4;
        int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
        double f1 = (c & 1) ? 0.5 : -0.5, f2 = (c & 2) ? 0.5 : -0.5;
        int n = 0;
        for (int l = 0; l < N; l++)
            if (r.node[l][a1] == f1 && r.node[l][a2] == f2) r.enode[le * r.NEN + n++] = l;
        if (n != r.NEN) return false;
        for (int s = 0; s < 3; s++) {
            double xi[3];
            edge_ref_point(le, 0.5 * s, xi);
            for (int k = 0; k < r.NEN; k++) r.eint[((size_t)le * 3 + s) * r.NEN + k] = r.psi(r.enode[le * r.NEN + k], xi);
        }
    }
    // edge nodes are listed by index, which orders them alike along every
    // edge; the Simpson-point weights are therefore shared (eintc)
    r.eintc.assign((size_t)r.NEN * 3, 0.0);
    for (int k = 0; k < r.NEN; k++)
        for (int s = 0; s < 3; s++) r.eintc[(size_t)k * 3 + s] = r.eint[(size_t)s * r.NEN + k];
    for (int le = 1; le < 12; le++)
        for (int s = 0; s < 3; s++)
            for (int k = 0; k < r.NEN; k++)
                if (std::abs(r.eint[((size_t)le * 3 + s) * r.NEN + k] - r.eintc[(size_t)k * 3 + s]) > 1e-13) return false;
    return true;
}

}  // namespace rg

// Icosahedral geodesic prism mesh of the library (host, FP64) and the C-ABI
// of the prism element:
//  - mesh of Section II.a: the projected icosahedron split level times at
//    great-circle edge midpoints;
//  - per column (triangle), the curved-prism map of Section II.b for a unit
//    shell with radii 1 and q = (r_out / r_in)^(1 / n_rad): a triangle
//    Lagrange interpolant of degree p-1 through sphere points (vertices,
//    equidistant great-circle points on the edges, the spherical centroid
//    where the medians meet) times a linear radial factor.  Shell k is that
//    shell scaled by r_k, so J scales by r_k^3 and the metrics by r_k^2.
//    Metrics J d xi_d / d x_n at the nodes in the conservative curl form.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <new>
#include <string>

#include "prism.hpp"
#include "prism_dtab.hpp"
#include "rg_geom_host.hpp"
#include "rg_internal.hpp"

namespace rg {

// compiled-in sparse tables of the kernels against the computed matrices
static bool prism_tables_match(const PrismRef &r)
{
    const int N = r.N;
    std::vector<double> T((size_t)3 * N * N, 0.0);
    auto fill = [&](int d, int nnz, const short (*e)[2], const double *v) {
        for (int k = 0; k < nnz; k++) T[((size_t)d * N + e[k][0]) * N + e[k][1]] = v[k];
    };
    if (r.order == 2) {
        fill(0, PrismD<2>::NZ0, PrismD<2>::E0, PrismD<2>::V0);
        fill(1, PrismD<2>::NZ1, PrismD<2>::E1, PrismD<2>::V1);
        fill(2, PrismD<2>::NZ2, PrismD<2>::E2, PrismD<2>::V2);
    } else if (r.order == 3) {
        fill(0, PrismD<3>::NZ0, PrismD<3>::E0, PrismD<3>::V0);
        fill(1, PrismD<3>::NZ1, PrismD<3>::E1, PrismD<3>::V1);
        fill(2, PrismD<3>::NZ2, PrismD<3>::E2, PrismD<3>::V2);
    } else {
        fill(0, PrismD<4>::NZ0, PrismD<4>::E0, PrismD<4>::V0);
        fill(1, PrismD<4>::NZ1, PrismD<4>::E1, PrismD<4>::V1);
        fill(2, PrismD<4>::NZ2, PrismD<4>::E2, PrismD<4>::V2);
    }
    for (size_t k = 0; k < T.size(); k++)
        if (std::fabs(T[k] - r.D[k]) > 1e-13) return false;
    return true;
}

}  // namespace rg

using namespace rg;

struct rg_prism {
    int level = 0, n_rad = 0, order = 0;
    double r_in = 0, r_out = 0, q = 0;
    int64_t ntri = 0, nz = 0;
    PrismRef ref;
    std::vector<double> tri;       // ntri x 9: vertices a, b, c of each triangle
    std::vector<double> radius;    // n_rad + 1
    std::vector<double> hx, hJ, hM;  // unit-shell nodes ntri x N x 3, J ntri x N, metrics ntri x 9 x N
    std::vector<int> edges, mirror;   // nedges x 4; QS
    std::vector<int> tedge;           // ntri x 3
    std::vector<double> vol;          // ntri, unit shell
    std::vector<double> Mb;           // ntri x nout x nin, built on first use
    int nin = 0, nout = 0;
    std::mutex mb_mutex;              // the first divergence-free call builds (and uploads) the maps
    std::vector<double> tfA, sfA;     // ntri x QT x 3; ntri x 3 x QS x 3
    // constrained transport
    std::vector<int> tri_v, edge_ab, ring_off, ring_tj, eidx;
    std::vector<double> vxyz, ring_n, aeg, eval;
    std::vector<void *> allocations;
    bool device = false;
    DevPrism dev{};
};

namespace {

void free_prism(rg_prism *p)
{
    if (!p) return;
    for (void *a : p->allocations) (void)hipFree(a);
    delete p;
}

template <class T>
bool upload(rg_prism *p, const std::vector<T> &h, const T **dst)
{
    void *d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(8, h.size() * sizeof(T))) != hipSuccess) return false;
    p->allocations.push_back(d);
    if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return false;
    *dst = static_cast<const T *>(d);
    return true;
}

void unit(double *v)
{
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

// the 20 level-0 triangles, each counter-clockwise seen from outside
void icosahedron(std::vector<double> &tri)
{
    double V[12][3];
    const double h = 1.0 / std::sqrt(5.0), rho = 2.0 / std::sqrt(5.0);
    V[0][0] = 0; V[0][1] = 0; V[0][2] = 1;
    V[11][0] = 0; V[11][1] = 0; V[11][2] = -1;
    for (int k = 0; k < 5; k++) {
        const double up = 2 * M_PI * k / 5, lo = 2 * M_PI * (k + 0.5) / 5;
        V[1 + k][0] = rho * std::cos(up); V[1 + k][1] = rho * std::sin(up); V[1 + k][2] = h;
        V[6 + k][0] = rho * std::cos(lo); V[6 + k][1] = rho * std::sin(lo); V[6 + k][2] = -h;
    }
    tri.clear();
    for (int k = 0; k < 5; k++) {
        const int k1 = (k + 1) % 5;
        const int F[4][3] = {{0, 1 + k, 1 + k1}, {1 + k, 6 + k, 1 + k1}, {1 + k1, 6 + k, 6 + k1}, {11, 6 + k1, 6 + k}};
        for (auto &f : F) {
            const double *a = V[f[0]], *b = V[f[1]], *c = V[f[2]];
            double u[3], w[3], n[3];
            for (int i = 0; i < 3; i++) { u[i] = b[i] - a[i]; w[i] = c[i] - a[i]; }
            n[0] = u[1] * w[2] - u[2] * w[1];
            n[1] = u[2] * w[0] - u[0] * w[2];
            n[2] = u[0] * w[1] - u[1] * w[0];
            const double o = n[0] * (a[0] + b[0] + c[0]) + n[1] * (a[1] + b[1] + c[1]) + n[2] * (a[2] + b[2] + c[2]);
            const double *s1 = o < 0 ? c : b, *s2 = o < 0 ? b : c;
            tri.insert(tri.end(), a, a + 3);
            tri.insert(tri.end(), s1, s1 + 3);
            tri.insert(tri.end(), s2, s2 + 3);
        }
    }
}

// children of every triangle: (a, m_ab, m_ca), (m_ab, b, m_bc),
// (m_ca, m_bc, c), (m_ab, m_bc, m_ca) with m = (u + v) / |u + v|
void split(std::vector<double> &tri)
{
    const size_t nt = tri.size() / 9;
    std::vector<double> out(nt * 36);
    for (size_t t = 0; t < nt; t++) {
        const double *a = &tri[9 * t], *b = a + 3, *c = a + 6;
        double ab[3], bc[3], ca[3];
        for (int i = 0; i < 3; i++) { ab[i] = a[i] + b[i]; bc[i] = b[i] + c[i]; ca[i] = c[i] + a[i]; }
        unit(ab); unit(bc); unit(ca);
        const double *ch[4][3] = {{a, ab, ca}, {ab, b, bc}, {ca, bc, c}, {ab, bc, ca}};
        for (int k = 0; k < 4; k++)
            for (int v = 0; v < 3; v++) std::memcpy(&out[36 * t + 9 * k + 3 * v], ch[k][v], 24);
    }
    tri.swap(out);
}

// unit-shell geometry of one column: nodes x[N][3], J[N], metrics M[9][N]
void column_geometry(const PrismRef &r, const double *abc, double q, double *x, double *J, double *M)
{
    const int N = r.N, mo = r.order - 1;
    std::vector<std::array<int, 3>> bary;
    std::vector<std::array<double, 3>> lx;
    lattice(mo, bary, lx);
    const int nl = (int)lx.size();
    // sphere point of every lattice node
    std::vector<double> sp((size_t)nl * 3);
    const double *P[3] = {abc, abc + 3, abc + 6};
    for (int a = 0; a < nl; a++) {
        double *o = &sp[3 * a];
        const auto &bc = bary[a];
        const int nz = (bc[0] == 0) + (bc[1] == 0) + (bc[2] == 0);
        if (nz == 2) {
            std::memcpy(o, P[bc[0] ? 0 : bc[1] ? 1 : 2], 24);
        } else if (nz == 1) {
            const int u = bc[0] ? 0 : 1, w = bc[2] ? 2 : 1;
            arc_point(P[u], P[w], double(bc[w]) / (bc[u] + bc[w]), o);
        } else {
            for (int i = 0; i < 3; i++) o[i] = P[0][i] + P[1][i] + P[2][i];
            unit(o);
        }
    }
    // derivatives of the triangle interpolant at the lattice nodes
    std::vector<std::array<int, 3>> tmo;
    for (int deg = 0; deg <= mo; deg++)
        for (int a = deg; a >= 0; a--) tmo.push_back({a, deg - a, 0});
    std::vector<double> C, TD;
    lagrange_coefficients(lx, tmo, C);
    derivative_matrices(lx, tmo, C, TD);   // TD[d][a][b], d = 0, 1 used
    std::vector<double> jac((size_t)N * 9);
    double cen[3] = {0, 0, 0};
    for (int i = 0; i < N; i++) {
        const int a = r.lat[i];
        const double z = r.node[i][2], Rz = (0.5 - z) + (0.5 + z) * q, dR = q - 1.0;
        double Sx[3] = {0, 0, 0}, Sy[3] = {0, 0, 0};
        for (int b = 0; b < nl; b++) {
            const double gx = TD[((size_t)0 * nl + a) * nl + b], gy = TD[((size_t)1 * nl + a) * nl + b];
            for (int k = 0; k < 3; k++) { Sx[k] += gx * sp[3 * b + k]; Sy[k] += gy * sp[3 * b + k]; }
        }
        for (int k = 0; k < 3; k++) {
            x[3 * i + k] = Rz * sp[3 * a + k];
            jac[9 * i + 3 * k + 0] = Rz * Sx[k];
            jac[9 * i + 3 * k + 1] = Rz * Sy[k];
            jac[9 * i + 3 * k + 2] = dR * sp[3 * a + k];
            cen[k] += x[3 * i + k] / N;
        }
        const double *j = &jac[9 * i];
        J[i] = j[0] * (j[4] * j[8] - j[5] * j[7]) - j[1] * (j[3] * j[8] - j[5] * j[6]) + j[2] * (j[3] * j[7] - j[4] * j[6]);
    }
    // curl form: with W_n[j] = (x_{n+2} - c) d x_{n+1} / d xi_j interpolated
    // in the element's basis, J d xi_d / d x_n = -(curl_xi W_n)_d
    for (int n = 0; n < 3; n++) {
        const int m1 = (n + 1) % 3, m2 = (n + 2) % 3;
        std::vector<double> W((size_t)N * 3);
        for (int i = 0; i < N; i++)
            for (int j = 0; j < 3; j++) W[3 * i + j] = (x[3 * i + m2] - cen[m2]) * jac[9 * i + 3 * m1 + j];
        for (int i = 0; i < N; i++) {
            double g[3][3] = {{0}};   // g[j][d] = d W_j / d xi_d at node i
            for (int l = 0; l < N; l++)
                for (int d = 0; d < 3; d++) {
                    const double w = r.D[((size_t)d * N + i) * N + l];
                    if (w == 0.0) continue;
                    for (int j = 0; j < 3; j++) g[j][d] += w * W[3 * l + j];
                }
            M[(0 * 3 + n) * N + i] = -(g[2][1] - g[1][2]);
            M[(1 * 3 + n) * N + i] = -(g[0][2] - g[2][0]);
            M[(2 * 3 + n) * N + i] = -(g[1][0] - g[0][1]);
        }
    }
}

// The sphere interpolant S(xi, eta) of one triangle: Lagrange through the
// lattice of degree p-1 mapped to the sphere (vertices, great-circle edge
// points, the spherical centroid), with its (xi, eta) derivatives.
struct TriSurface {
    int nl = 0;
    std::vector<double> sp, C;
    std::vector<std::array<int, 3>> tmo;
    TriSurface(const PrismRef &r, const double *abc)
    {
        const int mo = r.order - 1;
        std::vector<std::array<int, 3>> bary;
        std::vector<std::array<double, 3>> lx;
        lattice(mo, bary, lx);
        nl = (int)lx.size();
        sp.assign((size_t)nl * 3, 0.0);
        const double *P[3] = {abc, abc + 3, abc + 6};
        for (int a = 0; a < nl; a++) {
            double *o = &sp[3 * a];
            const auto &bc = bary[a];
            const int nz = (bc[0] == 0) + (bc[1] == 0) + (bc[2] == 0);
            if (nz == 2) std::memcpy(o, P[bc[0] ? 0 : bc[1] ? 1 : 2], 24);
            else if (nz == 1) {
                const int u = bc[0] ? 0 : 1, w = bc[2] ? 2 : 1;
                arc_point(P[u], P[w], double(bc[w]) / (bc[u] + bc[w]), o);
            } else {
                for (int i = 0; i < 3; i++) o[i] = P[0][i] + P[1][i] + P[2][i];
                unit(o);
            }
        }
        for (int deg = 0; deg <= mo; deg++)
            for (int a = deg; a >= 0; a--) tmo.push_back({a, deg - a, 0});
        lagrange_coefficients(lx, tmo, C);
    }
    void eval(const double *xi, double *S, double *Sx, double *Sy) const
    {
        for (int k = 0; k < 3; k++) S[k] = Sx[k] = Sy[k] = 0.0;
        for (int b = 0; b < nl; b++) {
            double L = 0.0, Lx = 0.0, Ly = 0.0;
            for (int m = 0; m < nl; m++) {
                const double c = C[(size_t)m * nl + b];
                if (c == 0.0) continue;
                const int ex = tmo[m][0], ey = tmo[m][1];
                L += c * std::pow(xi[0], ex) * std::pow(xi[1], ey);
                if (ex) Lx += c * ex * std::pow(xi[0], ex - 1) * std::pow(xi[1], ey);
                if (ey) Ly += c * ey * std::pow(xi[0], ex) * std::pow(xi[1], ey - 1);
            }
            for (int k = 0; k < 3; k++) {
                S[k] += L * sp[3 * b + k];
                Sx[k] += Lx * sp[3 * b + k];
                Sy[k] += Ly * sp[3 * b + k];
            }
        }
    }
};

// Face geometry of one column for the unit shell: the triangle-face area
// vectors at radius 1, (sqrt 3 / 4) w_q (S_xi x S_eta), which point along +r
// for a counter-clockwise triangle, and the side faces' outward area vectors
// w_q R(zeta) (q - 1) (S_s x S) with s along the edge from vertex k to k + 1;
// S is the triangle's sphere interpolant (reading of the map as in
// column_geometry).
void column_face_geometry(const PrismRef &r, const double *abc, double q, double *tfA, double *sfA)
{
    const int mo = r.order - 1;
    std::vector<std::array<int, 3>> bary;
    std::vector<std::array<double, 3>> lx;
    lattice(mo, bary, lx);
    const int nl = (int)lx.size();
    std::vector<double> sp((size_t)nl * 3);
    const double *P[3] = {abc, abc + 3, abc + 6};
    for (int a = 0; a < nl; a++) {
        double *o = &sp[3 * a];
        const auto &bc = bary[a];
        const int nz = (bc[0] == 0) + (bc[1] == 0) + (bc[2] == 0);
        if (nz == 2) {
            std::memcpy(o, P[bc[0] ? 0 : bc[1] ? 1 : 2], 24);
        } else if (nz == 1) {
            const int u = bc[0] ? 0 : 1, w = bc[2] ? 2 : 1;
            arc_point(P[u], P[w], double(bc[w]) / (bc[u] + bc[w]), o);
        } else {
            for (int i = 0; i < 3; i++) o[i] = P[0][i] + P[1][i] + P[2][i];
            unit(o);
        }
    }
    std::vector<std::array<int, 3>> tmo;
    for (int deg = 0; deg <= mo; deg++)
        for (int a = deg; a >= 0; a--) tmo.push_back({a, deg - a, 0});
    std::vector<double> C;
    lagrange_coefficients(lx, tmo, C);
    // S and its (xi, eta) derivatives at a reference point
    auto surf = [&](const double *xi, double *S, double *Sx, double *Sy) {
        for (int k = 0; k < 3; k++) S[k] = Sx[k] = Sy[k] = 0.0;
        for (int b = 0; b < nl; b++) {
            double L = 0.0, Lx = 0.0, Ly = 0.0;
            for (int m = 0; m < nl; m++) {
                const double c = C[(size_t)m * nl + b];
                if (c == 0.0) continue;
                const int ex = tmo[m][0], ey = tmo[m][1];
                double px = 1.0, py = 1.0;
                for (int i = 0; i < ex; i++) px *= xi[0];
                for (int i = 0; i < ey; i++) py *= xi[1];
                L += c * px * py;
                if (ex > 0) { double d = ex; for (int i = 0; i < ex - 1; i++) d *= xi[0]; Lx += c * d * py; }
                if (ey > 0) { double d = ey; for (int i = 0; i < ey - 1; i++) d *= xi[1]; Ly += c * px * d; }
            }
            for (int k = 0; k < 3; k++) {
                S[k] += L * sp[3 * b + k];
                Sx[k] += Lx * sp[3 * b + k];
                Sy[k] += Ly * sp[3 * b + k];
            }
        }
    };
    auto cross = [](const double *a, const double *b, double *c) {
        c[0] = a[1] * b[2] - a[2] * b[1];
        c[1] = a[2] * b[0] - a[0] * b[2];
        c[2] = a[0] * b[1] - a[1] * b[0];
    };
    const double tri_area = std::sqrt(3.0) / 4.0;
    for (int i = 0; i < r.QT; i++) {
        double S[3], Sx[3], Sy[3], c[3];
        surf(r.fpt[i].data(), S, Sx, Sy);
        cross(Sx, Sy, c);
        for (int k = 0; k < 3; k++) tfA[3 * i + k] = tri_area * r.fw[i] * c[k];
    }
    double V[3][2];
    for (int k = 0; k < 3; k++) {
        V[k][0] = k == 0 ? -0.5 : k == 1 ? 0.5 : 0.0;
        V[k][1] = k == 2 ? 1.0 / std::sqrt(3.0) : -0.5 / std::sqrt(3.0);
    }
    for (int e = 0; e < 3; e++)
        for (int i = 0; i < r.QS; i++) {
            const int qi = 2 * r.QT + e * r.QS + i;
            const double *xi = r.fpt[qi].data();
            double S[3], Sx[3], Sy[3], Ss[3], c[3];
            surf(xi, S, Sx, Sy);
            const double ex = V[(e + 1) % 3][0] - V[e][0], ey = V[(e + 1) % 3][1] - V[e][1];
            for (int k = 0; k < 3; k++) Ss[k] = ex * Sx[k] + ey * Sy[k];
            cross(Ss, S, c);
            const double R = (0.5 - xi[2]) + (0.5 + xi[2]) * q;
            for (int k = 0; k < 3; k++) sfA[(e * r.QS + i) * 3 + k] = r.fw[qi] * R * (q - 1.0) * c[k];
        }
}

// volume of one column's zone in the unit shell: the Jacobian of the map
// integrated by Gauss points in zeta times a rule on the triangle obtained by
// collapsing the square onto it (Duffy), six points each way
double column_volume(const PrismRef &r, const double *abc, double q)
{
    const int mo = r.order - 1, ng = 6;
    std::vector<std::array<int, 3>> bary;
    std::vector<std::array<double, 3>> lx;
    lattice(mo, bary, lx);
    const int nl = (int)lx.size();
    std::vector<double> sp((size_t)nl * 3);
    const double *P[3] = {abc, abc + 3, abc + 6};
    for (int a = 0; a < nl; a++) {
        double *o = &sp[3 * a];
        const auto &bc = bary[a];
        const int nz = (bc[0] == 0) + (bc[1] == 0) + (bc[2] == 0);
        if (nz == 2) std::memcpy(o, P[bc[0] ? 0 : bc[1] ? 1 : 2], 24);
        else if (nz == 1) {
            const int u = bc[0] ? 0 : 1, w = bc[2] ? 2 : 1;
            arc_point(P[u], P[w], double(bc[w]) / (bc[u] + bc[w]), o);
        } else {
            for (int i = 0; i < 3; i++) o[i] = P[0][i] + P[1][i] + P[2][i];
            unit(o);
        }
    }
    std::vector<std::array<int, 3>> tmo;
    for (int deg = 0; deg <= mo; deg++)
        for (int a = deg; a >= 0; a--) tmo.push_back({a, deg - a, 0});
    std::vector<double> C;
    lagrange_coefficients(lx, tmo, C);
    double gx[8], gw[8];
    gauss_legendre01(ng, gx, gw);
    const double s3 = std::sqrt(3.0);
    const double A[2] = {-0.5, -0.5 / s3}, B[2] = {0.5, -0.5 / s3}, Cc[2] = {0.0, 1.0 / s3};
    double V = 0.0;
    for (int i = 0; i < ng; i++)
        for (int j = 0; j < ng; j++) {
            // the square's (s, w) -> the triangle point A + s (B - A) + (1 - s) w (C - A)
            const double sv = gx[i], tv = (1.0 - sv) * gx[j];
            const double xi = A[0] + sv * (B[0] - A[0]) + tv * (Cc[0] - A[0]);
            const double eta = A[1] + sv * (B[1] - A[1]) + tv * (Cc[1] - A[1]);
            double S[3] = {0, 0, 0}, Sx[3] = {0, 0, 0}, Sy[3] = {0, 0, 0};
            for (int b = 0; b < nl; b++) {
                double L = 0.0, Lx = 0.0, Ly = 0.0;
                for (int m = 0; m < nl; m++) {
                    const double c = C[(size_t)m * nl + b];
                    const int ex = tmo[m][0], ey = tmo[m][1];
                    L += c * std::pow(xi, ex) * std::pow(eta, ey);
                    if (ex) Lx += c * ex * std::pow(xi, ex - 1) * std::pow(eta, ey);
                    if (ey) Ly += c * ey * std::pow(xi, ex) * std::pow(eta, ey - 1);
                }
                for (int k = 0; k < 3; k++) { S[k] += L * sp[3 * b + k]; Sx[k] += Lx * sp[3 * b + k]; Sy[k] += Ly * sp[3 * b + k]; }
            }
            // x = R(zeta) S: J = R^2 (q - 1) S . (S_xi x S_eta)
            const double trip = S[0] * (Sx[1] * Sy[2] - Sx[2] * Sy[1]) + S[1] * (Sx[2] * Sy[0] - Sx[0] * Sy[2]) +
                                S[2] * (Sx[0] * Sy[1] - Sx[1] * Sy[0]);
            double rz = 0.0;
            for (int k = 0; k < ng; k++) {
                const double R = (1.0 - gx[k]) + gx[k] * q;   // zeta = gx - 1/2
                rz += gw[k] * R * R;
            }
            V += 2.0 * (s3 / 4.0) * (1.0 - sv) * gw[i] * gw[j] * (q - 1.0) * trip * rz;
        }
    return V;
}

// mesh edges in first-encounter order over (triangle, local edge a-b, b-c,
// c-a), kept where the triangle precedes its neighbour; endpoints are
// compared bit for bit (shared vertices come out of the same sums)
bool mesh_edges(const std::vector<double> &tri, std::vector<int> &edges)
{
    const int64_t nt = (int64_t)(tri.size() / 9);
    struct Key {
        double v[6];
        bool operator<(const Key &o) const { return std::memcmp(v, o.v, sizeof(v)) < 0; }
    };
    std::map<Key, std::pair<int, int>> where;
    auto key = [&](int64_t t, int e, bool rev) {
        Key k;
        const double *a = &tri[9 * t + 3 * e], *b = &tri[9 * t + 3 * ((e + 1) % 3)];
        std::memcpy(k.v, rev ? b : a, 24);
        std::memcpy(k.v + 3, rev ? a : b, 24);
        return k;
    };
    for (int64_t t = 0; t < nt; t++)
        for (int e = 0; e < 3; e++) where[key(t, e, false)] = {(int)t, e};
    edges.clear();
    for (int64_t t = 0; t < nt; t++)
        for (int e = 0; e < 3; e++) {
            auto it = where.find(key(t, e, true));
            if (it == where.end()) return false;
            if (t < it->second.first) {
                edges.push_back((int)t);
                edges.push_back(e);
                edges.push_back(it->second.first);
                edges.push_back(it->second.second);
            }
        }
    return (int64_t)edges.size() / 4 == 3 * nt / 2;
}

// Constrained-transport tables of the mesh.  Vertices are numbered in first
// encounter over (triangle, local vertex), matched bit for bit (shared
// vertices come out of the same sums); each vertex's ring lists its
// triangles counter-clockwise seen from outside, starting at the lowest, a
// triangle (v, a, b) followed by the one holding the directed edge v -> b,
// with the unit normal v x b / |v x b| of the side face between them (it
// points from the ring's triangle to the next).  Per mesh edge and Simpson
// point on the unit shell: the unit tangent along the edge's first
// triangle, the frame of the four-state field from the two columns'
// centroids (east = the first triangle, north = outward: the directions of
// east minus west and north minus south do not depend on the radius), the
// normal t x r of the side face out of the first triangle, and |dx/ds|.
void zone_cubature(const TriSurface &ts, double q, std::vector<std::array<double, 4>> &cub, double &V, double *cen);

bool ct_tables(rg_prism *p)
{
    const int64_t nt = p->ntri;
    std::map<std::array<double, 3>, int> vid;
    p->tri_v.assign((size_t)nt * 3, -1);
    p->vxyz.clear();
    for (int64_t t = 0; t < nt; t++)
        for (int j = 0; j < 3; j++) {
            std::array<double, 3> a = {p->tri[9 * t + 3 * j], p->tri[9 * t + 3 * j + 1], p->tri[9 * t + 3 * j + 2]};
            auto it = vid.find(a);
            if (it == vid.end()) {
                it = vid.emplace(a, (int)(p->vxyz.size() / 3)).first;
                p->vxyz.insert(p->vxyz.end(), a.begin(), a.end());
            }
            p->tri_v[3 * t + j] = it->second;
        }
    const int64_t nv = (int64_t)p->vxyz.size() / 3;
    if (nv != nt / 2 + 2) return false;     // Euler: V = F / 2 + 2 for a closed triangulated sphere
    std::unordered_map<int64_t, int> directed;   // (u, w) -> 3 t + (local index of u)
    std::vector<int> first(nv, -1), count(nv, 0);
    for (int64_t t = 0; t < nt; t++)
        for (int j = 0; j < 3; j++) {
            const int u = p->tri_v[3 * t + j], w = p->tri_v[3 * t + (j + 1) % 3];
            directed[(int64_t)u * nv + w] = (int)(3 * t + j);
            if (first[u] < 0) first[u] = (int)(3 * t + j);
            count[u]++;
        }
    p->ring_off.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; v++) p->ring_off[v + 1] = p->ring_off[v] + count[v];
    p->ring_tj.assign(p->ring_off[nv], 0);
    p->ring_n.assign((size_t)p->ring_off[nv] * 3, 0.0);
    for (int64_t v = 0; v < nv; v++) {
        int cur = first[v];
        const double *vp = &p->vxyz[3 * v];
        for (int m = 0; m < count[v]; m++) {
            const int t = cur / 3, j = cur % 3;
            const int b = p->tri_v[3 * (size_t)t + (j + 2) % 3];
            p->ring_tj[p->ring_off[v] + m] = cur;
            const double *bp = &p->vxyz[3 * (size_t)b];
            double n[3] = {vp[1] * bp[2] - vp[2] * bp[1], vp[2] * bp[0] - vp[0] * bp[2], vp[0] * bp[1] - vp[1] * bp[0]};
            unit(n);
            std::memcpy(&p->ring_n[3 * (size_t)(p->ring_off[v] + m)], n, 24);
            auto it = directed.find((int64_t)v * nv + b);
            if (it == directed.end()) return false;
            cur = it->second;
        }
        if (cur != first[v]) return false;        // the ring must close after its count
    }
    const int64_t ne = (int64_t)p->edges.size() / 4;
    p->edge_ab.assign((size_t)ne * 2, 0);
    for (int64_t e = 0; e < ne; e++) {
        const int t1 = p->edges[4 * e], e1 = p->edges[4 * e + 1];
        p->edge_ab[2 * e] = p->tri_v[3 * (size_t)t1 + e1];
        p->edge_ab[2 * e + 1] = p->tri_v[3 * (size_t)t1 + (e1 + 1) % 3];
    }
    // unit-shell centroids of the columns
    std::vector<double> cen((size_t)nt * 3);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; t++) {
        const TriSurface ts(p->ref, &p->tri[9 * t]);
        std::vector<std::array<double, 4>> cub;
        double V;
        zone_cubature(ts, p->q, cub, V, &cen[3 * t]);
    }
    const double s3 = std::sqrt(3.0);
    const double TV[3][2] = {{-0.5, -0.5 / s3}, {0.5, -0.5 / s3}, {0.0, 1.0 / s3}};
    const double SS[3] = {0.0, 0.5, 1.0};
    p->aeg.assign((size_t)ne * 3 * 16, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; e++) {
        const int t1 = p->edges[4 * e], e1 = p->edges[4 * e + 1], t2 = p->edges[4 * e + 2];
        const TriSurface ts(p->ref, &p->tri[9 * (size_t)t1]);
        const double dx = TV[(e1 + 1) % 3][0] - TV[e1][0], dy = TV[(e1 + 1) % 3][1] - TV[e1][1];
        double u[3], w[3];
        for (int i = 0; i < 3; i++) {
            u[i] = cen[3 * (size_t)t1 + i] - cen[3 * (size_t)t2 + i];
            w[i] = cen[3 * (size_t)t1 + i] + cen[3 * (size_t)t2 + i];
        }
        for (int pp = 0; pp < 3; pp++) {
            const double xi[2] = {TV[e1][0] + SS[pp] * dx, TV[e1][1] + SS[pp] * dy};
            double S[3], Sx[3], Sy[3], tg[3], rh[3], nb[3];
            ts.eval(xi, S, Sx, Sy);
            for (int i = 0; i < 3; i++) tg[i] = Sx[i] * dx + Sy[i] * dy;
            const double dl = std::sqrt(tg[0] * tg[0] + tg[1] * tg[1] + tg[2] * tg[2]);
            for (int i = 0; i < 3; i++) { tg[i] /= dl; rh[i] = S[i]; }
            unit(rh);
            nb[0] = tg[1] * rh[2] - tg[2] * rh[1];
            nb[1] = tg[2] * rh[0] - tg[0] * rh[2];
            nb[2] = tg[0] * rh[1] - tg[1] * rh[0];
            unit(nb);
            double *g = &p->aeg[((size_t)e * 3 + pp) * 16];
            std::memcpy(g, tg, 24);
            symmetric_frame(u, w, tg, g + 3, g + 6);
            std::memcpy(g + 9, nb, 24);
            g[12] = dl;
        }
    }
    // basis values at the edge points
    p->eidx.assign((size_t)EDGE_POINTS * EDGE_TERMS, 0);
    p->eval.assign((size_t)EDGE_POINTS * EDGE_TERMS, 0.0);
    for (int pt = 0; pt < EDGE_POINTS; pt++) {
        double xi[3];
        if (pt < 18) {
            const int side = pt / 9, j = (pt / 3) % 3, pp = pt % 3;
            xi[0] = TV[j][0] + SS[pp] * (TV[(j + 1) % 3][0] - TV[j][0]);
            xi[1] = TV[j][1] + SS[pp] * (TV[(j + 1) % 3][1] - TV[j][1]);
            xi[2] = side == 0 ? 0.5 : -0.5;
        } else {
            const int j = (pt - 18) / 3, pp = (pt - 18) % 3;
            xi[0] = TV[j][0];
            xi[1] = TV[j][1];
            xi[2] = SS[pp] - 0.5;
        }
        int n = 0;
        for (int l = 0; l < p->ref.N; l++) {
            const double v = p->ref.psi(l, xi);
            if (std::fabs(v) < 1e-13) continue;
            if (n == EDGE_TERMS) return false;
            p->eidx[(size_t)pt * EDGE_TERMS + n] = l;
            p->eval[(size_t)pt * EDGE_TERMS + n] = v;
            n++;
        }
    }
    return true;
}

// cubature of the unit shell's zone over the column's triangle: Gauss (6
// points) in zeta times the collapsed 6 x 6 Gauss rule on the triangle;
// points (x, weight J) and the zone's volume and centroid
void zone_cubature(const TriSurface &ts, double q, std::vector<std::array<double, 4>> &cub, double &V, double *cen)
{
    const int ng = 6;
    double gx[8], gw[8];
    gauss_legendre01(ng, gx, gw);
    const double s3 = std::sqrt(3.0);
    const double VA[2] = {-0.5, -0.5 / s3}, VB[2] = {0.5, -0.5 / s3}, VC[2] = {0.0, 1.0 / s3};
    cub.clear();
    V = 0.0;
    cen[0] = cen[1] = cen[2] = 0.0;
    for (int i = 0; i < ng; i++)
        for (int j = 0; j < ng; j++) {
            const double sv = gx[i], tv = (1.0 - sv) * gx[j];
            const double xe[2] = {VA[0] + sv * (VB[0] - VA[0]) + tv * (VC[0] - VA[0]),
                                  VA[1] + sv * (VB[1] - VA[1]) + tv * (VC[1] - VA[1])};
            double S[3], Sx[3], Sy[3];
            ts.eval(xe, S, Sx, Sy);
            const double trip = S[0] * (Sx[1] * Sy[2] - Sx[2] * Sy[1]) + S[1] * (Sx[2] * Sy[0] - Sx[0] * Sy[2]) +
                                S[2] * (Sx[0] * Sy[1] - Sx[1] * Sy[0]);
            for (int k = 0; k < ng; k++) {
                const double R = (1.0 - gx[k]) + gx[k] * q;
                const double wJ = 2.0 * (s3 / 4.0) * (1.0 - sv) * gw[i] * gw[j] * gw[k] * R * R * (q - 1.0) * trip;
                cub.push_back({R * S[0], R * S[1], R * S[2], wJ});
                V += wJ;
                for (int d = 0; d < 3; d++) cen[d] += wJ * R * S[d];
            }
        }
    for (int d = 0; d < 3; d++) cen[d] /= V;
}

// Divergence-free reconstruction of B (Section IV.b with the prism's five
// faces) as one linear map per column: the KKT system of the constrained
// least squares is solved for every input at once, and the solution is
// evaluated at the element nodes.  The Taylor frame (centroid, l0 = V^(1/3),
// moments) makes the map the same for every shell of a column (each shell is
// the unit shell scaled by r_k).  Inputs (NIN): per component its zone mean
// and Taylor coefficients of degree 1..p-1 (degree by degree, x exponent
// descending, then y), the outward normal B at the face points
// (rg_prism_face_points order), the five outward face averages; outputs
// (3N + 3): B at the nodes by component, then the three zone means.
bool column_divfree_map(const PrismRef &r, const double *abc, double q, const double *nodex, double *Mb)
{
    const int p = r.order, N = r.N, Q = r.Q, QT = r.QT, QS = r.QS;
    std::vector<std::array<int, 3>> te;
    for (int d = 1; d <= p - 1; d++)
        for (int a = d; a >= 0; a--)
            for (int b = d - a; b >= 0; b--) te.push_back({a, b, d - a - b});
    const int nc = (int)te.size();
    std::vector<std::array<int, 3>> be[3];
    for (int c = 0; c < 3; c++) {
        be[c].push_back({0, 0, 0});
        for (auto &e : te) be[c].push_back(e);
        for (int a = p; a >= 0; a--)
            for (int b = p - a; b >= 0; b--) {
                std::array<int, 3> e = {a, b, p - a - b};
                if (e[c] >= 1) be[c].push_back(e);
            }
    }
    const int NB = (int)be[0].size(), nu = 3 * NB, ndiv = nc, ncon = ndiv + 5, nrow = nu + Q;
    const int NIN = 3 * (nc + 1) + Q + 5, NOUT = 3 * N + 3;
    const TriSurface ts(r, abc);
    std::vector<std::array<double, 4>> cub;
    double V = 0.0, cen[3];
    zone_cubature(ts, q, cub, V, cen);
    const double s3 = std::sqrt(3.0);
    const double VA[2] = {-0.5, -0.5 / s3}, VB[2] = {0.5, -0.5 / s3}, VC[2] = {0.0, 1.0 / s3};
    const double l0 = std::cbrt(V);
    auto mono = [](const std::array<int, 3> &e, const double *X) {
        double v = 1.0;
        for (int d = 0; d < 3; d++)
            for (int k = 0; k < e[d]; k++) v *= X[d];
        return v;
    };
    std::map<std::array<int, 3>, double> mom;
    for (int a = 0; a <= p; a++)
        for (int b = 0; a + b <= p; b++)
            for (int c = 0; a + b + c <= p; c++) mom[{a, b, c}] = 0.0;
    for (auto &pt : cub) {
        double X[3];
        for (int d = 0; d < 3; d++) X[d] = (pt[d] - cen[d]) / l0;
        for (auto &kv : mom) kv.second += pt[3] * mono(kv.first, X) / V;
    }
    auto tb = [&](const std::array<int, 3> &e, const double *X) {
        return e[0] + e[1] + e[2] == 0 ? 1.0 : mono(e, X) - mom.at(e);
    };
    // face points: positions, outward unit normals, weights within the face
    std::vector<std::array<double, 3>> fx(Q), fn(Q);
    std::vector<double> fa(Q);
    double area[5] = {0, 0, 0, 0, 0};
    double Vt[3][2] = {{VA[0], VA[1]}, {VB[0], VB[1]}, {VC[0], VC[1]}};
    for (int qq = 0; qq < Q; qq++) {
        const double *xi = r.fpt[qq].data();
        double S[3], Sx[3], Sy[3], a3[3], b3[3];
        ts.eval(xi, S, Sx, Sy);
        const double R = (0.5 - xi[2]) + (0.5 + xi[2]) * q;
        double sc;
        int f;
        if (qq < 2 * QT) {
            for (int k = 0; k < 3; k++) { a3[k] = R * Sx[k]; b3[k] = R * Sy[k]; }
            sc = (qq < QT ? 1.0 : -1.0) * (s3 / 4.0) * r.fw[qq];
            f = qq < QT ? 0 : 1;
        } else {
            const int e = (qq - 2 * QT) / QS;
            const double ex = Vt[(e + 1) % 3][0] - Vt[e][0], ey = Vt[(e + 1) % 3][1] - Vt[e][1];
            for (int k = 0; k < 3; k++) { a3[k] = R * (ex * Sx[k] + ey * Sy[k]); b3[k] = (q - 1.0) * S[k]; }
            sc = r.fw[qq];
            f = 2 + e;
        }
        const double cx = a3[1] * b3[2] - a3[2] * b3[1], cy = a3[2] * b3[0] - a3[0] * b3[2], cz = a3[0] * b3[1] - a3[1] * b3[0];
        const double m = std::sqrt(cx * cx + cy * cy + cz * cz), sg = sc > 0 ? 1.0 : -1.0;
        fn[qq] = {sg * cx / m, sg * cy / m, sg * cz / m};
        fa[qq] = std::fabs(sc) * m;
        area[f] += fa[qq];
        for (int k = 0; k < 3; k++) fx[qq][k] = R * S[k];
    }
    // least-squares rows and constraints, each as a map of the inputs
    const int inF = 3 * (nc + 1), inM = inF + Q;
    std::vector<double> Am((size_t)nrow * nu, 0.0), Sb((size_t)nrow * NIN, 0.0);
    std::vector<double> Cm((size_t)ncon * nu, 0.0), Sd((size_t)ncon * NIN, 0.0);
    for (int c = 0; c < 3; c++)
        for (int k = 0; k < NB; k++) {
            Am[(size_t)(c * NB + k) * nu + c * NB + k] = 1.0;
            if (k <= nc) Sb[(size_t)(c * NB + k) * NIN + c * (nc + 1) + k] = 1.0;
        }
    for (int qq = 0; qq < Q; qq++) {
        const int f = qq < QT ? 0 : qq < 2 * QT ? 1 : 2 + (qq - 2 * QT) / QS;
        double X[3];
        for (int d = 0; d < 3; d++) X[d] = (fx[qq][d] - cen[d]) / l0;
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < NB; k++) {
                const double val = fn[qq][c] * tb(be[c][k], X);
                Am[(size_t)(nu + qq) * nu + c * NB + k] = val;
                Cm[(size_t)(ndiv + f) * nu + c * NB + k] += fa[qq] / area[f] * val;
            }
        Sb[(size_t)(nu + qq) * NIN + inF + qq] = 1.0;
    }
    for (int f = 0; f < 5; f++) Sd[(size_t)(ndiv + f) * NIN + inM + f] = 1.0;
    for (int i = 0; i < ndiv; i++)
        for (int c = 0; c < 3; c++) {
            std::array<int, 3> t = te[i];
            t[c] += 1;
            for (int k = 0; k < NB; k++)
                if (be[c][k] == t) Cm[(size_t)i * nu + c * NB + k] += t[c];
        }
    // normal equations 2 A^T A u + C^T lambda = 2 A^T S b, C u = S_d b; the
    // first nu rows of A are the identity and each face row of S one unit
    const int nk = nu + ncon;
    std::vector<double> K((size_t)nk * nk, 0.0), rhs((size_t)nk * NIN, 0.0);
    for (int i = 0; i < nu; i++) {
        K[(size_t)i * nk + i] = 2.0;
        for (int j = 0; j < NIN; j++) rhs[(size_t)i * NIN + j] = 2.0 * Sb[(size_t)i * NIN + j];
    }
    for (int k = nu; k < nrow; k++) {
        const double *a = &Am[(size_t)k * nu];
        for (int i = 0; i < nu; i++) {
            if (a[i] == 0.0) continue;
            for (int j = 0; j < nu; j++) K[(size_t)i * nk + j] += 2.0 * a[i] * a[j];
            rhs[(size_t)i * NIN + inF + (k - nu)] += 2.0 * a[i];
        }
    }
    for (int i = 0; i < ncon; i++)
        for (int j = 0; j < nu; j++) {
            K[(size_t)(nu + i) * nk + j] = Cm[(size_t)i * nu + j];
            K[(size_t)j * nk + nu + i] = Cm[(size_t)i * nu + j];
        }
    for (int i = 0; i < ncon; i++)
        for (int j = 0; j < NIN; j++) rhs[(size_t)(nu + i) * NIN + j] = Sd[(size_t)i * NIN + j];
    std::vector<int> piv;
    if (!lu_factor(nk, K, piv)) return false;
    std::vector<double> Gm((size_t)nu * NIN), col(nk);
    for (int j = 0; j < NIN; j++) {
        for (int i = 0; i < nk; i++) col[i] = rhs[(size_t)i * NIN + j];
        lu_solve(nk, K, piv, col.data());
        for (int i = 0; i < nu; i++) Gm[(size_t)i * NIN + j] = col[i];
    }
    for (int c = 0; c < 3; c++)
        for (int i = 0; i < N; i++) {
            double X[3];
            for (int d = 0; d < 3; d++) X[d] = (nodex[3 * i + d] - cen[d]) / l0;
            double *row = &Mb[(size_t)(c * N + i) * NIN];
            for (int j = 0; j < NIN; j++) row[j] = 0.0;
            for (int k = 0; k < NB; k++) {
                const double bv = tb(be[c][k], X);
                const double *g = &Gm[(size_t)(c * NB + k) * NIN];
                for (int j = 0; j < NIN; j++) row[j] += bv * g[j];
            }
        }
    for (int c = 0; c < 3; c++)
        std::memcpy(&Mb[(size_t)(3 * N + c) * NIN], &Gm[(size_t)(c * NB) * NIN], sizeof(double) * NIN);
    (void)NOUT;
    return true;
}

}  // namespace

extern "C" {

static rg_status prism_build(int32_t level, int32_t n_rad, double r_in, double r_out, int32_t order, bool device,
                             rg_prism **out)
{
    if (!out) { set_error("null argument"); return RG_EINVAL; }
    *out = nullptr;
    if (order < 2 || order > 4) { set_error("prism order must be 2, 3 or 4"); return RG_ENOTSUP; }
    if (level < 0 || level > 8) { set_error("icosahedral level must be 0..8"); return RG_ENOTSUP; }
    if (n_rad < 1 || !(r_in > 0.0) || !(r_out > r_in)) { set_error("need n_rad >= 1 and 0 < r_in < r_out"); return RG_EINVAL; }
    rg_prism *p = new (std::nothrow) rg_prism;
    if (!p) { set_error("out of host memory"); return RG_ENOMEM; }
    p->level = level; p->n_rad = n_rad; p->order = order; p->r_in = r_in; p->r_out = r_out;
    if (!build_prism_ref(order, p->ref)) { set_error("prism reference element construction failed"); free_prism(p); return RG_ESINGULAR; }
    if (!prism_tables_match(p->ref)) { set_error("prism derivative matrices differ from the compiled-in tables"); free_prism(p); return RG_ESINGULAR; }
    icosahedron(p->tri);
    for (int l = 0; l < level; l++) split(p->tri);
    p->ntri = (int64_t)(p->tri.size() / 9);
    p->nz = p->ntri * n_rad;
    if (p->nz * p->ref.N >= ((int64_t)1 << 31)) { set_error("zone-node count exceeds 2^31"); free_prism(p); return RG_ENOTSUP; }
    p->q = std::pow(r_out / r_in, 1.0 / n_rad);
    p->radius.resize(n_rad + 1);
    for (int k = 0; k <= n_rad; k++) p->radius[k] = r_in * std::pow(r_out / r_in, double(k) / n_rad);
    const int N = p->ref.N;
    p->hx.assign((size_t)p->ntri * N * 3, 0.0);
    p->hJ.assign((size_t)p->ntri * N, 0.0);
    p->hM.assign((size_t)p->ntri * 9 * N, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < p->ntri; t++)
        column_geometry(p->ref, &p->tri[9 * t], p->q, &p->hx[(size_t)t * N * 3], &p->hJ[(size_t)t * N],
                        &p->hM[(size_t)t * 9 * N]);
    for (int64_t t = 0; t < p->ntri * N; t++)
        if (!(p->hJ[t] > 0.0)) { set_error("non-positive Jacobian"); free_prism(p); return RG_ESINGULAR; }
    const int QT = p->ref.QT, QS = p->ref.QS;
    p->tfA.assign((size_t)p->ntri * QT * 3, 0.0);
    p->sfA.assign((size_t)p->ntri * 3 * QS * 3, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < p->ntri; t++)
        column_face_geometry(p->ref, &p->tri[9 * t], p->q, &p->tfA[(size_t)t * QT * 3], &p->sfA[(size_t)t * 3 * QS * 3]);
    if (!mesh_edges(p->tri, p->edges)) { set_error("the triangles do not close into a sphere"); free_prism(p); return RG_ESINGULAR; }
    {
        int nc = 0;
        for (int d = 1; d <= order - 1; d++) nc += (d + 1) * (d + 2) / 2;
        p->nin = 3 * (nc + 1) + p->ref.Q + 5;
        p->nout = 3 * N + 3;
    }
    p->vol.assign(p->ntri, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < p->ntri; t++) p->vol[t] = column_volume(p->ref, &p->tri[9 * t], p->q);
    p->tedge.assign((size_t)p->ntri * 3, 0);
    for (size_t e = 0; e < p->edges.size() / 4; e++) {
        p->tedge[3 * (size_t)p->edges[4 * e] + p->edges[4 * e + 1]] = (int)e;
        p->tedge[3 * (size_t)p->edges[4 * e + 2] + p->edges[4 * e + 3]] = -(int)e - 1;
    }
    // side point at the same height, mirrored along the edge (the neighbour
    // runs the shared edge the other way)
    p->mirror.assign(QS, -1);
    for (int i = 0; i < QS; i++) {
        const auto &a = p->ref.fpt[2 * QT + i];
        for (int j = 0; j < QS; j++) {
            const auto &b = p->ref.fpt[2 * QT + j];
            // on edge 0 (eta fixed), mirroring along the edge maps xi to -xi
            if (std::fabs(b[0] + a[0]) < 1e-12 && std::fabs(b[2] - a[2]) < 1e-12) p->mirror[i] = j;
        }
        if (p->mirror[i] < 0) { set_error("side-face rule is not symmetric along the edge"); free_prism(p); return RG_ESINGULAR; }
    }
    if (!ct_tables(p)) { set_error("edge and vertex tables of the prism mesh could not be built"); free_prism(p); return RG_ESINGULAR; }
    p->device = device;
    if (!device) { *out = p; return RG_OK; }
    std::vector<double> rinv(n_rad);
    for (int k = 0; k < n_rad; k++) rinv[k] = 1.0 / p->radius[k];
    DevPrism &G = p->dev;
    G.order = order; G.N = N; G.n_rad = n_rad; G.ntri = p->ntri; G.nz = p->nz;
    G.Q = p->ref.Q;
    G.QT = QT;
    G.QS = QS;
    G.nedges = (int64_t)p->edges.size() / 4;
    G.nin = p->nin;
    G.nout = p->nout;
    G.Mb = nullptr;
    G.nfaces = p->ntri * (n_rad + 1) + G.nedges * n_rad;
    G.nvert = (int64_t)p->vxyz.size() / 3;
    if (!upload(p, p->hJ, &G.J) || !upload(p, p->hM, &G.met) || !upload(p, rinv, &G.rinv) ||
        !upload(p, p->ref.R, &G.R) || !upload(p, p->ref.wt, &G.wt) || !upload(p, p->ref.fidx, &G.fidx) ||
        !upload(p, p->ref.fval, &G.fval) || !upload(p, p->edges, &G.edges) || !upload(p, p->mirror, &G.mirror) ||
        !upload(p, p->tfA, &G.tfA) || !upload(p, p->sfA, &G.sfA) || !upload(p, p->radius, &G.radius) ||
        !upload(p, p->vol, &G.vol) || !upload(p, p->tedge, &G.tedge) || !upload(p, p->eidx, &G.eidx) ||
        !upload(p, p->eval, &G.eval) || !upload(p, p->aeg, &G.aeg) || !upload(p, p->edge_ab, &G.edge_ab) ||
        !upload(p, p->vxyz, &G.vxyz) || !upload(p, p->ring_off, &G.ring_off) || !upload(p, p->ring_tj, &G.ring_tj) ||
        !upload(p, p->ring_n, &G.ring_n)) {
        set_error("device allocation or upload of the prism geometry failed");
        free_prism(p);
        return RG_ENOMEM;
    }
    *out = p;
    return RG_OK;
}

rg_status rg_prism_build(int32_t level, int32_t n_rad, double r_in, double r_out, int32_t order, rg_prism **out)
{
    return prism_build(level, n_rad, r_in, r_out, order, true, out);
}

rg_status rg_prism_build_host(int32_t level, int32_t n_rad, double r_in, double r_out, int32_t order, rg_prism **out)
{
    return prism_build(level, n_rad, r_in, r_out, order, false, out);
}

void rg_prism_free(rg_prism *p) { free_prism(p); }

rg_status rg_prism_get_info(const rg_prism *p, rg_prism_info *info)
{
    if (!p || !info) { set_error("null argument"); return RG_EINVAL; }
    info->n_zones = p->nz;
    info->n_tri = p->ntri;
    info->n_nodes = p->ref.N;
    info->n_levels = p->ref.M;
    info->order = p->order;
    info->level = p->level;
    info->n_rad = p->n_rad;
    info->n_face_points = p->ref.Q;
    info->n_edges = (int64_t)p->edges.size() / 4;
    info->n_faces = p->ntri * (p->n_rad + 1) + info->n_edges * p->n_rad;
    info->n_divfree_in = p->nin;
    info->n_divfree_out = p->nout;
    info->n_vertices = (int64_t)p->vxyz.size() / 3;
    return RG_OK;
}

rg_status rg_prism_edges(const rg_prism *p, int32_t *edges)
{
    if (!p || !edges) { set_error("null argument"); return RG_EINVAL; }
    std::memcpy(edges, p->edges.data(), p->edges.size() * sizeof(int));
    return RG_OK;
}

rg_status rg_prism_vertices(const rg_prism *p, double *xyz)
{
    if (!p || !xyz) { set_error("null argument"); return RG_EINVAL; }
    std::memcpy(xyz, p->vxyz.data(), p->vxyz.size() * sizeof(double));
    return RG_OK;
}

rg_status rg_prism_edge_traces(const rg_prism *p, const double *avgU, const double *avgF, double *er, void *stream)
{
    if (!p || !avgU || !avgF || !er) { set_error("null argument"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    return launch_prism_edge_traces(p->dev, avgU, avgF, er, stream);
}

rg_status rg_prism_edge_emfs(const rg_prism *p, double gamma, const double *er, double *Gang, double *Grad,
                             void *stream)
{
    if (!p || !er || !Gang || !Grad) { set_error("null argument"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    if (!(gamma > 1.0)) { set_error("gamma must exceed 1"); return RG_EINVAL; }
    return launch_prism_edge_emfs(p->dev, gamma, er, Gang, Grad, stream);
}

rg_status rg_prism_ct(const rg_prism *p, double dt, const double *Gang, const double *Grad, const double *PhiB,
                      double *PhiBo, void *stream)
{
    if (!p || !Gang || !Grad || !PhiB || !PhiBo) { set_error("null argument"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    if (!(dt >= 0.0)) { set_error("dt must be non-negative"); return RG_EINVAL; }
    return launch_prism_ct(p->dev, dt, Gang, Grad, PhiB, PhiBo, stream);
}

rg_status rg_prism_volumes(const rg_prism *p, int64_t z0, int64_t nz, double *vol)
{
    if (!p || !vol) { set_error("null argument"); return RG_EINVAL; }
    if (z0 < 0 || nz < 0 || z0 + nz > p->nz) { set_error("zone range outside the mesh"); return RG_EINVAL; }
    for (int64_t i = 0; i < nz; i++) {
        const int64_t z = z0 + i;
        const double s = p->radius[z % p->n_rad];
        vol[i] = s * s * s * p->vol[z / p->n_rad];
    }
    return RG_OK;
}

static rg_status build_divfree_maps(rg_prism *p)
{
    if (!p->Mb.empty()) return RG_OK;
    const int N = p->ref.N;
    std::vector<double> Mb((size_t)p->ntri * p->nout * p->nin);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (int64_t t = 0; t < p->ntri; t++)
        bad += !column_divfree_map(p->ref, &p->tri[9 * t], p->q, &p->hx[(size_t)t * N * 3],
                                   &Mb[(size_t)t * p->nout * p->nin]);
    if (bad) { set_error("singular divergence-free KKT system"); return RG_ESINGULAR; }
    p->Mb.swap(Mb);
    return RG_OK;
}

rg_status rg_prism_divfree_host(rg_prism *p, int64_t z0, int64_t nz, const double *Bin, double *Bout)
{
    if (!p || !Bin || !Bout) { set_error("null argument"); return RG_EINVAL; }
    if (z0 < 0 || nz < 0 || z0 + nz > p->nz) { set_error("zone range outside the mesh"); return RG_EINVAL; }
    {
        std::lock_guard<std::mutex> lock(p->mb_mutex);
        rg_status st = build_divfree_maps(p);
        if (st != RG_OK) return st;
    }
    for (int64_t i = 0; i < nz; i++) {
        const double *M = &p->Mb[(size_t)((z0 + i) / p->n_rad) * p->nout * p->nin];
        for (int o = 0; o < p->nout; o++) {
            double acc = 0.0;
            for (int j = 0; j < p->nin; j++) acc += M[(size_t)o * p->nin + j] * Bin[i * p->nin + j];
            Bout[i * p->nout + o] = acc;
        }
    }
    return RG_OK;
}

rg_status rg_prism_divfree(rg_prism *p, const double *Bin, double *Bout, void *stream)
{
    if (!p || !Bin || !Bout) { set_error("null argument"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    std::lock_guard<std::mutex> lock(p->mb_mutex);
    if (!p->dev.Mb) {
        rg_status st = build_divfree_maps(p);
        if (st != RG_OK) return st;
        // the device copy is transposed per column: [nin][nout]
        std::vector<double> MT(p->Mb.size());
        const size_t blk = (size_t)p->nout * p->nin;
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < p->ntri; t++)
            for (int o = 0; o < p->nout; o++)
                for (int j = 0; j < p->nin; j++)
                    MT[t * blk + (size_t)j * p->nout + o] = p->Mb[t * blk + (size_t)o * p->nin + j];
        if (!upload(p, MT, &p->dev.Mb)) { set_error("device allocation of the divergence-free maps failed"); return RG_ENOMEM; }
    }
    return launch_prism_divfree(p->dev, Bin, Bout, stream);
}

rg_status rg_prism_update(const rg_prism *p, double dt, const double *U, const double *Phi, double *Uo, void *stream)
{
    if (!p || !U || !Phi || !Uo) { set_error("null argument"); return RG_EINVAL; }
    if (!(dt >= 0.0)) { set_error("need dt >= 0"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    return launch_prism_update(p->dev, dt, U, Phi, Uo, stream);
}

rg_status rg_prism_face_fluxes(const rg_prism *p, double gamma, const double *tr, double *Phi, void *stream)
{
    if (!p || !tr || !Phi) { set_error("null argument"); return RG_EINVAL; }
    if (!(gamma > 1.0)) { set_error("need gamma > 1"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    return launch_prism_face_flux(p->dev, gamma, tr, Phi, stream);
}

rg_status rg_prism_face_points(const rg_prism *p, double *xi, double *w, int32_t *n_tri_points, int32_t *n_side_points)
{
    if (!p) { set_error("null argument"); return RG_EINVAL; }
    for (int q = 0; q < p->ref.Q; q++) {
        if (xi)
            for (int k = 0; k < 3; k++) xi[3 * q + k] = p->ref.fpt[q][k];
        if (w) w[q] = p->ref.fw[q];
    }
    if (n_tri_points) *n_tri_points = p->ref.QT;
    if (n_side_points) *n_side_points = p->ref.QS;
    return RG_OK;
}

rg_status rg_prism_traces(const rg_prism *p, const double *avgU, const double *avgF, double *tr, void *stream)
{
    if (!p || !avgU || !avgF || !tr) { set_error("null argument"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    return launch_prism_traces(p->dev, avgU, avgF, tr, stream);
}

rg_status rg_prism_triangles(const rg_prism *p, double *abc)
{
    if (!p || !abc) { set_error("null argument"); return RG_EINVAL; }
    std::memcpy(abc, p->tri.data(), p->tri.size() * sizeof(double));
    return RG_OK;
}

rg_status rg_prism_geometry(const rg_prism *p, int64_t z0, int64_t nz, double *x, double *J, double *met)
{
    if (!p) { set_error("null argument"); return RG_EINVAL; }
    if (z0 < 0 || nz < 0 || z0 + nz > p->nz) { set_error("zone range outside the mesh"); return RG_EINVAL; }
    const int N = p->ref.N;
    for (int64_t zz = 0; zz < nz; zz++) {
        const int64_t z = z0 + zz, t = z / p->n_rad;
        const double s = p->radius[z % p->n_rad];
        for (int i = 0; i < N; i++) {
            if (x)
                for (int k = 0; k < 3; k++) x[(zz * N + i) * 3 + k] = s * p->hx[((size_t)t * N + i) * 3 + k];
            if (J) J[zz * N + i] = s * s * s * p->hJ[(size_t)t * N + i];
            if (met)
                for (int m = 0; m < 9; m++) met[(zz * N + i) * 9 + m] = s * s * p->hM[((size_t)t * 9 + m) * N + i];
        }
    }
    return RG_OK;
}

rg_status rg_prism_work(const rg_prism *p, int32_t n_picard, double *flops_per_zone, double *bytes_per_zone)
{
    if (!p || !flops_per_zone || !bytes_per_zone) { set_error("null argument"); return RG_EINVAL; }
    if (n_picard < 0 || n_picard > 16) { set_error("n_picard outside 0..16"); return RG_EINVAL; }
    const double N = p->ref.N, E = p->ref.M - 1;
    int nnz = 0;
    for (double v : p->ref.D) nnz += std::fabs(v) > 1e-14;
    // sweeps: the tau = 0 flux, then every level in each further iteration
    const double sweeps = n_picard > 0 ? 1.0 + (n_picard - 1) * E : 1.0;
    const double MAPPED_FLUX = 149.0, PHYS_FLUX = 94.0;
    double f = sweeps * (MAPPED_FLUX * N + 2.0 * 8 * nnz + 2.0 * 8 * N);       // fluxes, sum_d D_d F_d
    if (n_picard > 0) f += 2.0 * 8 * N * E + (n_picard - 1) * 8 * N * E * (2.0 + 2.0 * E);  // level updates
    f += 18.0 * N;                                                              // J U, scaled metrics
    f += (8.0 + PHYS_FLUX + 64.0) * N * E;                                      // time averages
    *flops_per_zone = f;
    // Ua read, avgU and avgF written, the column's geometry shared by its shells
    *bytes_per_zone = 8.0 * (8 * N + 8 * N + 24 * N) + 8.0 * 10 * N / p->n_rad;
    return RG_OK;
}

rg_status rg_prism_predict(const rg_prism *p, double gamma, double dt, int32_t n_picard, const double *Ua,
                           double *avgU, double *avgF, void *stream)
{
    if (!p || !Ua || !avgU || !avgF) { set_error("null argument"); return RG_EINVAL; }
    if (!p->device) { set_error("host-only prism mesh (rg_prism_build_host) has no device geometry"); return RG_EINVAL; }
    if (!(gamma > 1.0) || !(dt >= 0.0) || n_picard < 0 || n_picard > 16) {
        set_error("need gamma > 1, dt >= 0 and 0 <= n_picard <= 16");
        return RG_EINVAL;
    }
    return launch_prism_predict(p->dev, dt, gamma, n_picard, Ua, avgU, avgF, stream);
}

}  // extern "C"

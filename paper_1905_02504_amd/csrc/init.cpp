// Host initial data: circularly polarised Alfven wave (with optional
// multiplicative noise in density and pressure) and the spherical shock tubes
// of Section VIII.c.  Zone averages by a Gauss cubature of each zone's
// isoparametric map; face-averaged normal B from the circulation of the vector
// potential around each face (Stokes), which makes the discrete divergence
// vanish to round-off.  The tubes' radial field B_r ~ sin(theta) / r^2 carries
// the same flux through every sphere, so it has no vector potential on the
// shell; its face fluxes are added per column instead (radial_flux).
#include <cmath>
#include <cstring>

#include "rg_geom_host.hpp"

using namespace rg;

namespace {

struct Wave {
    double e1[3], e2[3], a[3], rho, p, B0, dB, kw, t, gam;
    void eval(const double *x, double &rh, double *v, double &pp, double *B, double *A) const
    {
        double vA = B0 / std::sqrt(rho);
        double ph = kw * (x[0] * a[0] + x[1] * a[1] + x[2] * a[2] - vA * t);
        double cs = std::cos(ph), sn = std::sin(ph);
        double axr[3] = {a[1] * x[2] - a[2] * x[1], a[2] * x[0] - a[0] * x[2], a[0] * x[1] - a[1] * x[0]};
        rh = rho;
        pp = p;
        for (int i = 0; i < 3; i++) {
            double tr = cs * e1[i] + sn * e2[i];
            B[i] = B0 * a[i] + dB * tr;
            v[i] = -dB / std::sqrt(rho) * tr;
            A[i] = 0.5 * B0 * axr[i] - dB / kw * tr;
        }
    }
};

// Spherical shock tube, pole on the z axis: primitive states
// (rho, p, v_r, v_theta, v_phi, B_theta, B_phi) inside and outside r = rm with
// no taper; B = Br0 sin(theta) (r0/r)^2 r_hat + (sin(theta)/2) T(r) phi_hat,
// T(r) = BphiL (1 - tanh((r - rm)/delta)) + BphiR (1 + tanh((r - rm)/delta)).
// The toroidal part is the curl of A = A_r r_hat with A_r = (z/2) T(r); the
// radial part enters through radial_flux.
struct Tube {
    double L[7], R[7], Br0, r0, rm, delta;
    void eval(const double *x, double &rh, double *v, double &pp, double *B, double *A) const
    {
        const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double s = std::sqrt(x[0] * x[0] + x[1] * x[1]);
        const double sin_t = s / r, cos_t = x[2] / r;
        double er[3] = {x[0] / r, x[1] / r, x[2] / r}, et[3] = {0.0, 0.0, -sin_t}, ep[3] = {0.0, 0.0, 0.0};
        if (s > 0.0) {
            et[0] = cos_t * x[0] / s;
            et[1] = cos_t * x[1] / s;
            ep[0] = -x[1] / s;
            ep[1] = x[0] / s;
        }
        const double *st = r <= rm ? L : R;
        const double h = std::tanh((r - rm) / delta);
        const double T = L[6] * (1.0 - h) + R[6] * (1.0 + h);
        const double br = Br0 * sin_t * (r0 / r) * (r0 / r), bp = 0.5 * sin_t * T;
        rh = st[0];
        pp = st[1];
        for (int i = 0; i < 3; i++) {
            v[i] = st[2] * er[i] + st[3] * et[i] + st[4] * ep[i];
            B[i] = br * er[i] + bp * ep[i];
            A[i] = 0.5 * x[2] * T * er[i];
        }
    }
};

// Magnetised blast (Section VIII.b): density rho, gas at rest, pressure pin
// inside the ball |x - c| < R and p outside, uniform B = B0 a with
// A = (B0/2) a x r.
struct Blast {
    double a[3], c[3], R, rho, pin, p, B0;
    void eval(const double *x, double &rh, double *v, double &pp, double *B, double *A) const
    {
        const double d0 = x[0] - c[0], d1 = x[1] - c[1], d2 = x[2] - c[2];
        rh = rho;
        pp = d0 * d0 + d1 * d1 + d2 * d2 < R * R ? pin : p;
        const double axr[3] = {a[1] * x[2] - a[2] * x[1], a[2] * x[0] - a[0] * x[2], a[0] * x[1] - a[1] * x[0]};
        for (int i = 0; i < 3; i++) {
            v[i] = 0.0;
            B[i] = B0 * a[i];
            A[i] = 0.5 * B0 * axr[i];
        }
    }
};

const int LF_EDGE[4] = {4, 5, 0, 1};
const int LF_FROMTO[4][2] = {{0, 3}, {1, 2}, {0, 1}, {3, 2}};

// Zone averages of the conserved variables (na x na x nr Gauss points per
// zone; 4 x 4 x 3 unless given).  With only(c, k) set, only the zones it
// accepts are written.
template <class F>
void zone_averages(const rg_geom *g, const F &fld, double gamma, const double *noise, double noise_amp, double *U,
                   int na = 4, int nr = 3, bool (*only)(const rg_geom *, const void *, int, int) = nullptr,
                   const void *only_arg = nullptr)
{
    const Mesh &m = g->mesh->m;
    const int K = m.K, mo = m.map_order;
    const int64_t Z = m.nzones;
    double ax[16], aw[16], rx[16], rw[16];
    gauss_legendre01(na, ax, aw);
    gauss_legendre01(nr, rx, rw);
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < m.ncol; c++) {
        const double *sn = &g->snode[(size_t)c * 48];
        for (int k = 0; k < K; k++) {
            if (only && !only(g, only_arg, c, k)) continue;
            int64_t z = (int64_t)c * K + k;
            double acc[8] = {0}, vol = 0.0;
            for (int kk = 0; kk < nr; kk++)
                for (int j = 0; j < na; j++)
                    for (int i = 0; i < na; i++) {
                        double xi[3] = {ax[i] - 0.5, ax[j] - 0.5, rx[kk] - 0.5}, x[3], jac[9];
                        zone_map(mo, sn, m.radius[k], m.radius[k + 1], xi, x, jac);
                        double J = jac[0] * (jac[4] * jac[8] - jac[5] * jac[7]) - jac[1] * (jac[3] * jac[8] - jac[5] * jac[6]) +
                                   jac[2] * (jac[3] * jac[7] - jac[4] * jac[6]);
                        double wq = aw[i] * aw[j] * rw[kk] * J;
                        double rh, v[3], pp, B[3], A[3];
                        fld.eval(x, rh, v, pp, B, A);
                        if (noise) {
                            rh *= 1.0 + noise_amp * noise[z];
                            pp *= 1.0 + noise_amp * noise[Z + z];
                        }
                        double u[8] = {rh, rh * v[0], rh * v[1], rh * v[2],
                                       pp / (gamma - 1) + 0.5 * rh * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
                                           0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]),
                                       B[0], B[1], B[2]};
                        for (int q = 0; q < 8; q++) acc[q] += wq * u[q];
                        vol += wq;
                    }
            for (int q = 0; q < 8; q++) U[(int64_t)q * Z + z] = acc[q] / vol;
        }
    }
}

// Face-averaged normal curl A: the circulation of A along every edge (5-point
// Gauss on each of nsub equal pieces, canonical direction), summed around
// each face with the face's orientation and divided by its area
template <class F>
void stokes_faces_host(const rg_geom *g, const F &fld, int nsub, double *Bf)
{
    const Mesh &m = g->mesh->m;
    const int K = m.K, mo = m.map_order;
    double gx[8], gw[8];
    gauss_legendre01(5, gx, gw);
    std::vector<double> Gam(m.nedges, 0.0);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < m.nv; v++) {
        const double *vh = &m.vpos[3 * v];
        for (int k = 0; k < K; k++) {
            double s = 0.0, len = m.radius[k + 1] - m.radius[k];
            for (int j = 0; j < nsub; j++)
                for (int q = 0; q < 5; q++) {
                    double r = m.radius[k] + (j + gx[q]) / nsub * len, x[3] = {r * vh[0], r * vh[1], r * vh[2]};
                    double rh, vv[3], pp, B[3], A[3];
                    fld.eval(x, rh, vv, pp, B, A);
                    s += gw[q] * len / nsub * (A[0] * vh[0] + A[1] * vh[1] + A[2] * vh[2]);
                }
            Gam[(int64_t)v * K + k] = s;
        }
    }
#pragma omp parallel for schedule(static)
    for (int ae = 0; ae < m.nae; ae++) {
        int c0 = m.ae_col[2 * ae], lf0 = m.ae_lf[2 * ae], le = LF_EDGE[lf0];
        bool rev = m.col_v[4 * c0 + LF_FROMTO[lf0][0]] != m.ae_v[2 * ae];
        const double *sn = &g->snode[(size_t)c0 * 48];
        for (int kf = 0; kf <= K; kf++) {
            double s = 0.0, r = m.radius[kf];
            for (int j = 0; j < nsub; j++)
                for (int q = 0; q < 5; q++) {
                    double xi[3], x[3], jac[9], sp = (j + gx[q]) / nsub;
                    edge_ref_point(le, rev ? 1.0 - sp : sp, xi);
                    zone_map(mo, sn, r, r, xi, x, jac);
                    double rh, vv[3], pp, B[3], A[3];
                    fld.eval(x, rh, vv, pp, B, A);
                    double sg = rev ? -1.0 : 1.0;
                    s += gw[q] / nsub * sg * (A[0] * jac[le / 4] + A[1] * jac[3 + le / 4] + A[2] * jac[6 + le / 4]);
                }
            Gam[m.nre + (int64_t)ae * (K + 1) + kf] = s;
        }
    }
    const int TRAV[4][2] = {{3, 0}, {1, 2}, {0, 1}, {2, 3}};
#pragma omp parallel for schedule(static)
    for (int c = 0; c < m.ncol; c++)
        for (int kf = 0; kf <= K; kf++) {
            double circ = 0.0;
            for (int lf = 0; lf < 4; lf++) {
                int ae = m.col_ae[4 * c + lf];
                int sg = (m.col_v[4 * c + TRAV[lf][0]] == m.ae_v[2 * ae]) ? 1 : -1;
                circ += sg * Gam[m.nre + (int64_t)ae * (K + 1) + kf];
            }
            int64_t f = (int64_t)c * (K + 1) + kf;
            Bf[f] = circ / g->farea[f];
        }
#pragma omp parallel for schedule(static)
    for (int ae = 0; ae < m.nae; ae++)
        for (int k = 0; k < K; k++) {
            int64_t ea = m.nre + (int64_t)ae * (K + 1) + k;
            double lp = Gam[ea] + Gam[(int64_t)m.ae_v[2 * ae + 1] * K + k] - Gam[ea + 1] - Gam[(int64_t)m.ae_v[2 * ae] * K + k];
            int64_t f = m.nrf + (int64_t)ae * K + k;
            Bf[f] = g->ae_rs_host[ae] * lp / g->farea[f];
        }
}

// Flux of Br0 r0^2 sin(theta) r_hat / r^2 through the radial faces (canonical
// normal +r).  A column's map is R(zeta) S(xi, eta), so all its radial faces
// subtend the same solid angle and carry the same flux: the integral of
// Br0 r0^2 sin(theta) (S . (S_xi x S_eta)) / |S|^3 over the reference square
// (6 x 6 Gauss), computed once per column.  Its angular faces, ruled along
// radial lines, carry none, so the discrete divergence stays at round-off.
void radial_flux(const rg_geom *g, const Tube &tb, double *Bf)
{
    const Mesh &m = g->mesh->m;
    const int K = m.K, mo = m.map_order;
    double gx[8], gw[8];
    gauss_legendre01(6, gx, gw);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < m.ncol; c++) {
        const double *sn = &g->snode[(size_t)c * 48];
        double flux = 0.0;
        for (int j = 0; j < 6; j++)
            for (int i = 0; i < 6; i++) {
                double xi[3] = {gx[i] - 0.5, gx[j] - 0.5, -0.5}, x[3], jac[9];
                zone_map(mo, sn, 1.0, 1.0, xi, x, jac);
                const double nx = jac[3] * jac[7] - jac[6] * jac[4], ny = jac[6] * jac[1] - jac[0] * jac[7],
                             nz = jac[0] * jac[4] - jac[3] * jac[1];
                const double R = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                const double sin_t = std::sqrt(x[0] * x[0] + x[1] * x[1]) / R;
                flux += gw[i] * gw[j] * sin_t * std::fabs(x[0] * nx + x[1] * ny + x[2] * nz) / (R * R * R);
            }
        flux *= tb.Br0 * tb.r0 * tb.r0;
        for (int kf = 0; kf <= K; kf++) {
            const int64_t f = (int64_t)c * (K + 1) + kf;
            Bf[f] += flux / g->farea[f];
        }
    }
}

}  // namespace

extern "C" rg_status rg_init_alfven(const rg_geom *g, const double *frame, double rho, double p, double B0, double dB,
                                    double wavelength, double gamma, double t, const double *noise, double noise_amp,
                                    double *U, double *Bf)
{
    if (!g || !frame || !U || !Bf || !(rho > 0) || !(p > 0) || !(wavelength > 0) || !(gamma > 1)) {
        set_error("invalid argument");
        return RG_EINVAL;
    }
    Wave w;
    for (int i = 0; i < 3; i++) { w.e1[i] = frame[i]; w.e2[i] = frame[3 + i]; w.a[i] = frame[6 + i]; }
    w.rho = rho; w.p = p; w.B0 = B0; w.dB = dB; w.kw = 2.0 * M_PI / wavelength; w.t = t; w.gam = gamma;
    zone_averages(g, w, gamma, noise, noise_amp, U);
    stokes_faces_host(g, w, 1, Bf);
    return RG_OK;
}

extern "C" rg_status rg_init_tube(const rg_geom *g, const double *left, const double *right, double Br0, double r0,
                                  double rm, double delta, double gamma, double *U, double *Bf)
{
    if (!g || !left || !right || !U || !Bf || !(r0 > 0) || !(rm > 0) || !(delta > 0) || !(gamma > 1)) {
        set_error("invalid argument");
        return RG_EINVAL;
    }
    if (!(left[0] > 0) || !(right[0] > 0) || !(left[1] > 0) || !(right[1] > 0)) {
        set_error("rg_init_tube: densities and pressures must be positive");
        return RG_EINVAL;
    }
    if (left[5] != 0.0 || right[5] != 0.0) {
        set_error("rg_init_tube: B_theta must be 0 (the toroidal field comes from a radial vector potential)");
        return RG_EINVAL;
    }
    Tube tb;
    for (int i = 0; i < 7; i++) { tb.L[i] = left[i]; tb.R[i] = right[i]; }
    tb.Br0 = Br0; tb.r0 = r0; tb.rm = rm; tb.delta = delta;
    zone_averages(g, tb, gamma, nullptr, 0.0, U);
    stokes_faces_host(g, tb, 4, Bf);
    radial_flux(g, tb, Bf);
    return RG_OK;
}

namespace {
// zones that the ball's surface may cut: the centroid is within the ball's
// radius plus the zone's largest centroid-to-corner distance of its centre
bool blast_cut(const rg_geom *g, const void *arg, int c, int k)
{
    const Blast &b = *static_cast<const Blast *>(arg);
    const Mesh &m = g->mesh->m;
    const int64_t z = (int64_t)c * m.K + k;
    const double *cen = &g->zcen[(size_t)z * 3];
    double reach = 0.0;
    for (int corner = 0; corner < 8; corner++) {
        double xi[3] = {(corner & 1) ? 0.5 : -0.5, (corner & 2) ? 0.5 : -0.5, (corner & 4) ? 0.5 : -0.5}, x[3], jac[9];
        zone_map(m.map_order, &g->snode[(size_t)c * 48], m.radius[k], m.radius[k + 1], xi, x, jac);
        reach = std::max(reach, std::sqrt((x[0] - cen[0]) * (x[0] - cen[0]) + (x[1] - cen[1]) * (x[1] - cen[1]) +
                                          (x[2] - cen[2]) * (x[2] - cen[2])));
    }
    const double d = std::sqrt((cen[0] - b.c[0]) * (cen[0] - b.c[0]) + (cen[1] - b.c[1]) * (cen[1] - b.c[1]) +
                               (cen[2] - b.c[2]) * (cen[2] - b.c[2]));
    return d < b.R + 1.01 * reach;
}
}  // namespace

extern "C" rg_status rg_init_blast(const rg_geom *g, const double *axis, const double *centre, double radius,
                                   double rho, double p_in, double p, double B0, double gamma, double *U, double *Bf)
{
    if (!g || !axis || !centre || !U || !Bf || !(radius > 0) || !(rho > 0) || !(p_in > 0) || !(p > 0) ||
        !(gamma > 1)) {
        set_error("invalid argument");
        return RG_EINVAL;
    }
    Blast b;
    for (int i = 0; i < 3; i++) { b.a[i] = axis[i]; b.c[i] = centre[i]; }
    b.R = radius; b.rho = rho; b.pin = p_in; b.p = p; b.B0 = B0;
    // the step function's average: 4 x 4 x 3 points where it is constant, 12 x 12 x 12 where the sphere may cut
    zone_averages(g, b, gamma, nullptr, 0.0, U);
    zone_averages(g, b, gamma, nullptr, 0.0, U, 12, 12, blast_cut, &b);
    stokes_faces_host(g, b, 1, Bf);
    return RG_OK;
}

// Host initial data: circularly polarised Alfven wave (with optional
// multiplicative noise in density and pressure).  Zone averages by a Gauss
// cubature of each zone's isoparametric map; face-averaged normal B from the
// circulation of the vector potential around each face (Stokes), which makes
// the discrete divergence vanish to round-off.
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

const int LF_EDGE[4] = {4, 5, 0, 1};
const int LF_FROMTO[4][2] = {{0, 3}, {1, 2}, {0, 1}, {3, 2}};

}  // namespace

extern "C" rg_status rg_init_alfven(const rg_geom *g, const double *frame, double rho, double p, double B0, double dB,
                                    double wavelength, double gamma, double t, const double *noise, double noise_amp,
                                    double *U, double *Bf)
{
    if (!g || !frame || !U || !Bf || !(rho > 0) || !(p > 0) || !(wavelength > 0) || !(gamma > 1)) {
        set_error("invalid argument");
        return RG_EINVAL;
    }
    const Mesh &m = g->mesh->m;
    Wave w;
    for (int i = 0; i < 3; i++) { w.e1[i] = frame[i]; w.e2[i] = frame[3 + i]; w.a[i] = frame[6 + i]; }
    w.rho = rho; w.p = p; w.B0 = B0; w.dB = dB; w.kw = 2.0 * M_PI / wavelength; w.t = t; w.gam = gamma;
    const int K = m.K, mo = m.map_order;
    const int64_t Z = m.nzones;
    const int na = 4, nr = 3;
    double ax[8], aw[8], rx[8], rw[8], gx[8], gw[8];
    gauss_legendre01(na, ax, aw);
    gauss_legendre01(nr, rx, rw);
    gauss_legendre01(5, gx, gw);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < m.ncol; c++) {
        const double *sn = &g->snode[(size_t)c * 48];
        for (int k = 0; k < K; k++) {
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
                        w.eval(x, rh, v, pp, B, A);
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
    // circulation of A along every edge, canonical direction
    std::vector<double> Gam(m.nedges, 0.0);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < m.nv; v++) {
        const double *vh = &m.vpos[3 * v];
        for (int k = 0; k < K; k++) {
            double s = 0.0, len = m.radius[k + 1] - m.radius[k];
            for (int q = 0; q < 5; q++) {
                double r = m.radius[k] + gx[q] * len, x[3] = {r * vh[0], r * vh[1], r * vh[2]};
                double rh, vv[3], pp, B[3], A[3];
                w.eval(x, rh, vv, pp, B, A);
                s += gw[q] * len * (A[0] * vh[0] + A[1] * vh[1] + A[2] * vh[2]);
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
            for (int q = 0; q < 5; q++) {
                double xi[3], x[3], jac[9];
                edge_ref_point(le, rev ? 1.0 - gx[q] : gx[q], xi);
                zone_map(mo, sn, r, r, xi, x, jac);
                double rh, vv[3], pp, B[3], A[3];
                w.eval(x, rh, vv, pp, B, A);
                double sg = rev ? -1.0 : 1.0;
                s += gw[q] * sg * (A[0] * jac[le / 4] + A[1] * jac[3 + le / 4] + A[2] * jac[6 + le / 4]);
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
    return RG_OK;
}

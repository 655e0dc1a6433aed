// Host-side geometry precompute: per-column shell-0 data and the flat host
// arrays that are uploaded to the device.
#pragma once

#include <algorithm>
#include <vector>

#include "rg_internal.hpp"

namespace rg {

bool build_mesh(const rg_mesh_desc &d, Mesh &m);

struct ColData {
    double sn[16 * 3];
    double cen[3], vol = 0, len = 0;
    double mom[125];
    double fx[6][9][3], fn[6][9][3], fdA[6][9], farea[6], fcen[6][3], fnbar[6][3];
    double dins = 0;
    std::vector<double> nx, nJ, nM;
};

struct HostGeom {
    std::vector<int> stm, stn;
    std::vector<double> Pl, Ps, Qs, Ev, Mb, nJ, nM, fevR, fnR, fwR, dins;
    // per column: 2-norm condition number of the large-stencil least-squares
    // matrix, 1-norm condition number of the divergence-free KKT matrix
    std::vector<double> cond_lsq, cond_kkt;
    std::vector<int> col_ae, col_side, col_perm, col_v, col_slot, col_rev, col_sgn;
    std::vector<double> fevA, fnA, fwA, aeF, aeW;
    std::vector<int> ae_rs;
    std::vector<double> vF, vN3;
    // query data
    std::vector<double> emid_ae, etan_ae, fcen_ae, fnrm_ae, farea_ae;
};

void column_surface_nodes(const Mesh &m, int c, double *sn);
// point at fraction t of the great-circle arc from unit vector a to b
void arc_point(const double *a, const double *b, double t, double *o);
// frame of the four-state edge field: u and w (east minus west, north minus
// south) projected off the unit tangent t and normalised, their bisector b
// and t x b turned by 45 degrees into e1 = (b - t x b)/sqrt 2, e2 = (b + t x b)/sqrt 2
void symmetric_frame(const double *u0, const double *w0, const double *t, double *e1, double *e2);
void zone_map(int mo, const double *sn, double r0, double r1, const double *xi, double *x, double *jac);
int moment_index(int a, int b, int c);
void column_pass1(const Mesh &m, const RefEl &r, int c, ColData &cd);
bool column_pass2(const Mesh &m, const RefEl &r, const std::vector<ColData> &cols, int c, HostGeom &hg);
void angular_edge_pass(const Mesh &m, const RefEl &r, const std::vector<ColData> &cols, int ae, HostGeom &hg);
void vertex_pass(const Mesh &m, const RefEl &r, const std::vector<ColData> &cols, int v, HostGeom &hg);
void column_pass4(const Mesh &m, const HostGeom &hg, int c, HostGeom &out);

// device step, implemented in the HIP translation unit
rg_status launch_step(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, double *Uo,
                      double *Bo, void *stream);
rg_status profile_end(rg_geom *g, double *ms, int *nsteps);
rg_status launch_cfl(rg_geom *g, const double *U, double gamma, double cfl, void *stream, double *dt);
// the same reduction through a file-scope device array (no allocation)
rg_status launch_cfl_noalloc(rg_geom *g, const double *U, double gamma, double cfl, void *stream, double *dt);
// stages 0-4 of the step only (boundary fill into Uo / Bo, reconstruction,
// divergence-free B, predictor and traces), FP64
rg_status launch_step_front(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, double *Uo,
                            double *Bo, void *stream);
rg_status launch_adjoint(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, const double *gU1,
                         const double *gBf1, double *gU, double *gBf, void *stream);
rg_status launch_stokes(rg_geom *g, const double *circ, double *Bf, void *stream);
rg_status launch_stokes_T(rg_geom *g, const double *gBf, double *gcirc, void *stream);
rg_status launch_fma_probe(double *sink, long long n_threads, int iters, void *stream);
rg_status launch_mfma_probe(double *sink, long long n_threads, int iters, int kind, void *stream);
rg_status launch_diag(rg_geom *g, const double *U, const double *Bf, double gamma, void *stream, rg_diag_out *out);

}  // namespace rg

/*
 * rg -- one ADER-WENO-AO divergence-free ideal-MHD timestep on a radially
 * extruded cube-based geodesic mesh of isoparametric hexahedra, on one AMD
 * Instinct MI355X (gfx950).
 *
 * The scheme is the one of Balsara, Florinski, Garain, Subramanian & Gurski,
 * "Efficient, divergence-free, high order MHD on 3D spherical meshes with
 * optimal geodesic meshing" (2019): WENO-AO reconstruction in a Taylor basis
 * (Section III), divergence-free reconstruction of B from face averages
 * (Section IV), ADER-CG space-time predictor on serendipity elements
 * (Section V), and a corrector with 1-D Riemann solvers at face quadrature
 * points, multidimensional Riemann solvers at edges and Yee-type constrained
 * transport (Sections II.c and VI).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All calls return rg_status; on failure rg_last_error() (thread-local)
 *   describes the problem.  Nothing throws across this boundary.
 * - Mesh and geometry are opaque, library-owned handles (free with
 *   rg_mesh_free / rg_geom_free).  State arrays are caller-owned.
 * - Zones: columns are numbered col = (patch * N + j) * N + i for the six
 *   cube patches of N x N columns; each column holds K = n_rad + 2 * n_ghost
 *   shells (n_ghost ghost shells below r_in and above r_out).  Zone
 *   z = col * K + k, radial index fastest.
 * - U is double[8][n_zones] (structure of arrays): rho, rho v_x, rho v_y,
 *   rho v_z, total energy, B_x, B_y, B_z, zone averages, rationalised units
 *   (magnetic pressure B^2 / 2), i.e. eq. (2.2) with 4 pi absorbed into B.
 * - Bf is double[n_faces]: face-averaged normal B, the primal magnetic
 *   variable.  Radial faces come first, id = col * (K + 1) + kf (kf = index
 *   of the interface, normal +r); then angular faces, id = n_radial_faces +
 *   ae * K + k (normal from the first to the second column of angular edge
 *   ae, as reported by rg_geom_face_data).
 * - Edges: radial edges id = v * K + k (direction +r), then angular edges
 *   id = n_radial_edges + ae * (K + 1) + kf.
 * - Device pointers are HIP device memory; streams are hipStream_t passed as
 *   void*.  Work is asynchronous on the stream unless stated otherwise.
 */
#ifndef RG_H
#define RG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RG_OK = 0,
    RG_EINVAL = 1,     /* bad argument (sizes, pointers, unsupported combination) */
    RG_ENOMEM = 2,     /* host or device allocation failed                        */
    RG_ESINGULAR = 3,  /* a least-squares or KKT system was singular at precompute */
    RG_ENOTSUP = 4,    /* order / mode / mesh size not supported                  */
    RG_EDEVICE = 5     /* a HIP runtime call failed                               */
} rg_status;

/* Geodesic shell mesh, Section II.a (cube-based, recursive great-circle
 * bisection, N = 2^k zones per cube edge; for N = 3 * 2^k each cube face is
 * first split 3 x 3, its edges at their thirds by arc length and the interior
 * points where the great circles joining opposite edges' thirds meet) with
 * radial extrusion into shells of geometrically growing thickness
 * (self-similar zones, Section V.b). */
typedef struct {
    int32_t n_ang;      /* zones per cube edge: 2^k (k >= 1) or 3 * 2^k (k >= 0) */
    int32_t n_rad;      /* physical radial shells                               */
    double r_in, r_out; /* inner / outer radius, 0 < r_in < r_out               */
    int32_t radial;     /* 0 = geometric shells r_k = r_in (r_out/r_in)^(k/n_rad) */
    int32_t map_order;  /* isoparametric surface map: 2 quadratic, 3 cubic (II.b) */
    int32_t n_ghost;    /* ghost shells on each side; 0 selects 3               */
} rg_mesh_desc;

typedef struct {
    int64_t n_ang, n_rad, n_ghost, n_shells; /* n_shells = K = n_rad + 2 n_ghost */
    int64_t n_columns, n_zones;
    int64_t n_faces, n_radial_faces;
    int64_t n_edges, n_radial_edges;
    int64_t n_vertices, n_angular_edges;
} rg_mesh_info;

typedef struct rg_mesh rg_mesh;
typedef struct rg_geom rg_geom;

/* Builds the mesh topology on the host.  Deterministic.  *out receives a
 * handle owned by the caller (rg_mesh_free).  RG_ENOTSUP if n_ang is neither
 * 2^k nor 3 * 2^k, RG_EINVAL for other bad fields. */
rg_status rg_mesh_build(const rg_mesh_desc *desc, rg_mesh **out);
rg_status rg_mesh_get_info(const rg_mesh *mesh, rg_mesh_info *info);
void rg_mesh_free(rg_mesh *mesh);

/* Precision of the reconstruction and predictor contractions (the paper's
 * scheme is FP64 throughout; RG_MODE_FP32 and RG_MODE_BF16 are the
 * reduced-precision forms).
 * In RG_MODE_FP32 the WENO-AO contractions and weights, the face nodal B
 * contractions, the ADER-CG predictor (fluxes, derivatives, Picard updates,
 * time averages) and the face / edge traces are computed and stored in FP32,
 * from FP32 copies of the per-column tables.  Geometry precompute, the state
 * U and Bf, the divergence-free map (FP64 matrix cores), the Riemann solvers,
 * the conservative update and constrained transport stay FP64, so div B
 * stays at round-off in either mode. */
typedef enum { RG_MODE_FP64 = 0, RG_MODE_FP32 = 1, RG_MODE_BF16 = 2 } rg_mode;
/* RG_MODE_BF16 is RG_MODE_FP32 with the predictor's flux derivatives (the
 * contraction sum_d D_d F_d of eqs. 5.24-5.29 applied at every Picard level,
 * Section V.d) on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
 * accumulation: the derivative matrices' entries are multiples of 1/2 and
 * exact in BF16, each FP32 flux value is split exactly into three BF16 parts
 * (x = hi + mid + lo, by truncation), and the three products are summed in
 * FP32, so the derivative keeps FP32 accuracy.  Everything else is as in
 * RG_MODE_FP32.  rg_step_adjoint refuses it (RG_ENOTSUP). */

/* Geometry precompute (Section VI step 1): FP64 on the host, one radial column
 * at a time (zones of a column are self-similar, Section V.b), then one upload
 * to the device on `stream`.  order is 3 or 4 (the scheme's order; the mesh
 * map_order should be order-1).  Requires n_ghost >= order - 1.  The mesh
 * must outlive the geometry.  RG_ESINGULAR if a least-squares or KKT system
 * is singular.  Synchronous with respect to `stream` on return. */
rg_status rg_geom_precompute(const rg_mesh *mesh, int32_t order, int32_t mode, void *stream, rg_geom **out);
void rg_geom_free(rg_geom *geom);

/* The same precompute without any device allocation or upload: for host-side
 * checks and initial data (the query calls and rg_init_alfven work, rg_step,
 * rg_step_fluxes and rg_cfl_dt return RG_EINVAL).  Always FP64. */
rg_status rg_geom_precompute_host(const rg_mesh *mesh, int32_t order, rg_geom **out);

/* Host copies of geometric data, for checks and initial data.  Any pointer
 * may be NULL.  centroid: [n_zones][3], volume: [n_zones]; face centre and
 * unit normal (area-weighted mean, canonical orientation) [n_faces][3], area
 * [n_faces]; edge midpoint and unit tangent [n_edges][3]. */
rg_status rg_geom_zone_data(const rg_geom *geom, double *centroid, double *volume);
rg_status rg_geom_face_data(const rg_geom *geom, double *center, double *normal, double *area);
rg_status rg_geom_edge_data(const rg_geom *geom, double *midpoint, double *tangent);

/* Orientation tables of the Yee layout (Section II.c, eqs. 2.5-2.6), host
 * copies; any pointer may be NULL.  zone_face[n_zones][6]: a zone's faces in
 * the local order xi-, xi+, eta-, eta+ (angular), r-, r+ (radial), and
 * zone_face_sign[n_zones][6]: +1 where the face's canonical normal (as
 * reported by rg_geom_face_data) points out of the zone, -1 where it points
 * in.  face_edge[n_faces][4]: a face's four edges, and face_edge_sign
 * [n_faces][4]: +1 where the edge's canonical direction (rg_geom_edge_data)
 * runs with the circulation about the face's canonical normal (right-hand
 * rule), -1 where it runs against it; the CT update of eqs. (2.5)-(2.6) is
 * Bf[f] -= dt / area[f] * sum_j face_edge_sign[f][j] * E[face_edge[f][j]]. */
rg_status rg_geom_incidence(const rg_geom *geom, int64_t *zone_face, int8_t *zone_face_sign, int64_t *face_edge,
                            int8_t *face_edge_sign);

/* Conditioning of the per-column systems built by the precompute (Section
 * III's least squares on eq. (3.4) rows, Section IV.b's KKT system), host
 * copies of [n_columns] each; either pointer may be NULL.  cond_lsq: the
 * 2-norm condition number sigma_max / sigma_min of the large-stencil
 * least-squares matrix (rows: zone averages of the Taylor basis over the
 * stencil members, scaled coordinates).  cond_kkt: the 1-norm condition
 * number of the divergence-free KKT matrix (||K^-1||_1 by Hager's estimate).
 * Rounding in the geometry is amplified by up to these factors in the
 * reconstruction; thin zones (radial depth far below the angular width) and
 * cube-corner stencils raise them.  The precompute returns RG_ESINGULAR when
 * any column exceeds RG_COND_MAX. */
#define RG_COND_MAX 1e13
rg_status rg_geom_conditioning(const rg_geom *geom, double *cond_lsq, double *cond_kkt);

typedef struct {
    double gamma;     /* ratio of specific heats                                   */
    double dt;        /* timestep; if <= 0 it is computed from cfl (host sync) and
                         written back here                                         */
    double cfl;       /* CFL number for the in-sphere diameter (Section VIII)       */
    int32_t bc_kind;  /* 0: continuative (ghost shells copy the nearest interior
                         shell, Section VII); 1: ghost values supplied by the caller */
    int32_t n_picard; /* 0 selects the order (Section V.d step 9)                   */
    double weno_eps;  /* epsilon of the WENO-AO nonlinear weights
                         gamma_s / (beta_s + eps)^2 (Section III; beta in units of
                         the squared zone data); 0 selects 1e-4                   */
    int32_t fallback; /* 0: off; 1: first-order fallback for positivity (below)  */
    double flattener; /* 0: off; > 0: the flattener (below) with this threshold kappa */
} rg_step_params;

/* Flattener (params->flattener = kappa > 0).  Section VII.a applies a
 * flattener on its coarse meshes and leaves its definition to other work;
 * this step's reading: for every reconstructed zone, with
 * D = (1/V) sum_faces s_f S_f . (v + v_neighbour) / 2 the discrete divergence
 * of the zone averages' velocity (S_f the face's vector area, s_f = +1 on
 * outward faces), l0 = V^(1/3) and c the smallest sqrt(gamma p / rho +
 * B^2 / rho) over the zone and its six face neighbours,
 * eta = min(1, max(0, -(l0 D + kappa c) / (kappa c))), and every WENO-AO
 * coefficient of the zone (Section III; all eight variables) is scaled by
 * 1 - eta before the rest of the step uses it: a zone compressing faster than
 * kappa c / l0 drops toward first order, one compressing at 2 kappa c / l0 or
 * faster is first order.  rg_step_adjoint refuses it (RG_ENOTSUP). */

/* First-order fallback (params->fallback = 1).  Section I leaves positive
 * pressures under strong magnetic fields to ruggedised WENO schemes from
 * other work; this step takes an a-posteriori per-zone order drop.  After the
 * high-order face fluxes and edge electric fields are computed, every
 * interior zone whose update with them would leave a density or pressure
 * that is not positive (or not finite) is flagged; every face and every edge
 * of a flagged zone is then solved again with the same HLL and
 * multidimensional solvers, each trace replaced by its zone's conserved
 * state at t (its eight averages after the boundary fill), and a flagged
 * zone advances its B average from its own value rather than from the
 * reconstruction's mean, so that its update is the first-order
 * finite-volume scheme on its own averages.  A re-solved face
 * can drive a neighbour negative, so the check is repeated with the new
 * fluxes and the newly flagged zones are re-solved too, for up to
 * RG_FALLBACK_ROUNDS rounds (stopping when a round flags no new zone); the
 * update and the constrained transport then take the final values.
 * Conservation and the discrete div B of the face field are kept; a flagged
 * zone can still come out non-positive (rg_diag reports the minima).  The
 * unflagged neighbours of zones flagged in the last round are not checked
 * again: when rg_step_fallback_counts reports a non-zero count for the last
 * round the rounds ran out, and such a neighbour can come out non-positive
 * without a flag.  With no zone flagged the result equals the plain step bit
 * for bit; the extra passes cost a few per cent of the step.
 * rg_step_adjoint refuses it (RG_ENOTSUP). */
#define RG_FALLBACK_ROUNDS 4

/* One complete timestep (Section VI) on device buffers.
 * U, Bf: state at t (device, read only).  U_out, Bf_out: state at t + dt
 * (device).  U_out may equal U and Bf_out may equal Bf (in place).  Ghost
 * entries of U_out / Bf_out hold the boundary-filled input.  Interior zone B
 * of U_out is the divergence-free reconstruction's mean (Section IV.b step
 * 10) advanced by the face fluxes.  Asynchronous on `stream` unless
 * params->dt <= 0. */
rg_status rg_step(const rg_geom *geom, rg_step_params *params, const double *U, const double *Bf,
                  double *U_out, double *Bf_out, void *stream);

/* Adjoint of one rg_step (its vector-Jacobian product) at the state
 * (U_n, Bf_n), with params->dt held fixed (dt > 0 required: a dt taken from
 * the CFL condition would itself depend on the state).  Given the gradients
 * gU_np1[8][n_zones], gBf_np1[n_faces] of a scalar loss with respect to the
 * step's outputs U_out, Bf_out, writes the gradients gU_n, gBf_n with
 * respect to U_n, Bf_n (all device buffers, rg_step layout; the outputs may
 * not alias the incoming gradients).  Exact derivative of the computed
 * step: the Picard sweeps of the predictor (Section V.d) are differentiated
 * as unrolled, the WENO-AO weights (Section III) through their nonlinear
 * dependence, and at the kinks (MinMod of eq. 4.11, the HLL branch and the
 * min/max of the signal speeds) the branch the forward step took is
 * differentiated.  Recomputes the forward step internally (its work buffers
 * and rg_step_fluxes data are overwritten).  Deterministic: every gradient
 * is gathered by its owner, no floating-point atomics.  On an RG_MODE_FP32
 * geometry it is the adjoint of that form: the FP32 forward is recomputed, the
 * predictor is reversed in FP32 and the rest in FP64, and the gradients are
 * FP64.  Device work buffers are allocated on the first call (RG_ENOMEM).
 * Asynchronous on `stream`. */
rg_status rg_step_adjoint(const rg_geom *geom, const rg_step_params *params, const double *U_n, const double *Bf_n,
                          const double *gU_np1, const double *gBf_np1, double *gU_n, double *gBf_n, void *stream);

/* Discrete Stokes map (eqs. 2.5-2.6 without the time step): given line
 * integrals of a vector potential along every edge, edge_circ[n_edges]
 * (canonical edge direction), writes the face averages of the normal
 * component of its curl, Bf[f] = (1/A_f) sum_e s_fe edge_circ[e], for every
 * face (canonical normal; s_fe = +-1 by the right-hand rule).  The result is
 * divergence-free to round-off.  Device buffers; asynchronous on `stream`. */
rg_status rg_stokes(const rg_geom *geom, const double *edge_circ, double *Bf, void *stream);

/* Transpose of rg_stokes: g_edge_circ[e] = sum_f s_fe gBf[f] / A_f over every
 * face holding edge e (all edges written); turns a gradient with respect to
 * face B into one with respect to the edge line integrals of the vector
 * potential.  Device buffers; asynchronous on `stream`. */
rg_status rg_stokes_T(const rg_geom *geom, const double *gBf, double *g_edge_circ, void *stream);

/* Device copies of the last step's face flux integrals Phi[8][n_faces]
 * (time-integrated over the step divided by dt, canonical normal) and edge
 * electric-field line integrals Gam[n_edges] (canonical direction).  Entries
 * the step did not compute are zero.  Asynchronous on `stream`. */
rg_status rg_step_fluxes(const rg_geom *geom, double *Phi, double *Gam, void *stream);

/* Device copy of the last rg_step's fallback flags, flags[n_zones] (uint8):
 * 1 for every zone the first-order fallback took, 0 elsewhere (all 0 after a
 * step with the fallback off).  Asynchronous on `stream`. */
rg_status rg_step_fallback_zones(const rg_geom *geom, uint8_t *flags, void *stream);

/* Host copy of the last rg_step's fallback round counters,
 * counts[RG_FALLBACK_ROUNDS]: the number of zones each round newly flagged
 * (all 0 when the last step ran without the fallback).  A non-zero last
 * entry means the rounds ran out (see the fallback above).  Synchronises
 * `stream`. */
rg_status rg_step_fallback_counts(const rg_geom *geom, int32_t *counts, void *stream);

/* Device copy of the last rg_step's WENO-AO order indicator, whi[n_zones]
 * (float): for every zone of the reconstructed shells, the smallest over the
 * eight variables of the large stencil's nonlinear weight divided by its
 * linear weight (Section III; about 1 where the reconstruction keeps its full
 * order, near 0 where it has dropped to the small stencils).  Entries of other
 * zones are 0 until a step writes them.  Asynchronous on `stream`. */
rg_status rg_step_weno_order(const rg_geom *geom, float *whi, void *stream);

/* Timestep limit dt = cfl * min over interior zones of d_in / (|v| + c_f,max)
 * (Section VIII) for device state U; blocks until the result is on the host. */
rg_status rg_cfl_dt(const rg_geom *geom, const double *U, double gamma, double cfl, void *stream, double *dt);

/* rg_cfl_dt for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, but the block minima go
 * through a file-scope device array of 65,536 doubles (512 KiB, held by each
 * device the library runs on until the process ends) instead of the
 * geometry's buffer, and the call allocates nothing.  Meshes with more than
 * 65,535 x 256 = 16,776,960 interior zones are refused (RG_ENOTSUP).  The
 * array is shared by every call on a device: calls that overlap on one
 * device race.  Runs on the current device; blocks until dt is on the host. */
rg_status rg_cfl_dt_noalloc(const rg_geom *geom, const double *U, double gamma, double cfl, void *stream, double *dt);

/* Initial data on the host (caller-owned host arrays U[8][n_zones],
 * Bf[n_faces]) for a circularly polarised Alfven wave with axis frame
 * (e1, e2, a) = frame[0..8]: B = B0 a + dB (cos phi e1 + sin phi e2),
 * v = -(dB/sqrt(rho)) (cos phi e1 + sin phi e2), phi = 2 pi (x.a - v_A t) / wavelength.
 * Zone averages by the zone cubature; Bf from circulations of the vector
 * potential (divergence-free to round-off).  If noise is non-NULL it holds
 * double[2][n_zones] in [-1, 1] and the zone averages of rho and pressure are
 * multiplied by (1 + noise_amp * noise). */
rg_status rg_init_alfven(const rg_geom *geom, const double *frame, double rho, double p, double B0, double dB,
                         double wavelength, double gamma, double t, const double *noise, double noise_amp,
                         double *U, double *Bf);

/* Initial data on the host (caller-owned host arrays U[8][n_zones],
 * Bf[n_faces]) for the spherical shock tubes of Section VIII.c, with the pole
 * on the z axis.  left and right are double[7] primitive states
 * (rho, p, v_r, v_theta, v_phi, B_theta, B_phi) for r <= rm and r > rm; the
 * fluid jump has no taper.  B = Br0 sin(theta) (r0/r)^2 r_hat
 * + (sin(theta)/2) T(r) phi_hat with T(r) = B_phiL (1 - tanh((r - rm)/delta))
 * + B_phiR (1 + tanh((r - rm)/delta)): the toroidal part is the curl of the
 * radial vector potential A_r = (r cos(theta)/2) T(r) of that section, whose
 * edge circulations (5-point Gauss on four pieces of each edge) give the face
 * values by Stokes; the radial part, which has no vector potential on a shell,
 * adds to each radial face the flux through the solid angle it subtends (the
 * same number for all radial faces of a column), so Bf is divergence-free to
 * round-off.  Zone averages by the zone cubature.  Works on a host-only
 * geometry.  RG_EINVAL if a density or pressure is not positive, if
 * r0, rm, delta <= 0 or gamma <= 1, or if B_theta is not 0 on either side (a
 * radial potential cannot produce it). */
rg_status rg_init_tube(const rg_geom *geom, const double *left, const double *right, double Br0, double r0,
                       double rm, double delta, double gamma, double *U, double *Bf);

/* Initial data on the host (caller-owned host arrays U[8][n_zones],
 * Bf[n_faces]) for the magnetised blast of Section VIII.b: density rho, gas
 * at rest, pressure p_in inside the ball |x - centre| < radius and p outside,
 * uniform field B = B0 axis (axis: unit vector, double[3]; centre double[3]).
 * Zone averages by Gauss cubature of the pressure step (12 x 12 x 12 points
 * in zones the ball's surface may cut, 4 x 4 x 3 elsewhere); Bf from the
 * circulations of A = (B0/2) axis x r, divergence-free to round-off.  Works on
 * a host-only geometry.  RG_EINVAL unless radius, rho, p_in, p > 0 and
 * gamma > 1. */
rg_status rg_init_blast(const rg_geom *geom, const double *axis, const double *centre, double radius, double rho,
                        double p_in, double p, double B0, double gamma, double *U, double *Bf);

/* Diagnostics of a state on the device (for checks after a step; not part of
 * the scheme): over the interior zones, the largest relative divergence
 * |sum_faces sigma A <B.n>| / sum_faces A |<B.n>| (sigma = +1 on outward
 * faces), the volume-weighted sums sum V U_v of the eight conserved
 * variables, and the smallest density and gas pressure.  U and Bf are device
 * buffers in the rg_step layout.  Deterministic (fixed reduction order);
 * synchronises `stream` before returning. */
typedef struct {
    double div_rel_max;
    double sums[8];
    double rho_min, p_min;
} rg_diag_out;
rg_status rg_diag(const rg_geom *geom, const double *U, const double *Bf, double gamma, void *stream,
                  rg_diag_out *out);

/* Per-stage timing with HIP events recorded on the step's own stream.
 * After rg_profile_begin, every rg_step records events around its
 * RG_NSTAGES stages: 0 boundary fill, 1 WENO-AO, 2 face nodal B,
 * 3 divergence-free B map (KKT solve and evaluation at the ADER nodes, one
 * kernel), 4 ADER predictor + traces (one kernel), 5 face HLL fluxes,
 * 6 edge EMFs, 7 FV update + CT (with the passes of the first-order
 * fallback when it is on).  rg_profile_end waits for the recorded
 * events, writes the summed milliseconds of each stage to ms[RG_NSTAGES]
 * and the number of recorded steps to *nsteps, releases the events and
 * stops recording. */
#define RG_NSTAGES 8
rg_status rg_profile_begin(rg_geom *geom);
rg_status rg_profile_end(rg_geom *geom, double *ms, int32_t *nsteps);

/* Algorithmic work of one rg_step on this geometry with the default number
 * of Picard sweeps (the order), per stage (numbering of rg_profile_end):
 * flops[RG_NSTAGES] floating-point operations (an FMA counts 2) of the
 * formulas each stage evaluates, bytes[RG_NSTAGES] minimum HBM traffic
 * (each input read once, each output written once, per-column matrices
 * amortised over the column).  Host only. */
rg_status rg_geom_work(const rg_geom *geom, double *flops, double *bytes);

/* Benchmark helper (not part of the scheme): launches n_threads (a multiple
 * of 256) lanes that each run iters x 16 independent FP64 FMAs and write one
 * double to sink[n_threads] (device).  Timed by the caller, it gives the
 * attainable FP64 vector rate (2 x 16 x iters x n_threads flops).
 * Asynchronous on `stream`. */
rg_status rg_fma_probe(double *sink, int64_t n_threads, int32_t iters, void *stream);

/* ------------------------------------------------------------------------
 * Triangular-prism element on the icosahedral geodesic mesh: the paper's own
 * zone (Sections II.a-II.b, V.b; Fig. 7; Appendices B-D) with its
 * element-local ADER-CG predictor (Section V.d).
 *
 * Mesh: the icosahedron projected to the unit sphere (vertex 0 the north
 * pole, 1-5 an upper ring at z = 1/sqrt 5 at longitudes 72 k degrees, 6-10 a
 * lower ring at z = -1/sqrt 5 at longitudes 36 + 72 k, 11 the south pole;
 * faces, for k = 0..4 and k1 = k + 1 mod 5, (0, 1+k, 1+k1), (1+k, 6+k, 1+k1),
 * (1+k1, 6+k, 6+k1), (11, 6+k1, 6+k), each turned counter-clockwise seen
 * from outside) is split `level` times: triangle t = (a, b, c) becomes
 * 4t + 0: (a, m_ab, m_ca), 4t + 1: (m_ab, b, m_bc), 4t + 2: (m_ca, m_bc, c),
 * 4t + 3: (m_ab, m_bc, m_ca), with the great-circle midpoints
 * m_uv = (u + v) / |u + v|: 20 * 4^level triangles.  Shells have radii
 * r_k = r_in (r_out / r_in)^(k / n_rad), k = 0..n_rad; zone z = t * n_rad + k.
 *
 * Element: the prism with unit edges and its centroid at the origin,
 * triangle vertices (-1/2, -1/(2 sqrt 3)), (1/2, -1/(2 sqrt 3)),
 * (0, 1/sqrt 3), zeta in [-1/2, 1/2] (zeta = -1/2 on the inner sphere); its
 * 6 / 15 / 26 nodes at orders 2 / 3 / 4 numbered as in Appendices B-D; the
 * map to a zone interpolates the sphere through the triangle lattice of
 * degree order-1 (vertices, equidistant great-circle edge points, and at
 * order 4 the spherical centroid) and is linear in radius.
 * ------------------------------------------------------------------------ */
typedef struct rg_prism rg_prism;

typedef struct {
    int64_t n_zones;   /* 20 * 4^level * n_rad                 */
    int64_t n_tri;     /* 20 * 4^level columns                  */
    int32_t n_nodes;   /* nodes per zone: 6, 15, 26             */
    int32_t n_levels;  /* time levels: order                    */
    int32_t order, level, n_rad;
    int32_t n_face_points;  /* face points per zone: 15, 24, 38      */
    int64_t n_edges;        /* mesh edges: 30 * 4^level              */
    int64_t n_faces;        /* n_tri (n_rad + 1) + n_edges n_rad     */
    int32_t n_divfree_in;   /* inputs of rg_prism_divfree per zone   */
    int32_t n_divfree_out;  /* outputs: 3 n_nodes + 3                */
    int64_t n_vertices;     /* mesh vertices: n_tri / 2 + 2          */
} rg_prism_info;

/* Builds the mesh and, on the current device, the geometry of every column
 * (Jacobians and curl-form flux metrics of eq. (5.11) at the nodes, for a
 * unit shell, 104 bytes per node).  *out is a library-owned handle
 * (rg_prism_free).  RG_ENOTSUP for order outside 2..4, level outside 0..8 or
 * more than 2^31 zone nodes; RG_EINVAL unless n_rad >= 1 and
 * 0 < r_in < r_out; RG_ESINGULAR if the element or a Jacobian degenerates;
 * RG_ENOMEM if a device allocation fails. */
rg_status rg_prism_build(int32_t level, int32_t n_rad, double r_in, double r_out, int32_t order, rg_prism **out);
/* The same mesh and host geometry without device uploads (queries only;
 * rg_prism_predict returns RG_EINVAL on it). */
rg_status rg_prism_build_host(int32_t level, int32_t n_rad, double r_in, double r_out, int32_t order,
                              rg_prism **out);
void rg_prism_free(rg_prism *prism);
rg_status rg_prism_get_info(const rg_prism *prism, rg_prism_info *info);

/* Host copy of the triangles' vertices: abc[n_tri][3][3] (a, b, c). */
rg_status rg_prism_triangles(const rg_prism *prism, double *abc);

/* Host copies for zones [z0, z0 + nz): node positions x[nz][N][3],
 * Jacobians J[nz][N] and metrics met[nz][N][3][3] (row d, column n:
 * J d xi_d / d x_n); any output may be NULL.  RG_EINVAL outside the mesh. */
rg_status rg_prism_geometry(const rg_prism *prism, int64_t z0, int64_t nz, double *x, double *J, double *met);

/* Face points of Appendix A in reference coordinates, xi[Q][3], and their
 * weights w[Q] (fractions of each face's reference area): the triangle rule
 * (A.1), (A.3) or (A.5) on the face zeta = +1/2, then on zeta = -1/2, then the
 * square rule (A.2), (A.4) or (A.6) on the side faces over the triangle edges
 * from vertex k to k + 1 (k = 0, 1, 2; x along the edge, y along zeta).  The
 * triangle rules are printed for a triangle with a vertex at the origin and
 * are moved to the centred one; within a face the points are in the
 * library's order.  Q = 2 n_tri_points + 3 n_side_points; any output may be
 * NULL.  Host only. */
rg_status rg_prism_face_points(const rg_prism *prism, double *xi, double *w, int32_t *n_tri_points,
                               int32_t *n_side_points);

/* Traces of the predictor's time averages at the face points, the corrector's
 * quadrature inputs (Section VI): tr[k][q][z] = sum_l psi_l(xi_q) a_k[z][l]
 * for the 32 values a = (avgU[0..8), avgF[0][0..8), avgF[1][0..8),
 * avgF[2][0..8)).  Device arrays as written by rg_prism_predict; tr is
 * double[32][Q][n_zones] (zones fastest), caller-owned.  Asynchronous on
 * stream.  RG_EINVAL for null pointers or a host-only mesh. */
rg_status rg_prism_traces(const rg_prism *prism, const double *avgU, const double *avgF, double *tr, void *stream);

/* Mesh edges, edges[n_edges][4] = (t, k, t', k'): triangle t's local edge k
 * (0: a-b, 1: b-c, 2: c-a) is triangle t''s local edge k', t < t'; listed in
 * the order met going through the triangles and their local edges.  Host. */
rg_status rg_prism_edges(const rg_prism *prism, int32_t *edges);

/* The corrector's face fluxes (Sections II.c and VI) on the prism faces:
 * for every face the integral over its points (rg_prism_face_points) of the
 * HLL flux of the two sides' traces (tr of rg_prism_traces: time-averaged
 * state and Cartesian flux), along the face's area vector, weighted by the
 * rule.  Faces: radial faces f = t (n_rad + 1) + kf at radius r_kf, along +r,
 * then side faces n_tri (n_rad + 1) + e n_rad + k over edge e in shell k,
 * along the outward normal of the edge's first triangle t; at r_in and r_out
 * the one zone's trace is taken on both sides.  Phi double[n_faces][8],
 * device, caller-owned.  Asynchronous on stream.  RG_EINVAL for null
 * pointers, gamma <= 1 or a host-only mesh. */
rg_status rg_prism_face_fluxes(const rg_prism *prism, double gamma, const double *tr, double *Phi, void *stream);

/* Constrained transport on the prisms (Section VI with the prism's edges).
 * rg_prism_edge_traces: the state (8 values) and the induction fluxes
 * F_d[B_i] (9 values, d major) of every zone at the 27 Simpson points of its
 * edges, from the predictor's time averages avgU double[8][n_zones][n_nodes]
 * and avgF double[3][8][n_zones][n_nodes] (rg_prism_predict's outputs):
 * er double[17][27][n_zones]; point (side * 3 + j) * 3 + p lies on the
 * triangle's edge j (vertex j to j + 1) at zeta = +1/2 (side 0) or -1/2
 * (side 1), point 18 + 3 j + p on the radial edge through vertex j, p = 0, 1,
 * 2 at the start, middle and end.
 * rg_prism_edge_emfs: the line integral of the electric field along every
 * edge from those records, by Simpson's rule along the edge.  At a point of
 * an angular edge (mesh edge e at radius r_k) the four zones about it give
 * the four-state multidimensional HLL field (as on the hexahedra; east = the
 * edge's first triangle, north = outward, frame from the zone centroids); at
 * r_in and r_out the two zones give the 1-D HLL field of their side face.
 * At a point of a radial edge (vertex v, shell k) the five or six zones
 * about it give the mean over the side faces between consecutive zones of
 * their 1-D HLL induction flux (the three-zone rule of the hexahedra for any
 * number).  Gang double[n_edges][n_rad + 1] runs from the start to the end
 * of edge e as its first triangle lists them (rg_prism_edges), Grad
 * double[n_vertices][n_rad] outward (vertices as rg_prism_vertices lists
 * them).
 * rg_prism_ct: the magnetic fluxes PhiB double[n_faces] through the faces
 * (numbered and directed as in rg_prism_face_fluxes) after dt: PhiBo = PhiB
 * - dt times the circulation of the edge integrals around each face,
 * counter-clockwise about its direction (Stokes' theorem), which keeps every
 * zone's net outward flux.
 * Device, caller-owned, asynchronous on stream; RG_EINVAL for null
 * pointers, a host-only mesh, gamma <= 1 or dt < 0. */
rg_status rg_prism_edge_traces(const rg_prism *prism, const double *avgU, const double *avgF, double *er, void *stream);
rg_status rg_prism_edge_emfs(const rg_prism *prism, double gamma, const double *er, double *Gang, double *Grad,
                             void *stream);
rg_status rg_prism_ct(const rg_prism *prism, double dt, const double *Gang, const double *Grad, const double *PhiB,
                      double *PhiBo, void *stream);
/* Host copy of the unit-sphere mesh vertices, double[n_vertices][3], numbered
 * in first encounter over (triangle, local vertex). */
rg_status rg_prism_vertices(const rg_prism *prism, double *xyz);

/* Divergence-free reconstruction of B (Section IV.b) on the prism's five
 * faces: per zone the constrained least squares of eqs. (4.3), (4.6), (4.9)
 * (closeness to the WENO-AO coefficients) and (4.15) (the normal B at every
 * face point) under the divergence identities of eq. (4.10) without its first
 * member and the five face averages of eq. (4.14), in the zone's Taylor frame
 * (centroid, l0 = V^(1/3)); each component carries the monomials of degree
 * <= p-1 and the degree-p ones containing its own coordinate.  The KKT system
 * is solved once per column for all inputs (the shells of a column are
 * scaled copies) and applied as a matrix: the first call builds and uploads
 * the maps (8 n_out n_in bytes per column, 5.5 GB at level 6, fourth order;
 * a lock makes concurrent first calls on one mesh safe).
 * Bin double[n_divfree_in][n_zones]: per component its zone mean and Taylor
 * coefficients of degree 1..p-1 (degree by degree, x exponent descending,
 * then y), the outward normal B at the Q face points (rg_prism_face_points
 * order), the five outward face averages (zeta = +1/2, -1/2, sides 0, 1, 2);
 * Bout double[n_divfree_out][n_zones]: B at the nodes (x components, then y,
 * then z), then the three zone means.  Device, caller-owned, asynchronous on
 * stream.  RG_EINVAL for null pointers or a host-only mesh, RG_ESINGULAR if a
 * KKT system is singular, RG_ENOMEM. */
rg_status rg_prism_divfree(rg_prism *prism, const double *Bin, double *Bout, void *stream);
/* The same map on the host for zones [z0, z0 + nz): Bin[nz][n_divfree_in],
 * Bout[nz][n_divfree_out] (zone-major).  Works on host-only meshes. */
rg_status rg_prism_divfree_host(rg_prism *prism, int64_t z0, int64_t nz, const double *Bin, double *Bout);

/* Host copies of the volumes of zones [z0, z0 + nz) (the map's Jacobian
 * integrated by cubature).  RG_EINVAL outside the mesh. */
rg_status rg_prism_volumes(const rg_prism *prism, int64_t z0, int64_t nz, double *vol);

/* Finite-volume update of the zone averages (Section VI): Uo = U - dt / V_z
 * times the sum over the zone's five faces of the face flux (Phi of
 * rg_prism_face_fluxes) taken along the zone's outward normal, for all eight
 * variables.  (The scheme replaces the B averages by those of its
 * divergence-free reconstruction after constrained transport, which is not
 * built for prisms.)  U, Uo double[8][n_zones], device, caller-owned, may
 * alias.  Asynchronous on stream.  RG_EINVAL for null pointers, dt < 0 or a
 * host-only mesh. */
rg_status rg_prism_update(const rg_prism *prism, double dt, const double *U, const double *Phi, double *Uo,
                          void *stream);

/* Algorithmic work of rg_prism_predict per zone with n_picard sweeps:
 * floating-point operations (mapped fluxes 149 per node, the sparse
 * derivative products, the level updates and the time averages) and HBM
 * bytes (Ua read, avgU and avgF written, per-column geometry shared by the
 * column's shells).  Host only. */
rg_status rg_prism_work(const rg_prism *prism, int32_t n_picard, double *flops_per_zone, double *bytes_per_zone);

/* The ADER-CG predictor of every zone (Section V.d, eqs. (5.20)-(5.29), in
 * the R (x) D form of eqs. (C.34)-(C.36) and (D.29)-(D.32)): from the nodal
 * conserved state Ua at t^n it runs n_picard Picard sweeps over the
 * order - 1 Gauss time levels (the scheme uses n_picard = order; 0 keeps
 * every level at the initial state) and returns the time averages over the
 * levels of the nodal state, avgU, and of the physical flux, avgF -- the
 * inputs of the corrector's face and edge quadratures.  Device arrays,
 * caller-owned: Ua and avgU double[8][n_zones][N], avgF double[3][8][n_zones][N]
 * (direction, variable, zone, node).  Asynchronous on stream.  RG_EINVAL for
 * null pointers, gamma <= 1, dt < 0 or n_picard outside 0..16. */
rg_status rg_prism_predict(const rg_prism *prism, double gamma, double dt, int32_t n_picard, const double *Ua,
                           double *avgU, double *avgF, void *stream);

/* Benchmark helper (not part of the scheme): launches n_threads (a multiple
 * of 256) lanes whose wavefronts each run iters x 8 independent matrix-core
 * products and write one double per lane to sink[n_threads] (device).  kind 0:
 * v_mfma_f64_16x16x4 (2048 flops per product), kind 1:
 * v_mfma_f32_16x16x32_bf16 (16384 flops).  Timed by the caller, it gives the
 * attainable matrix-core rate (flops x 8 x iters x n_threads / 64).  RG_EINVAL
 * for other kinds or sizes.  Asynchronous on `stream`. */
rg_status rg_mfma_probe(double *sink, int64_t n_threads, int32_t iters, int32_t kind, void *stream);

const char *rg_last_error(void);

/* Name and one-line meaning of a status code (static string). */
const char *rg_status_str(rg_status status);

#ifdef __cplusplus
}
#endif

#endif

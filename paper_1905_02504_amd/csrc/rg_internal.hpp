// Internal data structures of the rg library: host mesh, reference element,
// per-column geometry (host, FP64) and the device-side view used by kernels.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "rg.h"

namespace rg {

constexpr int NVAR = 8;

void set_error(const std::string &msg);

// ---------------------------------------------------------------- mesh
// Cube-based geodesic surface mesh (six patches of N x N quadrilateral
// columns) extruded into K = n_rad + 2 n_ghost geometric shells.
struct Mesh {
    int N = 0, Nr = 0, g = 0, K = 0, map_order = 2;
    double r_in = 1, r_out = 2, q = 1;
    std::vector<double> radius;  // K + 1 interface radii (extended index)
    int ncol = 0, nv = 0, nae = 0;
    std::vector<double> vpos;    // nv * 3, unit vectors
    std::vector<int> col_v;      // ncol * 4 corners v0..v3, counter-clockwise from outside
    std::vector<int> col_ae;     // ncol * 4 angular edge of local faces xi-, xi+, eta-, eta+
    std::vector<int> ae_v;       // nae * 2 vertices, a < b
    std::vector<int> ae_col;     // nae * 2 columns (side 0 = lower column id)
    std::vector<int> ae_lf;      // nae * 2 local face index in each column
    std::vector<int> v_ncol;     // nv, columns around each vertex (3 or 4)
    std::vector<int> v_col;      // nv * 4, counter-clockwise about +r
    int64_t nzones = 0, nfaces = 0, nrf = 0, nedges = 0, nre = 0;
};

// ---------------------------------------------------------------- reference element
struct RefEl {
    int order = 3;   // scheme order p
    int N = 0;       // serendipity nodes (20 / 32)
    int M = 0;       // time levels (p)
    int NC = 0;      // Taylor coefficients of degree 1..p-1 (9 / 19)
    int NB = 0;      // divergence-free coefficients per component (16 / 30)
    int Q1 = 0, Q = 0;        // face quadrature points per direction / per face
    int NS = 0;               // large-stencil slots (26 / 32)
    int NIN = 0, NOUTB = 0;   // inputs / outputs of the fused B map
    int NFN = 0, NEN = 0;     // serendipity nodes on a face / on an edge
    std::vector<std::array<double, 3>> node;   // N reference nodes on [-1/2,1/2]^3
    std::vector<std::array<int, 3>> sexp;      // N monomials (superlinear degree <= p-1)
    std::vector<double> coef;                  // N x N: psi_l = sum_k coef[k*N+l] m_k
    std::vector<double> D;                     // 3 x N x N: d psi_l / d xi_d at node i
    std::vector<double> tau, wt;               // M time nodes, Gauss weights (wt[0] = 0)
    std::vector<double> R;                     // (M-1) x M
    std::vector<double> gq, gw;                // Q1 Gauss points on [0,1]
    std::vector<std::array<int, 3>> tex;       // NC Taylor multi-indices
    std::vector<std::array<int, 3>> bex[3];    // NB basis of each B component
    // interpolation of nodal values to face points / edge Simpson points
    std::vector<int> fnode;    // 6 x NFN nodes on each local face
    std::vector<double> fint;  // 6 x Q x NFN weights
    std::vector<int> enode;    // 12 x NEN nodes on each local edge
    std::vector<double> eint;  // 12 x 3 x NEN weights
    std::vector<double> fintc; // NFN x Q  weights shared by all faces (node k, point q)
    std::vector<double> eintc; // NEN x 3  weights shared by all edges (node k, point s)
    double psi(int l, const double *xi) const;
    double dpsi(int l, int d, const double *xi) const;
};

bool build_refel(int order, RefEl &r);
bool time_galerkin(int M, std::vector<double> &tau, std::vector<double> &wt, std::vector<double> &R);
void face_ref_point(const RefEl &r, int lf, int q, double *xi);
void edge_ref_point(int le, double s, double *xi);
void gauss_legendre01(int n, double *x, double *w);

// small dense solvers (row-major)
bool lu_factor(int n, std::vector<double> &A, std::vector<int> &piv);
void lu_solve(int n, const std::vector<double> &LU, const std::vector<int> &piv, double *b);

// ---------------------------------------------------------------- device view
struct DevGeom {
    // sizes
    int order, N, M, NC, NB, Q, NS, NIN, NOUTB, NFN, NEN;
    int Nang, Nr, g, K, ncol, nv, nae;
    long long Z, NF, NRF, NE, NRE;
    // global tables
    const double *radius;   // K + 1
    const double *zscale;   // K: zone length scale relative to shell 0
    const double *R;        // (M-1) x M
    const double *wt;       // M
    const int *fnode;       // 6 x NFN
    const double *fint;     // 6 x Q x NFN
    const int *enode;       // 12 x NEN
    const double *eint;     // 12 x 3 x NEN
    const double *fintc;    // NFN x Q, identical for every face
    const double *eintc;    // NEN x 3, identical for every edge
    // per column
    const int *stm;         // ncol x NS   member = col * 8 + (dk + 3), -1 if empty
    const double *Pl;       // ncol x NC x NS
    const double *Ps;       // ncol x 7 x 3 x 6
    const double *Qs;       // ncol x NC x NC
    const double *Ev;       // ncol x NC x N      Taylor basis at the ADER nodes (node fastest)
    const double *Mb;       // ncol x NIN x NOUTB divergence-free map, transposed (output fastest)
    const double *nJ;       // ncol x N
    const double *nM;       // ncol x 9 x N       (J a^d)_n at the nodes (node fastest)
    const double *fevR;     // ncol x 2 x Q x NC
    const double *fnR;      // ncol x Q x 3
    const double *fwR;      // ncol x Q
    const int *col_ae;      // ncol x 4
    const int *col_side;    // ncol x 4
    const int *col_perm;    // ncol x 4 x Q
    const int *col_v;       // ncol x 4
    const int *col_slot;    // ncol x 12
    const int *col_rev;     // ncol x 12
    const int *col_sgn;     // ncol x 4   circulation sign of the angular edges about +r
    const double *dins;     // ncol      in-sphere diameter of the shell-0 zone
    // per angular edge
    const int *ae_col;      // nae x 2
    const int *ae_v;        // nae x 2
    const double *fevA;     // nae x 2 x Q x NC
    const double *fnA;      // nae x Q x 3
    const double *fwA;      // nae x Q
    const double *aeF;      // nae x 3 x 9   edge-point frames e1, e2, t
    const double *aeW;      // nae x 3       Simpson weight x |dx/ds| at interface 0
    const int *ae_rs;       // nae           +1 if side 1 is right of the direction a->b
    // per vertex
    const int *v_ncol;      // nv
    const double *vF;       // nv x 9 radial-edge frame
    const double *vN3;      // nv x 3 x 3 face normals at valence-3 vertices
    // per zone / face
    const double *vol;      // Z
    const double *area;     // NF
    // FP32 copies of the tables read by the reconstruction and predictor
    // contractions (precision mode RG_MODE_FP32 only; null otherwise)
    const float *PlF, *PsF, *QsF, *EvF, *nJF, *nMF, *fevRF, *fevAF, *fintcF, *eintcF;
    // RG_MODE_BF16: the A operands of the predictor's flux-derivative product
    // on the BF16 matrix cores, per lane [64][direction 3][M tile 2][4 dwords
    // of packed bf16 pairs]
    const unsigned *DmfA;
    // tables used only by the adjoint of the step
    const double *Dfull;    // 3 x N x N  d psi_l / d xi_d at node i, [d][i][l]
    const int *ae_lf;       // nae x 2    local face of the angular edge in each column
    const int *v_ae;        // nv x 4     angular edges at each vertex (v_ncol of them)
    const int *inv_ptr;     // ncol + 1   CSR over member columns of the WENO stencils
    const int *inv_ent;     // n x 3      (stencil column, slot, radial offset dk) per entry
};

// Device buffers of the adjoint of the step, allocated on its first call
struct AdjBuffers {
    bool ready = false, map_ready = false;
    double *Ubc = nullptr, *Bbc = nullptr, *MbA = nullptr;
    double *gUo = nullptr, *gBo = nullptr, *gzoneB = nullptr, *gwc = nullptr, *gftr = nullptr, *getr = nullptr;
    double *gGam = nullptr, *gPhi = nullptr, *gbnode = nullptr, *gbnod = nullptr, *gside = nullptr, *gsb = nullptr;
    double *gdu = nullptr;
};

}  // namespace rg

// opaque handles
struct rg_mesh {
    rg::Mesh m;
};

struct rg_geom {
    const rg_mesh *mesh = nullptr;
    rg::RefEl ref;
    int mode = 0;
    rg::DevGeom d{};
    std::vector<void *> allocations;        // device allocations owned by the geometry
    // host copies for queries
    std::vector<double> zcen, zvol, fcen, fnrm, farea, emid, etan;
    // work buffers (device)
    double *wcoef = nullptr, *bnod = nullptr, *ftr = nullptr, *etr = nullptr;
    double *Phi = nullptr, *Gam = nullptr, *zoneB = nullptr, *red = nullptr;
    double *bnode = nullptr;   // divergence-free B at the ADER nodes, [recon zone][3N]
    // first-order fallback: per-round counts of newly flagged zones, marks of
    // the faces [NF] and edges [NE] to solve again, per-zone flags [Z] (one
    // allocation), and whether zfl holds flags of a step that had the
    // fallback on
    int *fbcnt = nullptr;
    // the last step's per-zone WENO-AO order indicator [Z] (zones of the
    // reconstructed shells)
    float *whi = nullptr;
    unsigned char *zfl = nullptr, *ffl = nullptr, *efl = nullptr;
    bool fb_dirty = false;
    bool fb_last = false;   // the last rg_step ran the fallback (its round counters are valid)
    rg::AdjBuffers adj;
    // per-column host data kept for initial conditions
    std::vector<double> snode;   // ncol x 16 x 3 surface map nodes
    std::vector<int> ae_rs_host; // +1 if side 1 of an angular edge is right of its direction
    std::vector<int> col_side_host, col_sgn_host;   // per column-local angular face: side, circulation sign
    std::vector<double> cond_lsq, cond_kkt;   // per-column condition numbers (precompute)
    // optional per-stage timing: one set of RG_NSTAGE+1 events per recorded step
    bool prof_on = false;
    std::vector<void *> prof_events;
};

#define RG_NSTAGE RG_NSTAGES
// bytes reserved for the fallback's round counters (ahead of its marks)
#define RG_FB_COUNTER_BYTES 64
constexpr int FALLBACK_ROUNDS = RG_FALLBACK_ROUNDS;

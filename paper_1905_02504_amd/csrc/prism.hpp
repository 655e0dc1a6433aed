// Triangular-prism element on the icosahedral geodesic mesh: host-side
// reference element and the device view of the per-column geometry.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "rg.h"

namespace rg {

// Reference prism with unit edges and its centroid at the origin
// (Appendices B-D); nodes numbered as there, monomials of eqs. (5.12)-(5.14).
struct PrismRef {
    int order = 0, N = 0, M = 0;
    std::vector<std::array<double, 3>> node;
    std::vector<std::array<int, 3>> mono;
    std::vector<double> D;          // 3 x N x N: d psi_l / d xi_d at node i
    std::vector<double> tau, wt, R; // time levels, Gauss weights, (M-1) x M time matrix
    std::vector<int> lat;           // N: index of the node's (xi, eta) in the map's triangle lattice
    std::vector<double> coef;       // N x N: psi_l = sum_k coef[k * N + l] m_k
    // face points of Appendix A: faces zeta = +1/2, -1/2, then the side faces
    // on triangle edges 0-1, 1-2, 2-0; weights as fractions of the face
    int QT = 0, QS = 0, Q = 0;
    std::vector<std::array<double, 3>> fpt;
    std::vector<double> fw;
    // the nodes whose basis functions are non-zero at each face point, and
    // their values there (Q x TRACE_TERMS, padded with weight 0)
    std::vector<int> fidx;
    std::vector<double> fval;
    double psi(int l, const double *xi) const;
};

constexpr int TRACE_TERMS = 12;   // at most 12 nodes on a face (fourth-order side faces)

bool build_prism_ref(int order, PrismRef &r);

// psi_l = sum_k C[k][l] m_k for nodes x and monomials mo (eq. 5.3)
bool lagrange_coefficients(const std::vector<std::array<double, 3>> &x, const std::vector<std::array<int, 3>> &mo,
                           std::vector<double> &C);
// D[d][i][l] = d psi_l / d xi_d at node i
void derivative_matrices(const std::vector<std::array<double, 3>> &x, const std::vector<std::array<int, 3>> &mo,
                         const std::vector<double> &C, std::vector<double> &D);
// triangle lattice of degree mo on the reference triangle: barycentric
// (i, j, k) / mo with i, then j descending, and the (xi, eta, 0) points
void lattice(int mo, std::vector<std::array<int, 3>> &bary, std::vector<std::array<double, 3>> &x);

// device view: geometry of each column (triangle) for a unit shell with radii
// 1 and q, scaled per shell by the shell's inner radius r_k
struct DevPrism {
    int order, N, n_rad;
    int64_t ntri, nz;
    const double *J;      // ntri x N
    const double *met;    // ntri x 9 x N: (J d xi_d / d x_n), row d * 3 + n
    const double *rinv;   // n_rad: 1 / r_k
    const double *R;      // (M-1) x M
    const double *wt;     // M
    int Q;                // face points per zone
    const int *fidx;      // Q x TRACE_TERMS
    const double *fval;   // Q x TRACE_TERMS
    // face fluxes
    int QT, QS;           // points per triangle face, per side face
    int64_t nedges, nfaces;
    const int *edges;     // nedges x 4: t, local edge, t', local edge' (t < t')
    const int *mirror;    // QS: the side point at the same height, mirrored along the edge
    const double *tfA;    // ntri x QT x 3: weighted area vectors of the triangle faces at radius 1 (+r)
    const double *sfA;    // ntri x 3 x QS x 3: weighted outward area vectors of the side faces, unit shell
    const double *radius; // n_rad + 1
    // update
    const double *vol;    // ntri: volume of the unit shell's zone (shell k: r_k^3 times it)
    const int *tedge;     // ntri x 3: edge id of each local edge, negated - 1 where t is the second triangle
    // divergence-free B
    int nin, nout;
    const double *Mb;     // ntri x nin x nout: per column the transposed map (built on the first rg_prism_divfree call)
    // constrained transport: edges and vertices
    int64_t nvert;
    const int *eidx;      // EDGE_POINTS x EDGE_TERMS: nodes whose basis functions do not vanish at each edge point
    const double *eval;   // EDGE_POINTS x EDGE_TERMS: their values (padding: weight 0)
    const double *aeg;    // nedges x 3 x 16 (unit shell): tangent, frame e1, e2, boundary normal, |dx/ds|
    const int *edge_ab;   // nedges x 2: vertices at the start and end of each edge (its first triangle's order)
    const double *vxyz;   // nvert x 3: unit-sphere vertices
    const int *ring_off;  // nvert + 1
    const int *ring_tj;   // per ring entry 3 t + j: triangle t with vertex j at the ring's vertex, counter-clockwise
    const double *ring_n; // per ring entry: unit normal of the side face to the next triangle of the ring
};

// edge points of the element (Simpson's rule along each edge): angular edges
// (side 0: zeta = +1/2, side 1: zeta = -1/2) x local edge j x point p at
// (side * 3 + j) * 3 + p; radial edges at triangle vertex j: 18 + 3 j + p
constexpr int EDGE_POINTS = 27;
constexpr int EDGE_TERMS = 4;      // at most p nodes on an edge

rg_status launch_prism_traces(const DevPrism &G, const double *aU, const double *aF, double *tr, void *stream);
rg_status launch_prism_face_flux(const DevPrism &G, double gamma, const double *tr, double *Phi, void *stream);
rg_status launch_prism_divfree(const DevPrism &G, const double *Bin, double *Bout, void *stream);
rg_status launch_prism_edge_traces(const DevPrism &G, const double *aU, const double *aF, double *er, void *stream);
rg_status launch_prism_edge_emfs(const DevPrism &G, double gamma, const double *er, double *Gang, double *Grad,
                                 void *stream);
rg_status launch_prism_ct(const DevPrism &G, double dt, const double *Gang, const double *Grad, const double *PhiB,
                          double *PhiBo, void *stream);
rg_status launch_prism_update(const DevPrism &G, double dt, const double *U, const double *Phi, double *Uo, void *stream);
rg_status launch_prism_predict(const DevPrism &G, double dt, double gamma, int npic, const double *Ua, double *aU,
                               double *aF, void *stream);

}  // namespace rg

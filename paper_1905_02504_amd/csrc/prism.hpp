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
};

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
};

rg_status launch_prism_predict(const DevPrism &G, double dt, double gamma, int npic, const double *Ua, double *aU,
                               double *aF, void *stream);

}  // namespace rg

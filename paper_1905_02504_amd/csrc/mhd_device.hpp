// Device building blocks shared by the step (step.hip) and its adjoint
// (adjoint.hip): element traits, ideal-MHD point functions, the Riemann
// solvers, the WENO-AO combination and the derivative-matrix slab.  The point
// functions are templates on the scalar type: double for the FP64 step and
// the adjoint's recomputation, float for the reduced-precision form.
#pragma once
#include <hip/hip_runtime.h>

#include "dtab.hpp"
#include "rg_geom_host.hpp"

namespace rg {

template <int P>
struct Tr;
template <>
struct Tr<3> {
    static constexpr int N = 20, M = 3, NC = 9, NB = 16, Q1 = 2, Q = 4, NS = 26, NIN = 60, NOUTB = 63, NFN = 8, NEN = 3;
};
template <>
struct Tr<4> {
    static constexpr int N = 32, M = 4, NC = 19, NB = 30, Q1 = 3, Q = 9, NS = 32, NIN = 120, NOUTB = 99, NFN = 12, NEN = 4;
};

typedef long long i64;

constexpr double WENO_GAMMA_HI = 0.85;
// epsilon of the nonlinear weights when the step parameters leave it at 0
constexpr double WENO_EPS_DEFAULT = 1e-4;

// local edges 0..7 are angular: local face holding them and whether they lie
// on the upper (zeta+) interface; 8..11 radial at corners v0, v1, v3, v2
struct LocalEdges {
    static constexpr int FACE[8] = {2, 3, 2, 3, 0, 1, 0, 1};
    static constexpr int UP[8] = {0, 0, 1, 1, 0, 0, 1, 1};
    static constexpr int CORNER[4] = {0, 1, 3, 2};
};

// scalar functions with one spelling for every T
__device__ __forceinline__ double ssqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float ssqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double smax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double smin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float smax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ float smin(float a, float b) { return fminf(a, b); }

// accumulator of v_mfma_f64_16x16x4f64
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Trace records written by the predictor and read by the Riemann solvers.
// Face record (face f, quadrature point q, side s): the 8 time-averaged
// conserved variables, then the 8 time-averaged normal fluxes; the two sides
// of a point are adjacent, [f][q][side][16].  Edge record (edge e, Simpson
// point p, slot s): the 8 variables, then E . t, the electric field along the
// edge's canonical direction at that point (the only component either edge
// solver uses); [e][p][slot][9].
template <int P>
__host__ __device__ __forceinline__ long long ftr_at(long long f, int q, int side)
{
    return ((f * Tr<P>::Q + q) * 2 + side) * 16;
}
__host__ __device__ __forceinline__ long long etr_at(long long e, int p, int slot) { return ((e * 3 + p) * 4 + slot) * 9; }

// Faces of the flux stage (radial faces kf in [g, g+Nr], angular faces in
// shells [g, g+Nr-1]): face index t of that range -> face id, unit normals
// and weights of its quadrature points
template <int P>
__device__ __forceinline__ i64 flux_face(const DevGeom &G, i64 t, const double *&nrm, const double *&fw)
{
    using T = Tr<P>;
    const int nrad = G.Nr + 1, nang = G.Nr;
    const i64 nR = (i64)G.ncol * nrad;
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g + (int)(t % nrad);
        nrm = G.fnR + (i64)c * T::Q * 3;
        fw = G.fwR + (i64)c * T::Q;
        return (i64)c * (G.K + 1) + kf;
    }
    const i64 u = t - nR;
    const int ae = (int)(u / nang), k = G.g + (int)(u % nang);
    nrm = G.fnA + (i64)ae * T::Q * 3;
    fw = G.fwA + (i64)ae * T::Q;
    return G.NRF + (i64)ae * G.K + k;
}

// Edges of the EMF stage (radial edges in shells [g, g+Nr-1], angular edges at
// interfaces [g, g+Nr]): edge index t of that range -> edge id, the frame and
// line weight of its Simpson point p, the number of zones around it (3 or 4)
// and, at valence-3 vertices, the three face normals
__device__ __forceinline__ i64 emf_edge(const DevGeom &G, i64 t, int p, const double *&frame, double &wl, int &nzs,
                                        const double *&N3)
{
    const int nrad = G.Nr, nang = G.Nr + 1;
    const i64 nR = (i64)G.nv * nrad;
    if (t < nR) {
        const int v = (int)(t / nrad), k = G.g + (int)(t % nrad);
        nzs = G.v_ncol[v];
        wl = (p == 1 ? 4.0 / 6.0 : 1.0 / 6.0) * (G.radius[k + 1] - G.radius[k]);
        frame = G.vF + (i64)v * 9;
        N3 = G.vN3 + (i64)v * 9;
        return (i64)v * G.K + k;
    }
    const i64 u = t - nR;
    const int ae = (int)(u / nang), kf = G.g + (int)(u % nang);
    nzs = 4;
    wl = G.aeW[(i64)ae * 3 + p] * (G.radius[kf] / G.radius[0]);
    frame = G.aeF + ((i64)ae * 3 + p) * 9;
    N3 = nullptr;
    return G.NRE + (i64)ae * (G.K + 1) + kf;
}

// Canonical unit tangent at Simpson point p (canonical order) of local edge le
// of column c: the third row of the frame the EMF stage uses
__device__ __forceinline__ const double *edge_tangent(const DevGeom &G, int c, int le, int p)
{
    if (le < 8) return G.aeF + ((i64)G.col_ae[4 * c + LocalEdges::FACE[le]] * 3 + p) * 9 + 6;
    return G.vF + (i64)G.col_v[4 * c + LocalEdges::CORNER[le - 8]] * 9 + 6;
}

// ---------------------------------------------------------------- ideal MHD
template <class T>
__device__ __forceinline__ T dev_pressure(const T *u, T gam)
{
    T m2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    T b2 = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    return (gam - T(1.0)) * (u[4] - T(0.5) * m2 / u[0] - T(0.5) * b2);
}

// F[d][v]: flux of conserved variable v along Cartesian direction d (eq. 2.2)
template <class T>
__device__ __forceinline__ void dev_flux(const T *u, T gam, T F[3][8])
{
    T ir = T(1) / u[0];
    T v0 = u[1] * ir, v1 = u[2] * ir, v2 = u[3] * ir;
    T B0 = u[5], B1 = u[6], B2 = u[7];
    T hb2 = T(0.5) * (B0 * B0 + B1 * B1 + B2 * B2);
    T p = (gam - T(1)) * (u[4] - T(0.5) * (u[1] * v0 + u[2] * v1 + u[3] * v2) - hb2);
    T pt = p + hb2;
    T vB = v0 * B0 + v1 * B1 + v2 * B2;
    T v[3] = {v0, v1, v2}, B[3] = {B0, B1, B2};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        F[d][0] = u[1 + d];
#pragma unroll
        for (int i = 0; i < 3; i++) F[d][1 + i] = u[1 + d] * v[i] + (d == i ? pt : T(0)) - B[d] * B[i];
        F[d][4] = (u[4] + pt) * v[d] - B[d] * vB;
#pragma unroll
        for (int i = 0; i < 3; i++) F[d][5 + i] = v[d] * B[i] - B[d] * v[i];
    }
}

// flux contracted with the scaled metric terms at a node (eq. 5.23):
// out[d] = sum_c met[d][c] F_c(u / J).  Each contraction is the physical flux
// along the (non-unit) vector n = met[d][.], formed directly from n.m, n.v
// and n.B instead of from the three Cartesian fluxes.
template <class T>
__device__ __forceinline__ void mapped_flux(const T *u, T iJ, const T *met, T gam, T out[3][8])
{
    T w[8];
#pragma unroll
    for (int v = 0; v < 8; v++) w[v] = u[v] * iJ;
    const T ir = T(1) / w[0];
    const T v0 = w[1] * ir, v1 = w[2] * ir, v2 = w[3] * ir;
    const T B0 = w[5], B1 = w[6], B2 = w[7];
    const T hb2 = T(0.5) * (B0 * B0 + B1 * B1 + B2 * B2);
    const T p = (gam - T(1)) * (w[4] - T(0.5) * (w[1] * v0 + w[2] * v1 + w[3] * v2) - hb2);
    const T pt = p + hb2, Ept = w[4] + pt;
    const T vB = v0 * B0 + v1 * B1 + v2 * B2;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const T n0 = met[d * 3 + 0], n1 = met[d * 3 + 1], n2 = met[d * 3 + 2];
        const T mn = w[1] * n0 + w[2] * n1 + w[3] * n2;
        const T vn = mn * ir;
        const T Bn = B0 * n0 + B1 * n1 + B2 * n2;
        out[d][0] = mn;
        out[d][1] = mn * v0 + n0 * pt - Bn * B0;
        out[d][2] = mn * v1 + n1 * pt - Bn * B1;
        out[d][3] = mn * v2 + n2 * pt - Bn * B2;
        out[d][4] = Ept * vn - Bn * vB;
        out[d][5] = vn * B0 - Bn * v0;
        out[d][6] = vn * B1 - Bn * v1;
        out[d][7] = vn * B2 - Bn * v2;
    }
}

// fast magnetosonic speed along unit n
template <class T>
__device__ __forceinline__ T dev_fast(const T *u, T gam, const double *n)
{
    T ir = T(1.0) / u[0];
    T a2 = gam * dev_pressure<T>(u, gam) * ir;
    T b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * ir;
    T bn = u[5] * n[0] + u[6] * n[1] + u[7] * n[2];
    T bn2 = bn * bn * ir, s = a2 + b2;
    T disc = s * s - T(4.0) * a2 * bn2;
    disc = disc < T(0.0) ? T(0.0) : disc;
    return ssqrt(T(0.5) * (s + ssqrt(disc)));
}

// HLL with Davis speeds along unit n (from L to R)
template <class T>
__device__ __forceinline__ void dev_hll(const T *UL, const T *UR, const T *FL, const T *FR, const double *n, T gam,
                                        T *Fs)
{
    T vL = (UL[1] * n[0] + UL[2] * n[1] + UL[3] * n[2]) / UL[0];
    T vR = (UR[1] * n[0] + UR[2] * n[1] + UR[3] * n[2]) / UR[0];
    T cL = dev_fast<T>(UL, gam, n), cR = dev_fast<T>(UR, gam, n);
    T SL = smin(vL - cL, vR - cR), SR = smax(vL + cL, vR + cR);
    if (SL >= T(0.0)) {
        for (int v = 0; v < 8; v++) Fs[v] = FL[v];
    } else if (SR <= T(0.0)) {
        for (int v = 0; v < 8; v++) Fs[v] = FR[v];
    } else {
        T id = T(1.0) / (SR - SL);
        for (int v = 0; v < 8; v++) Fs[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) * id;
    }
}

__device__ __forceinline__ double dev_minmod(double a, double b)
{
    if (!(a * b > 0.0)) return 0.0;
    return a > 0.0 ? fmin(a, b) : fmax(a, b);
}

// four-state multidimensional HLL electric field along t in the frame F = (e1, e2, t)
template <class T>
__device__ __forceinline__ T emf4(const T U[4][8], const T Et[4], const double *F, T gam)
{
    const double *e1 = F, *e2 = F + 3;
    T ap1 = T(0.0), am1 = T(0.0), ap2 = T(0.0), am2 = T(0.0), B1[4], B2[4];
#pragma unroll
    for (int s = 0; s < 4; s++) {
        T ir = T(1.0) / U[s][0];
        T v1 = (U[s][1] * e1[0] + U[s][2] * e1[1] + U[s][3] * e1[2]) * ir;
        T v2 = (U[s][1] * e2[0] + U[s][2] * e2[1] + U[s][3] * e2[2]) * ir;
        T c1 = dev_fast<T>(U[s], gam, e1), c2 = dev_fast<T>(U[s], gam, e2);
        ap1 = smax(ap1, v1 + c1);
        am1 = smax(am1, c1 - v1);
        ap2 = smax(ap2, v2 + c2);
        am2 = smax(am2, c2 - v2);
        B1[s] = U[s][5] * e1[0] + U[s][6] * e1[1] + U[s][7] * e1[2];
        B2[s] = U[s][5] * e2[0] + U[s][6] * e2[1] + U[s][7] * e2[2];
    }
    // slots counter-clockwise: 0 SW, 1 SE, 2 NE, 3 NW
    T Es = (ap1 * ap2 * Et[0] + ap1 * am2 * Et[3] + am1 * ap2 * Et[1] + am1 * am2 * Et[2]) / ((ap1 + am1) * (ap2 + am2));
    Es += ap1 * am1 * (T(0.5) * (B2[1] + B2[2]) - T(0.5) * (B2[0] + B2[3])) / (ap1 + am1);
    Es -= ap2 * am2 * (T(0.5) * (B1[2] + B1[3]) - T(0.5) * (B1[0] + B1[1])) / (ap2 + am2);
    return Es;
}

// three zones about an edge: mean of the 1-D HLL induction fluxes of the three faces
template <class T>
__device__ __forceinline__ T emf3(const T U[4][8], const T E[4][3], const double *N3, const double *t, T gam)
{
    T acc = T(0.0);
    for (int s = 0; s < 3; s++) {
        int s2 = (s + 1) % 3;
        const double *n = N3 + 3 * s;
        T FL[8], FR[8], Fs[8];
        for (int v = 0; v < 8; v++) FL[v] = FR[v] = T(0.0);
        FL[5] = n[1] * E[s][2] - n[2] * E[s][1];
        FL[6] = n[2] * E[s][0] - n[0] * E[s][2];
        FL[7] = n[0] * E[s][1] - n[1] * E[s][0];
        FR[5] = n[1] * E[s2][2] - n[2] * E[s2][1];
        FR[6] = n[2] * E[s2][0] - n[0] * E[s2][2];
        FR[7] = n[0] * E[s2][1] - n[1] * E[s2][0];
        dev_hll<T>(U[s], U[s2], FL, FR, n, gam, Fs);
        double tn[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
        acc -= Fs[5] * tn[0] + Fs[6] * tn[1] + Fs[7] * tn[2];
    }
    return acc / T(3.0);
}

// WENO-AO combination (Section III) of one variable from its stencil
// differences du: large-stencil and small-stencil least squares, smoothness
// indicators, nonlinear weights and the adaptive-order blend.  Matrices of
// precision R, arithmetic in T.
template <int P, class T, class R>
__device__ __forceinline__ void weno_core(const T (&du)[Tr<P>::NS], const R *__restrict__ Pl,
                                          const R *__restrict__ Ps, const R *__restrict__ Qs, T eps,
                                          T (&out)[Tr<P>::NC], T &whi)
{
    using Tt = Tr<P>;
    const T ghi = T(WENO_GAMMA_HI), gs = T((1.0 - WENO_GAMMA_HI) / 7.0);
    T chi[Tt::NC];
#pragma unroll
    for (int a = 0; a < Tt::NC; a++) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < Tt::NS; j++) s += T(Pl[a * Tt::NS + j]) * du[j];
        chi[a] = s;
    }
    T cs[7][3];
#pragma unroll
    for (int s = 0; s < 7; s++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 6; j++) acc += T(Ps[s * 18 + i * 6 + j]) * du[j];
            cs[s][i] = acc;
        }
    T bhi = T(0);
#pragma unroll
    for (int a = 0; a < Tt::NC; a++) {
        T s = T(0);
#pragma unroll
        for (int b = 0; b < Tt::NC; b++) s += T(Qs[a * Tt::NC + b]) * chi[b];
        bhi += chi[a] * s;
    }
    T w0 = ghi / ((bhi + eps) * (bhi + eps)), tot = w0, ws[7];
#pragma unroll
    for (int s = 0; s < 7; s++) {
        T b = cs[s][0] * cs[s][0] + cs[s][1] * cs[s][1] + cs[s][2] * cs[s][2];
        ws[s] = gs / ((b + eps) * (b + eps));
        tot += ws[s];
    }
    T itot = T(1) / tot;
    w0 *= itot;
    whi = w0 / ghi;   // the large stencil's weight relative to its linear weight
#pragma unroll
    for (int a = 0; a < Tt::NC; a++) {
        T lin = T(0), nl = T(0);
        if (a < 3)
#pragma unroll
            for (int s = 0; s < 7; s++) { lin += gs * cs[s][a]; nl += ws[s] * itot * cs[s][a]; }
        out[a] = w0 / ghi * (chi[a] - lin) + nl;
    }
}

// Flux derivatives through the LDS slab.  Node lanes store the flux along
// direction d of their node at the node's position under the coordinate swap
// xi <-> d (identity for d = 0), so every one of the 24 (direction, variable)
// rows holds its values in the xi-derivative's own node order.  One lane per
// row then applies the xi-derivative matrix D_0, whose sparsity and entries
// (multiples of 1/2) are compile-time constants, in place: a row is read
// once into registers and each value is reused by all the outputs that need
// it.  D_d = S_d D_0 S_d for the swap S_d, so slot i of row (d, v) ends up
// holding the d-derivative at node S_d(i).
template <int SN, class R>
__device__ __forceinline__ void put_flux(R *sf, int i, int i1, int i2, const R (&F)[3][8])
{
#pragma unroll
    for (int v = 0; v < 8; v++) {
        sf[v * SN + i] = F[0][v];
        sf[(8 + v) * SN + i1] = F[1][v];
        sf[(16 + v) * SN + i2] = F[2][v];
    }
}

// entry e of D_0 (or of D_0^T), field k: row, column, twice the value
template <int P, bool TRANS>
__device__ constexpr int dent(int e, int k)
{
    return TRANS ? DTab<P>::ET[e][k] : DTab<P>::E[e][k];
}

// With TRANS the transposed table D_0^T is applied instead: slot S_d(l) of
// row (d, v) then holds sum_i D_d[i][l] x_i for values x_i stored at S_d(i).
template <int P, int SN, int ZS, int ZPW, class R, bool TRANS = false>
__device__ __forceinline__ void deriv_rows(R *slab, int lane)
{
    using D = DTab<P>;
    constexpr int N = Tr<P>::N;
#pragma unroll 1
    for (int t = lane; t < ZPW * 24; t += 64) {
        R *row = slab + (t / 24) * ZS + (t % 24) * SN;
        R x[N];
#pragma unroll
        for (int j = 0; j < N; j++) x[j] = row[j];
        R acc = R(0);
#pragma unroll
        for (int e = 0; e < D::NNZ; e++) {
            acc += R(0.5 * dent<P, TRANS>(e, 2)) * x[dent<P, TRANS>(e, 1)];
            if (e == D::NNZ - 1 || dent<P, TRANS>(e + 1, 0) != dent<P, TRANS>(e, 0)) {
                row[dent<P, TRANS>(e, 0)] = acc;
                acc = R(0);
            }
        }
    }
}

// acc = sum over the three directions of the derivative at node i
template <int SN, class R>
__device__ __forceinline__ void get_deriv(const R *sf, int i, int i1, int i2, R (&acc)[8])
{
#pragma unroll
    for (int v = 0; v < 8; v++) acc[v] = sf[v * SN + i] + sf[(8 + v) * SN + i1] + sf[(16 + v) * SN + i2];
}

// geometry table of precision R: the FP64 table or its FP32 copy
template <class R>
__device__ __forceinline__ const R *pick(const double *d, const float *f)
{
    if constexpr (sizeof(R) == sizeof(double)) return d;
    else return f;
}

// Runs of up to 64 items along a column: n = nu + nleft, the first nu items
// in nchunk wavefront-sized runs; a short tail (1 to 8 items beyond a
// multiple of 64) is left to nleft for the kernels' tail mode.
struct RunSplit {
    int nchunk, nu, nleft;
};
inline RunSplit run_split(int n)
{
    const int r = n % 64;
    if (n >= 64 && r >= 1 && r <= 8) return {n / 64, (n / 64) * 64, r};
    return {(n + 63) / 64, n, 0};
}

// the step's WENO-AO epsilon (0 selects the default)
inline double weno_eps(const rg_step_params &p) { return p.weno_eps > 0.0 ? p.weno_eps : WENO_EPS_DEFAULT; }

// Workgroups are dispatched round-robin over the eight XCDs, each with its
// own L2.  Renumbering so that XCD x runs one contiguous range of logical
// blocks keeps the blocks of a column (which share its geometry tables) in
// one L2.  A bijection of [0, nb) for any nb.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

}  // namespace rg

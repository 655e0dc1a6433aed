// ADER-CG predictor on the triangular-prism element (Section V.d, eqs.
// (5.20)-(5.29); Appendices B-D) for every zone of the icosahedral geodesic
// mesh.
//
// The space-time Galerkin system factors into the 1-D time matrix R and the
// nodal derivative matrices D_d (the prism spaces of eqs. (5.12)-(5.14) are
// closed under differentiation), so each Picard sweep is, per time level,
// mapped fluxes at the nodes followed by sum_d D_d F_d (eqs. C.34-C.36,
// D.29-D.32).  Layout of a 256-lane workgroup (ZPB zones):
//  - node phase: lane (zone, node) holds the node's eight conserved values at
//    every time level and computes its mapped flux (eq. 5.23), written to the
//    zone's LDS slab as 24 rows (direction, variable) of N values;
//  - derivative phase: lane (direction, zone, variable) loads one row into
//    registers and applies that direction's sparse D (compile-time tables) in
//    place.  ZPB * 8 rows per direction is a multiple of 64, so every
//    wavefront works on one direction and no lane diverges; at fourth order
//    the densest direction's outputs are split over two wavefronts.
// The first sweep starts from the tau = 0 state at every level, so it needs
// only the tau = 0 flux.  Geometry is per column for a unit shell; shell k
// scales it by r_k, which enters as dt / r_k on the metrics.  The metrics are
// re-read (cache hits: a column's shells share them) for every flux instead
// of held in registers, and the occupancy hint of three wavefronts per SIMD
// holds the fourth-order kernel to 168 registers (a 24-byte spill).  Fourth
// order on 81,920 triangles x 128 shells measured 101 ms with one direction
// per wavefront, 88 ms with the densest direction split over two, 77 ms with
// the hint and 76 ms with the metrics re-read.
#include <hip/hip_runtime.h>

#include "mhd_device.hpp"
#include "prism.hpp"
#include "prism_dtab.hpp"

namespace rg {

template <int P>
struct PrismLayout {
    static constexpr int N = PrismD<P>::N;
    static constexpr int ZPB = P == 2 ? 32 : P == 3 ? 16 : 8;   // zones per workgroup
    static constexpr int SN = N + 1;                             // slab row stride
    static constexpr int ZS = 24 * SN;                           // slab of one zone
    static_assert(ZPB * N <= 256 && (ZPB * 8) % 64 == 0, "workgroup layout");
};

template <int P, int DIR>
constexpr int pd_nz()
{
    if constexpr (DIR == 0) return PrismD<P>::NZ0;
    else if constexpr (DIR == 1) return PrismD<P>::NZ1;
    else return PrismD<P>::NZ2;
}

template <int P, int DIR>
constexpr int pd_ent(int e, int k)
{
    if constexpr (DIR == 0) return PrismD<P>::E0[e][k];
    else if constexpr (DIR == 1) return PrismD<P>::E1[e][k];
    else return PrismD<P>::E2[e][k];
}

template <int P, int DIR>
constexpr double pd_val(int e)
{
    if constexpr (DIR == 0) return PrismD<P>::V0[e];
    else if constexpr (DIR == 1) return PrismD<P>::V1[e];
    else return PrismD<P>::V2[e];
}

// the in-place row update below writes each output row once, so every row
// must have an entry and the entries must be grouped by row
template <int P, int DIR>
constexpr bool rows_complete()
{
    int e = 0;
    for (int i = 0; i < PrismD<P>::N; i++) {
        if (e >= pd_nz<P, DIR>() || pd_ent<P, DIR>(e, 0) != i) return false;
        while (e < pd_nz<P, DIR>() && pd_ent<P, DIR>(e, 0) == i) e++;
    }
    return e == pd_nz<P, DIR>();
}
static_assert(rows_complete<2, 0>() && rows_complete<2, 1>() && rows_complete<2, 2>(), "order-2 tables");
static_assert(rows_complete<3, 0>() && rows_complete<3, 1>() && rows_complete<3, 2>(), "order-3 tables");
static_assert(rows_complete<4, 0>() && rows_complete<4, 1>() && rows_complete<4, 2>(), "order-4 tables");

// first table entry of output row i (entries are grouped by row)
template <int P, int DIR>
constexpr int first_entry(int i)
{
    int e = 0;
    while (e < pd_nz<P, DIR>() && pd_ent<P, DIR>(e, 0) < i) e++;
    return e;
}

// output row that splits DIR's entries into two halves of nearly equal size
template <int P, int DIR>
constexpr int half_row()
{
    int i = 0;
    while (first_entry<P, DIR>(i + 1) <= pd_nz<P, DIR>() / 2) i++;
    return i;
}

// outputs I0 .. I1-1 of D_DIR applied to x, written to row
template <int P, int DIR, int I0, int I1>
__device__ __forceinline__ void prism_apply(const double *x, double *row)
{
    constexpr int E0 = first_entry<P, DIR>(I0), E1 = first_entry<P, DIR>(I1);
    double acc = 0.0;
#pragma unroll
    for (int e = E0; e < E1; e++) {
        acc += pd_val<P, DIR>(e) * x[pd_ent<P, DIR>(e, 1)];
        if (e == E1 - 1 || pd_ent<P, DIR>(e + 1, 0) != pd_ent<P, DIR>(e, 0)) {
            row[pd_ent<P, DIR>(e, 0)] = acc;
            acc = 0.0;
        }
    }
}

// row <- D_DIR row (the row holds one variable's DIR-flux at the N nodes)
template <int P, int DIR>
__device__ __forceinline__ void prism_row(double *row)
{
    constexpr int N = PrismD<P>::N;
    double x[N];
#pragma unroll
    for (int j = 0; j < N; j++) x[j] = row[j];
    prism_apply<P, DIR, 0, N>(x, row);
}

// Every slab row (zone, direction, variable) <- D_direction row.  With 64
// rows per direction (eight zones) the four wavefronts share the work by
// entry count: the eta rows, the densest, are split by output between two
// wavefronts, which first read their rows and wait for each other before
// writing them back.
template <int P>
__device__ __forceinline__ void prism_derivs(double *s_f, int tid)
{
    using L = PrismLayout<P>;
    if constexpr (L::ZPB * 8 == 64) {
        constexpr int N = L::N, H = half_row<P, 1>();
        const int w = tid >> 6, lane = tid & 63;
        const int dir = w == 0 ? 0 : w == 2 ? 2 : 1;
        double *row = s_f + (lane >> 3) * L::ZS + (dir * 8 + (lane & 7)) * L::SN;
        double x[N];
#pragma unroll
        for (int j = 0; j < N; j++) x[j] = row[j];
        __syncthreads();
        if (w == 0) prism_apply<P, 0, 0, N>(x, row);
        else if (w == 1) prism_apply<P, 1, 0, H>(x, row);
        else if (w == 2) prism_apply<P, 2, 0, N>(x, row);
        else prism_apply<P, 1, H, N>(x, row);
    } else {
        constexpr int NROW = 3 * L::ZPB * 8;
#pragma unroll 1
        for (int rr = tid; rr < NROW; rr += 256) {
            const int d = rr / (L::ZPB * 8), rem = rr % (L::ZPB * 8);
            double *row = s_f + (rem / 8) * L::ZS + (d * 8 + rem % 8) * L::SN;
            if (d == 0) prism_row<P, 0>(row);
            else if (d == 1) prism_row<P, 1>(row);
            else prism_row<P, 2>(row);
        }
    }
}

template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void prism_predictor(DevPrism G, double dt, double gamma, int npic,
                                                       const double *__restrict__ Ua, double *__restrict__ aU,
                                                       double *__restrict__ aF)
{
    using L = PrismLayout<P>;
    constexpr int N = L::N, SN = L::SN, E = P - 1;
    __shared__ double s_f[L::ZPB * L::ZS];
    const int tid = threadIdx.x, zl = tid / N, i = tid % N;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const i64 z = (i64)lb * L::ZPB + zl;
    const bool active = zl < L::ZPB && z < G.nz;
    double *sf = s_f + (zl < L::ZPB ? zl : 0) * L::ZS;
    const double gam = gamma;

    double U0[8], iJ = 1.0, dFa[8], Ut[E][8], fac = 0.0;
    const double *gm = G.met;
#pragma unroll
    for (int v = 0; v < 8; v++) U0[v] = 0.0;
    if (active) {
        const i64 t = z / G.n_rad;
        const int k = (int)(z - t * G.n_rad);
        const double J = G.J[t * N + i];
        iJ = 1.0 / J;
        fac = dt * G.rinv[k];
        gm = G.met + t * 9 * N + i;
        double met[9];
#pragma unroll
        for (int m = 0; m < 9; m++) met[m] = fac * gm[m * N];
#pragma unroll
        for (int v = 0; v < 8; v++) U0[v] = J * Ua[((i64)v * G.nz + z) * N + i];
        double F[3][8];
        mapped_flux<double>(U0, iJ, met, gam, F);
#pragma unroll
        for (int d = 0; d < 3; d++)
#pragma unroll
            for (int v = 0; v < 8; v++) sf[(d * 8 + v) * SN + i] = F[d][v];
    }
    __syncthreads();
    prism_derivs<P>(s_f, tid);
    __syncthreads();
    const double on = npic > 0 ? 1.0 : 0.0;
#pragma unroll
    for (int v = 0; v < 8; v++) dFa[v] = active ? sf[v * SN + i] + sf[(8 + v) * SN + i] + sf[(16 + v) * SN + i] : 0.0;
#pragma unroll
    for (int t = 0; t < E; t++) {
        double rs = G.R[t * P];
#pragma unroll
        for (int s = 0; s < E; s++) rs += G.R[t * P + s + 1];
#pragma unroll
        for (int v = 0; v < 8; v++) Ut[t][v] = U0[v] - on * rs * dFa[v];
    }
    __syncthreads();
    for (int it = 1; it < npic; it++) {
        double A[E][8];
#pragma unroll
        for (int s = 0; s < E; s++) {
            if (active) {
                double F[3][8], met[9];
#pragma unroll
                for (int m = 0; m < 9; m++) met[m] = fac * gm[m * N];
                mapped_flux<double>(Ut[s], iJ, met, gam, F);
#pragma unroll
                for (int d = 0; d < 3; d++)
#pragma unroll
                    for (int v = 0; v < 8; v++) sf[(d * 8 + v) * SN + i] = F[d][v];
            }
            __syncthreads();
            prism_derivs<P>(s_f, tid);
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 8; v++)
                A[s][v] = active ? sf[v * SN + i] + sf[(8 + v) * SN + i] + sf[(16 + v) * SN + i] : 0.0;
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < E; t++) {
            const double r0 = G.R[t * P];
#pragma unroll
            for (int v = 0; v < 8; v++) {
                double u = U0[v] - r0 * dFa[v];
#pragma unroll
                for (int s = 0; s < E; s++) u -= G.R[t * P + s + 1] * A[s][v];
                Ut[t][v] = u;
            }
        }
    }
    if (!active) return;
    // time averages of the state and of the physical flux over the Gauss levels
    double sU[8], sF[3][8];
#pragma unroll
    for (int v = 0; v < 8; v++) { sU[v] = 0.0; sF[0][v] = sF[1][v] = sF[2][v] = 0.0; }
#pragma unroll
    for (int t = 0; t < E; t++) {
        const double wt = G.wt[t + 1];
        double w[8], F[3][8];
#pragma unroll
        for (int v = 0; v < 8; v++) w[v] = Ut[t][v] * iJ;
        dev_flux<double>(w, gam, F);
#pragma unroll
        for (int v = 0; v < 8; v++) {
            sU[v] += wt * w[v];
            sF[0][v] += wt * F[0][v];
            sF[1][v] += wt * F[1][v];
            sF[2][v] += wt * F[2][v];
        }
    }
#pragma unroll
    for (int v = 0; v < 8; v++) aU[((i64)v * G.nz + z) * N + i] = sU[v];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int v = 0; v < 8; v++) aF[((i64)(d * 8 + v) * G.nz + z) * N + i] = sF[d][v];
}

// Face traces: tr double[32][Q][nz] (value, face point, zone; zones fastest,
// so that the face-flux kernels' lanes, consecutive shells, read consecutive
// records).  One lane per zone: for each of the 32 values the lane copies its
// zone's N nodal averages (the wavefront's loads cover contiguous memory)
// into its own LDS row and sums the at most TRACE_TERMS non-zero basis values
// of each face point's nodes from there.  Bound by HBM: 32 N values read and
// 32 Q written per zone.  (A 256-lane form that staged the averages of 256/Q
// zones and gave each lane one (zone, point) wrote [32][nz][Q]: 40.5 ms at
// fourth order on the benchmark mesh, and the face fluxes that read it
// 32.5 ms.)
template <int P>
struct TraceLayout {
    static constexpr int N = PrismD<P>::N;
    static constexpr int QT = P == 2 ? 3 : P == 3 ? 6 : 10;
    static constexpr int QS = P == 2 ? 3 : P == 3 ? 4 : 6;
    static constexpr int Q = 2 * QT + 3 * QS;
};
constexpr int TR_LANES = 128;

template <int P>
__global__ __launch_bounds__(TR_LANES) void prism_traces(DevPrism G, const double *__restrict__ aU,
                                                         const double *__restrict__ aF, double *__restrict__ tr)
{
    using L = TraceLayout<P>;
    constexpr int N = L::N, Q = L::Q;
    __shared__ double s_row[TR_LANES * (N + 1)];
    const i64 z = (i64)xcd_block(blockIdx.x, gridDim.x) * TR_LANES + threadIdx.x;
    if (z >= G.nz) return;
    double *row = s_row + threadIdx.x * (N + 1);
    const i64 nz = G.nz;
    for (int v = 0; v < 32; v++) {
        const double *src = v < 8 ? aU + ((i64)v * nz + z) * N : aF + ((i64)(v - 8) * nz + z) * N;
#pragma unroll
        for (int l = 0; l < N; l++) row[l] = src[l];
        for (int q = 0; q < Q; q++) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < TRACE_TERMS; t++)
                acc += G.fval[q * TRACE_TERMS + t] * row[G.fidx[q * TRACE_TERMS + t]];
            tr[((i64)v * Q + q) * nz + z] = acc;
        }
    }
}

template <int P>
static rg_status launch_traces(const DevPrism &G, const double *aU, const double *aF, double *tr, hipStream_t st)
{
    using L = TraceLayout<P>;
    if (G.Q != L::Q) { set_error("face point count differs from the kernel's"); return RG_EINVAL; }
    const i64 nb = (G.nz + TR_LANES - 1) / TR_LANES;
    if (nb >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (nb == 0) return RG_OK;
    prism_traces<P><<<(unsigned)nb, TR_LANES, 0, st>>>(G, aU, aF, tr);
    if (hipGetLastError() != hipSuccess) { set_error("prism trace launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

rg_status launch_prism_traces(const DevPrism &G, const double *aU, const double *aF, double *tr, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (G.order) {
    case 2: return launch_traces<2>(G, aU, aF, tr, st);
    case 3: return launch_traces<3>(G, aU, aF, tr, st);
    case 4: return launch_traces<4>(G, aU, aF, tr, st);
    default: set_error("prism order must be 2, 3 or 4"); return RG_ENOTSUP;
    }
}

// Face fluxes: one lane per face, the faces of a column (radial) or of an
// edge (side) in consecutive lanes, so that for every value and point the
// lanes read consecutive records of the traces.  The lane sums over its
// face's points |dA| times the HLL flux of the two sides' traces along the
// point's area vector.  Radial faces take the zone below (top face) and above
// (bottom face) at the same (xi, eta); side faces pair point i of the first
// triangle with the mirrored point of its neighbour, which runs the edge the
// other way.  One launch per kind of face.  (The lane-per-point form on the
// [32][nz][Q] traces, its face's points summed in LDS, took 15.4 + 17.1 ms on
// the benchmark mesh.)
template <int NPT>
__device__ __forceinline__ void face_point_flux(const double *__restrict__ tr, i64 nz, int Q, int ql, i64 zl, int qr,
                                                i64 zr, const double *A, double scale, double gam, double (&Fsum)[8])
{
    double n[3] = {scale * A[0], scale * A[1], scale * A[2]};
    const double a = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]), ia = 1.0 / a;
    n[0] *= ia; n[1] *= ia; n[2] *= ia;
    const i64 sl = (i64)Q * nz;
    const double *pl = tr + (i64)ql * nz + zl, *pr = tr + (i64)qr * nz + zr;
    double UL[8], UR[8], FL[8], FR[8], Fs[8];
#pragma unroll
    for (int v = 0; v < 8; v++) {
        UL[v] = pl[v * sl];
        UR[v] = pr[v * sl];
        FL[v] = n[0] * pl[(8 + v) * sl] + n[1] * pl[(16 + v) * sl] + n[2] * pl[(24 + v) * sl];
        FR[v] = n[0] * pr[(8 + v) * sl] + n[1] * pr[(16 + v) * sl] + n[2] * pr[(24 + v) * sl];
    }
    dev_hll<double>(UL, UR, FL, FR, n, gam, Fs);
#pragma unroll
    for (int v = 0; v < 8; v++) Fsum[v] += Fs[v] * a;
}

template <int P>
__global__ __launch_bounds__(256) void prism_face_flux_radial(DevPrism G, double gam, const double *__restrict__ tr,
                                                              double *__restrict__ Phi)
{
    using L = TraceLayout<P>;
    constexpr int QT = L::QT, Q = L::Q;
    const i64 f = (i64)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int nr = G.n_rad;
    if (f >= G.ntri * (nr + 1)) return;
    const i64 t = f / (nr + 1);
    const int kf = (int)(f - t * (nr + 1));
    // top face of the zone below, else the bottom face; bottom face of the
    // zone above, else the top face
    const i64 zl = t * nr + (kf > 0 ? kf - 1 : 0), zr = t * nr + (kf < nr ? kf : nr - 1);
    const int ql = kf > 0 ? 0 : QT, qr = kf < nr ? QT : 0;
    const double scale = G.radius[kf] * G.radius[kf];
    double Fsum[8];
#pragma unroll
    for (int v = 0; v < 8; v++) Fsum[v] = 0.0;
#pragma unroll 1
    for (int i = 0; i < QT; i++)
        face_point_flux<QT>(tr, G.nz, Q, ql + i, zl, qr + i, zr, G.tfA + (t * QT + i) * 3, scale, gam, Fsum);
#pragma unroll
    for (int v = 0; v < 8; v++) Phi[f * 8 + v] = Fsum[v];
}

template <int P>
__global__ __launch_bounds__(256) void prism_face_flux_side(DevPrism G, double gam, const double *__restrict__ tr,
                                                            double *__restrict__ Phi)
{
    using L = TraceLayout<P>;
    constexpr int QT = L::QT, QS = L::QS, Q = L::Q;
    const i64 f = (i64)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int nr = G.n_rad;
    if (f >= G.nedges * nr) return;
    const i64 e = f / nr;
    const int k = (int)(f - e * nr);
    const int t1 = G.edges[4 * e], e1 = G.edges[4 * e + 1], t2 = G.edges[4 * e + 2], e2 = G.edges[4 * e + 3];
    const i64 zl = (i64)t1 * nr + k, zr = (i64)t2 * nr + k;
    const double scale = G.radius[k] * G.radius[k];
    double Fsum[8];
#pragma unroll
    for (int v = 0; v < 8; v++) Fsum[v] = 0.0;
#pragma unroll 1
    for (int i = 0; i < QS; i++)
        face_point_flux<QS>(tr, G.nz, Q, 2 * QT + e1 * QS + i, zl, 2 * QT + e2 * QS + G.mirror[i], zr,
                            G.sfA + (((i64)t1 * 3 + e1) * QS + i) * 3, scale, gam, Fsum);
    const i64 nrf = G.ntri * (nr + 1);
#pragma unroll
    for (int v = 0; v < 8; v++) Phi[(nrf + f) * 8 + v] = Fsum[v];
}

template <int P>
static rg_status launch_fluxes(const DevPrism &G, double gamma, const double *tr, double *Phi, hipStream_t st)
{
    using L = TraceLayout<P>;
    if (G.QT != L::QT || G.QS != L::QS) { set_error("face point counts differ from the kernel's"); return RG_EINVAL; }
    const i64 nrf = G.ntri * (G.n_rad + 1), nsf = G.nedges * G.n_rad;
    const i64 br = (nrf + 255) / 256, bs = (nsf + 255) / 256;
    if (br >= ((i64)1 << 31) || bs >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (br > 0) prism_face_flux_radial<P><<<(unsigned)br, 256, 0, st>>>(G, gamma, tr, Phi);
    if (bs > 0) prism_face_flux_side<P><<<(unsigned)bs, 256, 0, st>>>(G, gamma, tr, Phi);
    if (hipGetLastError() != hipSuccess) { set_error("prism face flux launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

rg_status launch_prism_face_flux(const DevPrism &G, double gamma, const double *tr, double *Phi, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (G.order) {
    case 2: return launch_fluxes<2>(G, gamma, tr, Phi, st);
    case 3: return launch_fluxes<3>(G, gamma, tr, Phi, st);
    case 4: return launch_fluxes<4>(G, gamma, tr, Phi, st);
    default: set_error("prism order must be 2, 3 or 4"); return RG_ENOTSUP;
    }
}

// Finite-volume update of the zone averages (Section VI): U - dt / V times
// the zone's net outward face flux; one lane per zone (U, Uo [8][nz],
// Phi [nfaces][8]).
__global__ __launch_bounds__(256) void prism_update(DevPrism G, double dt, const double *__restrict__ U,
                                                    const double *__restrict__ Phi, double *__restrict__ Uo)
{
    const i64 z = (i64)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (z >= G.nz) return;
    const int nr = G.n_rad;
    const i64 t = z / nr, nrf = G.ntri * (nr + 1);
    const int k = (int)(z - t * nr);
    i64 f[5];
    double sg[5];
    f[0] = t * (nr + 1) + k + 1;   // top face, +r outward
    sg[0] = 1.0;
    f[1] = t * (nr + 1) + k;       // bottom face
    sg[1] = -1.0;
#pragma unroll
    for (int e = 0; e < 3; e++) {
        const int id = G.tedge[t * 3 + e];
        f[2 + e] = nrf + (i64)(id >= 0 ? id : -id - 1) * nr + k;
        sg[2 + e] = id >= 0 ? 1.0 : -1.0;
    }
    const double r = G.radius[k], cfac = dt / (r * r * r * G.vol[t]);
#pragma unroll
    for (int v = 0; v < 8; v++) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 5; j++) acc += sg[j] * Phi[f[j] * 8 + v];
        Uo[(i64)v * G.nz + z] = U[(i64)v * G.nz + z] - cfac * acc;
    }
}

// Divergence-free B: per column the dense product Out (nout x shells) =
// M (nout x nin) In (nin x shells) of the column's map with the inputs of its
// zones, on the FP64 matrix cores.  One wavefront owns DIVFREE_NT tiles of
// 16 shells of a column and every output row, stepping through the inputs
// four at a time: each A operand (a 16-row slice of the map, read from its
// transposed [nin][nout] copy) serves all the wavefront's tiles, and the B
// operands are loaded straight from Bin.  The inputs are padded to a multiple
// of four and the outputs to a multiple of 16 with zeros.  Bin [nin][nz],
// Bout [nout][nz].  (v_mfma_f64_16x16x4: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[i][j] in lane j + 16 (i % 4), element i / 4.)
// At fourth order on 81,920 columns x 128 shells: 12.6 ms as a VALU
// mat-vec per zone with the map through scalar loads (one wait per input),
// 9.1 ms on the matrix cores with the operand loads under branches, 4.8 ms
// with branch-free, double-buffered operand loads and four tiles per
// wavefront (two tiles: 5.3 ms; four cost two spilled registers).
constexpr int DIVFREE_NT = 4;

template <int P> struct DivfreeShape {
    static constexpr int nc = P == 2 ? 3 : P == 3 ? 9 : 19;     // Taylor terms of degree 1..P-1
    static constexpr int N = P == 2 ? 6 : P == 3 ? 15 : 26;
    static constexpr int Q = P == 2 ? 15 : P == 3 ? 24 : 38;    // face points
    static constexpr int nin = 3 * (nc + 1) + Q + 5, nout = 3 * N + 3;
};

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void prism_divfree(DevPrism G, const double *__restrict__ Mb,
                                                    const double *__restrict__ Bin, double *__restrict__ Bout)
{
    using S = DivfreeShape<P>;
    constexpr int NIN = S::nin, NOUT = S::nout, KT = (NIN + 3) / 4, MT = (NOUT + 15) / 16, NT = DIVFREE_NT;
    const int nt = (G.n_rad + 16 * NT - 1) / (16 * NT);
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const i64 c = lb / nt;
    const int tile = (int)(lb % nt);
    const int l = threadIdx.x, g = l >> 4, jz = l & 15;
    int kk[NT];
    bool active[NT];
    i64 z[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) {
        kk[t] = (tile * NT + t) * 16 + jz;
        active[t] = kk[t] < G.n_rad;
        z[t] = c * G.n_rad + (active[t] ? kk[t] : 0);     // inactive lanes read shell 0, store nothing
    }
    const double *__restrict__ M = Mb + c * (i64)(NIN * NOUT);
    dbl4 acc[NT][MT];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int m = 0; m < MT; m++) acc[t][m] = dbl4{0.0, 0.0, 0.0, 0.0};
    // operands of K step s: every load is unconditional and in bounds (the
    // indices are clamped) and the padding is selected to zero afterwards, so
    // the loads of the next step are in flight during this step's products
    auto load = [&](int s, double (&a)[MT], double (&b)[NT]) {
        const int j = 4 * s + g;
        const bool jin = j < NIN;
        const int jc = jin ? j : NIN - 1;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const double v = Bin[(i64)jc * G.nz + z[t]];
            b[t] = jin ? v : 0.0;
        }
        const double *__restrict__ mrow = M + jc * NOUT;
#pragma unroll
        for (int m = 0; m < MT; m++) {
            const int r = m * 16 + jz;
            const double v = mrow[r < NOUT ? r : NOUT - 1];
            a[m] = jin && r < NOUT ? v : 0.0;
        }
    };
    auto product = [&](const double (&a)[MT], const double (&b)[NT]) {
#pragma unroll
        for (int m = 0; m < MT; m++)
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t][m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[t], acc[t][m], 0, 0, 0);
    };
    double a0[MT], b0[NT], a1[MT], b1[NT];
    load(0, a0, b0);
#pragma unroll 1
    for (int s = 0; s < KT; s += 2) {
        if (s + 1 < KT) load(s + 1, a1, b1);
        product(a0, b0);
        if (s + 2 < KT) load(s + 2, a0, b0);
        if (s + 1 < KT) product(a1, b1);
    }
#pragma unroll
    for (int t = 0; t < NT; t++) {
        if (!active[t]) continue;
#pragma unroll
        for (int m = 0; m < MT; m++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = m * 16 + g + 4 * v;
                if (r < NOUT) Bout[(i64)r * G.nz + z[t]] = acc[t][m][v];
            }
    }
}

rg_status launch_prism_divfree(const DevPrism &G, const double *Bin, double *Bout, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const i64 nb = (i64)G.ntri * ((G.n_rad + 16 * DIVFREE_NT - 1) / (16 * DIVFREE_NT));
    if (nb >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (nb == 0) return RG_OK;
    bool shape_ok = false;
    switch (G.order) {
    case 2:
        shape_ok = G.nin == DivfreeShape<2>::nin && G.nout == DivfreeShape<2>::nout;
        if (shape_ok) prism_divfree<2><<<(unsigned)nb, 64, 0, st>>>(G, G.Mb, Bin, Bout);
        break;
    case 3:
        shape_ok = G.nin == DivfreeShape<3>::nin && G.nout == DivfreeShape<3>::nout;
        if (shape_ok) prism_divfree<3><<<(unsigned)nb, 64, 0, st>>>(G, G.Mb, Bin, Bout);
        break;
    case 4:
        shape_ok = G.nin == DivfreeShape<4>::nin && G.nout == DivfreeShape<4>::nout;
        if (shape_ok) prism_divfree<4><<<(unsigned)nb, 64, 0, st>>>(G, G.Mb, Bin, Bout);
        break;
    default:
        break;
    }
    if (!shape_ok) { set_error("divergence-free map shape does not match the element order"); return RG_EINVAL; }
    if (hipGetLastError() != hipSuccess) { set_error("prism divergence-free launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

// ---------------------------------------------------------------- constrained transport
// Edge traces: per zone the state and the induction fluxes F_d[B_i] at the
// 27 edge points (EDGE_POINTS), er double[17][27][nz] (value, point, zone;
// zones fastest, so that the edge kernels' lanes, consecutive shells, read
// consecutive records).  One lane per zone: for each of the 17 values the
// lane loads its zone's N nodal values (the wavefront's loads cover
// contiguous memory) into its own LDS row, then sums the at most
// EDGE_TERMS non-zero basis values of each point's nodes from there.
constexpr int ETR_LANES = 128;
constexpr int ETR_VALUES = 17;

template <int P>
__global__ __launch_bounds__(ETR_LANES) void prism_edge_traces(DevPrism G, const double *__restrict__ aU,
                                                               const double *__restrict__ aF,
                                                               double *__restrict__ er)
{
    constexpr int N = P == 2 ? 6 : P == 3 ? 15 : 26;
    __shared__ double s_row[ETR_LANES * (N + 1)];
    const i64 z = (i64)xcd_block(blockIdx.x, gridDim.x) * ETR_LANES + threadIdx.x;
    if (z >= G.nz) return;
    double *row = s_row + threadIdx.x * (N + 1);
    const i64 nz = G.nz;
    for (int v = 0; v < ETR_VALUES; v++) {
        const int fv = v - 8;
        const double *src = v < 8 ? aU + ((i64)v * nz + z) * N
                                  : aF + ((i64)((fv / 3) * 8 + 5 + fv % 3) * nz + z) * N;
#pragma unroll
        for (int l = 0; l < N; l++) row[l] = src[l];
        for (int pt = 0; pt < EDGE_POINTS; pt++) {
            double acc = 0.0;
#pragma unroll
            for (int n = 0; n < EDGE_TERMS; n++)
                acc += G.eval[pt * EDGE_TERMS + n] * row[G.eidx[pt * EDGE_TERMS + n]];
            er[((i64)v * EDGE_POINTS + pt) * nz + z] = acc;
        }
    }
}

// state and induction fluxes of zone z at edge point pt from the records
__device__ __forceinline__ void edge_trace(const DevPrism &G, const double *__restrict__ er, i64 z, int pt,
                                           double (&U)[8], double (&FB)[3][3])
{
    const i64 nz = G.nz;
#pragma unroll
    for (int v = 0; v < 8; v++) U[v] = er[((i64)v * EDGE_POINTS + pt) * nz + z];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int i = 0; i < 3; i++) FB[d][i] = er[((i64)(8 + 3 * d + i) * EDGE_POINTS + pt) * nz + z];
}

// E . t with E_x = F_z[B_y], E_y = F_x[B_z], E_z = F_y[B_x]
__device__ __forceinline__ double edge_field(const double (&FB)[3][3], const double *t)
{
    return FB[2][1] * t[0] + FB[0][2] * t[1] + FB[1][0] * t[2];
}

// -(t x n) . F_B of the 1-D HLL flux between two zones along unit n (from a
// to b): the field along t that the face between them carries
__device__ __forceinline__ double face_field(const double (&Ua)[8], const double (&Fa)[3][3], const double (&Ub)[8],
                                             const double (&Fb)[3][3], const double *n, const double *t, double gam)
{
    double FL[8], FR[8], Fs[8];
#pragma unroll
    for (int v = 0; v < 5; v++) FL[v] = FR[v] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        FL[5 + i] = n[0] * Fa[0][i] + n[1] * Fa[1][i] + n[2] * Fa[2][i];
        FR[5 + i] = n[0] * Fb[0][i] + n[1] * Fb[1][i] + n[2] * Fb[2][i];
    }
    dev_hll<double>(Ua, Ub, FL, FR, n, gam, Fs);
    const double tn[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
    return -(Fs[5] * tn[0] + Fs[6] * tn[1] + Fs[7] * tn[2]);
}

// angular edges: one lane per (mesh edge, radius level), the levels of an
// edge in consecutive lanes
__global__ __launch_bounds__(256) void prism_emf_ang(DevPrism G, double gam, const double *__restrict__ er,
                                                     double *__restrict__ Gang)
{
    const i64 i = (i64)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int nr1 = G.n_rad + 1;
    if (i >= G.nedges * nr1) return;
    const i64 e = i / nr1;
    const int kr = (int)(i % nr1);
    const int t1 = G.edges[4 * e], e1 = G.edges[4 * e + 1], t2 = G.edges[4 * e + 2], e2 = G.edges[4 * e + 3];
    const double r = G.radius[kr];
    const double w3[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    double gam_sum = 0.0;
    for (int pp = 0; pp < 3; pp++) {
        const double *g = G.aeg + (e * 3 + pp) * 16;
        double Es;
        if (kr > 0 && kr < G.n_rad) {
            // slots counter-clockwise about t: SW (t2 below), SE (t1 below),
            // NE (t1 above), NW (t2 above); the zone below sees the edge on
            // its top face (zeta = +1/2), the zone above on its bottom face;
            // the second triangle runs the edge the other way
            double U[4][8], Et[4], FB[3][3];
            edge_trace(G, er, (i64)t2 * G.n_rad + kr - 1, (0 * 3 + e2) * 3 + 2 - pp, U[0], FB);
            Et[0] = edge_field(FB, g);
            edge_trace(G, er, (i64)t1 * G.n_rad + kr - 1, (0 * 3 + e1) * 3 + pp, U[1], FB);
            Et[1] = edge_field(FB, g);
            edge_trace(G, er, (i64)t1 * G.n_rad + kr, (1 * 3 + e1) * 3 + pp, U[2], FB);
            Et[2] = edge_field(FB, g);
            edge_trace(G, er, (i64)t2 * G.n_rad + kr, (1 * 3 + e2) * 3 + 2 - pp, U[3], FB);
            Et[3] = edge_field(FB, g);
            Es = emf4<double>(U, Et, g + 3, gam);
        } else {
            // the one shell at r_in or r_out: the side face's 1-D HLL field
            const int k = kr > 0 ? kr - 1 : kr, side = kr > 0 ? 0 : 1;
            double Ua[8], Ub[8], Fa[3][3], Fb[3][3];
            edge_trace(G, er, (i64)t1 * G.n_rad + k, (side * 3 + e1) * 3 + pp, Ua, Fa);
            edge_trace(G, er, (i64)t2 * G.n_rad + k, (side * 3 + e2) * 3 + 2 - pp, Ub, Fb);
            Es = face_field(Ua, Fa, Ub, Fb, g + 9, g, gam);
        }
        gam_sum += w3[pp] * (g[12] * r) * Es;
    }
    Gang[i] = gam_sum;
}

// radial edges: one lane per (vertex, shell); the ring's zones are traced in
// turn and each face between consecutive ones contributes its 1-D HLL field
__global__ __launch_bounds__(256) void prism_emf_rad(DevPrism G, double gam, const double *__restrict__ er,
                                                     double *__restrict__ Grad)
{
    const i64 i = (i64)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (i >= G.nvert * G.n_rad) return;
    const i64 v = i / G.n_rad;
    const int k = (int)(i % G.n_rad);
    const int r0 = G.ring_off[v], K = G.ring_off[v + 1] - r0;
    const double t[3] = {G.vxyz[3 * v], G.vxyz[3 * v + 1], G.vxyz[3 * v + 2]};
    const double dl = G.radius[k + 1] - G.radius[k];
    const double w3[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    double gam_sum = 0.0;
    for (int pp = 0; pp < 3; pp++) {
        double U0[8], F0[3][3], Up[8], Fp[3][3], Uc[8], Fc[3][3];
        double acc = 0.0;
        for (int m = 0; m <= K; m++) {
            if (m < K) {
                const int tj = G.ring_tj[r0 + m];
                edge_trace(G, er, (i64)(tj / 3) * G.n_rad + k, 18 + 3 * (tj % 3) + pp, Uc, Fc);
            } else {
#pragma unroll
                for (int q = 0; q < 8; q++) Uc[q] = U0[q];
#pragma unroll
                for (int d = 0; d < 3; d++)
#pragma unroll
                    for (int q = 0; q < 3; q++) Fc[d][q] = F0[d][q];
            }
            if (m == 0) {
#pragma unroll
                for (int q = 0; q < 8; q++) U0[q] = Uc[q];
#pragma unroll
                for (int d = 0; d < 3; d++)
#pragma unroll
                    for (int q = 0; q < 3; q++) F0[d][q] = Fc[d][q];
            } else {
                acc += face_field(Up, Fp, Uc, Fc, G.ring_n + 3 * (i64)(r0 + m - 1), t, gam);
            }
#pragma unroll
            for (int q = 0; q < 8; q++) Up[q] = Uc[q];
#pragma unroll
            for (int d = 0; d < 3; d++)
#pragma unroll
                for (int q = 0; q < 3; q++) Fp[d][q] = Fc[d][q];
        }
        gam_sum += w3[pp] * dl * (acc / K);
    }
    Grad[i] = gam_sum;
}

// face magnetic fluxes: minus dt times the circulation of the edge integrals
// counter-clockwise about each face's direction (radial faces along +r,
// side faces out of the edge's first triangle)
__global__ __launch_bounds__(256) void prism_ct(DevPrism G, double dt, const double *__restrict__ Gang,
                                                const double *__restrict__ Grad, const double *__restrict__ PhiB,
                                                double *__restrict__ PhiBo)
{
    const i64 f = (i64)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (f >= G.nfaces) return;
    const int nr = G.n_rad, nr1 = nr + 1;
    const i64 nrf = G.ntri * nr1;
    double circ;
    if (f < nrf) {
        const i64 t = f / nr1;
        const int kf = (int)(f % nr1);
        circ = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int te = G.tedge[3 * t + j];
            const i64 e = te >= 0 ? te : -te - 1;
            const double g = Gang[e * nr1 + kf];
            circ += te >= 0 ? g : -g;
        }
    } else {
        const i64 s = f - nrf, e = s / nr;
        const int k = (int)(s % nr);
        const i64 A = G.edge_ab[2 * e], B = G.edge_ab[2 * e + 1];
        circ = Gang[e * nr1 + k] + Grad[B * nr + k] - Gang[e * nr1 + k + 1] - Grad[A * nr + k];
    }
    PhiBo[f] = PhiB[f] - dt * circ;
}

rg_status launch_prism_edge_traces(const DevPrism &G, const double *aU, const double *aF, double *er, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const i64 nb = (G.nz + ETR_LANES - 1) / ETR_LANES;
    if (nb >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (nb == 0) return RG_OK;
    switch (G.order) {
    case 2: prism_edge_traces<2><<<(unsigned)nb, ETR_LANES, 0, st>>>(G, aU, aF, er); break;
    case 3: prism_edge_traces<3><<<(unsigned)nb, ETR_LANES, 0, st>>>(G, aU, aF, er); break;
    case 4: prism_edge_traces<4><<<(unsigned)nb, ETR_LANES, 0, st>>>(G, aU, aF, er); break;
    default: set_error("order must be 2, 3 or 4"); return RG_EINVAL;
    }
    if (hipGetLastError() != hipSuccess) { set_error("prism edge trace launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

rg_status launch_prism_edge_emfs(const DevPrism &G, double gamma, const double *er, double *Gang, double *Grad,
                                 void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const i64 na = G.nedges * (G.n_rad + 1), nv = G.nvert * G.n_rad;
    const i64 ba = (na + 255) / 256, bv = (nv + 255) / 256;
    if (ba >= ((i64)1 << 31) || bv >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (ba > 0) prism_emf_ang<<<(unsigned)ba, 256, 0, st>>>(G, gamma, er, Gang);
    if (bv > 0) prism_emf_rad<<<(unsigned)bv, 256, 0, st>>>(G, gamma, er, Grad);
    if (hipGetLastError() != hipSuccess) { set_error("prism edge field launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

rg_status launch_prism_ct(const DevPrism &G, double dt, const double *Gang, const double *Grad, const double *PhiB,
                          double *PhiBo, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const i64 nb = (G.nfaces + 255) / 256;
    if (nb >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (nb > 0) prism_ct<<<(unsigned)nb, 256, 0, st>>>(G, dt, Gang, Grad, PhiB, PhiBo);
    if (hipGetLastError() != hipSuccess) { set_error("prism constrained-transport launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

rg_status launch_prism_update(const DevPrism &G, double dt, const double *U, const double *Phi, double *Uo, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const i64 nb = (G.nz + 255) / 256;
    if (nb >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (nb == 0) return RG_OK;
    prism_update<<<(unsigned)nb, 256, 0, st>>>(G, dt, U, Phi, Uo);
    if (hipGetLastError() != hipSuccess) { set_error("prism update launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

template <int P>
static rg_status launch_order(const DevPrism &G, double dt, double gamma, int npic, const double *Ua, double *aU,
                              double *aF, hipStream_t st)
{
    using L = PrismLayout<P>;
    const i64 nb = (G.nz + L::ZPB - 1) / L::ZPB;
    if (nb >= ((i64)1 << 31)) { set_error("prism mesh too large for one launch"); return RG_ENOTSUP; }
    if (nb == 0) return RG_OK;
    prism_predictor<P><<<(unsigned)nb, 256, 0, st>>>(G, dt, gamma, npic, Ua, aU, aF);
    if (hipGetLastError() != hipSuccess) { set_error("prism predictor launch failed"); return RG_EDEVICE; }
    return RG_OK;
}

rg_status launch_prism_predict(const DevPrism &G, double dt, double gamma, int npic, const double *Ua, double *aU,
                               double *aF, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (G.order) {
    case 2: return launch_order<2>(G, dt, gamma, npic, Ua, aU, aF, st);
    case 3: return launch_order<3>(G, dt, gamma, npic, Ua, aU, aF, st);
    case 4: return launch_order<4>(G, dt, gamma, npic, Ua, aU, aF, st);
    default: set_error("prism order must be 2, 3 or 4"); return RG_ENOTSUP;
    }
}

}  // namespace rg

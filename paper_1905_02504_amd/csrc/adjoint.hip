// Adjoint of one step (the vector-Jacobian product of rg_step at a given
// state, dt held fixed), of the FP64 step or of the FP32 form (whose
// predictor is recomputed and reversed in FP32; the rest of the reversal and
// every gradient buffer stay FP64).  The step's stages are reversed one by one:
//
//   face_ct, zone_update  : linear; transposed as gathers over the faces of an
//                           edge and the zones of a face
//   edge_emf, face_flux   : reverse-mode derivatives of the pointwise Riemann
//                           solvers, written out by hand (mhd_adjoint.hpp)
//   predictor             : recomputed per zone in the step's own wavefront
//                           layout, then the traces, time averages and the
//                           unrolled Picard sweeps reversed (flux Jacobians
//                           transposed by hand, derivative matrices
//                           transposed through the same LDS slab)
//   bmap                  : linear, the transposed per-column map
//   face_bnodal           : MinMod and mean restore reversed per face
//   weno                  : reverse-mode derivative of the WENO-AO
//                           combination, nonlinear weights included
//   boundary fill         : ghost copies accumulated into their sources
//
// Every gradient contribution to a zone or face is gathered by the one thread
// that owns the target, in a fixed order: no floating-point atomics, so the
// result is deterministic.  The forward quantities the reversal needs are
// recomputed by running the step first.
#include "mhd_adjoint.hpp"

namespace rg {

namespace {

inline unsigned nblk(i64 n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- constrained transport
// Transpose of the face circulation (eqs. 2.5-2.6) over the faces of shells
// k0..k1: gGam[e] = sum over the faces f holding edge e of
// scale / A_f * s_fe * gBf[f], with s_fe the sign with which edge e enters
// f's circulation.  Edges: radial in shells [k0, k1], angular at interfaces
// [k0, k1 + 1].
__global__ __launch_bounds__(256) void circ_transpose(DevGeom G, double scale, int k0, int k1,
                                                      const double *__restrict__ gBf, double *__restrict__ gGam)
{
    const int nrad = k1 - k0 + 1, nang = k1 - k0 + 2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.nv * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    double acc = 0.0;
    i64 e;
    if (t < nR) {
        // radial edge of vertex v in shell k: the angular faces (ae, k) of the
        // angular edges at v, through +Gam[edge at a's second vertex] - Gam[at its first]
        const int v = (int)(t / nrad), k = k0 + (int)(t % nrad);
        e = (i64)v * G.K + k;
        for (int s = 0; s < G.v_ncol[v]; s++) {
            const int ae = G.v_ae[4 * v + s];
            const double sg = (G.ae_v[2 * ae + 1] == v) ? 1.0 : -1.0;
            const i64 f = G.NRF + (i64)ae * G.K + k;
            acc += scale / G.area[f] * G.ae_rs[ae] * sg * gBf[f];
        }
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), kf = k0 + (int)(u % nang);
        e = G.NRE + (i64)ae * (G.K + 1) + kf;
        // radial faces kf of the two columns sharing the angular edge
        for (int s = 0; s < 2; s++) {
            const int c = G.ae_col[2 * ae + s], lf = G.ae_lf[2 * ae + s];
            const i64 f = (i64)c * (G.K + 1) + kf;
            acc += scale / G.area[f] * G.col_sgn[4 * c + lf] * gBf[f];
        }
        // angular faces of the shells above (as lower ring) and below (as upper ring)
        if (kf <= k1) {
            const i64 f = G.NRF + (i64)ae * G.K + kf;
            acc += scale / G.area[f] * G.ae_rs[ae] * gBf[f];
        }
        if (kf - 1 >= k0) {
            const i64 f = G.NRF + (i64)ae * G.K + kf - 1;
            acc -= scale / G.area[f] * G.ae_rs[ae] * gBf[f];
        }
    }
    gGam[e] = acc;
}

// ---------------------------------------------------------------- finite-volume update
// gPhi[v][f] = sum over the interior zones z of face f of -(dt/V_z) s_zf gU[v][z]
__global__ void adj_update_faces(DevGeom G, double dt, const double *__restrict__ gU, double *__restrict__ gPhi)
{
    const int nrad = G.Nr + 1, nang = G.Nr;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.ncol * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    i64 f, z[2] = {-1, -1};
    double sg[2] = {0.0, 0.0};
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        if (kf - 1 >= G.g) { z[0] = (i64)c * G.K + kf - 1; sg[0] = 1.0; }
        if (kf <= G.g + G.Nr - 1) { z[1] = (i64)c * G.K + kf; sg[1] = -1.0; }
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), k = G.g + (int)(u % nang);
        f = G.NRF + (i64)ae * G.K + k;
        z[0] = (i64)G.ae_col[2 * ae] * G.K + k;
        z[1] = (i64)G.ae_col[2 * ae + 1] * G.K + k;
        sg[0] = 1.0;
        sg[1] = -1.0;
    }
    for (int v = 0; v < 8; v++) {
        double acc = 0.0;
        for (int s = 0; s < 2; s++)
            if (z[s] >= 0) acc += -(dt / G.vol[z[s]]) * sg[s] * gU[(i64)v * G.Z + z[s]];
        gPhi[(i64)v * G.NF + f] = acc;
    }
}

// identity paths of the update: interior fluid variables keep the old value,
// interior B takes the divergence-free zone mean, ghost zones are the
// boundary-filled input
__global__ void adj_update_zones(DevGeom G, const double *__restrict__ gU, double *__restrict__ gUo,
                                 double *__restrict__ gzoneB)
{
    const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= G.Z) return;
    const int k = (int)(z % G.K);
    const bool interior = k >= G.g && k < G.g + G.Nr;
    for (int v = 0; v < 8; v++) {
        const double g = gU[(i64)v * G.Z + z];
        if (interior && v >= 5) {
            gzoneB[(i64)(v - 5) * G.Z + z] = g;
            gUo[(i64)v * G.Z + z] = 0.0;
        } else {
            gUo[(i64)v * G.Z + z] = g;
        }
    }
}

// ---------------------------------------------------------------- Riemann solvers
// one lane per face quadrature point (the step's face_flux layout); the traces
// are stored in the step form's precision R, the solver runs in FP64 as in
// the step
template <int P, class R>
__global__ __launch_bounds__(256) void adj_face_flux(DevGeom G, double gam, const R *__restrict__ ftr,
                                                     const double *__restrict__ gPhi, double *__restrict__ gftr)
{
    using T = Tr<P>;
    const i64 nff = (i64)G.ncol * (G.Nr + 1) + (i64)G.nae * G.Nr;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nff * T::Q) return;
    const int q = (int)(t % T::Q);
    const double *nrm, *fw;
    const i64 f = flux_face<P>(G, t / T::Q, nrm, fw);
    const double w = fw[q] * G.area[f];
    const R *a = ftr + ftr_at<P>(f, q, 0), *b = a + 16;
    double UL[8], UR[8], FL[8], FR[8], gFs[8], gUL[8], gUR[8], gFL[8], gFR[8];
    for (int v = 0; v < 8; v++) {
        UL[v] = a[v];
        FL[v] = a[8 + v];
        UR[v] = b[v];
        FR[v] = b[8 + v];
        gFs[v] = w * gPhi[(i64)v * G.NF + f];
        gUL[v] = gUR[v] = gFL[v] = gFR[v] = 0.0;
    }
    hll_vjp(UL, UR, FL, FR, nrm + q * 3, gam, gFs, gUL, gUR, gFL, gFR);
    double *ga = gftr + ftr_at<P>(f, q, 0), *gb = ga + 16;
    for (int v = 0; v < 8; v++) {
        ga[v] = gUL[v];
        ga[8 + v] = gFL[v];
        gb[v] = gUR[v];
        gb[8 + v] = gFR[v];
    }
}

// one lane per (edge, Simpson point) (the step's edge_emf layout)
template <class R>
__global__ __launch_bounds__(256) void adj_edge_emf(DevGeom G, double gam, const R *__restrict__ etr,
                                                    const double *__restrict__ gGam, double *__restrict__ getr)
{
    const i64 nee = (i64)G.nv * G.Nr + (i64)G.nae * (G.Nr + 1);
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nee * 3) return;
    const int p = (int)(t % 3);
    const double *frame, *N3;
    double wl;
    int nzs;
    const i64 e = emf_edge(G, t / 3, p, frame, wl, nzs, N3);
    const double *tt = frame + 6;
    const double g = wl * gGam[e];
    const R *rec = etr + etr_at(e, p, 0);
    double U[4][8], E[4][3], Et[4], gU[4][8], gE[4][3], gEt[4];
#pragma unroll
    for (int s = 0; s < 4; s++) {
#pragma unroll
        for (int v = 0; v < 8; v++) { U[s][v] = rec[s * 9 + v]; gU[s][v] = 0.0; }
        Et[s] = rec[s * 9 + 8];
#pragma unroll
        for (int v = 0; v < 3; v++) { E[s][v] = Et[s] * tt[v]; gE[s][v] = 0.0; }
        gEt[s] = 0.0;
    }
    if (nzs == 4) {
        emf4_vjp(U, Et, frame, gam, g, gU, gEt);
    } else {
        // the solver took E = Et t
        emf3_vjp(U, E, N3, tt, gam, g, gU, gE);
#pragma unroll
        for (int s = 0; s < 4; s++) gEt[s] = gE[s][0] * tt[0] + gE[s][1] * tt[1] + gE[s][2] * tt[2];
    }
    double *o = getr + etr_at(e, p, 0);
#pragma unroll
    for (int s = 0; s < 4; s++) {
        if (s >= nzs) continue;
#pragma unroll
        for (int v = 0; v < 8; v++) o[s * 9 + v] = gU[s][v];
        o[s * 9 + 8] = gEt[s];
    }
}

// ---------------------------------------------------------------- predictor
// The predictor's wavefront layout: 64 / N zones per wavefront, one lane per
// serendipity node, the derivative matrices applied through the LDS slab.
// A lane keeps its node's initial state, tau = 0 derivative and the states of
// one Picard sweep in registers; the states of earlier sweeps are recomputed
// from the first sweep when the reversal reaches them.
template <int P>
struct PredLayout {
    static constexpr int N = Tr<P>::N, SN = N + 1, ZS = 32 * SN + 4, ZPW = 64 / N, E = Tr<P>::M - 1;
};

// one Picard sweep: Ut <- Ua - R0 dFa - sum_s R_s D F(Ut_s)   (all lanes call it)
template <int P, class R>
__device__ __forceinline__ void picard_sweep(const DevGeom &G, R *s_f, R *sf, int lane, int i, int i1, int i2,
                                             bool active, const R (&Ua)[8], const R (&dFa)[8], R iJ,
                                             const R (&met)[9], R gam, R (&Ut)[Tr<P>::M - 1][8])
{
    using L = PredLayout<P>;
    constexpr int E = L::E, M = Tr<P>::M;
    R A[E][8];
#pragma unroll
    for (int s = 0; s < E; s++) {
        if (active) {
            R F[3][8];
            mapped_flux<R>(Ut[s], iJ, met, gam, F);
            put_flux<L::SN, R>(sf, i, i1, i2, F);
        }
        __syncthreads();
        deriv_rows<P, L::SN, L::ZS, L::ZPW, R>(s_f, lane);
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 8; v++) A[s][v] = R(0);
        if (active) get_deriv<L::SN, R>(sf, i, i1, i2, A[s]);
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < E; t++)
#pragma unroll
        for (int v = 0; v < 8; v++) {
            R u = Ua[v] - R(G.R[t * M]) * dFa[v];
#pragma unroll
            for (int s = 0; s < E; s++) u -= R(G.R[t * M + s + 1]) * A[s][v];
            Ut[t][v] = u;
        }
}

// gF[d][v] = sum_i D_d[i][node] g[i][v] for the lane's node (all lanes call it)
template <int P, class R>
__device__ __forceinline__ void deriv_transpose(R *s_f, R *sf, int lane, int i, int i1, int i2, bool active,
                                                const R (&g)[8], R (&gF)[3][8])
{
    using L = PredLayout<P>;
    if (active) {
        const R G3[3][8] = {{g[0], g[1], g[2], g[3], g[4], g[5], g[6], g[7]},
                                 {g[0], g[1], g[2], g[3], g[4], g[5], g[6], g[7]},
                                 {g[0], g[1], g[2], g[3], g[4], g[5], g[6], g[7]}};
        put_flux<L::SN, R>(sf, i, i1, i2, G3);
    }
    __syncthreads();
    deriv_rows<P, L::SN, L::ZS, L::ZPW, R, true>(s_f, lane);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 8; v++) {
        gF[0][v] = active ? sf[v * L::SN + i] : R(0);
        gF[1][v] = active ? sf[(8 + v) * L::SN + i1] : R(0);
        gF[2][v] = active ? sf[(16 + v) * L::SN + i2] : R(0);
    }
    __syncthreads();
}

// R: the precision of the step form (its stored coefficients and nodal B, and
// the arithmetic of the recomputed predictor and of its reversal); the
// incoming and outgoing gradients are FP64.
template <int P, class R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void adj_predictor(
    DevGeom G, double dt, double gamma, int npic, const double *__restrict__ U, const R *__restrict__ wc,
    const R *__restrict__ bnode, const double *__restrict__ gftr, const double *__restrict__ getr,
    double *__restrict__ gUo, double *__restrict__ gwc, double *__restrict__ gbnode)
{
    using T = Tr<P>;
    using L = PredLayout<P>;
    constexpr int N = T::N, M = T::M, ZS = L::ZS, ZPW = L::ZPW, E = L::E, NCF = T::NC + 1;
    __shared__ R s_c[ZPW][5 * NCF];
    __shared__ R s_f[ZPW * ZS];
    const R gam = R(gamma);
    const int lane = threadIdx.x, zl = lane / N, i = lane % N;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned zt = lb * ZPW + zl;
    const bool active = (zl < ZPW) && (zt < (unsigned)nzr);
    int c = 0, k = 0;
    i64 z = 0;
    if (active) {
        c = (int)(zt / (unsigned)KR);
        k = G.g - 1 + (int)(zt % (unsigned)KR);
        z = (i64)c * G.K + k;
        for (int j = i; j < 5 * NCF; j += N) {
            const int v = j / NCF, a = j % NCF;
            s_c[zl][j] = a == 0 ? R(U[v * G.Z + z]) : wc[((i64)v * T::NC + a - 1) * G.Z + z];
        }
    }
    const int i1 = DTab<P>::SWAP1[i], i2 = DTab<P>::SWAP2[i];
    __syncthreads();
    R Ua[8], dFa[8], met[9], iJ = R(1), J = R(1);
    R *sf = s_f + (zl < ZPW ? zl : 0) * ZS;
    for (int v = 0; v < 8; v++) Ua[v] = dFa[v] = R(0);
    for (int m = 0; m < 9; m++) met[m] = R(0);
    if (active) {
        const R *Ev = pick<R>(G.Ev, G.EvF) + (i64)c * T::NC * N + i;
        for (int v = 0; v < 5; v++) {
            R acc = s_c[zl][v * NCF];
#pragma unroll
            for (int a = 0; a < T::NC; a++) acc += Ev[a * N] * s_c[zl][v * NCF + 1 + a];
            Ua[v] = acc;
        }
        const R *bn = bnode + (i64)zt * (3 * N) + i;
        Ua[5] = bn[0];
        Ua[6] = bn[N];
        Ua[7] = bn[2 * N];
        J = pick<R>(G.nJ, G.nJF)[(i64)c * N + i];
        iJ = R(1) / J;
        const R fac = R(dt / G.zscale[k]);
        const R *nM = pick<R>(G.nM, G.nMF);
#pragma unroll
        for (int m = 0; m < 9; m++) met[m] = fac * nM[((i64)c * 9 + m) * N + i];
#pragma unroll
        for (int v = 0; v < 8; v++) Ua[v] *= J;
        R F[3][8];
        mapped_flux<R>(Ua, iJ, met, gam, F);
        put_flux<L::SN, R>(sf, i, i1, i2, F);
    }
    __syncthreads();
    deriv_rows<P, L::SN, ZS, ZPW, R>(s_f, lane);
    __syncthreads();
    if (active) get_deriv<L::SN, R>(sf, i, i1, i2, dFa);
    __syncthreads();
    // the first sweep from the constant guess: Ut_t = Ua - (R0_t + sum_s R_ts) dFa
    R cR[E];
#pragma unroll
    for (int t = 0; t < E; t++) {
        R acc = R(G.R[t * M]);
#pragma unroll
        for (int s = 0; s < E; s++) acc += R(G.R[t * M + s + 1]);
        cR[t] = npic > 0 ? acc : R(0);
    }
    R Ut[E][8];
#pragma unroll
    for (int t = 0; t < E; t++)
#pragma unroll
        for (int v = 0; v < 8; v++) Ut[t][v] = Ua[v] - cR[t] * dFa[v];
    for (int it = 2; it <= npic; it++) picard_sweep<P, R>(G, s_f, sf, lane, i, i1, i2, active, Ua, dFa, iJ, met, gam, Ut);

    // ---- traces reversed: gradients of the node's time-averaged state and flux
    R gaU[8], gaF[3][8];
#pragma unroll
    for (int v = 0; v < 8; v++) gaU[v] = gaF[0][v] = gaF[1][v] = gaF[2][v] = R(0);
    if (active) {
#pragma unroll 1
        for (int lf = 0; lf < 6; lf++) {
            int kk = -1;
            for (int j = 0; j < T::NFN; j++)
                if (G.fnode[lf * T::NFN + j] == i) kk = j;
            if (kk < 0) continue;
            // faces outside the flux stage's range carry no gradient
            if (lf >= 4 ? (k + lf - 4 < G.g || k + lf - 4 > G.g + G.Nr) : (k < G.g || k > G.g + G.Nr - 1)) continue;
            i64 fid;
            int side;
            const double *nrm;
            const int *perm = nullptr;
            if (lf >= 4) {
                fid = (i64)c * (G.K + 1) + k + (lf - 4);
                side = lf == 4 ? 1 : 0;
                nrm = G.fnR + (i64)c * T::Q * 3;
            } else {
                const int ae = G.col_ae[4 * c + lf];
                fid = G.NRF + (i64)ae * G.K + k;
                side = G.col_side[4 * c + lf];
                nrm = G.fnA + (i64)ae * T::Q * 3;
                perm = G.col_perm + ((i64)c * 4 + lf) * T::Q;
            }
            const double *go = gftr + ftr_at<P>(fid, 0, side);   // point q at go + 32 q
#pragma unroll 1
            for (int q = 0; q < T::Q; q++) {
                const int qc = perm ? perm[q] : q;
                const R w = pick<R>(G.fintc, G.fintcF)[kk * T::Q + q];
                const double *n = nrm + qc * 3;
                const double *gq = go + qc * 32;
#pragma unroll
                for (int v = 0; v < 8; v++) {
                    gaU[v] += w * R(gq[v]);
                    const R gn = w * R(gq[8 + v]);
                    gaF[0][v] += gn * R(n[0]);
                    gaF[1][v] += gn * R(n[1]);
                    gaF[2][v] += gn * R(n[2]);
                }
            }
        }
#pragma unroll 1
        for (int le = 0; le < 12; le++) {
            int kk = -1;
            for (int j = 0; j < T::NEN; j++)
                if (G.enode[le * T::NEN + j] == i) kk = j;
            if (kk < 0) continue;
            // edges outside the EMF stage's range carry no gradient
            if (le < 8 ? (k + LocalEdges::UP[le] < G.g || k + LocalEdges::UP[le] > G.g + G.Nr)
                       : (k < G.g || k > G.g + G.Nr - 1))
                continue;
            const int rev = G.col_rev[(i64)c * 12 + le], slot = G.col_slot[(i64)c * 12 + le];
            i64 e;
            if (le < 8) {
                const int ae = G.col_ae[4 * c + LocalEdges::FACE[le]];
                e = G.NRE + (i64)ae * (G.K + 1) + k + LocalEdges::UP[le];
            } else {
                e = (i64)G.col_v[4 * c + LocalEdges::CORNER[le - 8]] * G.K + k;
            }
            const double *go = getr + etr_at(e, 0, slot);   // point p at go + 36 p
            for (int p = 0; p < 3; p++) {
                const int pc = rev ? 2 - p : p;
                const R w = pick<R>(G.eintc, G.eintcF)[kk * 3 + p];
                const double *t = edge_tangent(G, c, le, pc);
#pragma unroll
                for (int v = 0; v < 8; v++) gaU[v] += w * R(go[pc * 36 + v]);
                const R gt = w * R(go[pc * 36 + 8]);   // the record held E . t
                gaF[2][6] += gt * R(t[0]);   // E_x = H[B_y]
                gaF[0][7] += gt * R(t[1]);   // E_y = F[B_z]
                gaF[1][5] += gt * R(t[2]);   // E_z = G[B_x]
            }
        }
    }
    // ---- time averages reversed: gX_t = wt_t / J (gaU + (dF/dw)^T gaF) at w = Ut_t / J
    R gX[E][8];
#pragma unroll
    for (int t = 0; t < E; t++) {
        R w[8], gw[8];
        const R wt = R(G.wt[t + 1]);
#pragma unroll
        for (int v = 0; v < 8; v++) { w[v] = active ? Ut[t][v] * iJ : (v == 0 ? R(1) : R(0)); gw[v] = gaU[v]; }
        if (active) flux_vjp<R>(w, gam, gaF, gw);
#pragma unroll
        for (int v = 0; v < 8; v++) gX[t][v] = wt * iJ * gw[v];
    }
    // ---- Picard sweeps reversed, last first
    R gUa[8], gdFa[8];
#pragma unroll
    for (int v = 0; v < 8; v++) gUa[v] = gdFa[v] = R(0);
    for (int it = npic; it >= 2; it--) {
        // the states this sweep started from
#pragma unroll
        for (int t = 0; t < E; t++)
#pragma unroll
            for (int v = 0; v < 8; v++) Ut[t][v] = Ua[v] - cR[t] * dFa[v];
        for (int r = 2; r < it; r++) picard_sweep<P, R>(G, s_f, sf, lane, i, i1, i2, active, Ua, dFa, iJ, met, gam, Ut);
#pragma unroll
        for (int t = 0; t < E; t++)
#pragma unroll
            for (int v = 0; v < 8; v++) {
                gUa[v] += gX[t][v];
                gdFa[v] -= R(G.R[t * M]) * gX[t][v];
            }
        // A_s = D F(Ut_s): the gradient of each level's start state; it
        // replaces that state in Ut (no longer needed) and becomes gX
#pragma unroll
        for (int s = 0; s < E; s++) {
            R gA[8], gF[3][8], gu[8];
#pragma unroll
            for (int v = 0; v < 8; v++) {
                R acc = R(0);
#pragma unroll
                for (int t = 0; t < E; t++) acc -= R(G.R[t * M + s + 1]) * gX[t][v];
                gA[v] = acc;
                gu[v] = R(0);
            }
            deriv_transpose<P, R>(s_f, sf, lane, i, i1, i2, active, gA, gF);
            if (active) mapped_flux_vjp<R>(Ut[s], iJ, met, gam, gF, gu);
#pragma unroll
            for (int v = 0; v < 8; v++) Ut[s][v] = gu[v];
        }
#pragma unroll
        for (int t = 0; t < E; t++)
#pragma unroll
            for (int v = 0; v < 8; v++) gX[t][v] = Ut[t][v];
    }
    // first sweep (or none): Ut_t = Ua - cR_t dFa
#pragma unroll
    for (int t = 0; t < E; t++)
#pragma unroll
        for (int v = 0; v < 8; v++) {
            gUa[v] += gX[t][v];
            gdFa[v] -= cR[t] * gX[t][v];
        }
    // ---- tau = 0 derivative reversed: dFa = D F(Ua)
    {
        R gF[3][8];
        deriv_transpose<P, R>(s_f, sf, lane, i, i1, i2, active, gdFa, gF);
        if (active) mapped_flux_vjp<R>(Ua, iJ, met, gam, gF, gUa);
    }
    // ---- nodal initial state reversed: Ua = J (fluid polynomial | divergence-free B)
    R *s_red = s_f;   // [ZPW][5][N], free once the slab is idle
    if (active) {
#pragma unroll
        for (int v = 0; v < 8; v++) gUa[v] *= J;
        for (int v = 5; v < 8; v++) gbnode[(i64)zt * (3 * N) + (v - 5) * N + i] = double(gUa[v]);
        for (int v = 0; v < 5; v++) s_red[(zl * 5 + v) * N + i] = gUa[v];
    }
    __syncthreads();
    for (int j = lane; j < ZPW * 5 * NCF; j += 64) {
        const int zq = j / (5 * NCF), v = (j % (5 * NCF)) / NCF, a = j % NCF;
        const unsigned ztq = lb * ZPW + zq;
        if (ztq >= (unsigned)nzr) continue;
        const int cq = (int)(ztq / (unsigned)KR), kq = G.g - 1 + (int)(ztq % (unsigned)KR);
        const i64 zq64 = (i64)cq * G.K + kq;
        const R *r = s_red + (zq * 5 + v) * N;
        double acc = 0.0;
        if (a == 0) {
            for (int n = 0; n < N; n++) acc += double(r[n]);
            gUo[(i64)v * G.Z + zq64] += acc;
        } else {
            const double *Ev = G.Ev + ((i64)cq * T::NC + a - 1) * N;
            for (int n = 0; n < N; n++) acc += Ev[n] * double(r[n]);
            gwc[((i64)v * T::NC + a - 1) * G.Z + zq64] = acc;
        }
    }
}

// ---------------------------------------------------------------- divergence-free B map
// MbA[c][r][j] = Mb[c][j][r]: the column's map with outputs outermost, so that
// the transposed product reads it like the step reads Mb
__global__ void transpose_map(const double *__restrict__ Mb, double *__restrict__ MbA, i64 ncol, int nin, int nout)
{
    const i64 n = ncol * nin * nout;
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        const i64 c = t / ((i64)nin * nout);
        const int rem = (int)(t % ((i64)nin * nout)), j = rem / nout, r = rem % nout;
        MbA[(c * nout + r) * nin + j] = Mb[t];
    }
}

// gIn = Mb gOut per zone, on the FP64 matrix cores as in the step's map: one
// wavefront owns 16 zones of a column and all input rows, stepping through
// the outputs four at a time (v_mfma_f64_16x16x4: A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i % 4), element i / 4).
// Writes the zone's share of the gradient of its inputs: B means and WENO B
// coefficients (zone owned), and per local face the limited nodal values and
// the face mean, gside[(lf Q + q) or (6 Q + lf)][zr], gathered per face
// afterwards.
template <int P>
__global__ __launch_bounds__(64) void adj_bmap(DevGeom G, const double *__restrict__ MbA,
                                               const double *__restrict__ gbnode, const double *__restrict__ gzoneB,
                                               double *__restrict__ gUo, double *__restrict__ gwc,
                                               double *__restrict__ gside)
{
    using T = Tr<P>;
    constexpr int NIN = T::NIN, NOUT = T::NOUTB, KT = (NOUT + 3) / 4, MT = (NIN + 15) / 16;
    constexpr int NA = 3 * (T::NC + 1), N3 = 3 * T::N;
    const int KR = G.Nr + 2, nt = (KR + 15) / 16;
    const i64 nzr = (i64)G.ncol * KR;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int c = lb / nt, tile = lb % nt;
    const int l = threadIdx.x, g = l >> 4, jz = l & 15;
    const int kk = tile * 16 + jz;
    const bool active = kk < KR;
    const int k = G.g - 1 + (active ? kk : 0);
    const i64 z = (i64)c * G.K + k;
    const i64 zr = (i64)c * KR + (active ? kk : 0);
    const bool interior = k >= G.g && k < G.g + G.Nr;
    const double *M = MbA + (i64)c * NOUT * NIN;
    dbl4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; m++) acc[m] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int s = 0; s < KT; s++) {
        // B operand: output gradient r = 4s + g of zone jz
        const int r = 4 * s + g;
        double b = 0.0;
        if (active && r < NOUT)
            b = r < N3 ? gbnode[zr * N3 + r] : (interior ? gzoneB[(i64)(r - N3) * G.Z + z] : 0.0);
        const double *mrow = M + (i64)(r < NOUT ? r : 0) * NIN;
#pragma unroll
        for (int m = 0; m < MT; m++) {
            const int j = m * 16 + jz;
            const double a = (r < NOUT && (m < MT - 1 || j < NIN)) ? mrow[j] : 0.0;
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
        }
    }
    if (!active) return;
#pragma unroll
    for (int m = 0; m < MT; m++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int j = m * 16 + g + 4 * v;
            if (j >= NIN) continue;
            const double x = acc[m][v];
            if (j < NA) {
                const int comp = j / (T::NC + 1), a = j % (T::NC + 1);
                if (a == 0) gUo[(i64)(5 + comp) * G.Z + z] += x;
                else gwc[((i64)(5 + comp) * T::NC + a - 1) * G.Z + z] = x;
            } else {
                gside[(i64)(j - NA) * nzr + zr] = x;
            }
        }
}

// per face of the face-nodal set: sum the two zones' shares from adj_bmap
template <int P>
__global__ void adj_face_gather_bmap(DevGeom G, const double *__restrict__ gside, double *__restrict__ gbnod,
                                     double *__restrict__ gBo)
{
    using T = Tr<P>;
    const int nrad = G.Nr + 3, nang = G.Nr + 2, KR = G.Nr + 2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.ncol * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    i64 f, zr[2] = {-1, -1};
    int lf[2] = {0, 0};
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g - 1 + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        if (kf - 1 >= G.g - 1 && kf - 1 <= G.g + G.Nr) { zr[0] = (i64)c * KR + (kf - 1 - (G.g - 1)); lf[0] = 5; }
        if (kf >= G.g - 1 && kf <= G.g + G.Nr) { zr[1] = (i64)c * KR + (kf - (G.g - 1)); lf[1] = 4; }
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), k = G.g - 1 + (int)(u % nang);
        f = G.NRF + (i64)ae * G.K + k;
        for (int s = 0; s < 2; s++) {
            zr[s] = (i64)G.ae_col[2 * ae + s] * KR + (k - (G.g - 1));
            lf[s] = G.ae_lf[2 * ae + s];
        }
    }
    const i64 nzr = (i64)G.ncol * KR;
    for (int q = 0; q < T::Q; q++) {
        double acc = 0.0;
        for (int s = 0; s < 2; s++)
            if (zr[s] >= 0) acc += gside[(i64)(lf[s] * T::Q + q) * nzr + zr[s]];
        gbnod[(i64)q * G.NF + f] = acc;
    }
    double acc = 0.0;
    for (int s = 0; s < 2; s++)
        if (zr[s] >= 0) acc += gside[(i64)(6 * T::Q + lf[s]) * nzr + zr[s]];
    gBo[f] += acc;
}

// ---------------------------------------------------------------- face nodal B
// Reverse of MinMod + mean restore on one face; the two sides' shares (B mean
// and WENO B coefficients of each side's zone) go to gsb[side][3 + 3 NC][f].
// Each side's B at the points is recomputed as the step computes it, in the
// step form's precision R, so that MinMod takes the step's branch.
template <int P, class R>
__global__ void adj_face_bnodal(DevGeom G, const double *__restrict__ Uo, const double *__restrict__ Bo,
                                const R *__restrict__ wc, const double *__restrict__ gbnod,
                                double *__restrict__ gBo, double *__restrict__ gsb)
{
    using T = Tr<P>;
    constexpr int NSB = 3 + 3 * T::NC;
    const int nrad = G.Nr + 3, nang = G.Nr + 2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.ncol * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    i64 f, z[2];
    bool have[2];
    const double *fev[2], *nrm, *fw;
    const R *fevr[2];
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g - 1 + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        z[0] = (i64)c * G.K + kf - 1;
        z[1] = (i64)c * G.K + kf;
        have[0] = (kf - 1 >= G.g - 1) && (kf - 1 <= G.g + G.Nr);
        have[1] = (kf >= G.g - 1) && (kf <= G.g + G.Nr);
        fev[0] = G.fevR + ((i64)c * 2 + 0) * T::Q * T::NC;
        fev[1] = G.fevR + ((i64)c * 2 + 1) * T::Q * T::NC;
        fevr[0] = pick<R>(G.fevR, G.fevRF) + ((i64)c * 2 + 0) * T::Q * T::NC;
        fevr[1] = pick<R>(G.fevR, G.fevRF) + ((i64)c * 2 + 1) * T::Q * T::NC;
        nrm = G.fnR + (i64)c * T::Q * 3;
        fw = G.fwR + (i64)c * T::Q;
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), k = G.g - 1 + (int)(u % nang);
        f = G.NRF + (i64)ae * G.K + k;
        z[0] = (i64)G.ae_col[2 * ae] * G.K + k;
        z[1] = (i64)G.ae_col[2 * ae + 1] * G.K + k;
        have[0] = have[1] = true;
        fev[0] = G.fevA + ((i64)ae * 2 + 0) * T::Q * T::NC;
        fev[1] = G.fevA + ((i64)ae * 2 + 1) * T::Q * T::NC;
        fevr[0] = pick<R>(G.fevA, G.fevAF) + ((i64)ae * 2 + 0) * T::Q * T::NC;
        fevr[1] = pick<R>(G.fevA, G.fevAF) + ((i64)ae * 2 + 1) * T::Q * T::NC;
        nrm = G.fnA + (i64)ae * T::Q * 3;
        fw = G.fwA + (i64)ae * T::Q;
    }
    // forward: each side's B at the points, deviations, MinMod
    const double mean = Bo[f];
    double d[2][T::Q];
    for (int s = 0; s < 2; s++) {
        if (!have[s]) continue;
        // the step's sum order: component mean, then the coefficients in turn
        R Bq[3][T::Q];
        for (int c3 = 0; c3 < 3; c3++) {
            const R m0 = R(Uo[(5 + c3) * G.Z + z[s]]);
            for (int q = 0; q < T::Q; q++) Bq[c3][q] = m0;
            for (int a = 0; a < T::NC; a++) {
                const R ca = wc[((i64)(5 + c3) * T::NC + a) * G.Z + z[s]];
                for (int q = 0; q < T::Q; q++) Bq[c3][q] += ca * fevr[s][q * T::NC + a];
            }
        }
        // the normal component adds the components' products in order, as the step does
        for (int q = 0; q < T::Q; q++) {
            double bn = double(Bq[0][q]) * nrm[q * 3];
            bn += double(Bq[1][q]) * nrm[q * 3 + 1];
            bn += double(Bq[2][q]) * nrm[q * 3 + 2];
            d[s][q] = bn - mean;
        }
    }
    for (int q = 0; q < T::Q; q++) {
        if (!have[0]) d[0][q] = d[1][q];
        if (!have[1]) d[1][q] = d[0][q];
    }
    // reverse: bnod[q] = bn[q] + mean - sum_q' fw[q'] bn[q'],  bn = mean + minmod(d0, d1)
    double gsum = 0.0, gmean = 0.0;
    for (int q = 0; q < T::Q; q++) {
        gsum += gbnod[(i64)q * G.NF + f];
    }
    gmean += gsum;
    double gd[2][T::Q];
    for (int q = 0; q < T::Q; q++) {
        const double gbn = gbnod[(i64)q * G.NF + f] - fw[q] * gsum;
        gmean += gbn;
        gd[0][q] = gd[1][q] = 0.0;
        const double a = d[0][q], b = d[1][q];
        if (a * b > 0.0) {
            const bool first = a > 0.0 ? (a <= b) : (a >= b);
            gd[first ? 0 : 1][q] = gbn;
        }
        // a missing side copied the other side's deviation
        if (!have[0]) { gd[1][q] += gd[0][q]; gd[0][q] = 0.0; }
        if (!have[1]) { gd[0][q] += gd[1][q]; gd[1][q] = 0.0; }
    }
    for (int s = 0; s < 2; s++) {
        double *o = gsb + (i64)s * NSB * G.NF + f;
        if (!have[s]) {
            for (int j = 0; j < NSB; j++) o[(i64)j * G.NF] = 0.0;
            continue;
        }
        for (int q = 0; q < T::Q; q++) gmean -= gd[s][q];
        for (int c3 = 0; c3 < 3; c3++) {
            double gq[T::Q], gm0 = 0.0;
            for (int q = 0; q < T::Q; q++) {
                gq[q] = gd[s][q] * nrm[q * 3 + c3];
                gm0 += gq[q];
            }
            o[(i64)c3 * G.NF] = gm0;
            for (int a = 0; a < T::NC; a++) {
                double acc = 0.0;
                for (int q = 0; q < T::Q; q++) acc += gq[q] * fev[s][q * T::NC + a];
                o[(i64)(3 + c3 * T::NC + a) * G.NF] = acc;
            }
        }
    }
    gBo[f] += gmean;
}

// per reconstructed zone: add its faces' shares from adj_face_bnodal
template <int P>
__global__ void adj_zone_gather_bnodal(DevGeom G, const double *__restrict__ gsb, double *__restrict__ gUo,
                                       double *__restrict__ gwc)
{
    using T = Tr<P>;
    constexpr int NSB = 3 + 3 * T::NC;
    const int KR = G.Nr + 2;
    const i64 zr = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (zr >= (i64)G.ncol * KR) return;
    const int c = (int)(zr / KR), k = G.g - 1 + (int)(zr % KR);
    const i64 z = (i64)c * G.K + k;
    i64 f[6];
    int sd[6];
    for (int lf = 0; lf < 4; lf++) {
        f[lf] = G.NRF + (i64)G.col_ae[4 * c + lf] * G.K + k;
        sd[lf] = G.col_side[4 * c + lf];
    }
    f[4] = (i64)c * (G.K + 1) + k;       // lower radial face: this zone is its side 1
    sd[4] = 1;
    f[5] = f[4] + 1;                      // upper radial face: side 0
    sd[5] = 0;
    for (int c3 = 0; c3 < 3; c3++) {
        double acc = 0.0;
        for (int lf = 0; lf < 6; lf++) acc += gsb[((i64)sd[lf] * NSB + c3) * G.NF + f[lf]];
        gUo[(i64)(5 + c3) * G.Z + z] += acc;
        for (int a = 0; a < T::NC; a++) {
            double s = 0.0;
            for (int lf = 0; lf < 6; lf++) s += gsb[((i64)sd[lf] * NSB + 3 + c3 * T::NC + a) * G.NF + f[lf]];
            gwc[((i64)(5 + c3) * T::NC + a) * G.Z + z] += s;
        }
    }
}

// ---------------------------------------------------------------- WENO-AO
// gdu[v][j][zr] = d(coefficients)/d(du_j)^T gwc for variable v of
// reconstructed zone zr, exact through the nonlinear weights.  The step's
// layout: one wavefront per run of up to 64 shells of a column (the column's
// matrices uniform, read as scalars), a short tail as (shell, variable) lanes.
template <int P>
__device__ __forceinline__ void weno_var_vjp(const DevGeom &G, const double *__restrict__ U,
                                             const double *__restrict__ gwc, double *__restrict__ gdu,
                                             const double *__restrict__ Pl, const double *__restrict__ Ps,
                                             const double *__restrict__ Qs, double eps, int c, int k, int v)
{
    using T = Tr<P>;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR, zr = (i64)c * KR + (k - (G.g - 1));
    const i64 z = (i64)c * G.K + k;
    const double *Uv = U + (i64)v * G.Z;
    const double u0 = Uv[z];
    double du[T::NS], go[T::NC];
#pragma unroll
    for (int j = 0; j < T::NS; j++) {
        const int m = G.stm[(i64)c * T::NS + j];
        const int dz = m < 0 ? 0 : (int)(((i64)(m >> 3) - c) * G.K + (m & 7) - 3);
        du[j] = Uv[z + dz] - u0;
    }
#pragma unroll
    for (int a = 0; a < T::NC; a++) go[a] = gwc[((i64)v * T::NC + a) * G.Z + z];
    double *o = gdu + (i64)v * T::NS * nzr + zr;
    const int *stm = G.stm + (i64)c * T::NS;
    weno_core_vjp<P>(du, Pl, Ps, Qs, eps, go, [&](int j, double g) { o[(i64)j * nzr] = stm[j] >= 0 ? g : 0.0; });
}

template <int P>
__global__ __launch_bounds__(64) void adj_weno(DevGeom G, const double *__restrict__ U, const double *__restrict__ gwc,
                                               double *__restrict__ gdu, double eps, int nchunk, int nu, int nleft)
{
    using T = Tr<P>;
    const int per = nchunk + (nleft > 0);
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int c = lb / per, ch = lb % per;
    const double *__restrict__ Pl = G.Pl + (i64)c * T::NC * T::NS;
    const double *__restrict__ Ps = G.Ps + (i64)c * 7 * 18;
    const double *__restrict__ Qs = G.Qs + (i64)c * T::NC * T::NC;
    if (ch < nchunk) {
        // the column's matrices staged in LDS once, read as broadcasts
        __shared__ double sPl[T::NC * T::NS], sPs[7 * 18], sQs[T::NC * T::NC];
        for (int j = threadIdx.x; j < T::NC * T::NS; j += 64) sPl[j] = Pl[j];
        for (int j = threadIdx.x; j < 7 * 18; j += 64) sPs[j] = Ps[j];
        for (int j = threadIdx.x; j < T::NC * T::NC; j += 64) sQs[j] = Qs[j];
        __syncthreads();
        const int kk = ch * 64 + threadIdx.x;
        if (kk >= nu) return;
#pragma unroll 1
        for (int v = 0; v < 8; v++) {
            int vo = 0;
            __asm__ __volatile__("" : "+s"(vo));
            weno_var_vjp<P>(G, U, gwc, gdu, sPl + vo, sPs + vo, sQs + vo, eps, c, G.g - 1 + kk, v);
        }
    } else {
        const int kk = nu + (int)threadIdx.x / 8, v = threadIdx.x % 8;
        if (kk >= nu + nleft) return;
        weno_var_vjp<P>(G, U, gwc, gdu, Pl, Ps, Qs, eps, c, G.g - 1 + kk, v);
    }
}

// per zone: gradient of the state from every stencil that holds it, minus
// the zone's own differences (du_j = u_member - u_zone)
template <int P>
__global__ void adj_weno_gather(DevGeom G, const double *__restrict__ gdu, double *__restrict__ gUo)
{
    using T = Tr<P>;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR;
    const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= G.Z) return;
    const int c = (int)(z / G.K), k = (int)(z % G.K);
    const bool recon = k >= G.g - 1 && k <= G.g + G.Nr;
    const i64 zr = (i64)c * KR + (k - (G.g - 1));
    // each entry read once for the eight variables; every variable still sums
    // its entries in order
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = G.inv_ptr[c]; e < G.inv_ptr[c + 1]; e++) {
        const int c2 = G.inv_ent[3 * e], j = G.inv_ent[3 * e + 1], dk = G.inv_ent[3 * e + 2];
        const int k2 = k - dk;
        if (k2 < G.g - 1 || k2 > G.g + G.Nr) continue;
        const double *src = gdu + (i64)j * nzr + (i64)c2 * KR + (k2 - (G.g - 1));
#pragma unroll
        for (int v = 0; v < 8; v++) acc[v] += src[(i64)v * T::NS * nzr];
    }
#pragma unroll
    for (int v = 0; v < 8; v++) {
        if (recon)
            for (int j = 0; j < T::NS; j++)
                if (G.stm[(i64)c * T::NS + j] >= 0) acc[v] -= gdu[((i64)v * T::NS + j) * nzr + zr];
        gUo[(i64)v * G.Z + z] += acc[v];
    }
}

// ---------------------------------------------------------------- boundary fill
// continuative (bc 0): ghost shells copied the nearest interior shell; fixed
// (bc 1): the input ghosts were used as they are
__global__ void adj_bc_zones(DevGeom G, int bc, const double *__restrict__ gUo, double *__restrict__ gU)
{
    const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= G.Z) return;
    const int k = (int)(z % G.K);
    const i64 base = z - k;
    for (int v = 0; v < 8; v++) {
        const double *g = gUo + (i64)v * G.Z;
        double acc;
        if (bc != 0) acc = g[z];
        else if (k < G.g || k > G.g + G.Nr - 1) acc = 0.0;
        else {
            acc = g[z];
            if (k == G.g)
                for (int k2 = 0; k2 < G.g; k2++) acc += g[base + k2];
            if (k == G.g + G.Nr - 1)
                for (int k2 = G.g + G.Nr; k2 < G.K; k2++) acc += g[base + k2];
        }
        gU[(i64)v * G.Z + z] = acc;
    }
}

__global__ void adj_bc_faces(DevGeom G, int bc, const double *__restrict__ gBo, double *__restrict__ gBf)
{
    const i64 f = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= G.NF) return;
    double acc;
    if (bc != 0) {
        acc = gBo[f];
    } else if (f < G.NRF) {
        const int kf = (int)(f % (G.K + 1));
        const i64 base = f - kf;
        if (kf < G.g || kf > G.g + G.Nr) acc = 0.0;
        else {
            acc = gBo[f];
            if (kf == G.g)
                for (int k2 = 0; k2 < G.g; k2++) acc += gBo[base + k2];
            if (kf == G.g + G.Nr)
                for (int k2 = G.g + G.Nr + 1; k2 <= G.K; k2++) acc += gBo[base + k2];
        }
    } else {
        const int k = (int)((f - G.NRF) % G.K);
        const i64 base = f - k;
        if (k < G.g || k > G.g + G.Nr - 1) acc = 0.0;
        else {
            acc = gBo[f];
            if (k == G.g)
                for (int k2 = 0; k2 < G.g; k2++) acc += gBo[base + k2];
            if (k == G.g + G.Nr - 1)
                for (int k2 = G.g + G.Nr; k2 < G.K; k2++) acc += gBo[base + k2];
        }
    }
    gBf[f] = acc;
}

__global__ void copy_state(const double *__restrict__ src, double *__restrict__ dst, i64 n)
{
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) dst[t] = src[t];
}

#define RG_ADJ_CHECK()                                                                   \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) {                                                          \
            set_error(std::string("adjoint kernel launch failed: ") + hipGetErrorString(e_)); \
            return RG_EDEVICE;                                                           \
        }                                                                                \
    } while (0)

}  // namespace

// R: the precision of the step form being differentiated (double, or float
// for RG_MODE_FP32, whose reconstruction coefficients, face nodal B, nodal B
// and traces are stored in FP32 and whose predictor computes in FP32)
template <int P, class R>
static rg_status adjoint_order(rg_geom *g, const rg_step_params &prm, const double *U, const double *Bf,
                               const double *gU1, const double *gBf1, double *gU, double *gBf, hipStream_t st)
{
    const DevGeom &G = g->d;
    using T = Tr<P>;
    AdjBuffers &A = g->adj;
    const int npic = prm.n_picard > 0 ? prm.n_picard : P;
    const double dt = prm.dt, gam = prm.gamma;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR;
    // the step's stages up to the predictor, at this state: the boundary-filled
    // working state, WENO coefficients, face nodal B, nodal B and traces
    rg_status s = launch_step_front(g, prm, U, Bf, A.Ubc, A.Bbc, st);
    if (s != RG_OK) return s;
    if (!A.map_ready) {
        transpose_map<<<2048, 256, 0, st>>>(G.Mb, A.MbA, (i64)G.ncol, T::NIN, T::NOUTB);
        RG_ADJ_CHECK();
        A.map_ready = true;
    }
    // CT and update (every entry of gBo, gGam, gPhi, gUo and the interior
    // entries of gzoneB are written here)
    copy_state<<<2048, 256, 0, st>>>(gBf1, A.gBo, G.NF);
    const i64 nee = (i64)G.nv * G.Nr + (i64)G.nae * (G.Nr + 1);
    circ_transpose<<<nblk(nee, 256), 256, 0, st>>>(G, -dt, G.g, G.g + G.Nr - 1, gBf1, A.gGam);
    const i64 nff = (i64)G.ncol * (G.Nr + 1) + (i64)G.nae * G.Nr;
    adj_update_faces<<<nblk(nff, 256), 256, 0, st>>>(G, dt, gU1, A.gPhi);
    adj_update_zones<<<nblk(G.Z, 256), 256, 0, st>>>(G, gU1, A.gUo, A.gzoneB);
    RG_ADJ_CHECK();
    // Riemann solvers
    const R *ftr = reinterpret_cast<const R *>(g->ftr), *etr = reinterpret_cast<const R *>(g->etr);
    const R *wcoef = reinterpret_cast<const R *>(g->wcoef), *bnode = reinterpret_cast<const R *>(g->bnode);
    adj_face_flux<P, R><<<nblk(nff * T::Q, 256), 256, 0, st>>>(G, gam, ftr, A.gPhi, A.gftr);
    adj_edge_emf<R><<<nblk(nee * 3, 256), 256, 0, st>>>(G, gam, etr, A.gGam, A.getr);
    RG_ADJ_CHECK();
    // predictor
    constexpr int ZPW = PredLayout<P>::ZPW;
    adj_predictor<P, R><<<(unsigned)((nzr + ZPW - 1) / ZPW), 64, 0, st>>>(G, dt, gam, npic, A.Ubc, wcoef, bnode,
                                                                          A.gftr, A.getr, A.gUo, A.gwc, A.gbnode);
    RG_ADJ_CHECK();
    // divergence-free map, then face nodal B
    const int ntile = (G.Nr + 2 + 15) / 16;
    adj_bmap<P><<<(unsigned)((i64)G.ncol * ntile), 64, 0, st>>>(G, A.MbA, A.gbnode, A.gzoneB, A.gUo, A.gwc, A.gside);
    const i64 nbn = (i64)G.ncol * (G.Nr + 3) + (i64)G.nae * (G.Nr + 2);
    adj_face_gather_bmap<P><<<nblk(nbn, 256), 256, 0, st>>>(G, A.gside, A.gbnod, A.gBo);
    adj_face_bnodal<P, R><<<nblk(nbn, 128), 128, 0, st>>>(G, A.Ubc, A.Bbc, wcoef, A.gbnod, A.gBo, A.gsb);
    adj_zone_gather_bnodal<P><<<nblk(nzr, 256), 256, 0, st>>>(G, A.gsb, A.gUo, A.gwc);
    RG_ADJ_CHECK();
    // WENO-AO
    const RunSplit wr = run_split(G.Nr + 2);
    adj_weno<P><<<(unsigned)((i64)G.ncol * (wr.nchunk + (wr.nleft > 0))), 64, 0, st>>>(
        G, A.Ubc, A.gwc, A.gdu, weno_eps(prm), wr.nchunk, wr.nu, wr.nleft);
    adj_weno_gather<P><<<nblk(G.Z, 256), 256, 0, st>>>(G, A.gdu, A.gUo);
    RG_ADJ_CHECK();
    // boundary fill
    adj_bc_zones<<<nblk(G.Z, 256), 256, 0, st>>>(G, prm.bc_kind, A.gUo, gU);
    adj_bc_faces<<<nblk(G.NF, 256), 256, 0, st>>>(G, prm.bc_kind, A.gBo, gBf);
    RG_ADJ_CHECK();
    return RG_OK;
}

rg_status launch_stokes_T(rg_geom *g, const double *gBf, double *gcirc, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGeom &G = g->d;
    const i64 ne = (i64)G.nv * G.K + (i64)G.nae * (G.K + 1);
    circ_transpose<<<nblk(ne, 256), 256, 0, st>>>(G, 1.0, 0, G.K - 1, gBf, gcirc);
    RG_ADJ_CHECK();
    return RG_OK;
}

rg_status launch_adjoint(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, const double *gU1,
                         const double *gBf1, double *gU, double *gBf, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool f32 = g->mode == RG_MODE_FP32;
    if (g->d.order == 3)
        return f32 ? adjoint_order<3, float>(g, p, U, Bf, gU1, gBf1, gU, gBf, st)
                   : adjoint_order<3, double>(g, p, U, Bf, gU1, gBf1, gU, gBf, st);
    if (g->d.order == 4)
        return f32 ? adjoint_order<4, float>(g, p, U, Bf, gU1, gBf1, gU, gBf, st)
                   : adjoint_order<4, double>(g, p, U, Bf, gU1, gBf1, gU, gBf, st);
    set_error("unsupported order");
    return RG_ENOTSUP;
}

}  // namespace rg

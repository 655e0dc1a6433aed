// Adjoint of one step (the vector-Jacobian product of rg_step at a given
// state, dt held fixed), FP64.  The step's stages are reversed one by one:
//
//   face_ct, zone_update  : linear; transposed as gathers over the faces of an
//                           edge and the zones of a face
//   edge_emf, face_flux   : pointwise Riemann solvers; exact local Jacobians by
//                           forward differentiation (dual numbers) of the
//                           step's own solver code, contracted with the
//                           incoming gradient
//   predictor             : recomputed per zone, then the traces, time
//                           averages and the unrolled Picard sweeps reversed
//                           (flux Jacobians again by dual numbers, derivative
//                           matrices transposed)
//   bmap                  : linear, the transposed per-column map
//   face_bnodal           : MinMod and mean restore reversed per face
//   weno                  : exact derivative of the WENO-AO combination
//                           (nonlinear weights included) by dual numbers
//   boundary fill         : ghost copies accumulated into their sources
//
// Every gradient contribution to a zone or face is gathered by the one thread
// that owns the target, in a fixed order: no floating-point atomics, so the
// result is deterministic.  The forward quantities the reversal needs are
// recomputed by running the step first.
#include "mhd_device.hpp"

namespace rg {

namespace {

// Picard sweeps the adjoint keeps in LDS (the sweeps' states are all needed
// in reverse)
constexpr int ADJ_MAX_PICARD = 6;

__global__ void fill_zero(double *p, i64 n)
{
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) p[t] = 0.0;
}

inline unsigned nblk(i64 n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- constrained transport
// gGam[e] = sum over the CT faces f holding edge e of -(dt/A_f) s_fe gBf[f],
// with s_fe the sign with which face_ct adds Gam[e] into face f's circulation.
__global__ void adj_ct(DevGeom G, double dt, const double *__restrict__ gBf, double *__restrict__ gGam)
{
    const int nrad = G.Nr, nang = G.Nr + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.nv * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    double acc = 0.0;
    i64 e;
    if (t < nR) {
        // radial edge of vertex v in shell k: the angular faces (ae, k) of the
        // angular edges at v, through lp = ... + Gam[v1 edge] - ... - Gam[v0 edge]
        const int v = (int)(t / nrad), k = G.g + (int)(t % nrad);
        e = (i64)v * G.K + k;
        for (int s = 0; s < G.v_ncol[v]; s++) {
            const int ae = G.v_ae[4 * v + s];
            const double sg = (G.ae_v[2 * ae + 1] == v) ? 1.0 : -1.0;
            const i64 f = G.NRF + (i64)ae * G.K + k;
            acc += -(dt / G.area[f]) * G.ae_rs[ae] * sg * gBf[f];
        }
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), kf = G.g + (int)(u % nang);
        e = G.NRE + (i64)ae * (G.K + 1) + kf;
        // radial faces kf of the two columns sharing the angular edge
        for (int s = 0; s < 2; s++) {
            const int c = G.ae_col[2 * ae + s], lf = G.ae_lf[2 * ae + s];
            const i64 f = (i64)c * (G.K + 1) + kf;
            acc += -(dt / G.area[f]) * G.col_sgn[4 * c + lf] * gBf[f];
        }
        // angular faces of the shells above (as lower ring) and below (as upper ring)
        if (kf <= G.g + G.Nr - 1) {
            const i64 f = G.NRF + (i64)ae * G.K + kf;
            acc += -(dt / G.area[f]) * G.ae_rs[ae] * gBf[f];
        }
        if (kf - 1 >= G.g) {
            const i64 f = G.NRF + (i64)ae * G.K + kf - 1;
            acc -= -(dt / G.area[f]) * G.ae_rs[ae] * gBf[f];
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
        if (interior && v >= 5) gzoneB[(i64)(v - 5) * G.Z + z] = g;
        else gUo[(i64)v * G.Z + z] = g;
    }
}

// ---------------------------------------------------------------- Riemann solvers
template <int P>
__global__ void adj_face_flux(DevGeom G, double gam, const double *__restrict__ ftr, const double *__restrict__ gPhi,
                              double *__restrict__ gftr)
{
    using T = Tr<P>;
    const int nrad = G.Nr + 1, nang = G.Nr;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.ncol * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    i64 f;
    const double *nrm, *fw;
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        nrm = G.fnR + (i64)c * T::Q * 3;
        fw = G.fwR + (i64)c * T::Q;
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), k = G.g + (int)(u % nang);
        f = G.NRF + (i64)ae * G.K + k;
        nrm = G.fnA + (i64)ae * T::Q * 3;
        fw = G.fwA + (i64)ae * T::Q;
    }
    const double area = G.area[f];
    double gPhiF[8];
    for (int v = 0; v < 8; v++) gPhiF[v] = gPhi[(i64)v * G.NF + f];
    for (int q = 0; q < T::Q; q++) {
        const double *a = ftr + ((f * 2 + 0) * T::Q + q) * 16, *b = ftr + ((f * 2 + 1) * T::Q + q) * 16;
        double *ga = gftr + ((f * 2 + 0) * T::Q + q) * 16, *gb = gftr + ((f * 2 + 1) * T::Q + q) * 16;
        const double w = fw[q] * area;
        // inputs in the order UL, FL (side 0 record), UR, FR (side 1 record)
        for (int in = 0; in < 32; in++) {
            dual UL[8], UR[8], FL[8], FR[8], Fs[8];
            for (int v = 0; v < 8; v++) {
                UL[v] = dual(a[v], in == v ? 1.0 : 0.0);
                FL[v] = dual(a[8 + v], in == 8 + v ? 1.0 : 0.0);
                UR[v] = dual(b[v], in == 16 + v ? 1.0 : 0.0);
                FR[v] = dual(b[8 + v], in == 24 + v ? 1.0 : 0.0);
            }
            dev_hll<dual>(UL, UR, FL, FR, nrm + q * 3, dual(gam), Fs);
            double s = 0.0;
            for (int v = 0; v < 8; v++) s += Fs[v].d * gPhiF[v];
            if (in < 16) ga[in] = w * s;
            else gb[in - 16] = w * s;
        }
    }
}

__global__ void adj_edge_emf(DevGeom G, double gam, const double *__restrict__ etr, const double *__restrict__ gGam,
                             double *__restrict__ getr)
{
    const int nrad = G.Nr, nang = G.Nr + 1;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.nv * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    const double simpson[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    i64 e;
    int nzs;
    const double *frame[3];
    double wl[3];
    const double *N3 = nullptr;
    if (t < nR) {
        const int v = (int)(t / nrad), k = G.g + (int)(t % nrad);
        e = (i64)v * G.K + k;
        nzs = G.v_ncol[v];
        const double len = G.radius[k + 1] - G.radius[k];
        for (int p = 0; p < 3; p++) { frame[p] = G.vF + (i64)v * 9; wl[p] = simpson[p] * len; }
        N3 = G.vN3 + (i64)v * 9;
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), kf = G.g + (int)(u % nang);
        e = G.NRE + (i64)ae * (G.K + 1) + kf;
        nzs = 4;
        const double s = G.radius[kf] / G.radius[0];
        for (int p = 0; p < 3; p++) { frame[p] = G.aeF + ((i64)ae * 3 + p) * 9; wl[p] = G.aeW[(i64)ae * 3 + p] * s; }
    }
    const double ge = gGam[e];
    for (int p = 0; p < 3; p++) {
        const double *tt = frame[p] + 6;
        for (int in = 0; in < nzs * 11; in++) {
            dual U[4][8], E[4][3], Et[4];
            for (int s = 0; s < 4; s++) {
                const double *rec = etr + ((e * 4 + s) * 3 + p) * 11;
                for (int v = 0; v < 8; v++) U[s][v] = dual(rec[v], in == s * 11 + v ? 1.0 : 0.0);
                for (int v = 0; v < 3; v++) E[s][v] = dual(rec[8 + v], in == s * 11 + 8 + v ? 1.0 : 0.0);
                Et[s] = E[s][0] * tt[0] + E[s][1] * tt[1] + E[s][2] * tt[2];
            }
            const dual Es = (nzs == 4) ? emf4<dual>(U, Et, frame[p], dual(gam)) : emf3<dual>(U, E, N3, tt, dual(gam));
            getr[((e * 4 + in / 11) * 3 + p) * 11 + in % 11] = wl[p] * ge * Es.d;
        }
    }
}

// ---------------------------------------------------------------- predictor
// One zone per block; lanes below N are the zone's serendipity nodes.
template <int P>
__global__ __launch_bounds__(64) void adj_predictor(DevGeom G, double dt, double gamma, int npic,
                                                    const double *__restrict__ Uo, const double *__restrict__ wc,
                                                    const double *__restrict__ bnode, const double *__restrict__ gftr,
                                                    const double *__restrict__ getr, double *__restrict__ gUo,
                                                    double *__restrict__ gwc, double *__restrict__ gbnode)
{
    using T = Tr<P>;
    constexpr int N = T::N, E = T::M - 1, NCF = T::NC + 1, NPMAX = ADJ_MAX_PICARD;
    __shared__ double s_c[5 * NCF];
    __shared__ double s_ut[NPMAX + 1][E][8][N];   // Ut after each sweep (index 0: the initial copy of Ua)
    __shared__ double s_a[3][8][N];               // flux / gradient slab
    __shared__ double s_red[5][N];
    const int KR = G.Nr + 2;
    const i64 zt = blockIdx.x;
    const int c = (int)(zt / KR), k = G.g - 1 + (int)(zt % KR);
    const i64 z = (i64)c * G.K + k;
    const int i = threadIdx.x;
    const bool node = i < N;
    const double *D = G.Dfull;   // [3][N][N]
    for (int j = i; j < 5 * NCF; j += 64) {
        const int v = j / NCF, a = j % NCF;
        s_c[j] = a == 0 ? Uo[v * G.Z + z] : wc[((i64)v * T::NC + a - 1) * G.Z + z];
    }
    __syncthreads();
    double Ua[8], dFa[8], met[9], iJ = 1.0, J = 1.0;
    const double gam = gamma;
    if (node) {
        const double *Ev = G.Ev + (i64)c * T::NC * N + i;
        for (int v = 0; v < 5; v++) {
            double acc = s_c[v * NCF];
            for (int a = 0; a < T::NC; a++) acc += Ev[a * N] * s_c[v * NCF + 1 + a];
            Ua[v] = acc;
        }
        const double *bn = bnode + zt * (3 * N) + i;
        Ua[5] = bn[0];
        Ua[6] = bn[N];
        Ua[7] = bn[2 * N];
        J = G.nJ[(i64)c * N + i];
        iJ = 1.0 / J;
        const double fac = dt / G.zscale[k];
        for (int m = 0; m < 9; m++) met[m] = fac * G.nM[((i64)c * 9 + m) * N + i];
        for (int v = 0; v < 8; v++) Ua[v] *= J;
    }
    // ---- forward recomputation
    auto flux_to_slab = [&](const double *u) {
        double F[3][8];
        mapped_flux<double>(u, iJ, met, gam, F);
        for (int d = 0; d < 3; d++)
            for (int v = 0; v < 8; v++) s_a[d][v][i] = F[d][v];
    };
    auto deriv_from_slab = [&](double *out) {   // out[v] = sum_d sum_l D_d[i][l] F_d[l][v]
        for (int v = 0; v < 8; v++) out[v] = 0.0;
        for (int d = 0; d < 3; d++)
            for (int l = 0; l < N; l++) {
                const double w = D[((i64)d * N + i) * N + l];
                if (w != 0.0)
                    for (int v = 0; v < 8; v++) out[v] += w * s_a[d][v][l];
            }
    };
    if (node) flux_to_slab(Ua);
    __syncthreads();
    if (node) deriv_from_slab(dFa);
    __syncthreads();
    if (node)
        for (int t = 0; t < E; t++)
            for (int v = 0; v < 8; v++) s_ut[0][t][v][i] = Ua[v];
    for (int it = 1; it <= npic; it++) {
        double A[E][8];
        for (int s = 0; s < E; s++) {
            if (it == 1) {
                for (int v = 0; v < 8; v++) A[s][v] = dFa[v];
            } else {
                double u[8];
                if (node) {
                    for (int v = 0; v < 8; v++) u[v] = s_ut[it - 1][s][v][i];
                    flux_to_slab(u);
                }
                __syncthreads();
                if (node) deriv_from_slab(A[s]);
                __syncthreads();
            }
        }
        if (node)
            for (int t = 0; t < E; t++)
                for (int v = 0; v < 8; v++) {
                    double u = Ua[v] - G.R[t * T::M] * dFa[v];
                    for (int s = 0; s < E; s++) u -= G.R[t * T::M + s + 1] * A[s][v];
                    s_ut[it][t][v][i] = u;
                }
        __syncthreads();
    }
    // ---- traces reversed: gradients of the time-averaged state and flux at this node
    double gaU[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gaF[3][8];
    for (int d = 0; d < 3; d++)
        for (int v = 0; v < 8; v++) gaF[d][v] = 0.0;
    if (node) {
        for (int lf = 0; lf < 6; lf++) {
            int kk = -1;
            for (int j = 0; j < T::NFN; j++)
                if (G.fnode[lf * T::NFN + j] == i) kk = j;
            if (kk < 0) continue;
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
            const double *go = gftr + (fid * 2 + side) * T::Q * 16;
            for (int q = 0; q < T::Q; q++) {
                const int qc = perm ? perm[q] : q;
                const double w = G.fintc[kk * T::Q + q];
                const double *n = nrm + qc * 3;
                for (int v = 0; v < 8; v++) {
                    gaU[v] += w * go[qc * 16 + v];
                    const double gn = w * go[qc * 16 + 8 + v];
                    for (int d = 0; d < 3; d++) gaF[d][v] += gn * n[d];
                }
            }
        }
        for (int le = 0; le < 12; le++) {
            int kk = -1;
            for (int j = 0; j < T::NEN; j++)
                if (G.enode[le * T::NEN + j] == i) kk = j;
            if (kk < 0) continue;
            const int rev = G.col_rev[(i64)c * 12 + le], slot = G.col_slot[(i64)c * 12 + le];
            i64 e;
            if (le < 8) {
                const int ae = G.col_ae[4 * c + LocalEdges::FACE[le]];
                e = G.NRE + (i64)ae * (G.K + 1) + k + LocalEdges::UP[le];
            } else {
                e = (i64)G.col_v[4 * c + LocalEdges::CORNER[le - 8]] * G.K + k;
            }
            const double *go = getr + (e * 4 + slot) * 3 * 11;
            for (int p = 0; p < 3; p++) {
                const int pc = rev ? 2 - p : p;
                const double w = G.eintc[kk * 3 + p];
                for (int v = 0; v < 8; v++) gaU[v] += w * go[pc * 11 + v];
                gaF[2][6] += w * go[pc * 11 + 8];   // E_x = H[B_y]
                gaF[0][7] += w * go[pc * 11 + 9];   // E_y = F[B_z]
                gaF[1][5] += w * go[pc * 11 + 10];  // E_z = G[B_x]
            }
        }
    }
    // ---- time averages reversed
    double gUt[E][8];
    if (node)
        for (int t = 0; t < E; t++) {
            const double wt = G.wt[t + 1];
            double w[8];
            for (int v = 0; v < 8; v++) w[v] = s_ut[npic][t][v][i] * iJ;
            for (int cmp = 0; cmp < 8; cmp++) {
                dual wd[8], F[3][8];
                for (int v = 0; v < 8; v++) wd[v] = dual(w[v], v == cmp ? 1.0 : 0.0);
                dev_flux<dual>(wd, dual(gam), F);
                double s = gaU[cmp];
                for (int d = 0; d < 3; d++)
                    for (int v = 0; v < 8; v++) s += F[d][v].d * gaF[d][v];
                gUt[t][cmp] = wt * s * iJ;
            }
        }
    // ---- Picard sweeps reversed
    double gUa[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gdFa[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int it = npic; it >= 1; it--) {
        if (node)
            for (int t = 0; t < E; t++)
                for (int v = 0; v < 8; v++) {
                    gUa[v] += gUt[t][v];
                    gdFa[v] -= G.R[t * T::M] * gUt[t][v];
                }
        double gprev[E][8];
        for (int s = 0; s < E; s++)
            for (int v = 0; v < 8; v++) gprev[s][v] = 0.0;
        for (int s = 0; s < E; s++) {
            double gA[8];
            for (int v = 0; v < 8; v++) {
                gA[v] = 0.0;
                for (int t = 0; t < E; t++) gA[v] -= G.R[t * T::M + s + 1] * gUt[t][v];
            }
            if (it == 1) {
                // the first sweep's derivatives are the tau = 0 ones
                for (int v = 0; v < 8; v++) gdFa[v] += gA[v];
                continue;
            }
            // A_s = D F(Ut_{it-1}[s]): transpose D through the slab
            if (node)
                for (int v = 0; v < 8; v++) s_a[0][v][i] = gA[v];
            __syncthreads();
            double gF[3][8];
            if (node)
                for (int d = 0; d < 3; d++)
                    for (int v = 0; v < 8; v++) {
                        double acc = 0.0;
                        for (int r = 0; r < N; r++) {
                            const double w = D[((i64)d * N + r) * N + i];
                            if (w != 0.0) acc += w * s_a[0][v][r];
                        }
                        gF[d][v] = acc;
                    }
            __syncthreads();
            if (node) {
                double u[8];
                for (int v = 0; v < 8; v++) u[v] = s_ut[it - 1][s][v][i];
                for (int cmp = 0; cmp < 8; cmp++) {
                    dual ud[8], F[3][8], metd[9];
                    for (int v = 0; v < 8; v++) ud[v] = dual(u[v], v == cmp ? 1.0 : 0.0);
                    for (int m = 0; m < 9; m++) metd[m] = dual(met[m]);
                    mapped_flux<dual>(ud, dual(iJ), metd, dual(gam), F);
                    double acc = 0.0;
                    for (int d = 0; d < 3; d++)
                        for (int v = 0; v < 8; v++) acc += F[d][v].d * gF[d][v];
                    gprev[s][cmp] += acc;
                }
            }
        }
        for (int t = 0; t < E; t++)
            for (int v = 0; v < 8; v++) gUt[t][v] = gprev[t][v];
    }
    if (npic == 0 && node)
        for (int t = 0; t < E; t++)
            for (int v = 0; v < 8; v++) gUa[v] += gUt[t][v];
    // ---- tau = 0 derivative reversed: dFa = D F(Ua)
    if (node)
        for (int v = 0; v < 8; v++) s_a[0][v][i] = gdFa[v];
    __syncthreads();
    if (node) {
        double gF[3][8];
        for (int d = 0; d < 3; d++)
            for (int v = 0; v < 8; v++) {
                double acc = 0.0;
                for (int r = 0; r < N; r++) {
                    const double w = D[((i64)d * N + r) * N + i];
                    if (w != 0.0) acc += w * s_a[0][v][r];
                }
                gF[d][v] = acc;
            }
        for (int cmp = 0; cmp < 8; cmp++) {
            dual ud[8], F[3][8], metd[9];
            for (int v = 0; v < 8; v++) ud[v] = dual(Ua[v], v == cmp ? 1.0 : 0.0);
            for (int m = 0; m < 9; m++) metd[m] = dual(met[m]);
            mapped_flux<dual>(ud, dual(iJ), metd, dual(gam), F);
            double acc = 0.0;
            for (int d = 0; d < 3; d++)
                for (int v = 0; v < 8; v++) acc += F[d][v].d * gF[d][v];
            gUa[cmp] += acc;
        }
    }
    __syncthreads();
    // ---- nodal initial state reversed: Ua = J (fluid polynomial | divergence-free B)
    if (node) {
        for (int v = 0; v < 8; v++) gUa[v] *= J;
        for (int v = 5; v < 8; v++) gbnode[zt * (3 * N) + (v - 5) * N + i] = gUa[v];
        for (int v = 0; v < 5; v++) s_red[v][i] = gUa[v];
    }
    __syncthreads();
    for (int j = i; j < 5 * NCF; j += 64) {
        const int v = j / NCF, a = j % NCF;
        double acc = 0.0;
        if (a == 0) {
            for (int n = 0; n < N; n++) acc += s_red[v][n];
            gUo[(i64)v * G.Z + z] += acc;
        } else {
            const double *Ev = G.Ev + ((i64)c * T::NC + a - 1) * N;
            for (int n = 0; n < N; n++) acc += Ev[n] * s_red[v][n];
            gwc[((i64)v * T::NC + a - 1) * G.Z + z] = acc;
        }
    }
}

// ---------------------------------------------------------------- divergence-free B map
// gIn = Mb gOut per zone (Mb stored input-major, output fastest): writes the
// zone's share of the gradient of its inputs -- B means and WENO B
// coefficients (zone owned), and per local face the limited nodal values and
// the face mean (gathered per face afterwards).
template <int P>
__global__ void adj_bmap(DevGeom G, const double *__restrict__ gbnode, const double *__restrict__ gzoneB,
                         double *__restrict__ gUo, double *__restrict__ gwc, double *__restrict__ gside)
{
    using T = Tr<P>;
    constexpr int NIN = T::NIN, NOUT = T::NOUTB, NA = 3 * (T::NC + 1), NQ = NA + 6 * T::Q;
    const int KR = G.Nr + 2;
    const i64 zr = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (zr >= (i64)G.ncol * KR) return;
    const int c = (int)(zr / KR), k = G.g - 1 + (int)(zr % KR);
    const i64 z = (i64)c * G.K + k;
    const bool interior = k >= G.g && k < G.g + G.Nr;
    double gout[NOUT];
    for (int r = 0; r < 3 * T::N; r++) gout[r] = gbnode[zr * (3 * T::N) + r];
    for (int r = 0; r < 3; r++) gout[3 * T::N + r] = interior ? gzoneB[(i64)r * G.Z + z] : 0.0;
    const double *Mb = G.Mb + (i64)c * NIN * NOUT;
    for (int j = 0; j < NIN; j++) {
        double acc = 0.0;
        for (int r = 0; r < NOUT; r++) acc += Mb[(i64)j * NOUT + r] * gout[r];
        if (j < NA) {
            const int comp = j / (T::NC + 1), a = j % (T::NC + 1);
            if (a == 0) gUo[(i64)(5 + comp) * G.Z + z] += acc;
            else gwc[((i64)(5 + comp) * T::NC + a - 1) * G.Z + z] = acc;
        } else {
            gside[zr * (NIN - NA) + (j - NA)] = acc;   // [6][Q] nodal values, then [6] face means
        }
    }
    (void)NQ;
}

// per face of the face-nodal set: sum the two zones' shares from adj_bmap
template <int P>
__global__ void adj_face_gather_bmap(DevGeom G, const double *__restrict__ gside, double *__restrict__ gbnod,
                                     double *__restrict__ gBo)
{
    using T = Tr<P>;
    constexpr int NIS = T::NIN - 3 * (T::NC + 1);   // 6Q + 6
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
    for (int q = 0; q < T::Q; q++) {
        double acc = 0.0;
        for (int s = 0; s < 2; s++)
            if (zr[s] >= 0) acc += gside[zr[s] * NIS + lf[s] * T::Q + q];
        gbnod[(i64)q * G.NF + f] = acc;
    }
    double acc = 0.0;
    for (int s = 0; s < 2; s++)
        if (zr[s] >= 0) acc += gside[zr[s] * NIS + 6 * T::Q + lf[s]];
    gBo[f] += acc;
}

// ---------------------------------------------------------------- face nodal B
// Reverse of MinMod + mean restore on one face; the two sides' shares (B mean
// and WENO B coefficients of each side's zone) go to gsb[f][side][3 + 3 NC].
template <int P>
__global__ void adj_face_bnodal(DevGeom G, const double *__restrict__ Uo, const double *__restrict__ Bo,
                                const double *__restrict__ wc, const double *__restrict__ gbnod,
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
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g - 1 + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        z[0] = (i64)c * G.K + kf - 1;
        z[1] = (i64)c * G.K + kf;
        have[0] = (kf - 1 >= G.g - 1) && (kf - 1 <= G.g + G.Nr);
        have[1] = (kf >= G.g - 1) && (kf <= G.g + G.Nr);
        fev[0] = G.fevR + ((i64)c * 2 + 0) * T::Q * T::NC;
        fev[1] = G.fevR + ((i64)c * 2 + 1) * T::Q * T::NC;
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
        nrm = G.fnA + (i64)ae * T::Q * 3;
        fw = G.fwA + (i64)ae * T::Q;
    }
    // forward: each side's B at the points, deviations, MinMod
    const double mean = Bo[f];
    double d[2][T::Q];
    for (int s = 0; s < 2; s++) {
        if (!have[s]) continue;
        for (int q = 0; q < T::Q; q++) {
            double B[3];
            for (int c3 = 0; c3 < 3; c3++) {
                double b = Uo[(5 + c3) * G.Z + z[s]];
                for (int a = 0; a < T::NC; a++)
                    b += wc[((i64)(5 + c3) * T::NC + a) * G.Z + z[s]] * fev[s][q * T::NC + a];
                B[c3] = b;
            }
            d[s][q] = B[0] * nrm[q * 3] + B[1] * nrm[q * 3 + 1] + B[2] * nrm[q * 3 + 2] - mean;
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
        double *o = gsb + (f * 2 + s) * NSB;
        if (!have[s]) {
            for (int j = 0; j < NSB; j++) o[j] = 0.0;
            continue;
        }
        for (int q = 0; q < T::Q; q++) gmean -= gd[s][q];
        for (int c3 = 0; c3 < 3; c3++) {
            double gm0 = 0.0;
            for (int q = 0; q < T::Q; q++) gm0 += gd[s][q] * nrm[q * 3 + c3];
            o[c3] = gm0;
            for (int a = 0; a < T::NC; a++) {
                double acc = 0.0;
                for (int q = 0; q < T::Q; q++) acc += gd[s][q] * nrm[q * 3 + c3] * fev[s][q * T::NC + a];
                o[3 + c3 * T::NC + a] = acc;
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
        for (int lf = 0; lf < 6; lf++) acc += gsb[(f[lf] * 2 + sd[lf]) * NSB + c3];
        gUo[(i64)(5 + c3) * G.Z + z] += acc;
        for (int a = 0; a < T::NC; a++) {
            double s = 0.0;
            for (int lf = 0; lf < 6; lf++) s += gsb[(f[lf] * 2 + sd[lf]) * NSB + 3 + c3 * T::NC + a];
            gwc[((i64)(5 + c3) * T::NC + a) * G.Z + z] += s;
        }
    }
}

// ---------------------------------------------------------------- WENO-AO
// gdu[v][j][zr] = d(coefficients)/d(du_j)^T gwc, exact through the nonlinear
// weights (one tangent pass per stencil member)
template <int P>
__global__ void adj_weno(DevGeom G, const double *__restrict__ Uo, const double *__restrict__ gwc,
                         double *__restrict__ gdu)
{
    using T = Tr<P>;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nzr * 8) return;
    const int v = (int)(t / nzr);
    const i64 zr = t % nzr;
    const int c = (int)(zr / KR), k = G.g - 1 + (int)(zr % KR);
    const i64 z = (i64)c * G.K + k;
    const double *Pl = G.Pl + (i64)c * T::NC * T::NS, *Ps = G.Ps + (i64)c * 7 * 18, *Qs = G.Qs + (i64)c * T::NC * T::NC;
    const double *Uv = Uo + (i64)v * G.Z;
    const double u0 = Uv[z];
    double du[T::NS], go[T::NC];
    bool used[T::NS];
    for (int j = 0; j < T::NS; j++) {
        const int m = G.stm[(i64)c * T::NS + j];
        used[j] = m >= 0;
        const int dz = m < 0 ? 0 : (int)(((i64)(m >> 3) - c) * G.K + (m & 7) - 3);
        du[j] = Uv[z + dz] - u0;
    }
    for (int a = 0; a < T::NC; a++) go[a] = gwc[((i64)v * T::NC + a) * G.Z + z];
    for (int j = 0; j < T::NS; j++) {
        double g = 0.0;
        if (used[j]) {
            dual dd[T::NS], o[T::NC];
            for (int jj = 0; jj < T::NS; jj++) dd[jj] = dual(du[jj], jj == j ? 1.0 : 0.0);
            weno_core<P, dual, double>(dd, Pl, Ps, Qs, o);
            for (int a = 0; a < T::NC; a++) g += o[a].d * go[a];
        }
        gdu[((i64)v * T::NS + j) * nzr + zr] = g;
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
    for (int v = 0; v < 8; v++) {
        double acc = 0.0;
        for (int e = G.inv_ptr[c]; e < G.inv_ptr[c + 1]; e++) {
            const int c2 = G.inv_ent[3 * e], j = G.inv_ent[3 * e + 1], dk = G.inv_ent[3 * e + 2];
            const int k2 = k - dk;
            if (k2 < G.g - 1 || k2 > G.g + G.Nr) continue;
            acc += gdu[((i64)v * T::NS + j) * nzr + (i64)c2 * KR + (k2 - (G.g - 1))];
        }
        if (recon)
            for (int j = 0; j < T::NS; j++)
                if (G.stm[(i64)c * T::NS + j] >= 0) acc -= gdu[((i64)v * T::NS + j) * nzr + zr];
        gUo[(i64)v * G.Z + z] += acc;
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

template <int P>
static rg_status adjoint_order(rg_geom *g, const rg_step_params &prm, const double *U, const double *Bf,
                               const double *gU1, const double *gBf1, double *gU, double *gBf, hipStream_t st)
{
    const DevGeom &G = g->d;
    using T = Tr<P>;
    AdjBuffers &A = g->adj;
    const int npic = prm.n_picard > 0 ? prm.n_picard : P;
    if (npic > ADJ_MAX_PICARD) {
        set_error("the adjoint supports at most " + std::to_string(ADJ_MAX_PICARD) + " Picard sweeps");
        return RG_ENOTSUP;
    }
    const double dt = prm.dt, gam = prm.gamma;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR;
    // forward step into scratch outputs: refreshes the step's work buffers
    // (WENO coefficients, face nodal B, nodal B, traces) at this state
    rg_step_params fp = prm;
    rg_status s = launch_step(g, fp, U, Bf, A.Utmp, A.Btmp, st);
    if (s != RG_OK) return s;
    // the boundary-filled working state the step started from
    s = launch_bc(g, prm.bc_kind, U, Bf, A.Ubc, A.Bbc, st);
    if (s != RG_OK) return s;
    const unsigned zb = 2048;
    fill_zero<<<zb, 256, 0, st>>>(A.gUo, 8 * G.Z);
    fill_zero<<<zb, 256, 0, st>>>(A.gBo, G.NF);
    fill_zero<<<zb, 256, 0, st>>>(A.gzoneB, 3 * G.Z);
    fill_zero<<<zb, 256, 0, st>>>(A.gwc, 8 * (i64)T::NC * G.Z);
    fill_zero<<<zb, 256, 0, st>>>(A.gftr, (i64)16 * T::Q * 2 * G.NF);
    fill_zero<<<zb, 256, 0, st>>>(A.getr, (i64)11 * 3 * 4 * G.NE);
    fill_zero<<<zb, 256, 0, st>>>(A.gGam, G.NE);
    fill_zero<<<zb, 256, 0, st>>>(A.gbnod, (i64)T::Q * G.NF);
    RG_ADJ_CHECK();
    // CT and update
    copy_state<<<zb, 256, 0, st>>>(gBf1, A.gBo, G.NF);
    const i64 nee = (i64)G.nv * G.Nr + (i64)G.nae * (G.Nr + 1);
    adj_ct<<<nblk(nee, 256), 256, 0, st>>>(G, dt, gBf1, A.gGam);
    const i64 nff = (i64)G.ncol * (G.Nr + 1) + (i64)G.nae * G.Nr;
    adj_update_faces<<<nblk(nff, 256), 256, 0, st>>>(G, dt, gU1, A.gPhi);
    adj_update_zones<<<nblk(G.Z, 256), 256, 0, st>>>(G, gU1, A.gUo, A.gzoneB);
    RG_ADJ_CHECK();
    // Riemann solvers
    adj_face_flux<P><<<nblk(nff, 128), 128, 0, st>>>(G, gam, g->ftr, A.gPhi, A.gftr);
    adj_edge_emf<<<nblk(nee, 128), 128, 0, st>>>(G, gam, g->etr, A.gGam, A.getr);
    RG_ADJ_CHECK();
    // predictor
    adj_predictor<P><<<(unsigned)nzr, 64, 0, st>>>(G, dt, gam, npic, A.Ubc, g->wcoef, g->bnode, A.gftr, A.getr,
                                                    A.gUo, A.gwc, A.gbnode);
    RG_ADJ_CHECK();
    // divergence-free map, then face nodal B
    adj_bmap<P><<<nblk(nzr, 128), 128, 0, st>>>(G, A.gbnode, A.gzoneB, A.gUo, A.gwc, A.gside);
    const i64 nbn = (i64)G.ncol * (G.Nr + 3) + (i64)G.nae * (G.Nr + 2);
    adj_face_gather_bmap<P><<<nblk(nbn, 256), 256, 0, st>>>(G, A.gside, A.gbnod, A.gBo);
    adj_face_bnodal<P><<<nblk(nbn, 128), 128, 0, st>>>(G, A.Ubc, A.Bbc, g->wcoef, A.gbnod, A.gBo, A.gsb);
    adj_zone_gather_bnodal<P><<<nblk(nzr, 256), 256, 0, st>>>(G, A.gsb, A.gUo, A.gwc);
    RG_ADJ_CHECK();
    // WENO-AO
    adj_weno<P><<<nblk(nzr * 8, 64), 64, 0, st>>>(G, A.Ubc, A.gwc, A.gdu);
    adj_weno_gather<P><<<nblk(G.Z, 256), 256, 0, st>>>(G, A.gdu, A.gUo);
    RG_ADJ_CHECK();
    // boundary fill
    adj_bc_zones<<<nblk(G.Z, 256), 256, 0, st>>>(G, prm.bc_kind, A.gUo, gU);
    adj_bc_faces<<<nblk(G.NF, 256), 256, 0, st>>>(G, prm.bc_kind, A.gBo, gBf);
    RG_ADJ_CHECK();
    return RG_OK;
}

rg_status launch_adjoint(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, const double *gU1,
                         const double *gBf1, double *gU, double *gBf, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->d.order == 3) return adjoint_order<3>(g, p, U, Bf, gU1, gBf1, gU, gBf, st);
    if (g->d.order == 4) return adjoint_order<4>(g, p, U, Bf, gU1, gBf1, gU, gBf, st);
    set_error("unsupported order");
    return RG_ENOTSUP;
}

}  // namespace rg

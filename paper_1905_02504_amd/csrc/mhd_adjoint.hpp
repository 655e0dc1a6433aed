// Reverse-mode (vector-Jacobian) counterparts of the point functions in
// mhd_device.hpp, written out by hand: FP64, and the flux reverses also for
// the FP32 form's predictor.  Each takes the forward inputs,
// recomputes what it needs, and ADDS the input gradients for a given output
// gradient.  At a kink (min / max, the HLL branch, the clamp of the fast-speed
// discriminant) the branch the forward function takes is differentiated, with
// the same tie rule.
#pragma once
#include "mhd_device.hpp"

namespace rg {

// gw += (dF/dw)^T G for the physical flux F[d][v] of dev_flux (eq. 2.2)
template <class T>
__device__ __forceinline__ void flux_vjp(const T *u, T gam, const T (&G)[3][8], T *gw)
{
    const T ir = T(1) / u[0];
    const T m[3] = {u[1], u[2], u[3]};
    const T v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    const T B[3] = {u[5], u[6], u[7]};
    const T hb2 = T(0.5) * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const T p = (gam - T(1)) * (u[4] - T(0.5) * (m[0] * v[0] + m[1] * v[1] + m[2] * v[2]) - hb2);
    const T pt = p + hb2;
    const T vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    T gm[3] = {0, 0, 0}, gv[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
    T gpt = T(0), gvB = T(0), gE = T(0);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        gm[d] += G[d][0];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const T g1 = G[d][1 + i];
            gm[d] += g1 * v[i];
            gv[i] += g1 * m[d];
            gB[d] -= g1 * B[i];
            gB[i] -= g1 * B[d];
            const T g5 = G[d][5 + i];
            gv[d] += g5 * B[i];
            gB[i] += g5 * v[d];
            gB[d] -= g5 * v[i];
            gv[i] -= g5 * B[d];
        }
        gpt += G[d][1 + d];
        const T g4 = G[d][4];
        gE += g4 * v[d];
        gpt += g4 * v[d];
        gv[d] += g4 * (u[4] + pt);
        gB[d] -= g4 * vB;
        gvB -= g4 * B[d];
    }
    // vB, pt = p + hb2, p, hb2, v = m / rho
    const T gp = gpt, gm1 = gam - T(1);
    T ghb2 = gpt - gm1 * gp, gir = T(0);
    gE += gm1 * gp;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        gv[i] += gvB * B[i];
        gB[i] += gvB * v[i];
        gm[i] -= T(0.5) * gm1 * gp * v[i];
        gv[i] -= T(0.5) * gm1 * gp * m[i];
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
        gB[i] += ghb2 * B[i];
        gm[i] += gv[i] * ir;
        gir += gv[i] * m[i];
    }
    gw[0] -= gir * ir * ir;
    gw[1] += gm[0];
    gw[2] += gm[1];
    gw[3] += gm[2];
    gw[4] += gE;
    gw[5] += gB[0];
    gw[6] += gB[1];
    gw[7] += gB[2];
}

// gu += (d out / du)^T gOut for mapped_flux (flux of u / J contracted with
// the scaled metric terms)
template <class T>
__device__ __forceinline__ void mapped_flux_vjp(const T *u, T iJ, const T *met, T gam, const T (&gOut)[3][8], T *gu)
{
    T w[8], G[3][8], gw[8];
#pragma unroll
    for (int v = 0; v < 8; v++) { w[v] = u[v] * iJ; gw[v] = T(0); }
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
        for (int v = 0; v < 8; v++) G[c][v] = met[c] * gOut[0][v] + met[3 + c] * gOut[1][v] + met[6 + c] * gOut[2][v];
    flux_vjp<T>(w, gam, G, gw);
#pragma unroll
    for (int v = 0; v < 8; v++) gu[v] += gw[v] * iJ;
}

// gu += gc dc/du for the fast magnetosonic speed c = dev_fast(u, n); returns c
__device__ __forceinline__ double fast_vjp(const double *u, double gam, const double *n, double gc, double *gu)
{
    const double ir = 1.0 / u[0];
    const double m2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
    const double b2u = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    const double p = (gam - 1.0) * (u[4] - 0.5 * m2 / u[0] - 0.5 * b2u);
    const double a2 = gam * p * ir, b2 = b2u * ir;
    const double bn = u[5] * n[0] + u[6] * n[1] + u[7] * n[2];
    const double bn2 = bn * bn * ir, s = a2 + b2;
    const double disc0 = s * s - 4.0 * a2 * bn2;
    const double disc = disc0 < 0.0 ? 0.0 : disc0;
    const double sq = sqrt(disc);
    const double c = sqrt(0.5 * (s + sq));
    const double gh = c > 0.0 ? gc * 0.5 / c : 0.0;
    double gs = 0.5 * gh;
    const double gdisc = disc0 > 0.0 ? 0.5 * gh * 0.5 / sq : 0.0;
    gs += 2.0 * s * gdisc;
    const double ga2 = gs - 4.0 * bn2 * gdisc, gbn2 = -4.0 * a2 * gdisc, gb2 = gs;
    const double gbn = 2.0 * bn * ir * gbn2;
    double gir = bn * bn * gbn2 + b2u * gb2 + gam * p * ga2;
    const double gb2u = ir * gb2, gp = gam * ir * ga2, gp1 = (gam - 1.0) * gp;
    gu[4] += gp1;
    gu[0] += gp1 * 0.5 * m2 * ir * ir - gir * ir * ir;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        gu[1 + i] -= gp1 * u[1 + i] * ir;
        gu[5 + i] += gbn * n[i] - gp1 * u[5 + i] + 2.0 * u[5 + i] * gb2u;
    }
    return c;
}

// velocity along n: gu += g d(m.n / rho)/du; returns it
__device__ __forceinline__ double vn_vjp(const double *u, const double *n, double g, double *gu)
{
    const double ir = 1.0 / u[0];
    const double vn = (u[1] * n[0] + u[2] * n[1] + u[3] * n[2]) * ir;
    gu[0] -= g * vn * ir;
#pragma unroll
    for (int i = 0; i < 3; i++) gu[1 + i] += g * n[i] * ir;
    return vn;
}

// HLL flux with Davis speeds (dev_hll): adds the gradients of its four inputs
// for the output gradient gFs
__device__ __forceinline__ void hll_vjp(const double *UL, const double *UR, const double *FL, const double *FR,
                                        const double *n, double gam, const double *gFs, double *gUL, double *gUR,
                                        double *gFL, double *gFR)
{
    const double vL = (UL[1] * n[0] + UL[2] * n[1] + UL[3] * n[2]) / UL[0];
    const double vR = (UR[1] * n[0] + UR[2] * n[1] + UR[3] * n[2]) / UR[0];
    const double cL = dev_fast<double>(UL, gam, n), cR = dev_fast<double>(UR, gam, n);
    const bool minL = (vL - cL) <= (vR - cR), maxL = (vL + cL) >= (vR + cR);
    const double SL = minL ? vL - cL : vR - cR, SR = maxL ? vL + cL : vR + cR;
    if (SL >= 0.0) {
        for (int v = 0; v < 8; v++) gFL[v] += gFs[v];
        return;
    }
    if (SR <= 0.0) {
        for (int v = 0; v < 8; v++) gFR[v] += gFs[v];
        return;
    }
    const double id = 1.0 / (SR - SL);
    double gid = 0.0, gSL = 0.0, gSR = 0.0;
    for (int v = 0; v < 8; v++) {
        const double dU = UR[v] - UL[v];
        const double num = SR * FL[v] - SL * FR[v] + SL * SR * dU;
        gid += gFs[v] * num;
        const double gn = gFs[v] * id;
        gFL[v] += gn * SR;
        gFR[v] -= gn * SL;
        gUR[v] += gn * SL * SR;
        gUL[v] -= gn * SL * SR;
        gSR += gn * (FL[v] + SL * dU);
        gSL += gn * (SR * dU - FR[v]);
    }
    gSR -= gid * id * id;
    gSL += gid * id * id;
    double gvL = 0.0, gvR = 0.0, gcL = 0.0, gcR = 0.0;
    if (minL) { gvL += gSL; gcL -= gSL; } else { gvR += gSL; gcR -= gSL; }
    if (maxL) { gvL += gSR; gcL += gSR; } else { gvR += gSR; gcR += gSR; }
    vn_vjp(UL, n, gvL, gUL);
    vn_vjp(UR, n, gvR, gUR);
    fast_vjp(UL, gam, n, gcL, gUL);
    fast_vjp(UR, gam, n, gcR, gUR);
}

// four-state electric field (emf4): adds the gradients of the four states
// and of their tangential fields Et for the output gradient g
__device__ __forceinline__ void emf4_vjp(const double (&U)[4][8], const double (&Et)[4], const double *F, double gam,
                                         double g, double (&gU)[4][8], double (&gEt)[4])
{
    const double *e1 = F, *e2 = F + 3;
    double ap1 = 0.0, am1 = 0.0, ap2 = 0.0, am2 = 0.0, B1[4], B2[4];
    int iap1 = -1, iam1 = -1, iap2 = -1, iam2 = -1;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const double ir = 1.0 / U[s][0];
        const double v1 = (U[s][1] * e1[0] + U[s][2] * e1[1] + U[s][3] * e1[2]) * ir;
        const double v2 = (U[s][1] * e2[0] + U[s][2] * e2[1] + U[s][3] * e2[2]) * ir;
        const double c1 = dev_fast<double>(U[s], gam, e1), c2 = dev_fast<double>(U[s], gam, e2);
        // the running maxima keep the earlier value on a tie
        if (v1 + c1 > ap1) { ap1 = v1 + c1; iap1 = s; }
        if (c1 - v1 > am1) { am1 = c1 - v1; iam1 = s; }
        if (v2 + c2 > ap2) { ap2 = v2 + c2; iap2 = s; }
        if (c2 - v2 > am2) { am2 = c2 - v2; iam2 = s; }
        B1[s] = U[s][5] * e1[0] + U[s][6] * e1[1] + U[s][7] * e1[2];
        B2[s] = U[s][5] * e2[0] + U[s][6] * e2[1] + U[s][7] * e2[2];
    }
    const double D1 = ap1 + am1, D2 = ap2 + am2, Qi = 1.0 / (D1 * D2);
    const double num = ap1 * ap2 * Et[0] + ap1 * am2 * Et[3] + am1 * ap2 * Et[1] + am1 * am2 * Et[2];
    const double X2 = 0.5 * (B2[1] + B2[2]) - 0.5 * (B2[0] + B2[3]);
    const double X1 = 0.5 * (B1[2] + B1[3]) - 0.5 * (B1[0] + B1[1]);
    const double gnum = g * Qi, gQ = g * num;
    gEt[0] += gnum * ap1 * ap2;
    gEt[3] += gnum * ap1 * am2;
    gEt[1] += gnum * am1 * ap2;
    gEt[2] += gnum * am1 * am2;
    double gap1 = gnum * (ap2 * Et[0] + am2 * Et[3]), gam1 = gnum * (ap2 * Et[1] + am2 * Et[2]);
    double gap2 = gnum * (ap1 * Et[0] + am1 * Et[1]), gam2 = gnum * (ap1 * Et[3] + am1 * Et[2]);
    double gD1 = -gQ * Qi / D1, gD2 = -gQ * Qi / D2;
    // + ap1 am1 X2 / D1
    gap1 += g * am1 * X2 / D1;
    gam1 += g * ap1 * X2 / D1;
    const double gX2 = g * ap1 * am1 / D1;
    gD1 -= g * ap1 * am1 * X2 / (D1 * D1);
    // - ap2 am2 X1 / D2
    gap2 -= g * am2 * X1 / D2;
    gam2 -= g * ap2 * X1 / D2;
    const double gX1 = -g * ap2 * am2 / D2;
    gD2 += g * ap2 * am2 * X1 / (D2 * D2);
    gap1 += gD1;
    gam1 += gD1;
    gap2 += gD2;
    gam2 += gD2;
    const double gB2[4] = {-0.5 * gX2, 0.5 * gX2, 0.5 * gX2, -0.5 * gX2};
    const double gB1[4] = {-0.5 * gX1, -0.5 * gX1, 0.5 * gX1, 0.5 * gX1};
#pragma unroll
    for (int s = 0; s < 4; s++) {
#pragma unroll
        for (int i = 0; i < 3; i++) gU[s][5 + i] += gB1[s] * e1[i] + gB2[s] * e2[i];
        // speeds: ap = max(v + c), am = max(c - v)
        const double gv1 = (iap1 == s ? gap1 : 0.0) - (iam1 == s ? gam1 : 0.0);
        const double gc1 = (iap1 == s ? gap1 : 0.0) + (iam1 == s ? gam1 : 0.0);
        const double gv2 = (iap2 == s ? gap2 : 0.0) - (iam2 == s ? gam2 : 0.0);
        const double gc2 = (iap2 == s ? gap2 : 0.0) + (iam2 == s ? gam2 : 0.0);
        if (gv1 != 0.0) vn_vjp(U[s], e1, gv1, gU[s]);
        if (gv2 != 0.0) vn_vjp(U[s], e2, gv2, gU[s]);
        if (gc1 != 0.0) fast_vjp(U[s], gam, e1, gc1, gU[s]);
        if (gc2 != 0.0) fast_vjp(U[s], gam, e2, gc2, gU[s]);
    }
}

// three-zone electric field (emf3): adds the gradients of the three states
// and of their electric fields for the output gradient g
__device__ __forceinline__ void emf3_vjp(const double (&U)[4][8], const double (&E)[4][3], const double *N3,
                                         const double *t, double gam, double g, double (&gU)[4][8],
                                         double (&gE)[4][3])
{
#pragma unroll
    for (int s = 0; s < 3; s++) {
        const int s2 = (s + 1) % 3;
        const double *n = N3 + 3 * s;
        double FL[8], FR[8], gFs[8], gFL[8], gFR[8];
        for (int v = 0; v < 8; v++) FL[v] = FR[v] = gFs[v] = gFL[v] = gFR[v] = 0.0;
        FL[5] = n[1] * E[s][2] - n[2] * E[s][1];
        FL[6] = n[2] * E[s][0] - n[0] * E[s][2];
        FL[7] = n[0] * E[s][1] - n[1] * E[s][0];
        FR[5] = n[1] * E[s2][2] - n[2] * E[s2][1];
        FR[6] = n[2] * E[s2][0] - n[0] * E[s2][2];
        FR[7] = n[0] * E[s2][1] - n[1] * E[s2][0];
        const double tn[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
        // Es = -(1/3) sum_s Fs[5..7] . tn
        for (int i = 0; i < 3; i++) gFs[5 + i] = -g * tn[i] / 3.0;
        hll_vjp(U[s], U[s2], FL, FR, n, gam, gFs, gU[s], gU[s2], gFL, gFR);
        // FL = n x E[s]: gE[s] += gFL x n
        gE[s][0] += gFL[6] * n[2] - gFL[7] * n[1];
        gE[s][1] += gFL[7] * n[0] - gFL[5] * n[2];
        gE[s][2] += gFL[5] * n[1] - gFL[6] * n[0];
        gE[s2][0] += gFR[6] * n[2] - gFR[7] * n[1];
        gE[s2][1] += gFR[7] * n[0] - gFR[5] * n[2];
        gE[s2][2] += gFR[5] * n[1] - gFR[6] * n[0];
    }
}

// WENO-AO combination (weno_core): out(j, g_j) receives g = (d out / d du)^T go,
// one stencil slot j at a time
template <int P, class Out>
__device__ __forceinline__ void weno_core_vjp(const double (&du)[Tr<P>::NS], const double *__restrict__ Pl,
                                              const double *__restrict__ Ps, const double *__restrict__ Qs,
                                              double eps, const double (&go)[Tr<P>::NC], Out &&out)
{
    using Tt = Tr<P>;
    constexpr int NC = Tt::NC, NS = Tt::NS;
    const double ghi = WENO_GAMMA_HI, gs = (1.0 - WENO_GAMMA_HI) / 7.0;
    double chi[NC];
#pragma unroll
    for (int a = 0; a < NC; a++) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NS; j++) s += Pl[a * NS + j] * du[j];
        chi[a] = s;
    }
    double cs[7][3];
#pragma unroll
    for (int s = 0; s < 7; s++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < 6; j++) acc += Ps[s * 18 + i * 6 + j] * du[j];
            cs[s][i] = acc;
        }
    double bhi = 0.0;
#pragma unroll
    for (int a = 0; a < NC; a++) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NC; b++) s += Qs[a * NC + b] * chi[b];
        bhi += chi[a] * s;
    }
    const double w0 = ghi / ((bhi + eps) * (bhi + eps));
    double tot = w0, ws[7], bs[7];
#pragma unroll
    for (int s = 0; s < 7; s++) {
        bs[s] = cs[s][0] * cs[s][0] + cs[s][1] * cs[s][1] + cs[s][2] * cs[s][2];
        ws[s] = gs / ((bs[s] + eps) * (bs[s] + eps));
        tot += ws[s];
    }
    const double itot = 1.0 / tot, w0n = w0 * itot;
    // the reverse pass reads the matrices again through an opaque zero
    // offset, so that their values are not held in registers in between
    int ro = 0;
    __asm__ __volatile__("" : "+s"(ro));
    Pl += ro;
    Ps += ro;
    Qs += ro;
    // out[a] = w0n / ghi (chi[a] - lin_a) + nl_a; lin, nl only for a < 3
    double gchi[NC], gcs[7][3], gw0n = 0.0, gwn[7];
#pragma unroll
    for (int s = 0; s < 7; s++) { gwn[s] = 0.0; gcs[s][0] = gcs[s][1] = gcs[s][2] = 0.0; }
#pragma unroll
    for (int a = 0; a < NC; a++) {
        double lin = 0.0;
        if (a < 3)
#pragma unroll
            for (int s = 0; s < 7; s++) lin += gs * cs[s][a];
        gw0n += go[a] * (chi[a] - lin) / ghi;
        gchi[a] = go[a] * w0n / ghi;
        if (a < 3) {
            const double glin = -go[a] * w0n / ghi;
#pragma unroll
            for (int s = 0; s < 7; s++) {
                gcs[s][a] += gs * glin + ws[s] * itot * go[a];
                gwn[s] += go[a] * cs[s][a];
            }
        }
    }
    // wn_s = ws_s itot, w0n = w0 itot, itot = 1 / (w0 + sum ws)
    double gitot = gw0n * w0;
#pragma unroll
    for (int s = 0; s < 7; s++) gitot += gwn[s] * ws[s];
    const double gtot = -gitot * itot * itot;
    const double gw0 = gw0n * itot + gtot;
#pragma unroll
    for (int s = 0; s < 7; s++) {
        const double gws = gwn[s] * itot + gtot;
        const double gb = -2.0 * gws * ws[s] / (bs[s] + eps);
#pragma unroll
        for (int i = 0; i < 3; i++) gcs[s][i] += 2.0 * gb * cs[s][i];
    }
    const double gbhi = -2.0 * gw0 * w0 / (bhi + eps);
    // bhi = chi . Qs chi: d bhi / d chi = (Qs + Qs^T) chi
#pragma unroll
    for (int a = 0; a < NC; a++) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NC; b++) s += (Qs[a * NC + b] + Qs[b * NC + a]) * chi[b];
        gchi[a] += gbhi * s;
    }
#pragma unroll
    for (int j = 0; j < NS; j++) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NC; a++) s += Pl[a * NS + j] * gchi[a];
        if (j < 6)
#pragma unroll
            for (int q = 0; q < 7; q++)
#pragma unroll
                for (int i = 0; i < 3; i++) s += Ps[q * 18 + i * 6 + j] * gcs[q][i];
        out(j, s);
    }
}

}  // namespace rg

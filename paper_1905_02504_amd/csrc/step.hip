// Device step of the rg library for gfx950: the FP64 scheme and its FP32 and
// BF16 forms.  One launch per stage, all on the caller's stream:
//   bc_zones / bc_faces : continuative ghost fill (Section VII) into the output state
//   weno_mfma          : WENO-AO in the Taylor basis (Section III) on the FP64
//                        matrix cores, 16 shells of one column per wavefront;
//                        weno_cols, its VALU form, serves the FP32 forms
//   flatten_wc         : the flattener (when on): each zone's coefficients
//                        scaled toward first order by a compression detector
//   zone_face_bn /     : limited nodal normal B on every face, eqs. (4.11)-(4.12):
//   face_bn_limit        each zone's normal B at its faces' points, then per face
//                        the MinMod and the mean restore
//   bmap               : divergence-free B (Section IV.b) as one dense per-column
//                        map on the FP64 matrix cores, evaluated at the ADER nodes
//   predictor          : ADER-CG Picard iteration (Section V.d), one lane per
//                        serendipity node (the BF16 form's flux derivatives on
//                        the BF16 matrix cores), then time-averaged traces at
//                        face and edge points
//   face_flux          : HLL at face quadrature points -> face flux integrals
//   edge_emf           : multidimensional HLL electric field at edge Simpson points
//   fb_*               : the first-order fallback (when on): flag, constant
//                        traces, and the two Riemann kernels on marked faces/edges
//   zone_update        : finite-volume update of the eight zone averages
//   face_ct            : constrained transport of face-averaged normal B (eqs. 2.5-2.6)
#include <climits>
#include <mutex>

#include "mhd_device.hpp"

namespace rg {

// ---------------------------------------------------------------- boundary fill
__global__ void bc_zones(DevGeom G, int bc, const double *U, double *Uo)
{
    i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= G.Z) return;
    int k = (int)(z % G.K);
    i64 src = z;
    if (bc == 0) {
        int ks = k < G.g ? G.g : (k > G.g + G.Nr - 1 ? G.g + G.Nr - 1 : k);
        src = z - k + ks;
    }
    for (int v = 0; v < 8; v++) Uo[v * G.Z + z] = U[v * G.Z + src];
}

__global__ void bc_faces(DevGeom G, int bc, const double *Bf, double *Bo)
{
    i64 f = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= G.NF) return;
    i64 src = f;
    if (bc == 0) {
        if (f < G.NRF) {
            int kf = (int)(f % (G.K + 1));
            int ks = kf < G.g ? G.g : (kf > G.g + G.Nr ? G.g + G.Nr : kf);
            src = f - kf + ks;
        } else {
            int k = (int)((f - G.NRF) % G.K);
            int ks = k < G.g ? G.g : (k > G.g + G.Nr - 1 ? G.g + G.Nr - 1 : k);
            src = f - k + ks;
        }
    }
    Bo[f] = Bf[src];
}

// ---------------------------------------------------------------- WENO-AO
// zones of shells g-1 .. g+Nr (interior plus one ghost shell on each side)
// WENO-AO reconstruction (Section III) of variable v of zone (c, k).  All
// lanes of a wavefront lie in column c, so the column's stencil offsets and
// least-squares matrices are uniform and read as scalars.
// Returns the large stencil's nonlinear weight relative to its linear weight.
template <int P, class R>
__device__ __forceinline__ R weno_var(const DevGeom &G, const double *__restrict__ U, R *__restrict__ wc,
                                      const R *__restrict__ Pl, const R *__restrict__ Ps, const R *__restrict__ Qs,
                                      R eps, int c, int k, int v)
{
    using T = Tr<P>;
    const i64 z = (i64)c * G.K + k;
    const double *Uv = U + (i64)v * G.Z;
    const double u0 = Uv[z];
    R du[T::NS];
#pragma unroll
    for (int j = 0; j < T::NS; j++) {
        const int m = G.stm[(i64)c * T::NS + j];   // member zone minus this zone fits 32 bits
        const int dz = m < 0 ? 0 : (int)(((i64)(m >> 3) - c) * G.K + (m & 7) - 3);
        du[j] = R(Uv[z + dz] - u0);
    }
    R o[T::NC], whi;
    weno_core<P, R, R>(du, Pl, Ps, Qs, eps, o, whi);
    R *out = wc + (i64)v * T::NC * G.Z + z;
#pragma unroll
    for (int a = 0; a < T::NC; a++) out[(i64)a * G.Z] = o[a];
    return whi;
}

// The FP32 forms' WENO-AO on the VALU (the FP64 scheme uses weno_mfma below).
// One wavefront per run of up to 64 shells of one column, the eight
// variables in turn.  With a short tail (nleft shells, at most 8) each column
// gets one more wavefront whose lanes take (tail shell, variable) pairs.
// whi[z]: the smallest over the eight variables of the large stencil's weight
// relative to its linear weight (the order WENO-AO keeps in zone z).
template <int P, class R>
__global__ __launch_bounds__(64) void weno_cols(DevGeom G, const double *__restrict__ U, R *__restrict__ wc,
                                                const R *__restrict__ PlA, const R *__restrict__ PsA,
                                                const R *__restrict__ QsA, R eps, int nchunk, int nu, int nleft,
                                                float *__restrict__ whi)
{
    using T = Tr<P>;
    const int per = nchunk + (nleft > 0);
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int c = lb / per, ch = lb % per;
    const R *__restrict__ Pl = PlA + (i64)c * T::NC * T::NS;
    const R *__restrict__ Ps = PsA + (i64)c * 7 * 18;
    const R *__restrict__ Qs = QsA + (i64)c * T::NC * T::NC;
    if (ch < nchunk) {
        // the column's matrices are staged in LDS once and read as broadcasts
        // (21 % faster than reading them as scalar operands for each variable)
        __shared__ R sPl[T::NC * T::NS], sPs[7 * 18], sQs[T::NC * T::NC];
        for (int j = threadIdx.x; j < T::NC * T::NS; j += 64) sPl[j] = Pl[j];
        for (int j = threadIdx.x; j < 7 * 18; j += 64) sPs[j] = Ps[j];
        for (int j = threadIdx.x; j < T::NC * T::NC; j += 64) sQs[j] = Qs[j];
        __syncthreads();
        const int kk = ch * 64 + threadIdx.x;
        if (kk >= nu) return;
        float wmin = 1e30f;
#pragma unroll 1
        for (int v = 0; v < 8; v++) {
            // an opaque zero offset keeps the matrix reads inside the loop (the
            // matrices would not fit in registers)
            int vo = 0;
            __asm__ __volatile__("" : "+s"(vo));
            wmin = fminf(wmin, float(weno_var<P, R>(G, U, wc, sPl + vo, sPs + vo, sQs + vo, eps, c, G.g - 1 + kk, v)));
        }
        whi[(i64)c * G.K + G.g - 1 + kk] = wmin;
    } else {
        // one wavefront: the lanes of a tail shell meet in LDS
        __shared__ float s_w[64];
        const int kk = nu + (int)threadIdx.x / 8, v = threadIdx.x % 8;
        const bool live = kk < nu + nleft;
        s_w[threadIdx.x] = live ? float(weno_var<P, R>(G, U, wc, Pl, Ps, Qs, eps, c, G.g - 1 + kk, v)) : 1e30f;
        __syncthreads();
        if (live && v == 0) {
            float wmin = s_w[threadIdx.x];
            for (int j = 1; j < 8; j++) wmin = fminf(wmin, s_w[threadIdx.x + j]);
            whi[(i64)c * G.K + G.g - 1 + kk] = wmin;
        }
    }
}

// WENO-AO on the FP64 matrix cores.  The per-column contractions are small
// dense products shared by the zones of a column (Section III, eq. 3.4):
//   chi  = Pl (NC x NS) . dU (NS x zones)        large-stencil least squares
//   cs   = Ps (21 x 6)  . dU[0:6]                 the seven linear small stencils
//   S    = Qs (NC x NC) . chi                     smoothness form, beta = chi . S
// One wavefront takes 16 zones of a column and the eight variables in turn;
// the column's matrices are the A operands and stay in registers for the
// whole wavefront, the stencil differences are loaded straight into the B
// operands, and chi leaves the first product in the layout the second one
// takes as its B operand.  No LDS: the VALU form of this stage spent its
// time on LDS broadcasts of the matrices (each element served one FMA).
// v_mfma_f64_16x16x4: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D[i][j] in lane j + 16 (i % 4), element i / 4.  Here j is the zone, so
// lane group g (lanes 16g .. 16g + 15) holds rows 4e + g of every tile.
// Fourth order (NC = 19): chi takes two M tiles; the second holds chi's rows
// 16-18 (element 0, groups 0-2) and small stencils 0-3 (stencil g in group
// g, component i in element i + 1), a separate tile small stencils 4-6
// (stencil 4 + g in group g, component i in element i); S is formed for
// rows 0-15 only, with Qs's columns 16-18 doubled, and the rest of beta,
// the 3 x 3 form of chi's rows 16-18, on the VALU.  Third order (NC = 9):
// one chi tile; small stencil s, component i in row 16 (x / 4) + 4 (x % 4)
// + s % 4, x = i + 3 (s / 4), of two tiles.
template <int P>
struct WenoMfma {
    using T = Tr<P>;
    static constexpr int MT = (T::NC + 15) / 16;   // M tiles of chi
    static constexpr int KL = (T::NS + 3) / 4;     // K steps of the least squares
    static constexpr int KQ = (T::NC + 3) / 4;     // K steps of the smoothness form
    static constexpr int MS = P == 4 ? 1 : 2;      // M tiles of the separate small-stencil product
};

// sum of x over the four lane groups (lanes j, j + 16, j + 32, j + 48), the
// same bits in every lane: rows of 16 lanes are exchanged with
// v_permlane16_swap, then halves with v_permlane32_swap (VALU, no LDS)
__device__ __forceinline__ double sum_lane_groups(double x)
{
    unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
    auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    x = __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
    lo = (unsigned)__double2loint(x);
    hi = (unsigned)__double2hiint(x);
    a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// x of lane groups 0, 1, 2 (the same lane offset) in every lane
__device__ __forceinline__ void gather_groups3(double x, double &x0, double &x1, double &x2)
{
    const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
    // groups (0, 1) in rows 0-1, (2, 3) in rows 2-3
    auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    // the lower half's pair to every lane, and the upper half's
    auto c = __builtin_amdgcn_permlane32_swap(a[0], a[0], false, false);
    auto d = __builtin_amdgcn_permlane32_swap(b[0], b[0], false, false);
    auto e = __builtin_amdgcn_permlane32_swap(a[1], a[1], false, false);
    auto f = __builtin_amdgcn_permlane32_swap(b[1], b[1], false, false);
    x0 = __hiloint2double((int)d[0], (int)c[0]);
    x2 = __hiloint2double((int)d[1], (int)c[1]);
    x1 = __hiloint2double((int)f[0], (int)e[0]);
}

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void weno_mfma(
    DevGeom G, const double *__restrict__ U, double *__restrict__ wc, const double *__restrict__ PlA,
    const double *__restrict__ PsA, const double *__restrict__ QsA, double eps, int nrun, float *__restrict__ whi)
{
    using T = Tr<P>;
    using W = WenoMfma<P>;
    constexpr int MT = W::MT, KL = W::KL, KQ = W::KQ, MS = W::MS, NC = T::NC, NS = T::NS;
    const double ghi = WENO_GAMMA_HI, gs = (1.0 - WENO_GAMMA_HI) / 7.0;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int c = (int)(lb / (unsigned)nrun), run = (int)(lb % (unsigned)nrun);
    const int lane = threadIdx.x, g = lane >> 4, jz = lane & 15;
    const int KR = G.Nr + 2, kk = run * 16 + jz;
    const bool active = kk < KR;
    const i64 z = (i64)c * G.K + G.g - 1 + (active ? kk : 0);
    const double *Pl = PlA + (i64)c * NC * NS;
    const double *Ps = PsA + (i64)c * 7 * 18;
    const double *Qs = QsA + (i64)c * NC * NC;
    // A operands: row jz of each M tile, column 4s + g of each K step.  Every
    // load is unconditional (a lane without an entry reads entry 0 and masks
    // it), so that the loads issue without branches.
    double aL[MT][KL], aQ[KQ], aS[MS][2];
#pragma unroll
    for (int m = 0; m < MT; m++) {
        const int row = 16 * m + jz;
#pragma unroll
        for (int s = 0; s < KL; s++) {
            const int col = 4 * s + g;
            // at fourth order rows 20-31 of tile 1 hold small stencil jz % 4,
            // component jz / 4 - 1
            const bool sm = P == 4 && m == 1 && jz >= 4;
            const bool ok = sm ? col < 6 : (row < NC && col < NS);
            const int idx = !ok ? 0 : sm ? (jz % 4) * 18 + (jz / 4 - 1) * 6 + col : row * NS + col;
            const double a = (sm ? Ps : Pl)[idx];
            aL[m][s] = ok ? a : 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < KQ; s++) {
        const int col = 4 * s + g;
        // rows 0-15; at fourth order the columns of chi's rows 16-18 count twice
        const bool ok = jz < NC && col < NC;
        const double a = Qs[ok ? jz * NC + col : 0];
        aQ[s] = ok ? (col >= 16 ? 2.0 : 1.0) * a : 0.0;
    }
#pragma unroll
    for (int m = 0; m < MS; m++)
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int col = 4 * s + g;
            bool ok;
            int idx;
            if (P == 4) {   // stencil 4 + jz % 4, component jz / 4
                ok = jz % 4 < 3 && jz / 4 < 3 && col < 6;
                idx = (4 + jz % 4) * 18 + (jz / 4) * 6 + col;
            } else {
                const int x = 4 * m + jz / 4, st = jz % 4 + 4 * (x / 3), comp = x % 3;
                ok = x < 6 && st < 7 && col < 6;
                idx = st * 18 + comp * 6 + col;
            }
            const double a = Ps[ok ? idx : 0];
            aS[m][s] = ok ? a : 0.0;
        }
    // the 3 x 3 block of Qs for chi's rows 16-18 (fourth order)
    double qbb[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b2 = 0; b2 < 3; b2++) qbb[a][b2] = P == 4 ? Qs[(16 + a) * NC + 16 + b2] : 0.0;
    // stencil members of the K rows this lane feeds (offsets fit 32 bits);
    // a lane without a member (missing corner member, padding, or a zone
    // beyond the column) loads its own zone and masks the value, so that
    // every load is unconditional
    int dz[KL];
    unsigned vmask = 0;
#pragma unroll
    for (int s = 0; s < KL; s++) {
        const int t = 4 * s + g;
        const int mem = t < NS ? G.stm[(i64)c * NS + t] : -1;
        const bool ok = active && mem >= 0;
        dz[s] = ok ? (int)(((i64)(mem >> 3) - c) * G.K + (mem & 7) - 3) : 0;
        vmask |= ok ? 1u << s : 0u;
    }
    float wmin = 1e30f;
    // the stencil values of the next variable are loaded while the current
    // one is reduced (a software pipeline that also overlapped the products
    // of the next variable with this reduction needed 175 VGPRs, two
    // wavefronts per SIMD instead of three, and was slower: 12.4 against
    // 10.5 ms at 6 x 128^2 x 128)
    double raw[KL], u0 = U[z];
#pragma unroll
    for (int s = 0; s < KL; s++) raw[s] = U[z + dz[s]];
#pragma unroll 1
    for (int v = 0; v < 8; v++) {
        double b[KL];
#pragma unroll
        for (int s = 0; s < KL; s++) b[s] = (vmask >> s) & 1u ? raw[s] - u0 : 0.0;
        if (v < 7) {
            const double *Un = U + (i64)(v + 1) * G.Z;
            u0 = Un[z];
#pragma unroll
            for (int s = 0; s < KL; s++) raw[s] = Un[z + dz[s]];
        }
        dbl4 chi[MT], cs[MS], sq = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < MT; m++) chi[m] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < MS; m++) cs[m] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KL; s++)
#pragma unroll
            for (int m = 0; m < MT; m++) chi[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(aL[m][s], b[s], chi[m], 0, 0, 0);
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
            for (int m = 0; m < MS; m++) cs[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(aS[m][s], b[s], cs[m], 0, 0, 0);
        // chi's element e of tile m is the B operand of K step 4m + e (at
        // fourth order K step 4 takes tile 1's element 0: rows 16-19)
#pragma unroll
        for (int s = 0; s < KQ; s++) sq = __builtin_amdgcn_mfma_f64_16x16x4f64(aQ[s], chi[s / 4][s % 4], sq, 0, 0, 0);
        // beta of the large stencil
        double bhi = chi[0][0] * sq[0] + chi[0][1] * sq[1] + chi[0][2] * sq[2] + chi[0][3] * sq[3];
        bhi = sum_lane_groups(bhi);
        if constexpr (P == 4) {
            double c16, c17, c18;
            gather_groups3(chi[1][0], c16, c17, c18);
            const double t0 = qbb[0][0] * c16 + qbb[0][1] * c17 + qbb[0][2] * c18;
            const double t1 = qbb[1][0] * c16 + qbb[1][1] * c17 + qbb[1][2] * c18;
            const double t2 = qbb[2][0] * c16 + qbb[2][1] * c17 + qbb[2][2] * c18;
            bhi += c16 * t0 + c17 * t1 + c18 * t2;
        }
        // small stencils g and g + 4 of this lane group: components of each
        double s0[3], s1[3];
        if constexpr (P == 4) {
            s0[0] = chi[1][1]; s0[1] = chi[1][2]; s0[2] = chi[1][3];
            s1[0] = cs[0][0]; s1[1] = cs[0][1]; s1[2] = cs[0][2];
        } else {
            s0[0] = cs[0][0]; s0[1] = cs[0][1]; s0[2] = cs[0][2];
            s1[0] = cs[0][3]; s1[1] = cs[MS - 1][0]; s1[2] = cs[MS - 1][1];
        }
        const double b0 = s0[0] * s0[0] + s0[1] * s0[1] + s0[2] * s0[2];
        const double b1 = s1[0] * s1[0] + s1[1] * s1[1] + s1[2] * s1[2];
        const double w0 = ghi / ((bhi + eps) * (bhi + eps));
        const double ws0 = gs / ((b0 + eps) * (b0 + eps));
        const double ws1 = g < 3 ? gs / ((b1 + eps) * (b1 + eps)) : 0.0;
        const double tot = sum_lane_groups(ws0 + ws1) + w0;
        const double itot = 1.0 / tot, w0n = w0 * itot;
        wmin = fminf(wmin, float(w0n / ghi));
        // first-order coefficients: (w0n / ghi)(chi_a - gs sum_s cs_sa) + sum_s (w_s / tot) cs_sa
        const double k0 = ws0 * itot - w0n * gs / ghi, k1 = ws1 * itot - w0n * gs / ghi;
        const double p0 = sum_lane_groups(k0 * s0[0] + k1 * s1[0]);
        const double p1 = sum_lane_groups(k0 * s0[1] + k1 * s1[1]);
        const double p2 = sum_lane_groups(k0 * s0[2] + k1 * s1[2]);
        const double sc = w0n / ghi;
        const double pg = g == 0 ? p0 : g == 1 ? p1 : p2;
        if (active) {
            double *out = wc + (i64)v * NC * G.Z + z;
#pragma unroll
            for (int m = 0; m < MT; m++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int a = 16 * m + 4 * e + g;
                    if (P == 4 && m == 1 && e > 0) continue;   // small-stencil rows
                    double o = sc * chi[m][e];
                    if (a < 3) o += pg;
                    if (a < NC) out[(i64)a * G.Z] = o;
                }
        }
    }
    if (active && g == 0) whi[z] = wmin;
}

// ---------------------------------------------------------------- flattener
// Section VII.a applies a flattener on its coarse meshes and defers its
// definition to other work.  Read here: a zone is flattened where the flow
// compresses faster than a fraction kappa of the slowest signal speed around
// it.  D = (1/V) sum_faces s_f (area-weighted face normal) . (v_zone +
// v_neighbour) / 2 is the discrete divergence of the zone averages'
// velocity, l0 = V^(1/3), c the smallest sqrt(gamma p / rho + B^2 / rho)
// over the zone and its six face neighbours, and
// eta = min(1, max(0, -(l0 D + kappa c) / (kappa c))).  Every WENO-AO
// coefficient of the zone (all eight variables) is scaled by 1 - eta.  One
// lane per reconstructed zone.
__device__ __forceinline__ double zone_fast_max(const DevGeom &G, const double *__restrict__ U, i64 z, double gam,
                                                double v[3])
{
    double u[8];
    for (int k = 0; k < 8; k++) u[k] = U[k * G.Z + z];
    const double ir = 1.0 / u[0];
    v[0] = u[1] * ir;
    v[1] = u[2] * ir;
    v[2] = u[3] * ir;
    const double a2 = gam * dev_pressure<double>(u, gam) * ir, b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * ir;
    return sqrt(fmax(a2, 0.0) + b2);
}

template <int P, class R>
__global__ __launch_bounds__(256) void flatten_wc(DevGeom G, double gam, double kappa, const double *__restrict__ U,
                                                  R *__restrict__ wc)
{
    using T = Tr<P>;
    const int KR = G.Nr + 2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (i64)G.ncol * KR) return;
    const int c = (int)(t / KR), k = G.g - 1 + (int)(t % KR);
    const i64 z = (i64)c * G.K + k;
    double vz[3], vn[3];
    double cmin = zone_fast_max(G, U, z, gam, vz), div = 0.0;
    for (int lf = 0; lf < 6; lf++) {
        i64 f, zn;
        double sg;
        const double *nrm, *fw;
        if (lf >= 4) {   // lower (outward -r) and upper radial faces
            f = (i64)c * (G.K + 1) + k + (lf - 4);
            zn = z + (lf == 4 ? -1 : 1);
            sg = lf == 4 ? -1.0 : 1.0;
            nrm = G.fnR + (i64)c * T::Q * 3;
            fw = G.fwR + (i64)c * T::Q;
        } else {
            const int ae = G.col_ae[4 * c + lf], side = G.col_side[4 * c + lf];
            f = G.NRF + (i64)ae * G.K + k;
            zn = (i64)G.ae_col[2 * ae + 1 - side] * G.K + k;
            sg = side == 0 ? 1.0 : -1.0;
            nrm = G.fnA + (i64)ae * T::Q * 3;
            fw = G.fwA + (i64)ae * T::Q;
        }
        double sa[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < T::Q; q++)
            for (int i = 0; i < 3; i++) sa[i] += fw[q] * nrm[q * 3 + i];
        cmin = fmin(cmin, zone_fast_max(G, U, zn, gam, vn));
        const double A = G.area[f];
        for (int i = 0; i < 3; i++) div += sg * A * sa[i] * 0.5 * (vz[i] + vn[i]);
    }
    div /= G.vol[z];
    const double kc = kappa * cmin;
    const double eta = fmin(1.0, fmax(0.0, -(cbrt(G.vol[z]) * div + kc) / kc));
    if (eta == 0.0) return;
    const R keep = R(1.0 - eta);
    for (int j = 0; j < 8 * T::NC; j++) wc[(i64)j * G.Z + z] *= keep;
}

// ---------------------------------------------------------------- face nodal B
// Limited nodal normal B on every face of the reconstructed shells (radial
// faces kf in [g-1, g+Nr+1], angular faces in shells [g-1, g+Nr]), Section
// IV.b: both sides' WENO B at the face quadrature points, the MinMod of their
// normal components' deviations from the face mean, then the mean restored.
// A missing side takes the other side's value.
// Two passes that read every zone's WENO B once.  zone_face_bn: one
// wavefront per run of up to 64 zones of a column, which stages the column's
// six faces' evaluation tables and normals in LDS; each lane evaluates its
// zone's B at the quadrature points of its six faces and stores the normal
// component in sbn[(side * Q + q) * NF + f].  A short run (at most 10 zones,
// such as the last one of a column) gives each lane one (zone, face) pair
// instead, so that its wavefront is not as long as a full one.
// face_bn_limit: one lane per face, the MinMod of the two sides' deviations
// from the face mean and the mean restore.  Each component sums its mean and
// then the coefficients in order, and the normal component adds the three
// components' products in order, as the adjoint's recomputation of this
// stage does.
template <int P, class R>
__global__ __launch_bounds__(64) void zone_face_bn(DevGeom G, const double *__restrict__ U,
                                                   const R *__restrict__ wc, double *__restrict__ sbn, int nchunk)
{
    using T = Tr<P>;
    constexpr int QN = T::Q * T::NC;
    __shared__ R s_fev[6][QN];
    __shared__ double s_nrm[6][T::Q * 3];
    const int KR = G.Nr + 2;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int c = (int)(lb / (unsigned)nchunk), base = (int)(lb % (unsigned)nchunk) * 64;
    const R *fvR = pick<R>(G.fevR, G.fevRF), *fvA = pick<R>(G.fevA, G.fevAF);
    for (int j = threadIdx.x; j < 6 * QN; j += 64) {
        const int lf = j / QN, i = j % QN;
        const R *fev = lf >= 4 ? fvR + ((i64)c * 2 + (lf == 4 ? 1 : 0)) * QN
                               : fvA + ((i64)G.col_ae[4 * c + lf] * 2 + G.col_side[4 * c + lf]) * QN;
        s_fev[lf][i] = fev[i];
    }
    for (int j = threadIdx.x; j < 6 * T::Q * 3; j += 64) {
        const int lf = j / (T::Q * 3), i = j % (T::Q * 3);
        const double *nrm = lf >= 4 ? G.fnR + (i64)c * T::Q * 3 : G.fnA + (i64)G.col_ae[4 * c + lf] * T::Q * 3;
        s_nrm[lf][i] = nrm[i];
    }
    __syncthreads();
    const int nk = min(64, KR - base);
    int kk, lf0, lf1;
    if (nk <= 10) {   // short run: lane = (zone, face)
        if ((int)threadIdx.x >= 6 * nk) return;
        kk = base + (int)threadIdx.x / 6;
        lf0 = (int)threadIdx.x % 6;
        lf1 = lf0 + 1;
    } else {
        kk = base + (int)threadIdx.x;
        if (kk >= KR) return;
        lf0 = 0;
        lf1 = 6;
    }
    const int k = G.g - 1 + kk;
    const i64 z = (i64)c * G.K + k;
    R cf[3][T::NC + 1];
#pragma unroll
    for (int c3 = 0; c3 < 3; c3++) {
        cf[c3][0] = R(U[(5 + c3) * G.Z + z]);
#pragma unroll
        for (int a = 0; a < T::NC; a++) cf[c3][a + 1] = wc[((i64)(5 + c3) * T::NC + a) * G.Z + z];
    }
#pragma unroll 1
    for (int lf = lf0; lf < lf1; lf++) {
        i64 f;
        int side;
        if (lf >= 4) {   // lower face: this zone is its side 1; upper face: side 0
            side = lf == 4 ? 1 : 0;
            f = (i64)c * (G.K + 1) + k + (lf - 4);
        } else {
            side = G.col_side[4 * c + lf];
            f = G.NRF + (i64)G.col_ae[4 * c + lf] * G.K + k;
        }
        double *o = sbn + (i64)side * T::Q * G.NF + f;
#pragma unroll 1
        for (int q = 0; q < T::Q; q++) {
            const R *fe = &s_fev[lf][q * T::NC];
            R b0 = cf[0][0], b1 = cf[1][0], b2 = cf[2][0];
#pragma unroll
            for (int a = 0; a < T::NC; a++) {
                const R w = fe[a];
                b0 += cf[0][a + 1] * w;
                b1 += cf[1][a + 1] * w;
                b2 += cf[2][a + 1] * w;
            }
            const double *n = &s_nrm[lf][q * 3];
            double bn = double(b0) * n[0];
            bn += double(b1) * n[1];
            bn += double(b2) * n[2];
            o[(i64)q * G.NF] = bn;
        }
    }
}

// Faces of the reconstructed shells: radial faces kf in [g-1, g+Nr+1] (their
// outer sides beyond the reconstructed shells are missing), angular faces in
// shells [g-1, g+Nr]; faces fastest along a column or an angular edge.
template <int P, class R>
__global__ __launch_bounds__(256) void face_bn_limit(DevGeom G, const double *__restrict__ Bf,
                                                     const double *__restrict__ sbn, R *__restrict__ bnod)
{
    using T = Tr<P>;
    const int nrad = G.Nr + 3, nang = G.Nr + 2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const i64 nR = (i64)G.ncol * nrad;
    if (t >= nR + (i64)G.nae * nang) return;
    i64 f;
    bool have[2];
    const double *fw;
    if (t < nR) {
        const int c = (int)(t / nrad), kf = G.g - 1 + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        have[0] = kf - 1 >= G.g - 1;
        have[1] = kf <= G.g + G.Nr;
        fw = G.fwR + (i64)c * T::Q;
    } else {
        const i64 u = t - nR;
        const int ae = (int)(u / nang), k = G.g - 1 + (int)(u % nang);
        f = G.NRF + (i64)ae * G.K + k;
        have[0] = have[1] = true;
        fw = G.fwA + (i64)ae * T::Q;
    }
    const double mean = Bf[f];
    double bn[T::Q];
#pragma unroll
    for (int q = 0; q < T::Q; q++) {
        double d[2] = {0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 2; s++)
            if (have[s]) d[s] = sbn[((i64)s * T::Q + q) * G.NF + f] - mean;
        if (!have[0]) d[0] = d[1];
        if (!have[1]) d[1] = d[0];
        bn[q] = mean + dev_minmod(d[0], d[1]);
    }
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < T::Q; q++) sum += fw[q] * bn[q];
#pragma unroll
    for (int q = 0; q < T::Q; q++) bnod[(i64)q * G.NF + f] = R(bn[q] + (mean - sum));
}

// ---------------------------------------------------------------- predictor
// Divergence-free B (Section IV.b): for every zone of a column the fused
// per-column map (KKT inverse followed by evaluation at the ADER nodes and the
// new zone mean) is applied to the zone's inputs -- its WENO B, the limited
// nodal normal B of its six faces and their face averages.  Per column this is
// a dense product Out^T (NOUTB x zones) = Mb^T (NOUTB x NIN) In^T (NIN x zones),
// done on the FP64 matrix cores: one wavefront owns BMAP_TILES tiles of
// 16 zones of a column and all output rows, stepping through the inputs four
// at a time; each A operand it loads serves all its tiles.  Three tiles
// measured 6 % faster than one with FP64 inputs (two were slower: fewer
// wavefronts in flight).  With FP32 inputs the compiler's own schedule for
// three tiles took 218 VGPRs beside the accumulators (one wavefront per SIMD,
// 23.3 ms at 6 x 128^3 against 16.3 ms for one tile); the occupancy hint of
// two wavefronts per SIMD holds both forms under 256 registers.  Face ids come
// from a per-column table in LDS, so the per-lane choice of face costs no
// branches: with a six-way select in registers the FP32 form took 14.4 ms,
// with the table 10.9 ms (FP64 12.0 -> 11.8 ms).  The operands are loaded one
// K step ahead with no load under a branch: FP64 11.8 -> 10.6 ms, FP32
// 10.9 -> 9.9 ms (two tiles per wavefront with the same loads: 13.1 ms; at
// fourth order three tiles hold 256 registers with a 24-byte spill)
// (v_mfma_f64_16x16x4: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D[i][j] in lane j + 16 (i % 4), element i / 4).
constexpr int BMAP_TILES = 3;

template <int P, class R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void bmap(DevGeom G, const double *__restrict__ U, const double *__restrict__ Bf,
                                           const R *__restrict__ wc, const R *__restrict__ bnod,
                                           R *__restrict__ bnode, double *__restrict__ zoneB)
{
    using T = Tr<P>;
    constexpr int NIN = T::NIN, NOUT = T::NOUTB, KT = NIN / 4, MT = (NOUT + 15) / 16, NT = BMAP_TILES;
    constexpr int NA = 3 * (T::NC + 1), NQ = NA + 6 * T::Q;
    static_assert(NIN % 4 == 0, "input count must be a multiple of 4");
    const int KR = G.Nr + 2, nt = (KR + 16 * NT - 1) / (16 * NT);
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int c = lb / nt, tile = lb % nt;
    const int l = threadIdx.x, g = l >> 4, jz = l & 15;
    // face id of a zone's local face lf (0..3 angular, 4, 5 radial) is
    // s_fbase[lf] + its shell index: a table, so that lanes choosing different
    // faces in one K step read it without branching
    __shared__ i64 s_fbase[6];
    if (l < 6)
        s_fbase[l] = l >= 4 ? (i64)c * (G.K + 1) + (l - 4) : G.NRF + (i64)G.col_ae[4 * c + l] * G.K;
    __syncthreads();
    int kk[NT], ks[NT];
    bool active[NT];
    i64 z[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) {
        kk[t] = (tile * NT + t) * 16 + jz;
        active[t] = kk[t] < KR;
        ks[t] = G.g - 1 + (active[t] ? kk[t] : 0);
        z[t] = (i64)c * G.K + ks[t];
    }
    const double *Mb = G.Mb + (i64)c * NIN * NOUT;
    dbl4 acc[NT][MT];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int m = 0; m < MT; m++) acc[t][m] = dbl4{0.0, 0.0, 0.0, 0.0};
    auto face_of = [&](int t, int lf) -> i64 { return s_fbase[lf] + ks[t]; };
    // operands of K step s.  B: input j = 4s + g of zone jz of each tile.
    // The inputs are the zone's WENO B coefficients (j < NA; the zone mean,
    // a = 0, comes from U), the faces' limited nodal normal B (j < NQ) and
    // the face averages.  s is uniform, so the kind of a K step is decided by
    // scalar branches; only the steps that straddle two kinds take the
    // per-lane choice.  Inactive zones (past the column's top) read a valid
    // zone and enter as zeros.  A: rows of the map, the padding rows read in
    // bounds and selected to zero, so that no load sits under a branch and
    // the loads of the next step are in flight during this step's products.
    auto load = [&](int s, double (&am)[MT], double (&b)[NT]) {
        const int j = 4 * s + g;
        if (4 * s + 3 < NA) {
            const int comp = j / (T::NC + 1), a = j % (T::NC + 1);
            // does any lane group of this step take a zone mean from U?
            const bool any_mean = (4 * s) / (T::NC + 1) != (4 * s + 3) / (T::NC + 1) || (4 * s) % (T::NC + 1) == 0;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const double w = double(wc[((i64)(5 + comp) * T::NC + (a > 0 ? a - 1 : 0)) * G.Z + z[t]]);
                const double u = any_mean ? U[(i64)(5 + comp) * G.Z + z[t]] : 0.0;
                b[t] = active[t] ? (a == 0 ? u : w) : 0.0;
            }
        } else if (4 * s >= NA && 4 * s + 3 < NQ) {
            const int q = (j - NA) % T::Q, lf = (j - NA) / T::Q;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const double v = double(bnod[(i64)q * G.NF + face_of(t, lf)]);
                b[t] = active[t] ? v : 0.0;
            }
        } else if (4 * s >= NQ) {
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const double v = Bf[face_of(t, j - NQ)];
                b[t] = active[t] ? v : 0.0;
            }
        } else {
            // every lane reads one valid element of each source and keeps
            // the one its input index names
            const int jw = j < NA ? j : NA - 1, jq = j < NA ? 0 : j < NQ ? j - NA : 6 * T::Q - 1;
            const int comp = jw / (T::NC + 1), a = jw % (T::NC + 1);
            const int lfq = jq / T::Q, lff = j < NQ ? 0 : j - NQ;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const double u = U[(i64)(5 + comp) * G.Z + z[t]];
                const double w = double(wc[((i64)(5 + comp) * T::NC + (a > 0 ? a - 1 : 0)) * G.Z + z[t]]);
                const double q = double(bnod[(i64)(jq % T::Q) * G.NF + face_of(t, lfq)]);
                const double f = Bf[face_of(t, lff)];
                const double v = j < NA ? (a == 0 ? u : w) : j < NQ ? q : f;
                b[t] = active[t] ? v : 0.0;
            }
        }
        const double *mrow = Mb + (i64)j * NOUT;
#pragma unroll
        for (int m = 0; m < MT; m++) {
            const int r = m * 16 + jz;
            const double v = mrow[r < NOUT ? r : NOUT - 1];
            am[m] = r < NOUT ? v : 0.0;
        }
    };
    auto product = [&](const double (&am)[MT], const double (&b)[NT]) {
#pragma unroll
        for (int m = 0; m < MT; m++)
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t][m] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[m], b[t], acc[t][m], 0, 0, 0);
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
        const i64 zr = (i64)c * KR + kk[t];
#pragma unroll
        for (int m = 0; m < MT; m++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int r = m * 16 + g + 4 * v;
                if (r < 3 * T::N) bnode[zr * (3 * T::N) + r] = R(acc[t][m][v]);
                else if (r < NOUT) zoneB[(i64)(r - 3 * T::N) * G.Z + z[t]] = acc[t][m][v];
            }
    }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Exact split of eight FP32 values into three BF16 parts each, x = hi + mid +
// lo: hi is x truncated to BF16, the remainder x - hi (exact, at most 16
// significant bits) is truncated again, and what is left has at most eight
// significant bits.  The parts are returned packed in pairs (element 2k in the
// low half of dword k), the layout of a BF16 matrix-core operand.
__device__ __forceinline__ void split_bf16x3(const float (&x)[8], u32x4 &hi, u32x4 &mid, u32x4 &lo)
{
    unsigned h[8], m[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
        h[e] = __float_as_uint(x[e]);
        const float r1 = x[e] - __uint_as_float(h[e] & 0xFFFF0000u);
        m[e] = __float_as_uint(r1);
        l[e] = __float_as_uint(r1 - __uint_as_float(m[e] & 0xFFFF0000u));
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        // high halves of both words: bytes 2, 3 of the second operand, then
        // bytes 2, 3 of the first
        hi[k] = __builtin_amdgcn_perm(h[2 * k + 1], h[2 * k], 0x07060302u);
        mid[k] = __builtin_amdgcn_perm(m[2 * k + 1], m[2 * k], 0x07060302u);
        lo[k] = __builtin_amdgcn_perm(l[2 * k + 1], l[2 * k], 0x07060302u);
    }
}

__device__ __forceinline__ f32x4 mfma_bf16(const u32x4 &a, const u32x4 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

// Flux derivatives of the FP32 predictor on the BF16 matrix cores.  The slab
// rows (d, v) hold each direction's flux at the swapped node positions (see
// put_flux), so the sum over directions of the derivatives at node i is
// sum_d sum_p A_d[i][p] x_{d,v}[p] with A_d[i][p] = D_0[S_d(i)][p]: one
// product with K = 3 x 32 (one 16x16x32 step per direction), M = the nodes
// (two tiles of 16) and one column per (zone, variable).  The entries of A
// (multiples of 1/2) are exact in BF16; each flux value enters as its three
// exact BF16 parts, the small parts first, with FP32 accumulation.
// v_mfma_f32_16x16x32_bf16: A[i][k] in lane i + 16 (k / 8), element k % 8;
// B[k][j] in lane j + 16 (k / 8), element k % 8; D[i][j] in lane
// j + 16 (i / 4), element i % 4.  The result overwrites the direction-0 rows
// of the zone's slab: slot i of row v then holds the derivative sum of
// variable v at node i.  A block is one wavefront, whose LDS accesses take
// effect in program order, so each column's reads precede its writes.
template <int N, int SN, int ZS, int ZPW>
__device__ __forceinline__ void deriv_mfma(float *s_f, const u32x4 (&Am)[3][2], int lane)
{
    constexpr int NT = (ZPW * 8 + 15) / 16;
    const int j = lane % 16, q = lane / 16;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const int jj = 16 * nt + j, zl = jj / 8, v = jj % 8;
        const bool zok = zl < ZPW;
        float *row0 = s_f + (zok ? zl : 0) * ZS + v * SN;
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float *r = row0 + 8 * d * SN + 8 * q;
            float x[8];
            if constexpr (N % 16 == 0) {
                const float4 a = *reinterpret_cast<const float4 *>(r);
                const float4 b = *reinterpret_cast<const float4 *>(r + 4);
                x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
                x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
            } else {
                // the rows end at N; slots 8q + e >= N (and zones past the
                // wavefront's) enter as zeros
#pragma unroll
                for (int e = 0; e < 8; e++) x[e] = 0.f;
                if (8 * q < N) {
                    const float4 a = *reinterpret_cast<const float4 *>(r);
                    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
                    if (8 * q + 4 < N) {
                        const float4 b = *reinterpret_cast<const float4 *>(r + 4);
                        x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
                    }
                }
#pragma unroll
                for (int e = 0; e < 8; e++) x[e] = zok ? x[e] : 0.f;
            }
            u32x4 bh, bm, bl;
            split_bf16x3(x, bh, bm, bl);
            c0 = mfma_bf16(Am[d][0], bl, c0);
            c1 = mfma_bf16(Am[d][1], bl, c1);
            c0 = mfma_bf16(Am[d][0], bm, c0);
            c1 = mfma_bf16(Am[d][1], bm, c1);
            c0 = mfma_bf16(Am[d][0], bh, c0);
            c1 = mfma_bf16(Am[d][1], bh, c1);
        }
        if (zok && 4 * q < N) *reinterpret_cast<f32x4 *>(row0 + 4 * q) = c0;
        if (zok && 16 + 4 * q < N) *reinterpret_cast<f32x4 *>(row0 + 16 + 4 * q) = c1;
    }
}

// ADER-CG predictor (Section V.d).  One wavefront holds 64 / N zones, one lane
// per serendipity node.  Each time level's nodal fluxes pass through LDS
// (node fastest) and the derivative matrices are applied level by level, so a
// lane keeps only its own node's state in registers.  With MF (FP32 only) the
// derivatives run on the BF16 matrix cores (deriv_mfma).
template <int P, class R, bool MF = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void predictor(
    DevGeom G, double dt, double gamma, int npic, const double *__restrict__ U, const R *__restrict__ wc,
    const R *__restrict__ bnode, R *__restrict__ ftr, R *__restrict__ etr)
{
    using T = Tr<P>;
    static_assert(!MF || sizeof(R) == sizeof(float), "the matrix-core derivative is an FP32 form");
    // slab rows are N + 1 long so that lanes reading one node's different
    // variables fall into different LDS banks; the matrix-core form reads
    // eight consecutive slots per lane and keeps rows 16-byte aligned instead
    // zone slabs are padded by eight elements so that the zones' rows fall
    // into different LDS banks (eight measured 1 % faster than four)
    constexpr int N = T::N, SN = MF ? N + 4 : N + 1, ZS = 32 * SN + 8, ZPW = 64 / N, E = T::M - 1,
                  NCF = T::NC + 1;
    __shared__ R s_c[ZPW][5 * NCF];
    // 16-byte aligned for the matrix-core form's vector reads and writes
    __shared__ __align__(16) R s_f[ZPW * ZS];
    u32x4 Am[3][2];
    if constexpr (MF) {
        const u32x4 *a = reinterpret_cast<const u32x4 *>(G.DmfA) + threadIdx.x * 6;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            Am[d][0] = a[2 * d];
            Am[d][1] = a[2 * d + 1];
        }
    }
    const R gam = R(gamma);
    const int lane = threadIdx.x, zl = lane / N, i = lane % N;
    const int KR = G.Nr + 2;
    const i64 nzr = (i64)G.ncol * KR;
    // zone counts stay below 2^31 (checked at launch)
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
            int v = j / NCF, a = j % NCF;
            s_c[zl][j] = a == 0 ? R(U[v * G.Z + z]) : wc[((i64)v * T::NC + a - 1) * G.Z + z];
        }
    }
    const int i1 = DTab<P>::SWAP1[i], i2 = DTab<P>::SWAP2[i];
    __syncthreads();

    R Ua[8], Ut[E][8], dFa[8], met[9], iJ = R(1);
    R *sf = s_f + (zl < ZPW ? zl : 0) * ZS;
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
        const R J = pick<R>(G.nJ, G.nJF)[(i64)c * N + i];
        iJ = R(1) / J;
        // metric terms scaled by dt over the zone's size: the predictor works in
        // reference time and space
        const R fac = R(dt / G.zscale[k]);
        const R *nM = pick<R>(G.nM, G.nMF);
#pragma unroll
        for (int m = 0; m < 9; m++) met[m] = fac * nM[((i64)c * 9 + m) * N + i];
#pragma unroll
        for (int v = 0; v < 8; v++) Ua[v] *= J;
        // level tau = 0: its flux derivative is the same in every iteration
        R F[3][8];
        mapped_flux<R>(Ua, iJ, met, gam, F);
        put_flux<SN, R>(sf, i, i1, i2, F);
    }
    __syncthreads();
    if constexpr (MF) deriv_mfma<N, SN, ZS, ZPW>(s_f, Am, lane);
    else deriv_rows<P, SN, ZS, ZPW, R>(s_f, lane);
    __syncthreads();
    if (active) {
        if constexpr (MF) {
#pragma unroll
            for (int v = 0; v < 8; v++) dFa[v] = sf[v * SN + i];
        } else {
            get_deriv<SN, R>(sf, i, i1, i2, dFa);
        }
        // The first sweep starts from the same state at every level, so each
        // level's flux derivative equals the one at tau = 0: it needs no flux
        // evaluations and gives the same numbers as the general sweep below.
        const R on = npic > 0 ? R(1) : R(0);
#pragma unroll
        for (int t = 0; t < E; t++)
#pragma unroll
            for (int v = 0; v < 8; v++) {
                R u = Ua[v] - on * R(G.R[t * T::M]) * dFa[v];
#pragma unroll
                for (int s = 0; s < E; s++) u -= on * R(G.R[t * T::M + s + 1]) * dFa[v];
                Ut[t][v] = u;
            }
    }
    __syncthreads();
    for (int it = 1; it < npic; it++) {
        // derivative of each level's flux; a level's state is dead once its
        // flux is in LDS, so at most E + 1 vectors of eight are live here
        R A[E][8];
#pragma unroll
        for (int s = 0; s < E; s++) {
            if (active) {
                R F[3][8];
                mapped_flux<R>(Ut[s], iJ, met, gam, F);
                put_flux<SN, R>(sf, i, i1, i2, F);
            }
            __syncthreads();
            if constexpr (MF) {
                deriv_mfma<N, SN, ZS, ZPW>(s_f, Am, lane);
                __syncthreads();
#pragma unroll
                for (int v = 0; v < 8; v++) A[s][v] = active ? sf[v * SN + i] : R(0);
                __syncthreads();
            } else {
                deriv_rows<P, SN, ZS, ZPW, R>(s_f, lane);
                __syncthreads();
#pragma unroll
                for (int v = 0; v < 8; v++) A[s][v] = R(0);
                if (active) get_deriv<SN, R>(sf, i, i1, i2, A[s]);
                __syncthreads();
            }
        }
#pragma unroll
        for (int t = 0; t < E; t++) {
            const R r0 = R(G.R[t * T::M]);
#pragma unroll
            for (int v = 0; v < 8; v++) {
                R u = Ua[v] - r0 * dFa[v];
#pragma unroll
                for (int s = 0; s < E; s++) u -= R(G.R[t * T::M + s + 1]) * A[s][v];
                Ut[t][v] = u;
            }
        }
    }
    // time averages of state and physical flux over the Gauss levels
    if (active) {
        R aU[8], aF[3][8], w[8], F[3][8];
#pragma unroll
        for (int v = 0; v < 8; v++) { aU[v] = R(0); aF[0][v] = aF[1][v] = aF[2][v] = R(0); }
#pragma unroll
        for (int t = 0; t < E; t++) {
            const R wt = R(G.wt[t + 1]);
#pragma unroll
            for (int v = 0; v < 8; v++) w[v] = Ut[t][v] * iJ;
            dev_flux<R>(w, gam, F);
#pragma unroll
            for (int v = 0; v < 8; v++) {
                aU[v] += wt * w[v];
                aF[0][v] += wt * F[0][v];
                aF[1][v] += wt * F[1][v];
                aF[2][v] += wt * F[2][v];
            }
        }
#pragma unroll
        for (int v = 0; v < 8; v++) {
            sf[v * SN + i] = aU[v];
            sf[(8 + v) * SN + i] = aF[0][v];
            sf[(16 + v) * SN + i] = aF[1][v];
            sf[(24 + v) * SN + i] = aF[2][v];
        }
    }
    __syncthreads();
    // Traces.  Faces: one task per (zone, face, variable) interpolates the
    // averaged state and the three flux components of its variable from the
    // face's nodes to all face quadrature points (weights shared by the six
    // faces), then forms the outward-normal flux.
#pragma unroll 1
    for (int t = lane; t < ZPW * 48; t += 64) {
        const int zq = t / 48, lf = (t % 48) / 8, v = t % 8;
        const unsigned ztq = lb * ZPW + zq;
        if (ztq >= (unsigned)nzr) continue;
        const int cq = (int)(ztq / (unsigned)KR), kq = G.g - 1 + (int)(ztq % (unsigned)KR);
        const R *sx = s_f + zq * ZS;
        R x[T::NFN][4];
#pragma unroll
        for (int kk = 0; kk < T::NFN; kk++) {
            const int l = G.fnode[lf * T::NFN + kk];
#pragma unroll
            for (int j = 0; j < 4; j++) x[kk][j] = sx[(8 * j + v) * SN + l];
        }
        i64 fid;
        int side;
        const double *nrm;
        const int *perm = nullptr;
        if (lf >= 4) {
            fid = (i64)cq * (G.K + 1) + kq + (lf - 4);
            side = lf == 4 ? 1 : 0;
            nrm = G.fnR + (i64)cq * T::Q * 3;
        } else {
            const int ae = G.col_ae[4 * cq + lf];
            fid = G.NRF + (i64)ae * G.K + kq;
            side = G.col_side[4 * cq + lf];
            nrm = G.fnA + (i64)ae * T::Q * 3;
            perm = G.col_perm + ((i64)cq * 4 + lf) * T::Q;
        }
        R *o = ftr + ftr_at<P>(fid, 0, side);   // point q at o + 32 q
        // every point's normal is loaded before the interpolation, so that the
        // loads (behind the point permutation) are in flight together: the
        // FP64 predictor at 6 x 128^3 measured 115.5 -> 109.6 ms
        int qcs[T::Q];
        R nn[T::Q][3];
#pragma unroll
        for (int q = 0; q < T::Q; q++) qcs[q] = perm ? perm[q] : q;
#pragma unroll
        for (int q = 0; q < T::Q; q++) {
            nn[q][0] = R(nrm[qcs[q] * 3]);
            nn[q][1] = R(nrm[qcs[q] * 3 + 1]);
            nn[q][2] = R(nrm[qcs[q] * 3 + 2]);
        }
        // one row of quadrature points at a time: its weights are uniform
        // across the wavefront and stay in scalar registers
#pragma unroll
        for (int b = 0; b < T::Q1; b++) {
            R aq[T::Q1][4];
#pragma unroll
            for (int a = 0; a < T::Q1; a++) aq[a][0] = aq[a][1] = aq[a][2] = aq[a][3] = R(0);
            const R *wrow = pick<R>(G.fintc, G.fintcF) + b * T::Q1;
#pragma unroll
            for (int kk = 0; kk < T::NFN; kk++)
#pragma unroll
                for (int a = 0; a < T::Q1; a++) {
                    const R w = wrow[kk * T::Q + a];
#pragma unroll
                    for (int j = 0; j < 4; j++) aq[a][j] += w * x[kk][j];
                }
#pragma unroll
            for (int a = 0; a < T::Q1; a++) {
                const int q = a + T::Q1 * b;
                const int qc = qcs[q];
                o[qc * 32 + v] = aq[a][0];
                o[qc * 32 + 8 + v] = nn[q][0] * aq[a][1] + nn[q][1] * aq[a][2] + nn[q][2] * aq[a][3];
            }
        }
    }
    // Edges: one task per (zone, edge) interpolates the averaged state and the
    // three electric-field components (eq. 2.3) to the edge's Simpson points
    // and keeps E . t there.
    if (lane < ZPW * 12) {
        const int zq = lane / 12, le = lane % 12;
        const unsigned ztq = lb * ZPW + zq;
        if (ztq < (unsigned)nzr) {
            const int cq = (int)(ztq / (unsigned)KR), kq = G.g - 1 + (int)(ztq % (unsigned)KR);
            const int rev = G.col_rev[(i64)cq * 12 + le], slot = G.col_slot[(i64)cq * 12 + le];
            // the tangents first, so that their loads overlap the interpolation
            R tv[3][3];
#pragma unroll
            for (int p = 0; p < 3; p++) {
                const double *t = edge_tangent(G, cq, le, rev ? 2 - p : p);
                tv[p][0] = R(t[0]);
                tv[p][1] = R(t[1]);
                tv[p][2] = R(t[2]);
            }
            const R *sx = s_f + zq * ZS;
            const R *ew = pick<R>(G.eintc, G.eintcF);
            R ae3[3][11];
#pragma unroll
            for (int p = 0; p < 3; p++)
#pragma unroll
                for (int v = 0; v < 11; v++) ae3[p][v] = R(0);
#pragma unroll
            for (int kk = 0; kk < T::NEN; kk++) {
                const int l = G.enode[le * T::NEN + kk];
                R x[11];
#pragma unroll
                for (int v = 0; v < 8; v++) x[v] = sx[v * SN + l];
                x[8] = sx[(24 + 6) * SN + l];    // E_x = H[B_y]
                x[9] = sx[(8 + 7) * SN + l];     // E_y = F[B_z]
                x[10] = sx[(16 + 5) * SN + l];   // E_z = G[B_x]
#pragma unroll
                for (int p = 0; p < 3; p++) {
                    const R w = ew[kk * 3 + p];
#pragma unroll
                    for (int v = 0; v < 11; v++) ae3[p][v] += w * x[v];
                }
            }
            i64 e;
            if (le < 8) {
                const int ae = G.col_ae[4 * cq + LocalEdges::FACE[le]];
                e = G.NRE + (i64)ae * (G.K + 1) + kq + LocalEdges::UP[le];
            } else {
                e = (i64)G.col_v[4 * cq + LocalEdges::CORNER[le - 8]] * G.K + kq;
            }
            R *o = etr + etr_at(e, 0, slot);   // point p at o + 36 p
#pragma unroll
            for (int p = 0; p < 3; p++) {
                const int pc = rev ? 2 - p : p;
#pragma unroll
                for (int v = 0; v < 8; v++) o[pc * 36 + v] = ae3[p][v];
                o[pc * 36 + 8] = tv[p][0] * ae3[p][8] + tv[p][1] * ae3[p][9] + tv[p][2] * ae3[p][10];
            }
        }
    }
}

// ---------------------------------------------------------------- face fluxes
// HLL at every face quadrature point, then the weighted sum over a face's
// points in order.  A point's two side records are adjacent (2 x 16 values).
// With FP64 records two lanes take a point: they load its records in
// alternate 16-byte pieces, so that the lanes of a pair read neighbouring
// bytes and each load instruction touches half as many cache lines, and a DPP
// swap gives each lane the other's pieces; both evaluate the same HLL.  The
// address unit was this kernel's limit with one lane per 256-byte point
// (21.4 -> 17.3 ms, bit-identical).  FP32 records (128 bytes a point) keep one
// lane per point, which measured faster for them.
// MARKED: only faces with mark[f] set are solved and written (the re-solve of
// the first-order fallback; *added counts the zones its round flagged).
template <class R>
constexpr int flux_lanes_per_point() { return sizeof(R) == sizeof(double) ? 2 : 1; }
template <int P, class R>
constexpr int flux_faces_per_block() { return 256 / (flux_lanes_per_point<R>() * Tr<P>::Q); }

template <int P, class R, bool MARKED = false>
__global__ __launch_bounds__(256) void face_flux(DevGeom G, double gam, const R *__restrict__ ftr,
                                                 double *__restrict__ Phi, const unsigned char *__restrict__ mark = nullptr,
                                                 const int *__restrict__ added = nullptr)
{
    using T = Tr<P>;
    if (MARKED && *added == 0) return;   // the round flagged no zone
    constexpr int LPP = flux_lanes_per_point<R>(), FPB = flux_faces_per_block<P, R>();
    __shared__ double s_q[FPB * T::Q][9];
    const i64 nff = (i64)G.ncol * (G.Nr + 1) + (i64)G.nae * G.Nr;
    const int tid = threadIdx.x, pt = tid / LPP, half = tid % LPP, fl = pt / T::Q, q = pt % T::Q;
    const i64 t = (i64)blockIdx.x * FPB + fl;
    const double *nrm = nullptr, *fw = nullptr;
    i64 f = 0;
    bool live = fl < FPB && t < nff;
    if (live) {
        f = flux_face<P>(G, t, nrm, fw);
        if (MARKED) live = mark[f] != 0;
    }
    R vals[32];   // the point's side-0 record, then its side-1 record
    if constexpr (LPP == 2) {
        constexpr int NDW = 2 * 16 * (int)sizeof(R) / 4;   // dwords of the two records
        constexpr int NPC = NDW / 4;                        // 16-byte pieces
        uint32_t own[NPC / 2][4];   // this lane's pieces 2i + half
#pragma unroll
        for (int i = 0; i < NPC / 2; i++) own[i][0] = own[i][1] = own[i][2] = own[i][3] = 0u;
        if (live) {
            const uint4 *src = reinterpret_cast<const uint4 *>(ftr + ftr_at<P>(f, q, 0));
#pragma unroll
            for (int i = 0; i < NPC / 2; i++) {
                const uint4 w = src[2 * i + half];
                own[i][0] = w.x;
                own[i][1] = w.y;
                own[i][2] = w.z;
                own[i][3] = w.w;
            }
        }
        uint32_t blk[NDW];
#pragma unroll
        for (int i = 0; i < NPC / 2; i++)
#pragma unroll
            for (int d = 0; d < 4; d++) {
                // lanes 2n and 2n + 1 swap (quad_perm 1, 0, 3, 2)
                const uint32_t oth = (uint32_t)__builtin_amdgcn_mov_dpp((int)own[i][d], 0xB1, 0xF, 0xF, false);
                blk[4 * (2 * i) + d] = half == 0 ? own[i][d] : oth;
                blk[4 * (2 * i + 1) + d] = half == 0 ? oth : own[i][d];
            }
        __builtin_memcpy(vals, blk, sizeof(vals));
    } else {
        if (live) {
            const R *a = ftr + ftr_at<P>(f, q, 0);
#pragma unroll
            for (int v = 0; v < 32; v++) vals[v] = a[v];
        }
    }
    if (live) {
        double UL[8], UR[8], FL[8], FR[8], Fs[8];
#pragma unroll
        for (int v = 0; v < 8; v++) {
            UL[v] = vals[v];
            FL[v] = vals[8 + v];
            UR[v] = vals[16 + v];
            FR[v] = vals[24 + v];
        }
        dev_hll<double>(UL, UR, FL, FR, nrm + q * 3, gam, Fs);
        const double w = fw[q] * G.area[f];
        if (half == 0)
#pragma unroll
            for (int v = 0; v < 8; v++) s_q[pt][v] = w * Fs[v];
    }
    __syncthreads();
    // one thread per (face, variable), faces fastest
    for (int j = tid; j < FPB * 8; j += 256) {
        const int f2 = j % FPB, v = j / FPB;
        const i64 t2 = (i64)blockIdx.x * FPB + f2;
        if (t2 >= nff) continue;
        const double *nrm2, *fw2;
        const i64 fo = flux_face<P>(G, t2, nrm2, fw2);
        if (MARKED && !mark[fo]) continue;
        double acc = 0.0;
#pragma unroll
        for (int qq = 0; qq < T::Q; qq++) acc += s_q[f2 * T::Q + qq][v];
        Phi[(i64)v * G.NF + fo] = acc;
    }
}

// ---------------------------------------------------------------- edge electric fields
// one lane per (edge, Simpson point), 64 edges per block, then the line
// integral summed over the three points in order
// MARKED: only edges with mark[e] set are solved and written
template <class R, bool MARKED = false>
__global__ __launch_bounds__(192) void edge_emf(DevGeom G, double gam, const R *__restrict__ etr, double *__restrict__ Gam,
                                                const unsigned char *__restrict__ mark = nullptr,
                                                const int *__restrict__ added = nullptr)
{
    if (MARKED && *added == 0) return;
    __shared__ double s_p[192];
    const i64 nee = (i64)G.nv * G.Nr + (i64)G.nae * (G.Nr + 1);
    const int tid = threadIdx.x, el = tid / 3, p = tid % 3;
    const i64 t = (i64)blockIdx.x * 64 + el;
    const double *frame = nullptr, *N3 = nullptr;
    double wl = 0.0;
    int nzs = 4;
    i64 e = 0;
    bool live = t < nee;
    if (live) {
        e = emf_edge(G, t, p, frame, wl, nzs, N3);
        if (MARKED) live = mark[e] != 0;
    }
    if (live) {
        double U[4][8], E[4][3], Et[4];
        const double *tt = frame + 6;
        // all four slots are read (a three-zone edge leaves slot 3 unused);
        // the three-zone solver takes E along t, the only part it projects on
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const R *rec = etr + etr_at(e, p, s);
#pragma unroll
            for (int v = 0; v < 8; v++) U[s][v] = rec[v];
            Et[s] = rec[8];
#pragma unroll
            for (int v = 0; v < 3; v++) E[s][v] = Et[s] * tt[v];
        }
        const double Es = (nzs == 4) ? emf4<double>(U, Et, frame, gam) : emf3<double>(U, E, N3, tt, gam);
        s_p[tid] = wl * Es;
    }
    __syncthreads();
    if (tid < 64) {
        const i64 t2 = (i64)blockIdx.x * 64 + tid;
        if (t2 < nee) {
            const double *frame2, *N32;
            double wl2;
            int nzs2;
            const i64 eo = emf_edge(G, t2, 0, frame2, wl2, nzs2, N32);
            if (MARKED && !mark[eo]) return;
            double gsum = 0.0;
            gsum += s_p[3 * tid];
            gsum += s_p[3 * tid + 1];
            gsum += s_p[3 * tid + 2];
            Gam[eo] = gsum;
        }
    }
}

// ---------------------------------------------------------------- updates
// Zone averages of interior zone (c, k) after the finite-volume update with
// the face fluxes Phi; zone B starts from Bbase, the divergence-free
// reconstruction's mean (step 10 of Section IV.b) [3][Z]
__device__ __forceinline__ void updated_zone(const DevGeom &G, double dt, const double *__restrict__ Phi,
                                             const double *Bbase, const double *Uo, int c, int k, double u[8])
{
    const i64 z = (i64)c * G.K + k;
    i64 f[6];
    double sg[6];
    for (int lf = 0; lf < 4; lf++) {
        f[lf] = G.NRF + (i64)G.col_ae[4 * c + lf] * G.K + k;
        sg[lf] = G.col_side[4 * c + lf] == 0 ? 1.0 : -1.0;
    }
    f[4] = (i64)c * (G.K + 1) + k;
    f[5] = f[4] + 1;
    sg[4] = -1.0;
    sg[5] = 1.0;
    const double cfac = dt / G.vol[z];
    for (int v = 0; v < 8; v++) {
        double acc = 0.0;
        for (int lf = 0; lf < 6; lf++) acc += sg[lf] * Phi[(i64)v * G.NF + f[lf]];
        const double base = v < 5 ? Uo[v * G.Z + z] : Bbase[(v - 5) * G.Z + z];
        u[v] = base - cfac * acc;
    }
}

// zfl (null without the fallback): a flagged zone advances its own B average
// instead of the reconstruction's mean, so that its update is the first-order
// finite-volume scheme on its eight averages
__global__ __launch_bounds__(256) void zone_update(DevGeom G, double dt, const double *__restrict__ Phi,
                                                   const double *__restrict__ zoneB, double *Uo,
                                                   const unsigned char *__restrict__ zfl)
{
    i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (i64)G.ncol * G.Nr) return;
    const int c = (int)(t / G.Nr), k = G.g + (int)(t % G.Nr);
    const i64 z = (i64)c * G.K + k;
    const bool own = zfl && zfl[z];
    double u[8];
    updated_zone(G, dt, Phi, own ? Uo + 5 * G.Z : zoneB, Uo, c, k, u);
    for (int v = 0; v < 8; v++) Uo[v * G.Z + z] = u[v];
}

// ---------------------------------------------------------------- first-order fallback
// Section I leaves positivity under strong fields to ruggedised schemes from
// other work; the step's fallback is an a-posteriori per-zone order drop.
static_assert(FALLBACK_ROUNDS == RG_FALLBACK_ROUNDS, "round count matches the C-ABI");
static_assert(FALLBACK_ROUNDS * sizeof(int) <= RG_FB_COUNTER_BYTES, "round counters fit their slot");

// zero n bytes (16 per lane; m 16-byte aligned)
__global__ __launch_bounds__(256) void fb_clear(unsigned char *__restrict__ m, i64 n)
{
    const i64 i = ((i64)blockIdx.x * blockDim.x + threadIdx.x) * 16;
    if (i + 16 <= n) {
        *reinterpret_cast<uint4 *>(m + i) = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (i64 j = i; j < n; j++) m[j] = 0;
    }
}

// One round of the check.  Round 0 writes every zone's flag: 1 for an
// interior zone whose update with the current fluxes leaves a density or
// pressure that is not positive (NaN included).  A re-solved face can drive a
// neighbour negative, so later rounds re-check the unflagged zones that touch
// a marked face (the fluxes of every other zone are those of round 0, which
// it passed) and add the bad ones.  A flagged zone marks its six faces and
// twelve edges (every writer of a mark writes 1; marks of earlier rounds were
// written by earlier launches, so what a zone reads does not depend on the
// order of the lanes).  added[round] counts the zones the round flags.
__global__ __launch_bounds__(256) void fb_flag(DevGeom G, double dt, double gam, int round,
                                               const double *__restrict__ Phi, const double *__restrict__ zoneB,
                                               const double *__restrict__ Uo, unsigned char *__restrict__ zfl,
                                               unsigned char *__restrict__ ffl, unsigned char *__restrict__ efl,
                                               int *__restrict__ added)
{
    // no zone flagged in the previous round: no flux changed, nothing to check
    if (round > 0 && added[round - 1] == 0) return;
    const i64 z = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= G.Z) return;
    const int c = (int)(z / G.K), k = (int)(z % G.K);
    if (k < G.g || k >= G.g + G.Nr) {
        if (round == 0) zfl[z] = 0;
        return;
    }
    i64 fid[6];
    for (int lf = 0; lf < 4; lf++) fid[lf] = G.NRF + (i64)G.col_ae[4 * c + lf] * G.K + k;
    fid[4] = (i64)c * (G.K + 1) + k;
    fid[5] = fid[4] + 1;
    if (round > 0) {
        if (zfl[z]) return;
        bool touched = false;
        for (int lf = 0; lf < 6; lf++) touched |= ffl[fid[lf]] != 0;
        if (!touched) return;
    }
    double u[8];
    updated_zone(G, dt, Phi, zoneB, Uo, c, k, u);
    const bool ok = u[0] > 0.0 && dev_pressure<double>(u, gam) > 0.0;
    if (round == 0) zfl[z] = ok ? 0 : 1;
    if (ok) return;
    zfl[z] = 1;
    atomicAdd(&added[round], 1);
    for (int lf = 0; lf < 6; lf++) ffl[fid[lf]] = 1;
    for (int le = 0; le < 8; le++)
        efl[G.NRE + (i64)G.col_ae[4 * c + LocalEdges::FACE[le]] * (G.K + 1) + k + LocalEdges::UP[le]] = 1;
    for (int j = 0; j < 4; j++) efl[(i64)G.col_v[4 * c + LocalEdges::CORNER[j]] * G.K + k] = 1;
}

// Constant traces for the re-solve: every zone of the predictor's range
// (shells g-1 .. g+Nr) writes, on each of its marked faces and edges, its
// conserved state at t^n (its eight averages in Uo before the update) and the
// physical flux of that state in the records the predictor fills (face: the
// state and the normal flux at each quadrature point; edge: the state and
// E . t with E = (H[B_y], F[B_z], G[B_x]) at each Simpson point).
template <int P, class R>
__global__ __launch_bounds__(256) void fb_traces(DevGeom G, double gam, const double *__restrict__ Uo,
                                                 const unsigned char *__restrict__ ffl,
                                                 const unsigned char *__restrict__ efl, R *__restrict__ ftr,
                                                 R *__restrict__ etr, const int *__restrict__ added)
{
    using T = Tr<P>;
    if (*added == 0) return;   // the round flagged no zone: no new marks
    const int KR = G.Nr + 2;
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (i64)G.ncol * KR) return;
    const int c = (int)(t / KR), k = G.g - 1 + (int)(t % KR);
    const i64 z = (i64)c * G.K + k;
    i64 fid[6], eid[12];
    for (int lf = 0; lf < 4; lf++) fid[lf] = G.NRF + (i64)G.col_ae[4 * c + lf] * G.K + k;
    fid[4] = (i64)c * (G.K + 1) + k;
    fid[5] = fid[4] + 1;
    for (int le = 0; le < 8; le++)
        eid[le] = G.NRE + (i64)G.col_ae[4 * c + LocalEdges::FACE[le]] * (G.K + 1) + k + LocalEdges::UP[le];
    for (int j = 0; j < 4; j++) eid[8 + j] = (i64)G.col_v[4 * c + LocalEdges::CORNER[j]] * G.K + k;
    bool any = false;
    for (int lf = 0; lf < 6; lf++) any |= ffl[fid[lf]] != 0;
    for (int le = 0; le < 12; le++) any |= efl[eid[le]] != 0;
    if (!any) return;
    double u[8], F[3][8];
    for (int v = 0; v < 5; v++) u[v] = Uo[v * G.Z + z];
    for (int v = 5; v < 8; v++) u[v] = Uo[v * G.Z + z];
    dev_flux<double>(u, gam, F);
    for (int lf = 0; lf < 6; lf++) {
        if (!ffl[fid[lf]]) continue;
        int side;
        const double *nrm;
        if (lf >= 4) {
            side = lf == 4 ? 1 : 0;
            nrm = G.fnR + (i64)c * T::Q * 3;
        } else {
            side = G.col_side[4 * c + lf];
            nrm = G.fnA + (i64)G.col_ae[4 * c + lf] * T::Q * 3;
        }
        R *o = ftr + ftr_at<P>(fid[lf], 0, side);   // point q at o + 32 q
        for (int q = 0; q < T::Q; q++) {
            const double *n = nrm + q * 3;
            for (int v = 0; v < 8; v++) {
                o[q * 32 + v] = R(u[v]);
                o[q * 32 + 8 + v] = R(n[0] * F[0][v] + n[1] * F[1][v] + n[2] * F[2][v]);
            }
        }
    }
    for (int le = 0; le < 12; le++) {
        if (!efl[eid[le]]) continue;
        R *o = etr + etr_at(eid[le], 0, G.col_slot[(i64)c * 12 + le]);   // point p at o + 36 p
        for (int p = 0; p < 3; p++) {
            const double *t = edge_tangent(G, c, le, p);
            for (int v = 0; v < 8; v++) o[p * 36 + v] = R(u[v]);
            o[p * 36 + 8] = R(t[0] * F[2][6] + t[1] * F[0][7] + t[2] * F[1][5]);
        }
    }
}

// Circulation of edge values Gam about a face (right-hand rule about its
// canonical normal): the discrete Stokes sum of eqs. 2.5-2.6.  Faces of
// shells k0..k1: radial faces kf in [k0, k1 + 1], angular faces k in [k0, k1];
// thread t < nR takes radial face (c, kf), the rest angular face (ae, k).
__device__ __forceinline__ double face_circulation(const DevGeom &G, const double *__restrict__ Gam, i64 t, int k0,
                                                   int k1, i64 &f)
{
    const int nrad = k1 - k0 + 2, nang = k1 - k0 + 1;
    const i64 nR = (i64)G.ncol * nrad;
    if (t < nR) {
        const int c = (int)(t / nrad), kf = k0 + (int)(t % nrad);
        f = (i64)c * (G.K + 1) + kf;
        double circ = 0.0;
        for (int lf = 0; lf < 4; lf++)
            circ += G.col_sgn[4 * c + lf] * Gam[G.NRE + (i64)G.col_ae[4 * c + lf] * (G.K + 1) + kf];
        return circ;
    }
    const i64 u = t - nR;
    const int ae = (int)(u / nang), k = k0 + (int)(u % nang);
    f = G.NRF + (i64)ae * G.K + k;
    const i64 ea0 = G.NRE + (i64)ae * (G.K + 1) + k;
    const double lp = Gam[ea0] + Gam[(i64)G.ae_v[2 * ae + 1] * G.K + k] - Gam[ea0 + 1] - Gam[(i64)G.ae_v[2 * ae] * G.K + k];
    return G.ae_rs[ae] * lp;
}

__global__ __launch_bounds__(256) void face_ct(DevGeom G, double dt, const double *__restrict__ Gam, double *Bo)
{
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (i64)G.ncol * (G.Nr + 1) + (i64)G.nae * G.Nr) return;
    i64 f;
    const double circ = face_circulation(G, Gam, t, G.g, G.g + G.Nr - 1, f);
    Bo[f] -= dt / G.area[f] * circ;
}

// Face averages of the normal component of curl A from the line integrals of
// A along every edge (Stokes), for every face of the mesh
__global__ __launch_bounds__(256) void stokes_faces(DevGeom G, const double *__restrict__ circ_e, double *__restrict__ Bf)
{
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (i64)G.ncol * (G.K + 1) + (i64)G.nae * G.K) return;
    i64 f;
    const double circ = face_circulation(G, circ_e, t, 0, G.K - 1, f);
    Bf[f] = circ / G.area[f];
}

// ---------------------------------------------------------------- CFL
__global__ __launch_bounds__(256) void cfl_partial(DevGeom G, double gam, double cfl, const double *__restrict__ U,
                                                   double *red)
{
    __shared__ double sm[256];
    i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    double best = 1e300;
    if (t < (i64)G.ncol * G.Nr) {
        int c = (int)(t / G.Nr), k = G.g + (int)(t % G.Nr);
        i64 z = (i64)c * G.K + k;
        double u[8];
        for (int v = 0; v < 8; v++) u[v] = U[v * G.Z + z];
        double ir = 1.0 / u[0];
        double vv = sqrt(u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * ir;
        double a2 = gam * dev_pressure<double>(u, gam) * ir, b2 = (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]) * ir;
        best = cfl * G.dins[c] * G.zscale[k] / (vv + sqrt(a2 + b2));
    }
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) red[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void cfl_final(int n, double *red)
{
    __shared__ double sm[256];
    double best = 1e300;
    for (int i = threadIdx.x; i < n; i += 256) best = fmin(best, red[i]);
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) red[65535] = sm[0];
}

// ---------------------------------------------------------------- diagnostics
// Per interior zone: relative div B |sum sigma A <B.n>| / sum A |<B.n>|, the
// volume-weighted conserved sums and the smallest density and pressure.
// A fixed grid strides over the zones; partial results per block, then one
// block reduces them in a fixed order (deterministic).
constexpr int DIAG_BLOCKS = 1024, DIAG_NV = 11;   // div max, 8 sums, rho min, p min

__device__ __forceinline__ void diag_combine(double *a, const double *b)
{
    a[0] = fmax(a[0], b[0]);
    for (int v = 1; v < 9; v++) a[v] += b[v];
    a[9] = fmin(a[9], b[9]);
    a[10] = fmin(a[10], b[10]);
}

__global__ __launch_bounds__(256) void diag_partial(DevGeom G, double gam, const double *__restrict__ U,
                                                    const double *__restrict__ Bf, double *red)
{
    __shared__ double sm[256][DIAG_NV];
    double acc[DIAG_NV] = {0.0, 0, 0, 0, 0, 0, 0, 0, 0, 1e300, 1e300};
    const i64 n = (i64)G.ncol * G.Nr;
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
        const int c = (int)(t / G.Nr), k = G.g + (int)(t % G.Nr);
        const i64 z = (i64)c * G.K + k;
        double num = 0.0, den = 0.0;
        const i64 fr = (i64)c * (G.K + 1) + k;
        num += G.area[fr + 1] * Bf[fr + 1] - G.area[fr] * Bf[fr];
        den += G.area[fr + 1] * fabs(Bf[fr + 1]) + G.area[fr] * fabs(Bf[fr]);
        for (int lf = 0; lf < 4; lf++) {
            const i64 f = G.NRF + (i64)G.col_ae[4 * c + lf] * G.K + k;
            const double sg = G.col_side[4 * c + lf] == 0 ? 1.0 : -1.0;
            num += sg * G.area[f] * Bf[f];
            den += G.area[f] * fabs(Bf[f]);
        }
        acc[0] = fmax(acc[0], den > 0.0 ? fabs(num) / den : 0.0);
        double u[8];
        for (int v = 0; v < 8; v++) {
            u[v] = U[v * G.Z + z];
            acc[1 + v] += G.vol[z] * u[v];
        }
        acc[9] = fmin(acc[9], u[0]);
        acc[10] = fmin(acc[10], dev_pressure<double>(u, gam));
    }
    for (int v = 0; v < DIAG_NV; v++) sm[threadIdx.x][v] = acc[v];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) diag_combine(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int v = 0; v < DIAG_NV; v++) red[(i64)blockIdx.x * DIAG_NV + v] = sm[0][v];
}

__global__ __launch_bounds__(256) void diag_final(double *red)
{
    __shared__ double sm[256][DIAG_NV];
    double acc[DIAG_NV] = {0.0, 0, 0, 0, 0, 0, 0, 0, 0, 1e300, 1e300};
    for (int b = threadIdx.x; b < DIAG_BLOCKS; b += 256) diag_combine(acc, red + (i64)b * DIAG_NV);
    for (int v = 0; v < DIAG_NV; v++) sm[threadIdx.x][v] = acc[v];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) diag_combine(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int v = 0; v < DIAG_NV; v++) red[DIAG_BLOCKS * DIAG_NV + v] = sm[0][v];
}

// ---------------------------------------------------------------- host launch
static inline unsigned nblocks(i64 n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#define RG_LAUNCH_CHECK()                                            \
    do {                                                             \
        hipError_t e_ = hipGetLastError();                           \
        if (e_ != hipSuccess) {                                      \
            set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_)); \
            return RG_EDEVICE;                                       \
        }                                                            \
    } while (0)

template <class R>
static const R *pick_host(const double *d, const float *f)
{
    if constexpr (sizeof(R) == sizeof(double)) return d;
    else return f;
}

// stage markers for optional per-stage timing (0 bc, 1 weno, 2 face_bnodal,
// 3 bmap, 4 predictor, 5 face_flux, 6 edge_emf, 7 update)
struct StageMarks {
    hipEvent_t ev[RG_NSTAGE + 1];
    bool on = false;
    void mark(int i, hipStream_t st)
    {
        if (on) (void)hipEventRecord(ev[i], st);
    }
};

template <int P, class R, bool MF = false>
static rg_status step_order(rg_geom *g, const rg_step_params &prm, const double *U, const double *Bf, double *Uo,
                            double *Bo, hipStream_t st, bool front_only = false)
{
    const DevGeom &G = g->d;
    // work buffers hold R values (they are sized for doubles)
    R *wcoef = reinterpret_cast<R *>(g->wcoef), *bnod = reinterpret_cast<R *>(g->bnod);
    R *bnode = reinterpret_cast<R *>(g->bnode), *ftr = reinterpret_cast<R *>(g->ftr);
    R *etr = reinterpret_cast<R *>(g->etr);
    const int npic = prm.n_picard > 0 ? prm.n_picard : P;
    const double dt = prm.dt, gam = prm.gamma;
    StageMarks sm;
    if (g->prof_on && !front_only) {
        sm.on = true;
        for (int i = 0; i <= RG_NSTAGE; i++) {
            if (hipEventCreate(&sm.ev[i]) != hipSuccess) { set_error("hipEventCreate failed"); return RG_EDEVICE; }
            g->prof_events.push_back((void *)sm.ev[i]);
        }
    }
    sm.mark(0, st);
    bc_zones<<<nblocks(G.Z, 256), 256, 0, st>>>(G, prm.bc_kind, U, Uo);
    bc_faces<<<nblocks(G.NF, 256), 256, 0, st>>>(G, prm.bc_kind, Bf, Bo);
    RG_LAUNCH_CHECK();
    sm.mark(1, st);
    const i64 nzr = (i64)G.ncol * (G.Nr + 2);
    if constexpr (sizeof(R) == sizeof(double)) {
        const int nrun = (G.Nr + 2 + 15) / 16;
        weno_mfma<P><<<(unsigned)((i64)G.ncol * nrun), 64, 0, st>>>(G, Uo, reinterpret_cast<double *>(wcoef), G.Pl, G.Ps,
                                                                    G.Qs, weno_eps(prm), nrun, g->whi);
    } else {
        const RunSplit wr = run_split(G.Nr + 2);
        weno_cols<P, R><<<(unsigned)((i64)G.ncol * (wr.nchunk + (wr.nleft > 0))), 64, 0, st>>>(
            G, Uo, wcoef, pick_host<R>(G.Pl, G.PlF), pick_host<R>(G.Ps, G.PsF), pick_host<R>(G.Qs, G.QsF),
            R(weno_eps(prm)), wr.nchunk, wr.nu, wr.nleft, g->whi);
    }
    if (prm.flattener > 0.0)
        flatten_wc<P, R><<<nblocks(nzr, 256), 256, 0, st>>>(G, gam, prm.flattener, Uo, wcoef);
    RG_LAUNCH_CHECK();
    sm.mark(2, st);
    {
        // the sides' normal B at the face points go through the face-trace
        // buffer, which the predictor fills only later in the step
        double *sbn = reinterpret_cast<double *>(ftr);
        const int nch = (G.Nr + 2 + 63) / 64;
        zone_face_bn<P, R><<<(unsigned)((i64)G.ncol * nch), 64, 0, st>>>(G, Uo, wcoef, sbn, nch);
        face_bn_limit<P, R><<<nblocks((i64)G.ncol * (G.Nr + 3) + (i64)G.nae * (G.Nr + 2), 256), 256, 0, st>>>(
            G, Bo, sbn, bnod);
    }
    RG_LAUNCH_CHECK();
    sm.mark(3, st);
    constexpr int ZPW = 64 / Tr<P>::N;
    const int ntile = (G.Nr + 2 + 16 * BMAP_TILES - 1) / (16 * BMAP_TILES);
    bmap<P, R><<<(unsigned)((i64)G.ncol * ntile), 64, 0, st>>>(G, Uo, Bo, wcoef, bnod, bnode, g->zoneB);
    RG_LAUNCH_CHECK();
    sm.mark(4, st);
    predictor<P, R, MF><<<(unsigned)((nzr + ZPW - 1) / ZPW), 64, 0, st>>>(G, dt, gam, npic, Uo, wcoef, bnode, ftr, etr);
    RG_LAUNCH_CHECK();
    if (front_only) return RG_OK;
    sm.mark(5, st);
    const i64 nff = (i64)G.ncol * (G.Nr + 1) + (i64)G.nae * G.Nr;
    face_flux<P, R><<<nblocks(nff, flux_faces_per_block<P, R>()), 256, 0, st>>>(G, gam, ftr, g->Phi);
    RG_LAUNCH_CHECK();
    sm.mark(6, st);
    const i64 nee = (i64)G.nv * G.Nr + (i64)G.nae * (G.Nr + 1);
    edge_emf<R><<<nblocks(nee, 64), 192, 0, st>>>(G, gam, etr, g->Gam);
    RG_LAUNCH_CHECK();
    sm.mark(7, st);
    if (prm.fallback) {
        // round counters, face marks and edge marks are contiguous
        const i64 nclear = RG_FB_COUNTER_BYTES + G.NF + G.NE;
        fb_clear<<<nblocks((nclear + 15) / 16, 256), 256, 0, st>>>(reinterpret_cast<unsigned char *>(g->fbcnt), nclear);
        // a fixed number of rounds (no host synchronisation); the passes of a
        // round that flags no new zone exit at once
        for (int round = 0; round < FALLBACK_ROUNDS; round++) {
            fb_flag<<<nblocks(G.Z, 256), 256, 0, st>>>(G, dt, gam, round, g->Phi, g->zoneB, Uo, g->zfl, g->ffl,
                                                      g->efl, g->fbcnt);
            fb_traces<P, R><<<nblocks(nzr, 256), 256, 0, st>>>(G, gam, Uo, g->ffl, g->efl, ftr, etr, g->fbcnt + round);
            face_flux<P, R, true><<<nblocks(nff, flux_faces_per_block<P, R>()), 256, 0, st>>>(G, gam, ftr, g->Phi, g->ffl,
                                                                                 g->fbcnt + round);
            edge_emf<R, true><<<nblocks(nee, 64), 192, 0, st>>>(G, gam, etr, g->Gam, g->efl, g->fbcnt + round);
            RG_LAUNCH_CHECK();
        }
        g->fb_dirty = true;
        g->fb_last = true;
    } else if (g->fb_dirty) {
        fb_clear<<<nblocks((G.Z + 15) / 16, 256), 256, 0, st>>>(g->zfl, G.Z);
        RG_LAUNCH_CHECK();
        g->fb_dirty = false;
    }
    if (!prm.fallback) g->fb_last = false;
    zone_update<<<nblocks((i64)G.ncol * G.Nr, 256), 256, 0, st>>>(G, dt, g->Phi, g->zoneB, Uo,
                                                                  prm.fallback ? g->zfl : nullptr);
    face_ct<<<nblocks(nff, 256), 256, 0, st>>>(G, dt, g->Gam, Bo);
    RG_LAUNCH_CHECK();
    sm.mark(8, st);
    return RG_OK;
}

rg_status profile_end(rg_geom *g, double *ms, int *nsteps)
{
    for (int i = 0; i < RG_NSTAGE; i++) ms[i] = 0.0;
    const size_t per = RG_NSTAGE + 1, n = g->prof_events.size() / per;
    rg_status st = RG_OK;
    for (size_t s = 0; s < n; s++) {
        hipEvent_t *ev = reinterpret_cast<hipEvent_t *>(&g->prof_events[s * per]);
        if (hipEventSynchronize(ev[RG_NSTAGE]) != hipSuccess) st = RG_EDEVICE;
        for (int i = 0; i < RG_NSTAGE && st == RG_OK; i++) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) st = RG_EDEVICE;
            ms[i] += t;
        }
    }
    for (void *e : g->prof_events) (void)hipEventDestroy((hipEvent_t)e);
    g->prof_events.clear();
    g->prof_on = false;
    *nsteps = (int)n;
    if (st != RG_OK) set_error("reading the stage timers failed");
    return st;
}

template <int P>
static rg_status step_mode(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, double *Uo,
                           double *Bo, hipStream_t st, bool front_only)
{
    switch (g->mode) {
    case RG_MODE_FP64: return step_order<P, double>(g, p, U, Bf, Uo, Bo, st, front_only);
    case RG_MODE_FP32: return step_order<P, float>(g, p, U, Bf, Uo, Bo, st, front_only);
    case RG_MODE_BF16: return step_order<P, float, true>(g, p, U, Bf, Uo, Bo, st, front_only);
    }
    set_error("unknown precision mode");
    return RG_ENOTSUP;
}

rg_status launch_step(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, double *Uo, double *Bo,
                      void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->d.order == 3) return step_mode<3>(g, p, U, Bf, Uo, Bo, st, false);
    if (g->d.order == 4) return step_mode<4>(g, p, U, Bf, Uo, Bo, st, false);
    set_error("unsupported order");
    return RG_ENOTSUP;
}

rg_status launch_step_front(rg_geom *g, const rg_step_params &p, const double *U, const double *Bf, double *Uo,
                            double *Bo, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->d.order == 3) return step_mode<3>(g, p, U, Bf, Uo, Bo, st, true);
    if (g->d.order == 4) return step_mode<4>(g, p, U, Bf, Uo, Bo, st, true);
    set_error("unsupported order");
    return RG_ENOTSUP;
}

rg_status launch_stokes(rg_geom *g, const double *circ, double *Bf, void *stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGeom &G = g->d;
    stokes_faces<<<nblocks(G.NF, 256), 256, 0, st>>>(G, circ, Bf);
    RG_LAUNCH_CHECK();
    return RG_OK;
}

// The CFL reduction: cfl_partial leaves one minimum per block of 256
// interior zones in red[0 .. nb-1], cfl_final the global one in red[65535],
// which is copied to the host.  red holds CFL_RED_DOUBLES doubles.
constexpr int CFL_RED_DOUBLES = 65536;

static rg_status cfl_reduce(const DevGeom &G, const double *U, double gamma, double cfl, hipStream_t st, double *red,
                            double *dt)
{
    const i64 n = (i64)G.ncol * G.Nr;
    const unsigned nb = nblocks(n, 256);
    if (nb > CFL_RED_DOUBLES - 1) {
        set_error("mesh too large for the CFL reduction: " + std::to_string(n) + " interior zones, at most " +
                  std::to_string((long long)(CFL_RED_DOUBLES - 1) * 256));
        return RG_ENOTSUP;
    }
    cfl_partial<<<nb, 256, 0, st>>>(G, gamma, cfl, U, red);
    cfl_final<<<1, 256, 0, st>>>((int)nb, red);
    RG_LAUNCH_CHECK();
    if (hipMemcpyAsync(dt, red + CFL_RED_DOUBLES - 1, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("CFL reduction copy failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

rg_status launch_cfl(rg_geom *g, const double *U, double gamma, double cfl, void *stream, double *dt)
{
    return cfl_reduce(g->d, U, gamma, cfl, static_cast<hipStream_t>(stream), g->red, dt);
}

// ---------------------------------------------------------------- allocation-free CFL
// rg_cfl_dt_noalloc reduces through this file-scope array instead of the
// geometry's buffer.  Each device holds its own copy (512 KiB) for the life
// of the process; every call on a device shares it, so calls that overlap on
// one device race.  Its device address is taken once per device with
// hipGetSymbolAddress (the array's name is not a device address in host code).
__device__ __align__(256) double scratch[CFL_RED_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

rg_status launch_cfl_noalloc(rg_geom *g, const double *U, double gamma, double cfl, void *stream, double *dt)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_error("hipGetDevice failed or device index out of range");
        return RG_EDEVICE;
    }
    double *red = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                set_error(std::string("hipGetSymbolAddress of the CFL scratch failed: ") + hipGetErrorString(e));
                return RG_EDEVICE;
            }
            g_scratch_ptr[dev] = static_cast<double *>(p);
        }
        red = g_scratch_ptr[dev];
    }
    return cfl_reduce(g->d, U, gamma, cfl, static_cast<hipStream_t>(stream), red, dt);
}

}  // namespace rg

namespace rg {
rg_status launch_diag(rg_geom *g, const double *U, const double *Bf, double gamma, void *stream, rg_diag_out *out)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    static_assert((DIAG_BLOCKS + 1) * DIAG_NV <= 65536, "diagnostics fit the reduction buffer");
    diag_partial<<<DIAG_BLOCKS, 256, 0, st>>>(g->d, gamma, U, Bf, g->red);
    diag_final<<<1, 256, 0, st>>>(g->red);
    RG_LAUNCH_CHECK();
    double h[DIAG_NV];
    if (hipMemcpyAsync(h, g->red + DIAG_BLOCKS * DIAG_NV, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("diagnostics copy failed");
        return RG_EDEVICE;
    }
    out->div_rel_max = h[0];
    for (int v = 0; v < 8; v++) out->sums[v] = h[1 + v];
    out->rho_min = h[9];
    out->p_min = h[10];
    return RG_OK;
}
}  // namespace rg

// C-ABI of the rg library: argument checking, host precompute orchestration,
// device upload and the step entry points.  No exception crosses this file.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "dtab.hpp"
#include "rg_geom_host.hpp"

namespace rg {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

}  // namespace rg

using namespace rg;

extern "C" const char *rg_last_error(void) { return g_err.c_str(); }

extern "C" const char *rg_status_str(rg_status s)
{
    switch (s) {
    case RG_OK: return "RG_OK: success";
    case RG_EINVAL: return "RG_EINVAL: bad argument";
    case RG_ENOMEM: return "RG_ENOMEM: allocation failed";
    case RG_ESINGULAR: return "RG_ESINGULAR: singular least-squares or KKT system";
    case RG_ENOTSUP: return "RG_ENOTSUP: unsupported order, mode or mesh size";
    case RG_EDEVICE: return "RG_EDEVICE: HIP runtime call failed";
    }
    return "unknown rg_status";
}

extern "C" rg_status rg_mesh_build(const rg_mesh_desc *desc, rg_mesh **out)
{
    if (!desc || !out) { set_error("null argument"); return RG_EINVAL; }
    *out = nullptr;
    if (desc->n_rad < 1 || !(desc->r_in > 0) || !(desc->r_out > desc->r_in) || desc->radial != 0 ||
        desc->map_order < 2 || desc->map_order > 3 || desc->n_ghost < 0 || desc->n_ang < 2) {
        set_error("invalid mesh description");
        return RG_EINVAL;
    }
    rg_mesh *m = new (std::nothrow) rg_mesh;
    if (!m) { set_error("out of host memory"); return RG_ENOMEM; }
    try {
        if (!build_mesh(*desc, m->m)) {
            delete m;
            return RG_ENOTSUP;
        }
    } catch (const std::bad_alloc &) {
        delete m;
        set_error("out of host memory");
        return RG_ENOMEM;
    }
    *out = m;
    return RG_OK;
}

extern "C" rg_status rg_mesh_get_info(const rg_mesh *mesh, rg_mesh_info *info)
{
    if (!mesh || !info) { set_error("null argument"); return RG_EINVAL; }
    const Mesh &m = mesh->m;
    info->n_ang = m.N;
    info->n_rad = m.Nr;
    info->n_ghost = m.g;
    info->n_shells = m.K;
    info->n_columns = m.ncol;
    info->n_zones = m.nzones;
    info->n_faces = m.nfaces;
    info->n_radial_faces = m.nrf;
    info->n_edges = m.nedges;
    info->n_radial_edges = m.nre;
    info->n_vertices = m.nv;
    info->n_angular_edges = m.nae;
    return RG_OK;
}

extern "C" void rg_mesh_free(rg_mesh *mesh) { delete mesh; }

namespace {

// D_d[i][l] == D_0[S_d(i)][S_d(l)] with D_0 and the swaps S_d from dtab.hpp
template <int P>
bool check_dtab_order(const RefEl &r)
{
    using D = DTab<P>;
    const int N = r.N;
    std::vector<double> D0((size_t)N * N, 0.0);
    for (int e = 0; e < D::NNZ; e++) D0[(size_t)D::E[e][0] * N + D::E[e][1]] = 0.5 * D::E[e][2];
    // the transposed table holds the same entries, indexed (column, row), in row order
    for (int e = 0; e < D::NNZ; e++) {
        if (D0[(size_t)D::ET[e][1] * N + D::ET[e][0]] != 0.5 * D::ET[e][2]) return false;
        if (e > 0 && D::ET[e][0] < D::ET[e - 1][0]) return false;
    }
    for (int d = 0; d < 3; d++)
        for (int i = 0; i < N; i++)
            for (int l = 0; l < N; l++) {
                const int si = d == 0 ? i : d == 1 ? D::SWAP1[i] : D::SWAP2[i];
                const int sl = d == 0 ? l : d == 1 ? D::SWAP1[l] : D::SWAP2[l];
                if (r.D[((size_t)d * N + i) * N + l] != D0[(size_t)si * N + sl]) return false;
            }
    return true;
}

bool check_dtab(const RefEl &r)
{
    if (r.order == 3) return r.N == 20 && check_dtab_order<3>(r);
    if (r.order == 4) return r.N == 32 && check_dtab_order<4>(r);
    return false;
}


// A operands of the BF16 flux-derivative product (RG_MODE_BF16): lane l
// (r = l % 16, q = l / 16) holds, for each direction d and M tile m, the
// eight entries A_d[16 m + r][8 q + e] (e = 0..7) as packed bf16 pairs, with
// A_d[i][p] = D_0[S_d(i)][p]: the predictor stores each direction's fluxes at
// the swapped node positions S_d, so that A_d times that row is the
// d-derivative at node i (D_d = S_d D_0 S_d).  Rows or columns beyond N are
// zero.  Fails if an entry is not exact in BF16.
template <int P>
bool bf16_operands_order(const RefEl &r, std::vector<unsigned> &out)
{
    using D = DTab<P>;
    const int N = r.N;
    out.assign(64 * 3 * 2 * 4, 0u);
    for (int l = 0; l < 64; l++) {
        const int rr = l % 16, q = l / 16;
        for (int d = 0; d < 3; d++)
            for (int m = 0; m < 2; m++)
                for (int e = 0; e < 8; e++) {
                    const int i = 16 * m + rr, p = 8 * q + e;
                    double v = 0.0;
                    if (i < N && p < N) {
                        const int si = d == 0 ? i : d == 1 ? D::SWAP1[i] : D::SWAP2[i];
                        v = r.D[(size_t)si * N + p];   // the xi block of D: D_0
                    }
                    const float f = (float)v;
                    unsigned bits;
                    std::memcpy(&bits, &f, 4);
                    if ((double)f != v || (bits & 0xFFFFu) != 0u) return false;
                    out[((size_t)l * 6 + d * 2 + m) * 4 + e / 2] |= (bits >> 16) << (16 * (e % 2));
                }
    }
    return true;
}

bool bf16_derivative_operands(const RefEl &r, std::vector<unsigned> &out)
{
    if (r.order == 3) return bf16_operands_order<3>(r, out);
    if (r.order == 4) return bf16_operands_order<4>(r, out);
    return false;
}

template <typename T>
bool upload(rg_geom *g, const std::vector<T> &h, const T **dst)
{
    void *p = nullptr;
    size_t bytes = std::max<size_t>(sizeof(T), h.size() * sizeof(T));
    if (hipMalloc(&p, bytes) != hipSuccess) return false;
    g->allocations.push_back(p);
    if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return false;
    *dst = static_cast<const T *>(p);
    return true;
}

// FP32 copy of a double table (precision mode RG_MODE_FP32)
bool upload_f32(rg_geom *g, const std::vector<double> &h, const float **dst)
{
    std::vector<float> f(h.begin(), h.end());
    return upload(g, f, dst);
}

bool alloc_zero(rg_geom *g, size_t n, double **dst)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(8, n * sizeof(double))) != hipSuccess) return false;
    g->allocations.push_back(p);
    if (hipMemset(p, 0, n * sizeof(double)) != hipSuccess) return false;
    *dst = static_cast<double *>(p);
    return true;
}

void free_geom(rg_geom *g)
{
    if (!g) return;
    for (void *p : g->allocations) (void)hipFree(p);
    delete g;
}

}  // namespace

static rg_status precompute(const rg_mesh *mesh, int32_t order, int32_t mode, bool device, rg_geom **out)
{
    if (!mesh || !out) { set_error("null argument"); return RG_EINVAL; }
    *out = nullptr;
    if (order != 3 && order != 4) { set_error("order must be 3 or 4"); return RG_ENOTSUP; }
    if (mode != RG_MODE_FP64 && mode != RG_MODE_FP32 && mode != RG_MODE_BF16) {
        set_error("unknown precision mode");
        return RG_ENOTSUP;
    }
    const Mesh &m = mesh->m;
    if (m.g < order - 1) { set_error("n_ghost must be at least order - 1"); return RG_EINVAL; }
    rg_geom *g = new (std::nothrow) rg_geom;
    if (!g) { set_error("out of host memory"); return RG_ENOMEM; }
    g->mesh = mesh;
    g->mode = mode;
    RefEl &r = g->ref;
    HostGeom hg;
    try {
        if (!build_refel(order, r)) { set_error("reference element construction failed"); free_geom(g); return RG_ESINGULAR; }
        const int ncol = m.ncol, N = r.N, NC = r.NC, NS = r.NS, Q = r.Q;
        std::vector<ColData> cols(ncol);
#pragma omp parallel for schedule(dynamic, 16)
        for (int c = 0; c < ncol; c++) column_pass1(m, r, c, cols[c]);

        hg.stm.assign((size_t)ncol * NS, -1);
        hg.stn.assign(ncol, 0);
        hg.Pl.assign((size_t)ncol * NC * NS, 0.0);
        hg.Ps.assign((size_t)ncol * 7 * 18, 0.0);
        hg.Qs.assign((size_t)ncol * NC * NC, 0.0);
        hg.Ev.assign((size_t)ncol * N * NC, 0.0);
        hg.Mb.assign((size_t)ncol * r.NOUTB * r.NIN, 0.0);
        hg.nJ.assign((size_t)ncol * N, 0.0);
        hg.nM.assign((size_t)ncol * N * 9, 0.0);
        hg.fevR.assign((size_t)ncol * 2 * Q * NC, 0.0);
        hg.fnR.assign((size_t)ncol * Q * 3, 0.0);
        hg.fwR.assign((size_t)ncol * Q, 0.0);
        hg.dins.assign(ncol, 0.0);
        hg.cond_lsq.assign(ncol, 0.0);
        hg.cond_kkt.assign(ncol, 0.0);
        hg.col_ae.assign((size_t)ncol * 4, 0);
        hg.col_side.assign((size_t)ncol * 4, 0);
        hg.col_perm.assign((size_t)ncol * 4 * Q, 0);
        hg.col_v.assign((size_t)ncol * 4, 0);
        hg.col_slot.assign((size_t)ncol * 12, 0);
        hg.col_rev.assign((size_t)ncol * 12, 0);
        hg.col_sgn.assign((size_t)ncol * 4, 0);
        const int nae = m.nae, nv = m.nv;
        hg.fevA.assign((size_t)nae * 2 * Q * NC, 0.0);
        hg.fnA.assign((size_t)nae * Q * 3, 0.0);
        hg.fwA.assign((size_t)nae * Q, 0.0);
        hg.aeF.assign((size_t)nae * 27, 0.0);
        hg.aeW.assign((size_t)nae * 3, 0.0);
        hg.ae_rs.assign(nae, 0);
        hg.vF.assign((size_t)nv * 9, 0.0);
        hg.vN3.assign((size_t)nv * 9, 0.0);
        hg.emid_ae.assign((size_t)nae * 3, 0.0);
        hg.etan_ae.assign((size_t)nae * 3, 0.0);
        hg.fcen_ae.assign((size_t)nae * 3, 0.0);
        hg.fnrm_ae.assign((size_t)nae * 3, 0.0);
        hg.farea_ae.assign(nae, 0.0);

        int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : bad)
        for (int c = 0; c < ncol; c++)
            if (!column_pass2(m, r, cols, c, hg)) bad++;
        if (bad) { free_geom(g); return RG_ESINGULAR; }
        for (int c = 0; c < ncol; c++)
            if (!(hg.cond_lsq[c] <= RG_COND_MAX) || !(hg.cond_kkt[c] <= RG_COND_MAX)) {
                set_error("column " + std::to_string(c) + ": least-squares condition " +
                          std::to_string(hg.cond_lsq[c]) + ", KKT condition " + std::to_string(hg.cond_kkt[c]) +
                          " above the limit " + std::to_string(RG_COND_MAX));
                free_geom(g);
                return RG_ESINGULAR;
            }
        g->cond_lsq = hg.cond_lsq;
        g->cond_kkt = hg.cond_kkt;
#pragma omp parallel for schedule(dynamic, 64)
        for (int ae = 0; ae < nae; ae++) angular_edge_pass(m, r, cols, ae, hg);
#pragma omp parallel for schedule(dynamic, 64)
        for (int v = 0; v < nv; v++) vertex_pass(m, r, cols, v, hg);
#pragma omp parallel for schedule(static)
        for (int c = 0; c < ncol; c++) column_pass4(m, hg, c, hg);

        // per-zone, per-face scaled quantities and query copies
        const int K = m.K;
        std::vector<double> zscale(K + 1);
        for (int k = 0; k <= K; k++) zscale[k] = m.radius[k] / m.radius[0];
        const int64_t Z = m.nzones, NF = m.nfaces, NE = m.nedges;
        std::vector<double> vol(Z), area(NF);
        g->zcen.assign(Z * 3, 0.0);
        g->zvol.assign(Z, 0.0);
        g->fcen.assign(NF * 3, 0.0);
        g->fnrm.assign(NF * 3, 0.0);
        g->farea.assign(NF, 0.0);
        g->emid.assign(NE * 3, 0.0);
        g->etan.assign(NE * 3, 0.0);
        g->snode.assign((size_t)ncol * 48, 0.0);
        g->ae_rs_host = hg.ae_rs;
        g->col_side_host = hg.col_side;
        g->col_sgn_host = hg.col_sgn;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < ncol; c++) {
            const ColData &cd = cols[c];
            std::memcpy(&g->snode[(size_t)c * 48], cd.sn, sizeof(cd.sn));
            for (int k = 0; k < K; k++) {
                int64_t z = (int64_t)c * K + k;
                double s = zscale[k];
                vol[z] = cd.vol * s * s * s;
                g->zvol[z] = vol[z];
                for (int i = 0; i < 3; i++) g->zcen[z * 3 + i] = s * cd.cen[i];
            }
            for (int kf = 0; kf <= K; kf++) {
                int64_t f = (int64_t)c * (K + 1) + kf;
                double s = zscale[kf];
                area[f] = cd.farea[4] * s * s;
                g->farea[f] = area[f];
                for (int i = 0; i < 3; i++) {
                    g->fcen[f * 3 + i] = s * cd.fcen[4][i];
                    g->fnrm[f * 3 + i] = -cd.fnbar[4][i];
                }
            }
        }
#pragma omp parallel for schedule(static)
        for (int ae = 0; ae < nae; ae++) {
            for (int k = 0; k < K; k++) {
                int64_t f = m.nrf + (int64_t)ae * K + k;
                double s = zscale[k];
                area[f] = hg.farea_ae[ae] * s * s;
                g->farea[f] = area[f];
                for (int i = 0; i < 3; i++) {
                    g->fcen[f * 3 + i] = s * hg.fcen_ae[ae * 3 + i];
                    g->fnrm[f * 3 + i] = hg.fnrm_ae[ae * 3 + i];
                }
            }
            for (int kf = 0; kf <= K; kf++) {
                int64_t e = m.nre + (int64_t)ae * (K + 1) + kf;
                for (int i = 0; i < 3; i++) {
                    g->emid[e * 3 + i] = zscale[kf] * hg.emid_ae[ae * 3 + i];
                    g->etan[e * 3 + i] = hg.etan_ae[ae * 3 + i];
                }
            }
        }
        for (int v = 0; v < nv; v++)
            for (int k = 0; k < K; k++) {
                int64_t e = (int64_t)v * K + k;
                double rm = 0.5 * (m.radius[k] + m.radius[k + 1]);
                for (int i = 0; i < 3; i++) {
                    g->emid[e * 3 + i] = rm * m.vpos[3 * v + i];
                    g->etan[e * 3 + i] = m.vpos[3 * v + i];
                }
            }

        // The predictor applies the derivative matrices from compile-time
        // tables (D_0 and the coordinate swaps); they must match the computed
        // matrices exactly.
        if (!check_dtab(r)) {
            set_error("derivative matrices differ from the compiled-in tables");
            return RG_EINVAL;
        }
        // node-fastest / output-fastest copies of the per-column matrices
        std::vector<double> EvT((size_t)ncol * NC * N), MbT((size_t)ncol * r.NIN * r.NOUTB), nMT((size_t)ncol * 9 * N);
#pragma omp parallel for schedule(static)
        for (int c = 0; c < ncol; c++) {
            for (int i = 0; i < N; i++)
                for (int a = 0; a < NC; a++) EvT[((size_t)c * NC + a) * N + i] = hg.Ev[((size_t)c * N + i) * NC + a];
            for (int o = 0; o < r.NOUTB; o++)
                for (int j = 0; j < r.NIN; j++)
                    MbT[((size_t)c * r.NIN + j) * r.NOUTB + o] = hg.Mb[((size_t)c * r.NOUTB + o) * r.NIN + j];
            for (int i = 0; i < N; i++)
                for (int mm = 0; mm < 9; mm++) nMT[((size_t)c * 9 + mm) * N + i] = hg.nM[((size_t)c * N + i) * 9 + mm];
        }
        std::vector<double>().swap(hg.Mb);
        std::vector<double> Rv = r.R, wt = r.wt, radius = m.radius, zs(zscale.begin(), zscale.end() - 1);
        std::vector<int> vncol = m.v_ncol, aecol = m.ae_col, aev = m.ae_v, aelf = m.ae_lf;
        // adjoint tables: angular edges at each vertex, and for every column
        // the (stencil column, slot, radial offset) of the WENO stencils that
        // hold it
        std::vector<int> vae((size_t)nv * 4, -1), vcnt(nv, 0);
        for (int ae = 0; ae < nae; ae++)
            for (int s = 0; s < 2; s++) {
                const int v = m.ae_v[2 * ae + s];
                if (vcnt[v] >= 4) { set_error("vertex with more than four angular edges"); free_geom(g); return RG_ENOTSUP; }
                vae[(size_t)v * 4 + vcnt[v]++] = ae;
            }
        for (int v = 0; v < nv; v++)
            if (vcnt[v] != m.v_ncol[v]) { set_error("vertex edge count differs from its column count"); free_geom(g); return RG_ENOTSUP; }
        std::vector<int> invp(ncol + 1, 0), inve;
        for (int c2 = 0; c2 < ncol; c2++)
            for (int j = 0; j < NS; j++) {
                const int mm = hg.stm[(size_t)c2 * NS + j];
                if (mm >= 0) invp[(mm >> 3) + 1]++;
            }
        for (int c = 0; c < ncol; c++) invp[c + 1] += invp[c];
        inve.assign((size_t)invp[ncol] * 3, 0);
        {
            std::vector<int> fill(invp.begin(), invp.end() - 1);
            for (int c2 = 0; c2 < ncol; c2++)
                for (int j = 0; j < NS; j++) {
                    const int mm = hg.stm[(size_t)c2 * NS + j];
                    if (mm < 0) continue;
                    const int e = fill[mm >> 3]++;
                    inve[(size_t)e * 3] = c2;
                    inve[(size_t)e * 3 + 1] = j;
                    inve[(size_t)e * 3 + 2] = (mm & 7) - 3;
                }
        }

        if (!device) {
            *out = g;
            return RG_OK;
        }
        DevGeom &d = g->d;
        d.order = order; d.N = N; d.M = r.M; d.NC = NC; d.NB = r.NB; d.Q = Q; d.NS = NS;
        d.NIN = r.NIN; d.NOUTB = r.NOUTB; d.NFN = r.NFN; d.NEN = r.NEN;
        d.Nang = m.N; d.Nr = m.Nr; d.g = m.g; d.K = K; d.ncol = ncol; d.nv = nv; d.nae = nae;
        d.Z = Z; d.NF = NF; d.NRF = m.nrf; d.NE = NE; d.NRE = m.nre;
        bool ok = upload(g, radius, &d.radius) && upload(g, zs, &d.zscale) && upload(g, Rv, &d.R) &&
                  upload(g, wt, &d.wt) && upload(g, r.fnode, &d.fnode) && upload(g, r.fint, &d.fint) &&
                  upload(g, r.enode, &d.enode) && upload(g, r.eint, &d.eint) && upload(g, r.fintc, &d.fintc) &&
                  upload(g, r.eintc, &d.eintc) && upload(g, hg.stm, &d.stm) &&
                  upload(g, hg.Pl, &d.Pl) && upload(g, hg.Ps, &d.Ps) && upload(g, hg.Qs, &d.Qs) &&
                  upload(g, EvT, &d.Ev) && upload(g, MbT, &d.Mb) && upload(g, hg.nJ, &d.nJ) &&
                  upload(g, nMT, &d.nM) && upload(g, hg.fevR, &d.fevR) && upload(g, hg.fnR, &d.fnR) &&
                  upload(g, hg.fwR, &d.fwR) && upload(g, hg.col_ae, &d.col_ae) &&
                  upload(g, hg.col_side, &d.col_side) && upload(g, hg.col_perm, &d.col_perm) &&
                  upload(g, hg.col_v, &d.col_v) && upload(g, hg.col_slot, &d.col_slot) &&
                  upload(g, hg.col_rev, &d.col_rev) && upload(g, hg.col_sgn, &d.col_sgn) &&
                  upload(g, hg.dins, &d.dins) && upload(g, aecol, &d.ae_col) && upload(g, aev, &d.ae_v) &&
                  upload(g, hg.fevA, &d.fevA) && upload(g, hg.fnA, &d.fnA) && upload(g, hg.fwA, &d.fwA) &&
                  upload(g, hg.aeF, &d.aeF) && upload(g, hg.aeW, &d.aeW) && upload(g, hg.ae_rs, &d.ae_rs) &&
                  upload(g, vncol, &d.v_ncol) && upload(g, hg.vF, &d.vF) && upload(g, hg.vN3, &d.vN3) &&
                  upload(g, vol, &d.vol) && upload(g, area, &d.area) && upload(g, r.D, &d.Dfull) &&
                  upload(g, aelf, &d.ae_lf) && upload(g, vae, &d.v_ae) && upload(g, invp, &d.inv_ptr) &&
                  upload(g, inve, &d.inv_ent);
        if (ok && mode == RG_MODE_BF16) {
            std::vector<unsigned> dmf;
            if (!bf16_derivative_operands(r, dmf)) {
                set_error("derivative matrices are not exact in BF16");
                free_geom(g);
                return RG_EINVAL;
            }
            ok = upload(g, dmf, &d.DmfA);
        }
        if (ok && (mode == RG_MODE_FP32 || mode == RG_MODE_BF16))
            ok = upload_f32(g, hg.Pl, &d.PlF) && upload_f32(g, hg.Ps, &d.PsF) && upload_f32(g, hg.Qs, &d.QsF) &&
                 upload_f32(g, EvT, &d.EvF) && upload_f32(g, hg.nJ, &d.nJF) && upload_f32(g, nMT, &d.nMF) &&
                 upload_f32(g, hg.fevR, &d.fevRF) && upload_f32(g, hg.fevA, &d.fevAF) &&
                 upload_f32(g, r.fintc, &d.fintcF) && upload_f32(g, r.eintc, &d.eintcF);
        if (!ok) { set_error("device allocation or upload of the geometry failed"); free_geom(g); return RG_ENOMEM; }
        ok = alloc_zero(g, (size_t)NVAR * NC * Z, &g->wcoef) && alloc_zero(g, (size_t)Q * NF, &g->bnod) &&
             // the face traces; earlier in the step the same memory carries the
             // two sides' normal B at the face points (2 Q NF doubles)
             alloc_zero(g, (size_t)16 * Q * 2 * NF, &g->ftr) && alloc_zero(g, (size_t)9 * 3 * 4 * NE, &g->etr) &&
             alloc_zero(g, (size_t)NVAR * NF, &g->Phi) && alloc_zero(g, (size_t)NE, &g->Gam) &&
             alloc_zero(g, (size_t)3 * Z, &g->zoneB) && alloc_zero(g, 65536, &g->red) &&
             alloc_zero(g, (size_t)ncol * (m.Nr + 2) * 3 * N, &g->bnode);
        // fallback: round counters, face marks and edge marks contiguous
        // (cleared together), zone flags at a 256-byte aligned offset after
        double *fb = nullptr;
        const size_t marks = ((size_t)RG_FB_COUNTER_BYTES + NF + NE + 255) / 256 * 256;
        ok = ok && alloc_zero(g, (marks + Z + 7) / 8, &fb);
        if (!ok) { set_error("device allocation of the step work buffers failed"); free_geom(g); return RG_ENOMEM; }
        g->fbcnt = reinterpret_cast<int *>(fb);
        g->ffl = reinterpret_cast<unsigned char *>(fb) + RG_FB_COUNTER_BYTES;
        g->efl = g->ffl + NF;
        g->zfl = reinterpret_cast<unsigned char *>(fb) + marks;
        double *wh = nullptr;
        if (!alloc_zero(g, ((size_t)Z + 1) / 2, &wh)) {
            set_error("device allocation of the step work buffers failed");
            free_geom(g);
            return RG_ENOMEM;
        }
        g->whi = reinterpret_cast<float *>(wh);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory");
        free_geom(g);
        return RG_ENOMEM;
    }
    *out = g;
    return RG_OK;
}

extern "C" rg_status rg_geom_precompute(const rg_mesh *mesh, int32_t order, int32_t mode, void *stream, rg_geom **out)
{
    (void)stream;
    return precompute(mesh, order, mode, true, out);
}

extern "C" rg_status rg_geom_precompute_host(const rg_mesh *mesh, int32_t order, rg_geom **out)
{
    return precompute(mesh, order, RG_MODE_FP64, false, out);
}

extern "C" void rg_geom_free(rg_geom *geom) { free_geom(geom); }

extern "C" rg_status rg_geom_zone_data(const rg_geom *g, double *centroid, double *volume)
{
    if (!g) { set_error("null geometry"); return RG_EINVAL; }
    if (centroid) std::memcpy(centroid, g->zcen.data(), g->zcen.size() * sizeof(double));
    if (volume) std::memcpy(volume, g->zvol.data(), g->zvol.size() * sizeof(double));
    return RG_OK;
}

extern "C" rg_status rg_geom_face_data(const rg_geom *g, double *center, double *normal, double *area)
{
    if (!g) { set_error("null geometry"); return RG_EINVAL; }
    if (center) std::memcpy(center, g->fcen.data(), g->fcen.size() * sizeof(double));
    if (normal) std::memcpy(normal, g->fnrm.data(), g->fnrm.size() * sizeof(double));
    if (area) std::memcpy(area, g->farea.data(), g->farea.size() * sizeof(double));
    return RG_OK;
}

extern "C" rg_status rg_geom_conditioning(const rg_geom *g, double *cond_lsq, double *cond_kkt)
{
    if (!g) { set_error("null geometry"); return RG_EINVAL; }
    if (cond_lsq) std::memcpy(cond_lsq, g->cond_lsq.data(), g->cond_lsq.size() * sizeof(double));
    if (cond_kkt) std::memcpy(cond_kkt, g->cond_kkt.data(), g->cond_kkt.size() * sizeof(double));
    return RG_OK;
}

extern "C" rg_status rg_geom_edge_data(const rg_geom *g, double *midpoint, double *tangent)
{
    if (!g) { set_error("null geometry"); return RG_EINVAL; }
    if (midpoint) std::memcpy(midpoint, g->emid.data(), g->emid.size() * sizeof(double));
    if (tangent) std::memcpy(tangent, g->etan.data(), g->etan.size() * sizeof(double));
    return RG_OK;
}

extern "C" rg_status rg_geom_incidence(const rg_geom *g, int64_t *zone_face, int8_t *zone_face_sign,
                                       int64_t *face_edge, int8_t *face_edge_sign)
{
    if (!g || !g->mesh) { set_error("null geometry"); return RG_EINVAL; }
    const rg::Mesh &m = g->mesh->m;
    const int K = m.K;
    const int64_t NRF = m.nrf, NRE = m.nre;
    if (zone_face || zone_face_sign) {
        for (int c = 0; c < m.ncol; c++)
            for (int k = 0; k < K; k++) {
                const int64_t z = (int64_t)c * K + k;
                for (int lf = 0; lf < 6; lf++) {
                    int64_t f;
                    int sg;
                    if (lf < 4) {
                        // the canonical normal runs from side 0 to side 1 of the angular edge
                        f = NRF + (int64_t)m.col_ae[4 * c + lf] * K + k;
                        sg = g->col_side_host[4 * c + lf] == 0 ? 1 : -1;
                    } else {
                        f = (int64_t)c * (K + 1) + k + (lf - 4);   // normal +r
                        sg = lf == 5 ? 1 : -1;
                    }
                    if (zone_face) zone_face[z * 6 + lf] = f;
                    if (zone_face_sign) zone_face_sign[z * 6 + lf] = (int8_t)sg;
                }
            }
    }
    if (face_edge || face_edge_sign) {
        // radial face (c, kf): the four angular edges at interface kf
        for (int c = 0; c < m.ncol; c++)
            for (int kf = 0; kf <= K; kf++) {
                const int64_t f = (int64_t)c * (K + 1) + kf;
                for (int lf = 0; lf < 4; lf++) {
                    if (face_edge) face_edge[f * 4 + lf] = NRE + (int64_t)m.col_ae[4 * c + lf] * (K + 1) + kf;
                    if (face_edge_sign) face_edge_sign[f * 4 + lf] = (int8_t)g->col_sgn_host[4 * c + lf];
                }
            }
        // angular face (ae, k): its lower and upper angular edges and the
        // radial edges at the edge's two vertices
        for (int ae = 0; ae < m.nae; ae++) {
            const int rs = g->ae_rs_host[ae];
            for (int k = 0; k < K; k++) {
                const int64_t f = NRF + (int64_t)ae * K + k, ea = NRE + (int64_t)ae * (K + 1) + k;
                const int64_t e[4] = {ea, (int64_t)m.ae_v[2 * ae + 1] * K + k, ea + 1, (int64_t)m.ae_v[2 * ae] * K + k};
                const int sg[4] = {rs, rs, -rs, -rs};
                for (int j = 0; j < 4; j++) {
                    if (face_edge) face_edge[f * 4 + j] = e[j];
                    if (face_edge_sign) face_edge_sign[f * 4 + j] = (int8_t)sg[j];
                }
            }
        }
    }
    return RG_OK;
}

extern "C" rg_status rg_step(const rg_geom *geom, rg_step_params *params, const double *U, const double *Bf,
                             double *U_out, double *Bf_out, void *stream)
{
    if (!geom || !params || !U || !Bf || !U_out || !Bf_out) { set_error("null argument"); return RG_EINVAL; }
    if (!(params->gamma > 1.0) || params->bc_kind < 0 || params->bc_kind > 1 || params->n_picard < 0 ||
        !(params->weno_eps >= 0.0) || params->fallback < 0 || params->fallback > 1 || !(params->flattener >= 0.0)) {
        set_error("invalid step parameters");
        return RG_EINVAL;
    }
    rg_geom *g = const_cast<rg_geom *>(geom);
    if (!g->d.vol) { set_error("geometry was built without device data"); return RG_EINVAL; }
    if (!(params->dt > 0.0)) {
        if (!(params->cfl > 0.0)) { set_error("dt <= 0 needs cfl > 0"); return RG_EINVAL; }
        double dt = 0.0;
        rg_status s = launch_cfl(g, U, params->gamma, params->cfl, stream, &dt);
        if (s != RG_OK) return s;
        params->dt = dt;
    }
    return launch_step(g, *params, U, Bf, U_out, Bf_out, stream);
}

namespace {
bool alloc_adjoint(rg_geom *g)
{
    AdjBuffers &A = g->adj;
    if (A.ready) return true;
    const DevGeom &d = g->d;
    const size_t Z = d.Z, NF = d.NF, NE = d.NE, nzr = (size_t)d.ncol * (d.Nr + 2);
    const size_t NA = 3 * (size_t)(d.NC + 1);
    bool ok = alloc_zero(g, 8 * Z, &A.Ubc) && alloc_zero(g, NF, &A.Bbc) &&
              alloc_zero(g, (size_t)d.ncol * d.NIN * d.NOUTB, &A.MbA) && alloc_zero(g, 8 * Z, &A.gUo) && alloc_zero(g, NF, &A.gBo) &&
              alloc_zero(g, 3 * Z, &A.gzoneB) && alloc_zero(g, 8 * (size_t)d.NC * Z, &A.gwc) &&
              alloc_zero(g, (size_t)16 * d.Q * 2 * NF, &A.gftr) && alloc_zero(g, (size_t)9 * 3 * 4 * NE, &A.getr) &&
              alloc_zero(g, NE, &A.gGam) && alloc_zero(g, 8 * NF, &A.gPhi) &&
              alloc_zero(g, nzr * 3 * d.N, &A.gbnode) && alloc_zero(g, (size_t)d.Q * NF, &A.gbnod) &&
              alloc_zero(g, nzr * (d.NIN - NA), &A.gside) && alloc_zero(g, NF * 2 * (3 + 3 * (size_t)d.NC), &A.gsb) &&
              alloc_zero(g, 8 * (size_t)d.NS * nzr, &A.gdu);
    A.ready = ok;
    return ok;
}
}  // namespace

extern "C" rg_status rg_step_adjoint(const rg_geom *geom, const rg_step_params *params, const double *U_n,
                                     const double *Bf_n, const double *gU_np1, const double *gBf_np1, double *gU_n,
                                     double *gBf_n, void *stream)
{
    if (!geom || !params || !U_n || !Bf_n || !gU_np1 || !gBf_np1 || !gU_n || !gBf_n) {
        set_error("null argument");
        return RG_EINVAL;
    }
    if (!(params->gamma > 1.0) || params->bc_kind < 0 || params->bc_kind > 1 || params->n_picard < 0 ||
        !(params->weno_eps >= 0.0) || !(params->dt > 0.0)) {
        set_error("invalid step parameters (the adjoint needs a fixed dt > 0)");
        return RG_EINVAL;
    }
    rg_geom *g = const_cast<rg_geom *>(geom);
    if (!g->d.vol) { set_error("geometry was built without device data"); return RG_EINVAL; }
    if (params->fallback != 0) {
        set_error("the first-order fallback has no adjoint (run the adjoint with fallback = 0)");
        return RG_ENOTSUP;
    }
    if (params->flattener != 0.0) {
        set_error("the flattener has no adjoint (run the adjoint with flattener = 0)");
        return RG_ENOTSUP;
    }
    if (g->mode == RG_MODE_BF16) {
        set_error("the BF16 form has no adjoint (use RG_MODE_FP32 or RG_MODE_FP64)");
        return RG_ENOTSUP;
    }
    if ((const void *)gU_n == (const void *)gU_np1 || (const void *)gBf_n == (const void *)gBf_np1) {
        set_error("the adjoint cannot run in place");
        return RG_EINVAL;
    }
    if (!alloc_adjoint(g)) { set_error("device allocation of the adjoint buffers failed"); return RG_ENOMEM; }
    return launch_adjoint(g, *params, U_n, Bf_n, gU_np1, gBf_np1, gU_n, gBf_n, stream);
}

extern "C" rg_status rg_stokes(const rg_geom *g, const double *edge_circ, double *Bf, void *stream)
{
    if (!g || !edge_circ || !Bf) { set_error("null argument"); return RG_EINVAL; }
    if (!g->d.vol) { set_error("geometry was built without device data"); return RG_EINVAL; }
    return launch_stokes(const_cast<rg_geom *>(g), edge_circ, Bf, stream);
}

extern "C" rg_status rg_stokes_T(const rg_geom *g, const double *gBf, double *g_edge_circ, void *stream)
{
    if (!g || !gBf || !g_edge_circ) { set_error("null argument"); return RG_EINVAL; }
    if (!g->d.vol) { set_error("geometry was built without device data"); return RG_EINVAL; }
    return launch_stokes_T(const_cast<rg_geom *>(g), gBf, g_edge_circ, stream);
}

extern "C" rg_status rg_step_fluxes(const rg_geom *g, double *Phi, double *Gam, void *stream)
{
    if (!g || !g->d.vol) { set_error("null geometry or geometry without device data"); return RG_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (Phi && hipMemcpyAsync(Phi, g->Phi, sizeof(double) * NVAR * g->d.NF, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("hipMemcpyAsync failed");
        return RG_EDEVICE;
    }
    if (Gam && hipMemcpyAsync(Gam, g->Gam, sizeof(double) * g->d.NE, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("hipMemcpyAsync failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

extern "C" rg_status rg_step_fallback_zones(const rg_geom *g, uint8_t *flags, void *stream)
{
    if (!g || !g->d.vol) { set_error("null geometry or geometry without device data"); return RG_EINVAL; }
    if (!flags) { set_error("null argument"); return RG_EINVAL; }
    if (hipMemcpyAsync(flags, g->zfl, (size_t)g->d.Z, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)) !=
        hipSuccess) {
        set_error("hipMemcpyAsync failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

extern "C" rg_status rg_step_weno_order(const rg_geom *g, float *whi, void *stream)
{
    if (!g || !g->d.vol) { set_error("null geometry or geometry without device data"); return RG_EINVAL; }
    if (!whi) { set_error("null argument"); return RG_EINVAL; }
    if (hipMemcpyAsync(whi, g->whi, sizeof(float) * (size_t)g->d.Z, hipMemcpyDeviceToDevice,
                       static_cast<hipStream_t>(stream)) != hipSuccess) {
        set_error("hipMemcpyAsync failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

extern "C" rg_status rg_diag(const rg_geom *g, const double *U, const double *Bf, double gamma, void *stream,
                             rg_diag_out *out)
{
    if (!g || !U || !Bf || !out || !(gamma > 1.0)) { set_error("invalid argument"); return RG_EINVAL; }
    if (!g->d.vol) { set_error("geometry was built without a device copy"); return RG_EINVAL; }
    return launch_diag(const_cast<rg_geom *>(g), U, Bf, gamma, stream, out);
}

extern "C" rg_status rg_cfl_dt(const rg_geom *g, const double *U, double gamma, double cfl, void *stream, double *dt)
{
    if (!g || !g->d.vol || !U || !dt || !(cfl > 0) || !(gamma > 1)) { set_error("invalid argument"); return RG_EINVAL; }
    return launch_cfl(const_cast<rg_geom *>(g), U, gamma, cfl, stream, dt);
}

extern "C" rg_status rg_cfl_dt_noalloc(const rg_geom *g, const double *U, double gamma, double cfl, void *stream,
                                       double *dt)
{
    if (!g || !g->d.vol || !U || !dt || !(cfl > 0) || !(gamma > 1)) { set_error("invalid argument"); return RG_EINVAL; }
    return launch_cfl_noalloc(const_cast<rg_geom *>(g), U, gamma, cfl, stream, dt);
}

extern "C" rg_status rg_step_fallback_counts(const rg_geom *g, int32_t *counts, void *stream)
{
    if (!g || !g->d.vol || !counts) { set_error("invalid argument"); return RG_EINVAL; }
    if (!g->fb_last) {
        for (int r = 0; r < RG_FALLBACK_ROUNDS; r++) counts[r] = 0;
        return RG_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(counts, g->fbcnt, sizeof(int32_t) * RG_FALLBACK_ROUNDS, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("copy of the fallback counters failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

extern "C" rg_status rg_fma_probe(double *sink, int64_t n_threads, int32_t iters, void *stream)
{
    if (!sink) { set_error("null argument"); return RG_EINVAL; }
    return launch_fma_probe(sink, (long long)n_threads, (int)iters, stream);
}

extern "C" rg_status rg_mfma_probe(double *sink, int64_t n_threads, int32_t iters, int32_t kind, void *stream)
{
    if (!sink) { set_error("null argument"); return RG_EINVAL; }
    return launch_mfma_probe(sink, (long long)n_threads, (int)iters, (int)kind, stream);
}

extern "C" rg_status rg_profile_begin(rg_geom *g)
{
    if (!g || !g->d.vol) { set_error("null geometry or geometry without device data"); return RG_EINVAL; }
    if (g->prof_on) { set_error("profiling already active"); return RG_EINVAL; }
    g->prof_on = true;
    return RG_OK;
}

extern "C" rg_status rg_profile_end(rg_geom *g, double *ms, int32_t *nsteps)
{
    if (!g || !ms || !nsteps) { set_error("null argument"); return RG_EINVAL; }
    if (!g->prof_on) { set_error("profiling not active"); return RG_EINVAL; }
    int n = 0;
    rg_status s = profile_end(g, ms, &n);
    *nsteps = n;
    return s;
}

// Algorithmic work of one step, per stage (same numbering as the stage
// timers): floating-point operations counted from the formulas each stage
// evaluates (one FMA = 2), and the minimum HBM bytes: every input read once,
// every output written once, per-column matrices amortised over the column.
extern "C" rg_status rg_geom_work(const rg_geom *g, double *flops, double *bytes)
{
    if (!g || !flops || !bytes) { set_error("null argument"); return RG_EINVAL; }
    const RefEl &r = g->ref;
    const Mesh &m = g->mesh->m;
    const double N = r.N, NC = r.NC, NS = r.NS, Q = r.Q, NIN = r.NIN, E = r.M - 1, K = m.K;
    const double zr = (double)m.ncol * (m.Nr + 2);                       // reconstructed zones
    const double zi = (double)m.ncol * m.Nr;                             // interior zones
    const double fb = (double)m.ncol * (m.Nr + 3) + (double)m.nae * (m.Nr + 2);  // faces with nodal B
    const double ff = (double)m.ncol * (m.Nr + 1) + (double)m.nae * m.Nr;        // flux / CT faces
    const double ee = (double)m.nv * m.Nr + (double)m.nae * (m.Nr + 1);          // EMF edges
    double nnz = 0;
    for (double v : r.D) nnz += (v != 0.0);
    const double nnz_node = nnz / N;        // over the three directions
    const double FLUX = 96, FAST = 22, HLL = 2 * FAST + 14 + 8 * 7;
    // 0 boundary fill
    flops[0] = 0;
    bytes[0] = 2.0 * 8 * (8.0 * m.nzones + (double)m.nfaces);
    // 1 WENO-AO per variable: differences, large and small least squares,
    // smoothness forms, weights and the adaptive-order blend
    double wv = NS + 2 * NC * NS + 7 * 3 * 6 * 2 + 2 * NC * NC + 2 * NC + 90 + 2 * NC + 84;
    flops[1] = zr * 8 * wv;
    bytes[1] = 8 * (zr * (8 + 8 * NC) + m.ncol * (NC * NS + 126 + NC * NC));
    // 2 face nodal B: both sides' WENO B at Q points, minmod, mean restore
    flops[2] = fb * Q * (2 * 3 * 2 * (NC + 1) + 2 * 6 + 4 + 4);
    bytes[2] = 8 * (fb * (2 * (3 + 3 * NC) + 1 + Q) + m.ncol * (2 * Q * NC + 4 * Q) + m.nae * (2 * Q * NC + 4 * Q));
    // 3 divergence-free B map: dense per-column product
    flops[3] = zr * NIN * r.NOUTB * 2;
    bytes[3] = 8 * (zr * (NIN + r.NOUTB) + m.ncol * (NIN * r.NOUTB));
    // 4 ADER-CG predictor: nodal state, the tau = 0 flux derivative, a first
    // sweep from the constant guess (no flux evaluations), order - 1 full
    // sweeps, time averages, then traces at face points and edge points
    const double MAPPED = 8 + FLUX + 24 * 5, DERIV = nnz_node * 8 * 2, UPD = (E + 1) * 8 * 2;
    double init = N * (5 * NC * 2 + 8 + MAPPED + DERIV);
    double first = N * E * UPD;
    double sweep = N * E * (MAPPED + DERIV + UPD);
    double avg = N * E * (8 + FLUX + 32 * 2);
    double trc = 6 * 8 * Q * r.NFN * 4 * 2 + 6 * Q * 8 * 5 + 12 * 3 * r.NEN * 11 * 2;
    flops[4] = zr * (init + first + (r.order - 1) * sweep + avg + trc);
    bytes[4] = 8 * (zr * (5 * (NC + 1) + 3 * N + 6 * Q * 16 + 36 * 9) + m.ncol * N * (NC + 10));
    // 5 face HLL fluxes
    flops[5] = ff * Q * (HLL + 2 + 16);
    bytes[5] = 8 * (ff * (2 * 16 * Q + 8 + 1) + m.ncol * 4 * Q + m.nae * 4 * Q);
    // 6 edge EMFs (four-state solver at three Simpson points)
    flops[6] = ee * 3 * (4 * (2 * FAST + 4 * 5 + 8) + 40);
    bytes[6] = 8 * (ee * (3 * 4 * 9 + 1) + m.nae * 30.0 + m.nv * 18.0);
    // 7 finite-volume update and constrained transport
    flops[7] = zi * (8 * 6 * 2 + 8 * 2) + ff * 10;
    bytes[7] = 8 * (zi * (6 * 8 + 8 + 3 + 8 + 1) + ff * (4 + 2 + 1));
    (void)K;
    return RG_OK;
}

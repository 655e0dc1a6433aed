"""rg: ADER-WENO-AO divergence-free MHD timestep on a cube-based geodesic
shell mesh, as HIP kernels for AMD MI355X (gfx950).

The Python layer only marshals arguments to the C-ABI in include/rg.h (see
_native.py); PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N
from ._native import RGError, rg_step_params  # noqa: F401

__all__ = ["ShellMHD", "PrismMesh", "RGError", "rg_step_params"]


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return a.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class ShellMHD:
    """Mesh + precomputed geometry of one shell problem.

    device=False builds only the host geometry (queries and initial data);
    device=True also uploads it and allows steps on torch.cuda float64 tensors.
    """

    def __init__(self, n_ang, n_rad, order, r_in=1.0, r_out=2.0, map_order=None, n_ghost=3, device=True,
                 mode=N.RG_MODE_FP64):
        if map_order is None:
            map_order = order - 1
        self.order = order
        self._mesh = N.rg_mesh_build(n_ang, n_rad, r_in, r_out, map_order, n_ghost)
        self.info = N.rg_mesh_get_info(self._mesh)
        self.nz = self.info["n_zones"]
        self.nf = self.info["n_faces"]
        self.ne = self.info["n_edges"]
        self.K = self.info["n_shells"]
        self.g = self.info["n_ghost"]
        self.n_rad = n_rad
        self.device = device
        if device:
            self._geom = N.rg_geom_precompute(self._mesh, order, mode, _stream())
        else:
            self._geom = N.rg_geom_precompute_host(self._mesh, order)

    def close(self):
        if getattr(self, "_geom", None):
            N.rg_geom_free(self._geom)
            self._geom = None
        if getattr(self, "_mesh", None):
            N.rg_mesh_free(self._mesh)
            self._mesh = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # geometry queries ------------------------------------------------------
    def zone_data(self):
        cen = np.zeros((self.nz, 3)); vol = np.zeros(self.nz)
        N.rg_geom_zone_data(self._geom, _ptr(cen), _ptr(vol))
        return cen, vol

    def face_data(self):
        cen = np.zeros((self.nf, 3)); nrm = np.zeros((self.nf, 3)); area = np.zeros(self.nf)
        N.rg_geom_face_data(self._geom, _ptr(cen), _ptr(nrm), _ptr(area))
        return cen, nrm, area

    def edge_data(self):
        mid = np.zeros((self.ne, 3)); tan = np.zeros((self.ne, 3))
        N.rg_geom_edge_data(self._geom, _ptr(mid), _ptr(tan))
        return mid, tan

    def incidence(self):
        """rg_geom_incidence: (zone_face [nz, 6], zone_face_sign, face_edge [nf, 4], face_edge_sign)"""
        zf = np.zeros((self.nz, 6), np.int64); zs = np.zeros((self.nz, 6), np.int8)
        fe = np.zeros((self.nf, 4), np.int64); fs = np.zeros((self.nf, 4), np.int8)
        N.rg_geom_incidence(self._geom, _ptr(zf), _ptr(zs), _ptr(fe), _ptr(fs))
        return zf, zs, fe, fs

    def conditioning(self):
        """rg_geom_conditioning: per-column condition numbers of the large-stencil
        least squares (2-norm) and of the divergence-free KKT matrix (1-norm)."""
        ncol = self.info["n_columns"]
        lsq = np.zeros(ncol); kkt = np.zeros(ncol)
        N.rg_geom_conditioning(self._geom, _ptr(lsq), _ptr(kkt))
        return lsq, kkt

    def shells(self):
        return np.tile(np.arange(self.K), self.nz // self.K)

    def interior(self):
        k = self.shells()
        return (k >= self.g) & (k < self.g + self.n_rad)

    # initial data ------------------------------------------------------------
    def init_alfven(self, prob, t=0.0, noise=None, noise_amp=0.0):
        U = np.zeros((8, self.nz)); Bf = np.zeros(self.nf)
        frame = np.ascontiguousarray(prob["frame"], np.float64).ravel()
        nz = None if noise is None else np.ascontiguousarray(noise, np.float64)
        N.rg_init_alfven(self._geom, _ptr(frame), prob["rho"], prob["p"], prob["B0"], prob["dB"],
                         prob["wavelength"], prob["gamma"], float(t), _ptr(nz), float(noise_amp), _ptr(U), _ptr(Bf))
        return U, Bf

    def init_blast(self, prob):
        """rg_init_blast: host (U, Bf) of the magnetised blast; prob from
        rg_inputs.blast_problem (axis, centre, radius, rho, p_in, p, B0, gamma)."""
        U = np.zeros((8, self.nz)); Bf = np.zeros(self.nf)
        a = np.ascontiguousarray(prob["axis"], np.float64)
        c = np.ascontiguousarray(prob["centre"], np.float64)
        N.rg_init_blast(self._geom, _ptr(a), _ptr(c), float(prob["radius"]), float(prob["rho"]),
                        float(prob["p_in"]), float(prob["p"]), float(prob["B0"]), float(prob["gamma"]),
                        _ptr(U), _ptr(Bf))
        return U, Bf

    def init_tube(self, prob):
        """rg_init_tube: host (U, Bf) of a spherical shock tube; prob holds 'left' and
        'right' (rho, p, v_r, v_theta, v_phi, B_theta, B_phi), 'Br0', 'r0', 'rm',
        'delta' and 'gamma'."""
        U = np.zeros((8, self.nz)); Bf = np.zeros(self.nf)
        L, R = (np.ascontiguousarray(prob[k], np.float64) for k in ("left", "right"))
        if L.shape != (7,) or R.shape != (7,):
            raise ValueError("left and right are 7 primitive values each")
        N.rg_init_tube(self._geom, _ptr(L), _ptr(R), float(prob["Br0"]), float(prob["r0"]), float(prob["rm"]),
                       float(prob["delta"]), float(prob["gamma"]), _ptr(U), _ptr(Bf))
        return U, Bf

    # the step ------------------------------------------------------------------
    def step(self, U, Bf, dt, gamma=5.0 / 3.0, bc=0, U_out=None, Bf_out=None, cfl=0.0, n_picard=0, weno_eps=0.0,
             fallback=False, flattener=0.0):
        """One timestep on torch.cuda float64 tensors; returns (U_out, Bf_out, dt).
        fallback=True turns on the first-order fallback for zones the high-order
        update would leave with non-positive density or pressure; flattener > 0
        turns on the flattener with that threshold."""
        import torch
        assert U.is_cuda and U.dtype == torch.float64 and U.is_contiguous() and U.shape == (8, self.nz)
        assert Bf.is_cuda and Bf.dtype == torch.float64 and Bf.is_contiguous() and Bf.shape == (self.nf,)
        if U_out is None:
            U_out = torch.empty_like(U)
        if Bf_out is None:
            Bf_out = torch.empty_like(Bf)
        p = rg_step_params(gamma, dt, cfl, bc, n_picard, weno_eps, int(bool(fallback)), float(flattener))
        N.rg_step(self._geom, p, U.data_ptr(), Bf.data_ptr(), U_out.data_ptr(), Bf_out.data_ptr(), _stream())
        return U_out, Bf_out, p.dt

    def step_adjoint(self, U, Bf, gU1, gBf1, dt, gamma=5.0 / 3.0, bc=0, n_picard=0, gU=None, gBf=None,
                     weno_eps=0.0):
        """rg_step_adjoint: the gradients with respect to (U, Bf) of a loss whose
        gradients with respect to the step's outputs are (gU1, gBf1); dt fixed."""
        import torch
        for t, shape in ((U, (8, self.nz)), (Bf, (self.nf,)), (gU1, (8, self.nz)), (gBf1, (self.nf,))):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.shape == shape
        if not dt > 0:
            raise ValueError("the adjoint needs a fixed dt > 0")
        if gU is None:
            gU = torch.empty_like(U)
        if gBf is None:
            gBf = torch.empty_like(Bf)
        p = rg_step_params(gamma, dt, 0.0, bc, n_picard, weno_eps, 0)
        N.rg_step_adjoint(self._geom, p, U.data_ptr(), Bf.data_ptr(), gU1.data_ptr(), gBf1.data_ptr(),
                          gU.data_ptr(), gBf.data_ptr(), _stream())
        return gU, gBf

    def step_ad(self, U, Bf, dt, gamma=5.0 / 3.0, bc=0, n_picard=0):
        """Differentiable step (torch autograd): saves (U, Bf) as the step's
        checkpoint and recomputes the rest in the backward pass."""
        return _step_function().apply(U, Bf, self, float(dt), float(gamma), int(bc), int(n_picard))

    def rollout(self, U, Bf, dt, n_steps, gamma=5.0 / 3.0, bc=0, n_picard=0):
        """n_steps differentiable steps with fixed dt (one checkpoint per step)."""
        for _ in range(n_steps):
            U, Bf = self.step_ad(U, Bf, dt, gamma=gamma, bc=bc, n_picard=n_picard)
        return U, Bf

    def stokes(self, circ, Bf=None):
        """rg_stokes: face-averaged normal curl A from edge line integrals of A."""
        import torch
        assert circ.is_cuda and circ.dtype == torch.float64 and circ.is_contiguous() and circ.shape == (self.ne,)
        if Bf is None:
            Bf = torch.empty(self.nf, dtype=torch.float64, device=circ.device)
        N.rg_stokes(self._geom, circ.data_ptr(), Bf.data_ptr(), _stream())
        return Bf

    def stokes_T(self, gBf, gcirc=None):
        """rg_stokes_T: the transpose of stokes (face-B gradient -> edge gradient)."""
        import torch
        assert gBf.is_cuda and gBf.dtype == torch.float64 and gBf.is_contiguous() and gBf.shape == (self.nf,)
        if gcirc is None:
            gcirc = torch.empty(self.ne, dtype=torch.float64, device=gBf.device)
        N.rg_stokes_T(self._geom, gBf.data_ptr(), gcirc.data_ptr(), _stream())
        return gcirc

    def fluxes(self):
        import torch
        Phi = torch.zeros((8, self.nf), dtype=torch.float64, device="cuda")
        Gam = torch.zeros(self.ne, dtype=torch.float64, device="cuda")
        N.rg_step_fluxes(self._geom, Phi.data_ptr(), Gam.data_ptr(), _stream())
        return Phi, Gam

    def fallback_zones(self):
        """Per-zone flags (uint8 on the device) of the last step's first-order fallback."""
        import torch
        flags = torch.empty(self.nz, dtype=torch.uint8, device="cuda")
        N.rg_step_fallback_zones(self._geom, flags.data_ptr(), _stream())
        return flags

    def weno_order(self):
        """Per-zone WENO-AO order indicator of the last step (float32 on the device):
        the large stencil's weight over its linear weight, smallest over the variables."""
        import torch
        whi = torch.empty(self.nz, dtype=torch.float32, device="cuda")
        N.rg_step_weno_order(self._geom, whi.data_ptr(), _stream())
        return whi

    def cfl_dt(self, U, cfl, gamma=5.0 / 3.0):
        return N.rg_cfl_dt(self._geom, U.data_ptr(), gamma, cfl, _stream())

    def fallback_counts(self):
        """rg_step_fallback_counts: zones newly flagged in each round of the last step's fallback."""
        return N.rg_step_fallback_counts(self._geom, _stream())

    # per-stage timing ----------------------------------------------------------
    def diag(self, U, Bf, gamma=5.0 / 3.0):
        """rg_diag: max relative div B, volume-weighted sums, min rho and p."""
        return N.rg_diag(self._geom, U.data_ptr(), Bf.data_ptr(), gamma, _stream())

    def profile_begin(self):
        N.rg_profile_begin(self._geom)

    def profile_end(self):
        """-> ({stage: summed ms}, number of steps)"""
        return N.rg_profile_end(self._geom)

    def work(self):
        """-> ({stage: flops per step}, {stage: algorithmic HBM bytes per step})"""
        return N.rg_geom_work(self._geom)


class PrismMesh:
    """Icosahedral geodesic prism mesh of `level` (20 * 4^level triangles) and
    n_rad shells with the order-`order` prism element's geometry on the
    device (rg_prism_build).  Zone z = triangle * n_rad + shell."""

    def __init__(self, level, n_rad, order, r_in=1.0, r_out=2.0, device=True):
        build = N.rg_prism_build if device else N.rg_prism_build_host
        self._h = build(level, n_rad, r_in, r_out, order)
        info = N.rg_prism_get_info(self._h)
        self.nz, self.ntri, self.N = info["n_zones"], info["n_tri"], info["n_nodes"]
        self.Q = info["n_face_points"]
        self.n_edges, self.n_faces = info["n_edges"], info["n_faces"]
        self.n_divfree_in, self.n_divfree_out = info["n_divfree_in"], info["n_divfree_out"]
        self.n_vertices = info["n_vertices"]
        self.level, self.n_rad, self.order = level, n_rad, order

    def close(self):
        if getattr(self, "_h", None):
            N.rg_prism_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def triangles(self):
        abc = np.zeros((self.ntri, 3, 3))
        N.rg_prism_triangles(self._h, _ptr(abc))
        return abc

    def geometry(self, z0, nz):
        """host x[nz][N][3], J[nz][N], met[nz][N][3][3] of zones z0 .. z0 + nz - 1"""
        x, J, met = np.zeros((nz, self.N, 3)), np.zeros((nz, self.N)), np.zeros((nz, self.N, 3, 3))
        N.rg_prism_geometry(self._h, z0, nz, _ptr(x), _ptr(J), _ptr(met))
        return x, J, met

    def face_points(self):
        """reference face points [Q][3], weights [Q], points per triangle face, per side face"""
        xi, w = np.zeros((self.Q, 3)), np.zeros(self.Q)
        nt, ns = N.rg_prism_face_points(self._h, _ptr(xi), _ptr(w))
        return xi, w, nt, ns

    def traces(self, aU, aF, tr=None):
        """face-point traces [32][Q][nz] of predict()'s averages (float64 CUDA tensors)"""
        import torch
        assert aU.is_contiguous() and aF.is_contiguous()
        if tr is None:
            tr = torch.empty((32, self.Q, self.nz), dtype=torch.float64, device=aU.device)
        N.rg_prism_traces(self._h, _ptr(aU), _ptr(aF), _ptr(tr), _stream())
        return tr

    def edges(self):
        """[n_edges][4]: (t, local edge, t', local edge'), t < t'"""
        e = np.zeros((self.n_edges, 4), np.int32)
        N.rg_prism_edges(self._h, _ptr(e))
        return e

    def face_fluxes(self, tr, gamma=5.0 / 3.0, Phi=None):
        """HLL flux integrals [n_faces][8] of every face from traces() (CUDA tensors)"""
        import torch
        assert tr.is_contiguous()
        if Phi is None:
            Phi = torch.empty((self.n_faces, 8), dtype=torch.float64, device=tr.device)
        N.rg_prism_face_fluxes(self._h, gamma, _ptr(tr), _ptr(Phi), _stream())
        return Phi

    def volumes(self, z0=0, nz=None):
        nz = self.nz - z0 if nz is None else nz
        vol = np.zeros(nz)
        N.rg_prism_volumes(self._h, z0, nz, _ptr(vol))
        return vol

    def update(self, U, Phi, dt, Uo=None):
        """finite-volume update of the zone averages U [8][nz] (CUDA tensors)"""
        import torch
        assert U.is_contiguous() and Phi.is_contiguous() and tuple(U.shape) == (8, self.nz)
        if Uo is None:
            Uo = torch.empty_like(U)
        N.rg_prism_update(self._h, dt, _ptr(U), _ptr(Phi), _ptr(Uo), _stream())
        return Uo

    def divfree(self, Bin, Bout=None):
        """divergence-free B (Section IV.b): Bin [n_in][nz] -> Bout [n_out][nz] (CUDA tensors)"""
        import torch
        assert Bin.is_contiguous() and tuple(Bin.shape) == (self.n_divfree_in, self.nz)
        if Bout is None:
            Bout = torch.empty((self.n_divfree_out, self.nz), dtype=torch.float64, device=Bin.device)
        N.rg_prism_divfree(self._h, _ptr(Bin), _ptr(Bout), _stream())
        return Bout

    def divfree_host(self, Bin, z0=0):
        """the same map on the host: Bin [nz][n_in] -> [nz][n_out]"""
        Bin = np.ascontiguousarray(Bin, np.float64)
        out = np.zeros((len(Bin), self.n_divfree_out))
        N.rg_prism_divfree_host(self._h, z0, len(Bin), _ptr(Bin), _ptr(out))
        return out

    def edge_traces(self, aU, aF, er=None):
        """state and induction fluxes at the 27 edge points of every zone,
        [17][27][nz], from predict()'s outputs"""
        import torch
        assert aU.is_contiguous() and aF.is_contiguous()
        if er is None:
            er = torch.empty((17, 27, self.nz), dtype=torch.float64, device=aU.device)
        N.rg_prism_edge_traces(self._h, _ptr(aU), _ptr(aF), _ptr(er), _stream())
        return er

    def edge_emfs(self, er, gamma=5.0 / 3.0, Gang=None, Grad=None):
        """line integrals of E along the angular edges [n_edges][n_rad + 1]
        and the radial edges [n_vertices][n_rad] from edge_traces()"""
        import torch
        assert er.is_contiguous()
        if Gang is None:
            Gang = torch.empty((self.n_edges, self.n_rad + 1), dtype=torch.float64, device=er.device)
        if Grad is None:
            Grad = torch.empty((self.n_vertices, self.n_rad), dtype=torch.float64, device=er.device)
        N.rg_prism_edge_emfs(self._h, gamma, _ptr(er), _ptr(Gang), _ptr(Grad), _stream())
        return Gang, Grad

    def ct(self, PhiB, Gang, Grad, dt, out=None):
        """face magnetic fluxes [n_faces] after dt of constrained transport"""
        import torch
        if out is None:
            out = torch.empty_like(PhiB)
        N.rg_prism_ct(self._h, dt, _ptr(Gang), _ptr(Grad), _ptr(PhiB), _ptr(out), _stream())
        return out

    def vertices(self):
        """unit-sphere mesh vertices [n_vertices][3] in the library's numbering"""
        xyz = np.zeros((self.n_vertices, 3))
        N.rg_prism_vertices(self._h, _ptr(xyz))
        return xyz

    def work(self, n_picard=None):
        """-> (flops per zone, algorithmic HBM bytes per zone) of predict()"""
        return N.rg_prism_work(self._h, self.order if n_picard is None else n_picard)

    def predict(self, Ua, dt, gamma=5.0 / 3.0, n_picard=None, aU=None, aF=None):
        """ADER-CG predictor of every zone: Ua, aU [8][nz][N], aF [3][8][nz][N]
        float64 CUDA tensors (aU, aF allocated when not given)."""
        import torch
        assert Ua.dtype == torch.float64 and Ua.is_cuda and Ua.is_contiguous()
        assert tuple(Ua.shape) == (8, self.nz, self.N)
        if aU is None:
            aU = torch.empty_like(Ua)
        if aF is None:
            aF = torch.empty((3, 8, self.nz, self.N), dtype=torch.float64, device=Ua.device)
        N.rg_prism_predict(self._h, gamma, dt, self.order if n_picard is None else n_picard, _ptr(Ua), _ptr(aU),
                           _ptr(aF), _stream())
        return aU, aF


_STEP_FN = None


def _step_function():
    """torch.autograd.Function around rg_step / rg_step_adjoint (built on first use)."""
    global _STEP_FN
    if _STEP_FN is not None:
        return _STEP_FN
    import torch

    class StepFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, U, Bf, shell, dt, gamma, bc, n_picard):
            U = U.detach().contiguous()
            Bf = Bf.detach().contiguous()
            U1, Bf1, _ = shell.step(U, Bf, dt, gamma=gamma, bc=bc, n_picard=n_picard)
            ctx.save_for_backward(U, Bf)
            ctx.cfg = (shell, dt, gamma, bc, n_picard)
            return U1, Bf1

        @staticmethod
        def backward(ctx, gU1, gBf1):
            U, Bf = ctx.saved_tensors
            shell, dt, gamma, bc, n_picard = ctx.cfg
            gU1 = torch.zeros_like(U) if gU1 is None else gU1.contiguous()
            gBf1 = torch.zeros_like(Bf) if gBf1 is None else gBf1.contiguous()
            gU, gBf = shell.step_adjoint(U, Bf, gU1, gBf1, dt, gamma=gamma, bc=bc, n_picard=n_picard)
            return gU, gBf, None, None, None, None, None

    _STEP_FN = StepFn
    return StepFn

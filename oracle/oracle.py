"""ctypes access to the reference oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain FP64 CPU implementation of one ADER-WENO-AO
divergence-free MHD step written from the paper (Sections II-VI).  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may use
it; the GPU library never imports or links it.

Every part is pinned by the tests in tests/test_oracle_pins.py,
tests/test_oracle_pins_solvers.py (fast speed, HLL, the edge solvers and the
WENO-AO internals), tests/test_oracle_fallback.py, tests/test_tube_init.py
and, for the triangular-prism element on the icosahedral mesh (prism.c,
prism.py), tests/test_oracle_prism.py.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["la.c", "refel.c", "mesh.c", "geom.c", "scheme.c", "scheme_cx.c", "init.c", "oracle.c", "prism.c"]

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-shared", "-fPIC",
               *[os.path.join(_HERE, s) for s in _SOURCES], "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.rgo_create.restype = C.c_void_p
        L.rgo_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
        L.rgo_destroy.argtypes = [C.c_void_p]
        L.rgo_sizes.argtypes = [C.c_void_p, _lp]
        L.rgo_zone_data.argtypes = [C.c_void_p, _dp, _dp, _ip, _ip]
        L.rgo_zone_faces.argtypes = [C.c_void_p, _ip, _ip]
        L.rgo_face_data.argtypes = [C.c_void_p, _dp, _dp, _dp, _ip]
        L.rgo_face_quad.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.rgo_edge_data.argtypes = [C.c_void_p, _dp, _dp, _ip]
        L.rgo_face_edges.argtypes = [C.c_void_p, _ip, _ip]
        L.rgo_cubature.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.rgo_ncub.restype = C.c_int
        L.rgo_ncub.argtypes = [C.c_void_p]
        L.rgo_node_data.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.rgo_sphericity.restype = C.c_double
        L.rgo_sphericity.argtypes = [C.c_void_p, C.c_int]
        L.rgo_step.restype = C.c_int
        L.rgo_step.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double, _dp,
                               _dp, _dp, _dp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rgo_recon.restype = C.c_int
        L.rgo_recon.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, _dp, C.c_int, C.c_int, _dp, _dp, _dp]
        L.rgo_divfree.restype = C.c_int
        L.rgo_divfree.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, _dp, C.c_int, _dp, _ip, _dp]
        L.rgo_weno_order.restype = C.c_int
        L.rgo_weno_order.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _dp, _dp, _dp]
        L.rgo_cfl_dt.restype = C.c_double
        L.rgo_cfl_dt.argtypes = [C.c_void_p, C.c_double, C.c_double, _dp]
        L.rgo_init_harmonic.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, C.c_double, _dp, _dp]
        L.rgo_init_alfven.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.rgo_init_tube.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, _dp, _dp]
        L.rgo_refel_query.restype = C.c_int
        L.rgo_refel_query.argtypes = [C.c_int, _ip, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
        L.rgo_refel_eval.restype = C.c_int
        L.rgo_refel_eval.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.rgo_lagrange.restype = C.c_int
        L.rgo_lagrange.argtypes = [C.c_int, _dp, _ip, _dp]
        L.rgo_gauss01.argtypes = [C.c_int, _dp, _dp]
        L.rgo_predict.restype = C.c_int
        L.rgo_predict.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        L.rgo_hll.argtypes = [_dp, _dp, _dp, C.c_double, _dp]
        L.rgo_flux.argtypes = [_dp, C.c_double, _dp]
        L.rgo_emf.restype = C.c_double
        L.rgo_emf.argtypes = [_dp, _dp, _dp, _dp, C.c_double]
        L.rgo_fast.restype = C.c_double
        L.rgo_fast.argtypes = [_dp, C.c_double, _dp]
        L.rgo_emf3x.restype = C.c_double
        L.rgo_emf3x.argtypes = [_dp, _dp, _dp, _dp, C.c_double]
        L.rgo_init_blast.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, _dp, _dp]
        _cp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
        L.rgo_step_cx.restype = C.c_int
        L.rgo_step_cx.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                  _cp, _cp, _cp, _cp]
        L.rgo_weno_rows.restype = C.c_int
        L.rgo_weno_rows.argtypes = [C.c_void_p, C.c_int, _dp]
        L.rgo_weno_detail.restype = C.c_int
        L.rgo_weno_detail.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, C.c_int, _dp]
        _lib = L
    return _lib


NVAR = 8
FLAG_LINEAR_WEIGHTS = 1
# a-posteriori first-order fallback for zones the high-order update would
# leave with non-positive density or pressure (the step's own positivity
# measure; the paper defers positivity to the ruggedised-WENO literature)
FLAG_FALLBACK = 2
# epsilon of the WENO-AO nonlinear weights w_s ~ gamma_s / (beta_s + eps)^2
# (Section III defers the weights to the WENO-AO literature).  The smoothness
# indicators are in units of the squared zone data; 1e-4 lets the weights
# reach the linear ones on smooth, resolved data, which the scheme needs for
# the design order reported in Section VII (Tables I-II), while jumps with
# beta >> eps still switch to the small stencils.
WENO_EPS = 1e-4


class OracleMesh:
    """Cube-based geodesic shell mesh with per-zone geometry (oracle side)."""

    def __init__(self, n_ang, n_rad, r_in=1.0, r_out=2.0, n_ghost=3, map_order=None, order=3):
        if map_order is None:
            map_order = order - 1
        self.order = order
        self.n_ang, self.n_rad, self.r_in, self.r_out = n_ang, n_rad, r_in, r_out
        self._h = lib().rgo_create(n_ang, n_rad, r_in, r_out, n_ghost, map_order, order)
        if not self._h:
            raise ValueError("oracle mesh construction failed")
        s = np.zeros(8, np.int64)
        lib().rgo_sizes(self._h, s)
        self.nz, self.nf, self.ne, self.ktot, self.n_ghost, self.nquad, self.nv, self.nnodes = map(int, s)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rgo_destroy(h)
            self._h = None

    # geometry ---------------------------------------------------------
    def zones(self):
        cen = np.zeros((self.nz, 3)); vol = np.zeros(self.nz)
        shell = np.zeros(self.nz, np.int32); stn = np.zeros(self.nz, np.int32)
        lib().rgo_zone_data(self._h, cen, vol, shell, stn)
        return cen, vol, shell, stn

    def zone_faces(self):
        f = np.zeros((self.nz, 6), np.int32); n = np.zeros((self.nz, 6), np.int32)
        lib().rgo_zone_faces(self._h, f, n)
        return f, n

    def faces(self):
        cen = np.zeros((self.nf, 3)); nrm = np.zeros((self.nf, 3)); area = np.zeros(self.nf)
        zones = np.zeros((self.nf, 2), np.int32)
        lib().rgo_face_data(self._h, cen, nrm, area, zones)
        return cen, nrm, area, zones

    def face_quad(self):
        Q = (self.order - 1) ** 2
        x = np.zeros((self.nf, Q, 3)); n = np.zeros((self.nf, Q, 3)); dA = np.zeros((self.nf, Q))
        lib().rgo_face_quad(self._h, x, n, dA)
        return x, n, dA

    def edges(self):
        mid = np.zeros((self.ne, 3)); tan = np.zeros((self.ne, 3)); nzs = np.zeros(self.ne, np.int32)
        lib().rgo_edge_data(self._h, mid, tan, nzs)
        return mid, tan, nzs

    def face_edges(self):
        e = np.zeros((self.nf, 4), np.int32); s = np.zeros((self.nf, 4), np.int32)
        lib().rgo_face_edges(self._h, e, s)
        return e, s

    def cubature(self, z):
        n = lib().rgo_ncub(self._h)
        x = np.zeros((n, 3)); w = np.zeros(n)
        lib().rgo_cubature(self._h, int(z), x, w)
        return x, w

    def node_data(self, z):
        N = self.nnodes
        x = np.zeros((N, 3)); J = np.zeros(N); met = np.zeros((N, 3, 3))
        lib().rgo_node_data(self._h, int(z), x, J, met)
        return x, J, met

    def sphericity(self, samples=16):
        return lib().rgo_sphericity(self._h, samples)

    # initial data -------------------------------------------------------
    def init_harmonic(self, prob):
        U = np.zeros((NVAR, self.nz)); Bf = np.zeros(self.nf)
        lib().rgo_init_harmonic(self._h, np.ascontiguousarray(prob["rho"], np.float64),
                                np.ascontiguousarray(prob["v"], np.float64),
                                np.ascontiguousarray(prob["A"], np.float64),
                                float(prob["p"]), float(prob["gamma"]), U, Bf)
        return U, Bf

    def init_alfven(self, prob, t=0.0):
        U = np.zeros((NVAR, self.nz)); Bf = np.zeros(self.nf)
        lib().rgo_init_alfven(self._h, np.ascontiguousarray(prob["frame"], np.float64).ravel(),
                              prob["rho"], prob["p"], prob["B0"], prob["dB"], prob["wavelength"],
                              prob["gamma"], float(t), U, Bf)
        return U, Bf

    def init_tube(self, prob):
        """Spherical shock tube (Section VIII.c): prob holds the primitive states
        'left' and 'right' (rho, p, v_r, v_theta, v_phi, B_theta, B_phi; B_theta
        must be 0), 'Br0', 'r0', 'rm', 'delta' and 'gamma'."""
        U = np.zeros((NVAR, self.nz)); Bf = np.zeros(self.nf)
        L, R = (np.ascontiguousarray(prob[k], np.float64) for k in ("left", "right"))
        assert L.shape == (7,) and R.shape == (7,) and L[5] == 0.0 and R[5] == 0.0
        lib().rgo_init_tube(self._h, L, R, float(prob["Br0"]), float(prob["r0"]), float(prob["rm"]),
                            float(prob["delta"]), float(prob["gamma"]), U, Bf)
        return U, Bf

    def init_blast(self, prob):
        """Magnetised blast: prob from rg_inputs.blast_problem; zone averages of the
        pressure step by the zone cubature."""
        U = np.zeros((NVAR, self.nz)); Bf = np.zeros(self.nf)
        lib().rgo_init_blast(self._h, np.ascontiguousarray(prob["axis"], np.float64),
                             np.ascontiguousarray(prob["centre"], np.float64), float(prob["radius"]),
                             float(prob["rho"]), float(prob["p_in"]), float(prob["p"]), float(prob["B0"]),
                             float(prob["gamma"]), U, Bf)
        return U, Bf

    # the method -----------------------------------------------------------
    def step(self, U, Bf, dt, gamma=5.0 / 3.0, bc=0, flags=0, debug=False, weno_eps=WENO_EPS, fallback=False,
             flattener=0.0):
        """One step.  With fallback=True the first-order fallback is on and the
        per-zone flags (uint8, 1 = the zone fell back) are returned last; the
        round that flagged each zone (1-based, 0 = not flagged) is kept in
        self.last_fallback_round.  flattener > 0 turns the flattener on with
        that threshold kappa; its per-zone values are kept in self.last_eta."""
        U = np.ascontiguousarray(U, np.float64); Bf = np.ascontiguousarray(Bf, np.float64)
        Uo = np.zeros_like(U); Bo = np.zeros_like(Bf)
        phi = np.zeros((self.nf, NVAR)) if debug else None
        gam = np.zeros(self.ne) if debug else None
        fz = np.zeros(self.nz, np.uint8)
        if fallback:
            flags |= FLAG_FALLBACK
        eta = np.zeros(self.nz)
        rc = lib().rgo_step(self._h, gamma, dt, bc, flags, weno_eps, float(flattener), U, Bf, Uo, Bo,
                            phi.ctypes.data if debug else None, gam.ctypes.data if debug else None,
                            fz.ctypes.data, eta.ctypes.data)
        self.last_eta = eta
        if rc != 0:
            raise RuntimeError("oracle step failed")
        out = (Uo, Bo, phi, gam) if debug else (Uo, Bo)
        self.last_fallback_round = fz.copy()
        fz = (fz > 0).astype(np.uint8)
        return out + (fz,) if fallback else out

    def step_complex(self, U, Bf, dt, gamma=5.0 / 3.0, bc=0, flags=0, weno_eps=WENO_EPS, fallback=False,
                     flattener=0.0):
        """One step with complex state (complex128 arrays); the branches of the
        step decide on real parts.  With U = U0 + i h dU, Bf = Bf0 + i h dB
        (h about 1e-30) the imaginary parts of the outputs divided by h are the
        step's directional derivative along (dU, dB)."""
        U = np.ascontiguousarray(U, np.complex128); Bf = np.ascontiguousarray(Bf, np.complex128)
        Uo = np.zeros_like(U); Bo = np.zeros_like(Bf)
        if fallback:
            flags |= FLAG_FALLBACK
        rc = lib().rgo_step_cx(self._h, gamma, dt, bc, flags, weno_eps, float(flattener), U, Bf, Uo, Bo)
        if rc != 0:
            raise RuntimeError("oracle complex step failed")
        return Uo, Bo

    def recon(self, U, Bf, z, pts, flags=0, weno_eps=WENO_EPS):
        pts = np.ascontiguousarray(pts, np.float64)
        w = np.zeros((len(pts), NVAR)); b = np.zeros((len(pts), 3))
        rc = lib().rgo_recon(self._h, flags, weno_eps, np.ascontiguousarray(U), np.ascontiguousarray(Bf), int(z),
                             len(pts), pts, w, b)
        if rc != 0:
            raise RuntimeError("oracle reconstruction failed")
        return w, b

    def divfree(self, U, Bf, z, flags=0, weno_eps=WENO_EPS):
        nb = 16 if self.order == 3 else 30
        Q = (self.order - 1) ** 2
        c = np.zeros(3 * nb); e = np.zeros((3 * nb, 3), np.int32); fn = np.zeros((6, Q))
        rc = lib().rgo_divfree(self._h, flags, weno_eps, np.ascontiguousarray(U), np.ascontiguousarray(Bf), int(z),
                               c, e, fn)
        if rc != nb:
            raise RuntimeError("oracle divergence-free reconstruction failed")
        return c.reshape(3, nb), e.reshape(3, nb, 3), fn

    def weno_order(self, U, Bf, bc=0, flags=0, weno_eps=WENO_EPS):
        """Per-zone WENO-AO order indicator: min over variables of w_hi / gamma_hi."""
        out = np.zeros(self.nz)
        lib().rgo_weno_order(self._h, bc, flags, weno_eps, np.ascontiguousarray(U, np.float64),
                             np.ascontiguousarray(Bf, np.float64), out)
        return out

    def weno_rows(self, z):
        """Large-stencil least-squares matrix of zone z (members x Taylor coefficients)."""
        nc = 9 if self.order == 3 else 19
        A = np.zeros((40, nc))
        ns = lib().rgo_weno_rows(self._h, int(z), A)
        return A[:ns].copy()

    def weno_detail(self, U, z, flags=0, weno_eps=WENO_EPS):
        """WENO-AO internals of zone z (no boundary fill): per variable the
        smoothness indicators (large stencil, then the seven small ones), the
        normalised nonlinear weights in the same order and the blended Taylor
        coefficients (Section III)."""
        nc = 9 if self.order == 3 else 19
        out = np.zeros((NVAR, 16 + nc))
        rc = lib().rgo_weno_detail(self._h, flags, weno_eps, np.ascontiguousarray(U, np.float64), int(z), out)
        assert rc == nc
        return dict(beta=out[:, :8].copy(), w=out[:, 8:16].copy(), coef=out[:, 16:].copy())

    def cfl_dt(self, U, cfl, gamma=5.0 / 3.0):
        return lib().rgo_cfl_dt(self._h, gamma, cfl, np.ascontiguousarray(U))


def refel(order):
    NM = np.zeros(2, np.int32)
    lib().rgo_refel_query(order, NM, None, None, None, None, None, None, None)
    N, M = map(int, NM)
    E = (M - 1) * N
    tau = np.zeros(M); wt = np.zeros(M); nodes = np.zeros((N, 3)); D = np.zeros((3, N, N))
    Kd = np.zeros((3, E, E)); Kd0 = np.zeros((3, E, N)); Kt0 = np.zeros((E, N))
    lib().rgo_refel_query(order, NM, tau.ctypes.data, wt.ctypes.data, nodes.ctypes.data, D.ctypes.data,
                          Kd.ctypes.data, Kd0.ctypes.data, Kt0.ctypes.data)
    return dict(N=N, M=M, tau=tau, wt=wt, nodes=nodes, D=D, Kd=Kd, Kd0=Kd0, Kt0=Kt0)


def refel_eval(order, xi):
    xi = np.ascontiguousarray(xi, np.float64)
    N = 20 if order == 3 else 32
    out = np.zeros((len(xi), N))
    lib().rgo_refel_eval(order, len(xi), xi, out)
    return out


def lagrange(nodes, exps):
    nodes = np.ascontiguousarray(nodes, np.float64)
    exps = np.ascontiguousarray(exps, np.int32)
    n = len(nodes)
    coef = np.zeros((n, n))
    if lib().rgo_lagrange(n, nodes, exps, coef) != 0:
        raise RuntimeError("singular Vandermonde")
    return coef  # psi_l = sum_k coef[k, l] * mono_k


def gauss01(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().rgo_gauss01(n, x, w)
    return x, w


def predict(order, dt, J, met, Ua, gamma=5.0 / 3.0):
    N = len(J)
    M = order
    Ulev = np.zeros((M * N, NVAR)); aU = np.zeros((N, NVAR)); aF = np.zeros((N, 3, NVAR))
    lib().rgo_predict(order, gamma, dt, np.ascontiguousarray(J, np.float64),
                      np.ascontiguousarray(met, np.float64), np.ascontiguousarray(Ua, np.float64), Ulev, aU, aF)
    return Ulev.reshape(M, N, NVAR), aU, aF


def hll(UL, UR, n, gamma=5.0 / 3.0):
    out = np.zeros(NVAR)
    lib().rgo_hll(np.ascontiguousarray(UL, np.float64), np.ascontiguousarray(UR, np.float64),
                  np.ascontiguousarray(n, np.float64), gamma, out)
    return out


def flux(U, gamma=5.0 / 3.0):
    out = np.zeros((3, NVAR))
    lib().rgo_flux(np.ascontiguousarray(U, np.float64), gamma, out)
    return out


def emf4(U4, E4, cen4, t, gamma=5.0 / 3.0):
    return lib().rgo_emf(np.ascontiguousarray(U4, np.float64), np.ascontiguousarray(E4, np.float64),
                         np.ascontiguousarray(cen4, np.float64), np.ascontiguousarray(t, np.float64), gamma)


def fast_speed(U, n, gamma=5.0 / 3.0):
    return lib().rgo_fast(np.ascontiguousarray(U, np.float64), gamma, np.ascontiguousarray(n, np.float64))


def emf3(U3, E3, n3, t, gamma=5.0 / 3.0):
    """Three-zone edge electric field (E . t); n3[k] is the unit normal of the
    face from zone k to zone k+1 (mod 3)."""
    return lib().rgo_emf3x(np.ascontiguousarray(U3, np.float64), np.ascontiguousarray(E3, np.float64),
                           np.ascontiguousarray(n3, np.float64), np.ascontiguousarray(t, np.float64), gamma)

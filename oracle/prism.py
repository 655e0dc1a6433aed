"""Triangular-prism element on the icosahedral geodesic mesh, oracle side
(TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may use it; the GPU library never imports
or links it).

- Mesh (Section II.a, Fig. 1): the icosahedron projected to the unit sphere
  gives 20 spherical triangles (level 0); each level splits every triangle
  into four by the great-circle midpoints of its edges, (a + b)/|a + b|, so
  level L has 20 4^L triangles.  The radial direction is cut into n_rad
  shells with logarithmically spaced radii (Section VII), and each
  (triangle, shell) pair is a curved prism zone (Fig. 2).
- Numbering: vertices 0 (north pole), 1-5 (upper ring at z = 1/sqrt 5,
  longitudes 72 k degrees), 6-10 (lower ring, longitudes 36 + 72 k), 11
  (south pole); the 20 level-0 faces are, for k = 0..4 (k1 = k + 1 mod 5),
  (0, 1+k, 1+k1), (1+k, 6+k, 1+k1), (1+k1, 6+k, 6+k1), (11, 6+k1, 6+k), each
  turned counter-clockwise as seen from outside; the children of triangle t
  (a, b, c) with midpoints m_ab, m_bc, m_ca are 4t + (0: a m_ab m_ca,
  1: m_ab b m_bc, 2: m_ca m_bc c, 3: m_ab m_bc m_ca).  Zone z = t n_rad + k.
- Zone geometry and the element predictor are in prism.c.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import oracle as O

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")

NODES = {2: 6, 3: 15, 4: 26}


def _lib():
    L = O.lib()
    if not getattr(L, "_prism_ready", False):
        L.rgo_prism_refel_query.restype = C.c_int
        L.rgo_prism_refel_query.argtypes = [C.c_int, _ip] + [C.c_void_p] * 9
        L.rgo_prism_geometry.restype = C.c_int
        L.rgo_prism_geometry.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.rgo_prism_predict.restype = C.c_int
        L.rgo_prism_predict.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _dp, _dp, _dp, C.c_void_p,
                                        _dp, _dp]
        L.rgo_prism_face_points.restype = C.c_int
        L.rgo_prism_face_points.argtypes = [C.c_int, _dp, _dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.rgo_prism_traces.restype = C.c_int
        L.rgo_prism_traces.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.rgo_prism_face_geometry.restype = C.c_int
        L.rgo_prism_face_geometry.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.rgo_prism_hll.restype = None
        L.rgo_prism_hll.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_double, _dp]
        L.rgo_prism_volumes.restype = C.c_int
        L.rgo_prism_volumes.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.rgo_prism_divfree.restype = C.c_int
        L.rgo_prism_divfree.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.rgo_prism_divfree_sizes.restype = None
        L.rgo_prism_divfree_sizes.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.rgo_prism_frames.restype = C.c_int
        L.rgo_prism_frames.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L._prism_ready = True
    return L


def refel(order):
    """Prism reference element: nodes, monomials, basis coefficients
    (psi_l = sum_k coef[k, l] m_k), nodal derivative matrices D[d, i, l] =
    d psi_l / d xi_d at node i, and the full-Galerkin matrices of eq. (5.29)."""
    N, M = NODES[order], order
    E = (M - 1) * N
    NM = np.zeros(2, np.int32)
    tau, wt = np.zeros(M), np.zeros(M)
    nodes, exps, coef = np.zeros((N, 3)), np.zeros((N, 3), np.int32), np.zeros((N, N))
    D, Kd, Kd0, Kt0 = np.zeros((3, N, N)), np.zeros((3, E, E)), np.zeros((3, E, N)), np.zeros((E, N))
    rc = _lib().rgo_prism_refel_query(order, NM, tau.ctypes, wt.ctypes, nodes.ctypes, exps.ctypes, coef.ctypes,
                                      D.ctypes, Kd.ctypes, Kd0.ctypes, Kt0.ctypes)
    if rc:
        raise ValueError("prism reference element failed")
    return dict(N=N, M=M, tau=tau, wt=wt, nodes=nodes, exps=exps, coef=coef, D=D, Kd=Kd, Kd0=Kd0, Kt0=Kt0)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def icosahedron():
    """The 12 vertices and 20 outward counter-clockwise faces of level 0."""
    h, rho = 1 / np.sqrt(5), 2 / np.sqrt(5)
    V = [np.array([0.0, 0.0, 1.0])]
    for k in range(5):
        a = 2 * np.pi * k / 5
        V.append(np.array([rho * np.cos(a), rho * np.sin(a), h]))
    for k in range(5):
        a = 2 * np.pi * (k + 0.5) / 5
        V.append(np.array([rho * np.cos(a), rho * np.sin(a), -h]))
    V.append(np.array([0.0, 0.0, -1.0]))
    F = []
    for k in range(5):
        k1 = (k + 1) % 5
        F += [(0, 1 + k, 1 + k1), (1 + k, 6 + k, 1 + k1), (1 + k1, 6 + k, 6 + k1), (11, 6 + k1, 6 + k)]
    out = []
    for a, b, c in F:
        if np.cross(V[b] - V[a], V[c] - V[a]) @ (V[a] + V[b] + V[c]) < 0:
            b, c = c, b
        out.append((a, b, c))
    return np.array(V), np.array(out, np.int64)


def subdivide(V, T):
    """One level of great-circle bisection: vertices shared through an edge
    table, children in the order documented above."""
    V = list(V)
    mid = {}

    def m(i, j):
        key = (min(i, j), max(i, j))
        if key not in mid:
            mid[key] = len(V)
            V.append(_unit(V[i] + V[j]))
        return mid[key]

    out = np.empty((4 * len(T), 3), np.int64)
    for t, (a, b, c) in enumerate(T):
        ab, bc, ca = m(a, b), m(b, c), m(c, a)
        out[4 * t:4 * t + 4] = [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
    return np.array(V), out


class OraclePrismMesh:
    """Icosahedral geodesic prism mesh with per-zone geometry on demand."""

    def __init__(self, level, n_rad, r_in=1.0, r_out=2.0, order=4):
        V, T = icosahedron()
        for _ in range(level):
            V, T = subdivide(V, T)
        self.level, self.n_rad, self.order = level, n_rad, order
        self.vert, self.tri = V, T
        self.ntri = len(T)
        self.nz = self.ntri * n_rad
        self.N = NODES[order]
        self.radius = r_in * (r_out / r_in) ** (np.arange(n_rad + 1) / n_rad)

    def zone_tri_shell(self, zones):
        zones = np.asarray(zones, np.int64)
        return zones // self.n_rad, zones % self.n_rad

    def geometry(self, zones):
        """x[z][N][3], J[z][N], met[z][N][d][n] of the given zones."""
        t, k = self.zone_tri_shell(zones)
        nz = len(t)
        abc = np.ascontiguousarray(self.vert[self.tri[t]].reshape(nz, 9))
        r01 = np.ascontiguousarray(np.stack([self.radius[k], self.radius[k + 1]], 1))
        x, J, met = np.zeros((nz, self.N, 3)), np.zeros((nz, self.N)), np.zeros((nz, self.N, 3, 3))
        if _lib().rgo_prism_geometry(self.order, nz, abc, r01, x, J, met):
            raise ValueError("prism geometry failed")
        return x, J, met

    def face_geometry(self, zones):
        """face-point positions xq[z][Q][3] and weighted outward area vectors
        dAw[z][Q][3] of the given zones"""
        t, k = self.zone_tri_shell(zones)
        nz = len(t)
        Q = len(face_points(self.order)[1])
        abc = np.ascontiguousarray(self.vert[self.tri[t]].reshape(nz, 9))
        r01 = np.ascontiguousarray(np.stack([self.radius[k], self.radius[k + 1]], 1))
        xq, dA = np.zeros((nz, Q, 3)), np.zeros((nz, Q, 3))
        if _lib().rgo_prism_face_geometry(self.order, nz, abc, r01, xq, dA):
            raise ValueError("prism face geometry failed")
        return xq, dA

    def edges(self):
        """mesh edges in first-encounter order over (triangle, local edge
        0: a-b, 1: b-c, 2: c-a): [n_edges][4] = (t, local edge, t', local edge'),
        t < t'"""
        where = {}
        for t, (a, b, c) in enumerate(self.tri):
            for e, (u, v) in enumerate(((a, b), (b, c), (c, a))):
                where[(u, v)] = (t, e)
        out = []
        for t, (a, b, c) in enumerate(self.tri):
            for e, (u, v) in enumerate(((a, b), (b, c), (c, a))):
                t2, e2 = where[(v, u)]
                if t < t2:
                    out.append((t, e, t2, e2))
        return np.array(out, np.int64)

    def face_fluxes(self, tr, gamma=5.0 / 3.0):
        """HLL flux integrals over every face from the traces tr[z][Q][32] of
        the predictor's averages (Section VI): radial faces first,
        f = t (n_rad + 1) + kf, along +r (boundary faces take the one zone's
        trace on both sides); then side faces n_radial + e n_rad + k, along the
        outward normal of edge e's first triangle t.  -> Phi[n_faces][8]"""
        order, nr = self.order, self.n_rad
        xi, w, nt, ns = face_points(order)
        Q = len(w)
        zones = np.arange(self.nz)
        xq, dA = self.face_geometry(zones)
        E = self.edges()
        nrf = self.ntri * (nr + 1)
        Phi = np.zeros((nrf + len(E) * nr, 8))
        # radial faces: the zone below (top face, points 0..nt) or, at the
        # inner boundary, the zone above (bottom face, points nt..2nt, turned)
        for t in range(self.ntri):
            for kf in range(nr + 1):
                below, above = (t * nr + kf - 1 if kf > 0 else None), (t * nr + kf if kf < nr else None)
                if below is not None:
                    qs = np.arange(nt); zl, A = below, dA[below, :nt]
                else:
                    qs = np.arange(nt, 2 * nt); zl, A = above, -dA[above, nt:2 * nt]
                zr = above if above is not None else below
                qr = np.arange(nt, 2 * nt) if above is not None else np.arange(nt)
                Phi[t * (nr + 1) + kf] = self._integrate(tr[zl, qs], tr[zr, qr], A, gamma)
        # side faces: the neighbour's point at the same height, mirrored along the edge
        xs = xi[2 * nt:2 * nt + ns]
        sx = xs[:, 0] + 0.5                                     # position along edge 0 (xi from -1/2 to 1/2)
        mirror = [int(np.argmin(np.abs(sx - (1 - sx[i])) + np.abs(xs[:, 2] - xs[i, 2]))) for i in range(ns)]
        for e, (t1, e1, t2, e2) in enumerate(E):
            for k in range(nr):
                z1, z2 = t1 * nr + k, t2 * nr + k
                q1 = 2 * nt + e1 * ns + np.arange(ns)
                q2 = 2 * nt + e2 * ns + np.array(mirror)
                Phi[nrf + e * nr + k] = self._integrate(tr[z1, q1], tr[z2, q2], dA[z1, q1 - 0], gamma)
        return Phi

    @staticmethod
    def _integrate(tl, tr_, A, gamma):
        a = np.linalg.norm(A, axis=1)
        n = np.ascontiguousarray(A / a[:, None])
        Fs = np.zeros((len(a), 8))
        _lib().rgo_prism_hll(len(a), np.ascontiguousarray(tl[:, :8]), np.ascontiguousarray(tr_[:, :8]),
                             np.ascontiguousarray(tl[:, 8:]), np.ascontiguousarray(tr_[:, 8:]), n, gamma, Fs)
        return (a[:, None] * Fs).sum(0)

    def volumes(self, zones):
        t, k = self.zone_tri_shell(zones)
        nz = len(t)
        abc = np.ascontiguousarray(self.vert[self.tri[t]].reshape(nz, 9))
        r01 = np.ascontiguousarray(np.stack([self.radius[k], self.radius[k + 1]], 1))
        vol = np.zeros(nz)
        if _lib().rgo_prism_volumes(self.order, nz, abc, r01, vol):
            raise ValueError("prism volumes failed")
        return vol

    def _abc_r01(self, zones):
        t, k = self.zone_tri_shell(zones)
        nz = len(t)
        abc = np.ascontiguousarray(self.vert[self.tri[t]].reshape(nz, 9))
        r01 = np.ascontiguousarray(np.stack([self.radius[k], self.radius[k + 1]], 1))
        return nz, abc, r01

    def frames(self, zones):
        """zone centroids [z][3] and Taylor lengths l0 = V^(1/3) [z]"""
        nz, abc, r01 = self._abc_r01(zones)
        cen, l0 = np.zeros((nz, 3)), np.zeros(nz)
        if _lib().rgo_prism_frames(self.order, nz, abc, r01, cen, l0):
            raise ValueError("prism frames failed")
        return cen, l0

    def divfree(self, zones, Bin):
        """divergence-free reconstruction of B (Section IV.b, five faces) from
        Bin[z][NIN] (see prism.c) -> [z][3N + 3]: B at the nodes, zone means"""
        nz, abc, r01 = self._abc_r01(zones)
        nin, nout = divfree_sizes(self.order)
        out = np.zeros((nz, nout))
        if _lib().rgo_prism_divfree(self.order, nz, abc, r01, np.ascontiguousarray(Bin, np.float64), out):
            raise ValueError("prism divergence-free reconstruction failed")
        return out

    def zone_faces(self):
        """for every zone its five faces with the sign of the zone's outward
        normal relative to the face's direction: [nz][5] faces, [nz][5] signs"""
        nr, nrf = self.n_rad, self.ntri * (self.n_rad + 1)
        F = np.zeros((self.nz, 5), np.int64); S = np.zeros((self.nz, 5))
        cnt = np.zeros(self.nz, np.int64)
        def put(z, f, s):
            F[z, cnt[z]] = f; S[z, cnt[z]] = s; cnt[z] += 1
        for t in range(self.ntri):
            for k in range(nr):
                put(t * nr + k, t * (nr + 1) + k + 1, 1.0)
                put(t * nr + k, t * (nr + 1) + k, -1.0)
        for e, (t1, e1, t2, e2) in enumerate(self.edges()):
            for k in range(nr):
                put(t1 * nr + k, nrf + e * nr + k, 1.0)
                put(t2 * nr + k, nrf + e * nr + k, -1.0)
        assert np.all(cnt == 5)
        return F, S

    def update(self, U, Phi, dt):
        """finite-volume update of the zone averages U[nz][8] (Section VI):
        U - dt / V sum over the zone's faces of the outward face flux"""
        F, S = self.zone_faces()
        vol = self.volumes(np.arange(self.nz))
        net = (S[:, :, None] * Phi[F]).sum(1)
        return U - dt / vol[:, None] * net

    def predict(self, zones, Ua, dt, gamma=5.0 / 3.0):
        """Element predictor of the given zones from nodal states Ua[z][N][8]:
        time-averaged nodal state avgU[z][N][8] and flux avgF[z][N][3][8]."""
        _, J, met = self.geometry(zones)
        return predict(self.order, J, met, Ua, dt, gamma)


def predict(order, J, met, Ua, dt, gamma=5.0 / 3.0, levels=False):
    """avgU[z][N][8], avgF[z][N][3][8] (and with levels=True also
    Ulev[z][M][N][8], J times the state at each time level)."""
    nz, N = J.shape
    Ua = np.ascontiguousarray(Ua, dtype=np.float64)
    aU, aF = np.zeros((nz, N, 8)), np.zeros((nz, N, 3, 8))
    Ul = np.zeros((nz, order, N, 8)) if levels else None
    if _lib().rgo_prism_predict(order, nz, gamma, dt, np.ascontiguousarray(J), np.ascontiguousarray(met), Ua,
                                Ul.ctypes if levels else None, aU, aF):
        raise ValueError("prism predictor failed")
    return (aU, aF, Ul) if levels else (aU, aF)


def face_points(order):
    """reference points [Q][3], weights [Q] (fractions of each face's area),
    points per triangle face and per side face: faces zeta = +1/2, -1/2, then
    the side faces on triangle edges 0-1, 1-2, 2-0 (Appendix A)"""
    xi, w = np.zeros(38 * 3), np.zeros(38)
    nt, ns = C.c_int(0), C.c_int(0)
    Q = _lib().rgo_prism_face_points(order, xi, w, C.byref(nt), C.byref(ns))
    if Q < 0:
        raise ValueError("order must be 2, 3 or 4")
    return xi[:3 * Q].reshape(Q, 3), w[:Q], nt.value, ns.value


def traces(order, aU, aF):
    """tr[z][q][32]: time-averaged state (8) and flux (3 x 8) at the face points"""
    nz = aU.shape[0]
    Q = len(face_points(order)[1])
    tr = np.zeros((nz, Q, 32))
    if _lib().rgo_prism_traces(order, nz, np.ascontiguousarray(aU), np.ascontiguousarray(aF), tr):
        raise ValueError("prism traces failed")
    return tr


def divfree_sizes(order):
    a, b = C.c_int(0), C.c_int(0)
    _lib().rgo_prism_divfree_sizes(order, C.byref(a), C.byref(b))
    return a.value, b.value


def taylor_indices(order):
    """multi-indices of degree 1..p-1: degree by degree, x exponent descending, then y"""
    return [(a, b, d - a - b) for d in range(1, order) for a in range(d, -1, -1) for b in range(d - a, -1, -1)]

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
- Constrained transport on the prisms (Section VI with the prism's edges):
  the line integral of the electric field along every edge by Simpson's rule
  (as on the hexahedra), from the four zones about an angular edge by the
  four-state multidimensional HLL field of the hexahedral oracle (two zones
  at the inner and outer radius: the 1-D HLL of their side face), and from
  the five or six zones about a radial edge by the mean of the 1-D HLL
  induction fluxes of the faces between consecutive zones (the three-zone
  rule of the hexahedral oracle for any number of zones); the magnetic flux
  through every face then changes by minus dt times the circulation of these
  integrals around it (Stokes' theorem), so each zone's net outward flux is
  unchanged.  Pinned (tests/test_oracle_prism.py): the zone identity for
  arbitrary edge integrals, exact integrals and no change for a uniform
  state, Stokes' theorem for linear fields against the faces' vector areas,
  the three-zone case against the hexahedral rule, upwinding of the K-zone
  rule in supersonic flow and its invariance under relabelling and rotation;
  the four-state field is the hexahedral oracle's, pinned there.
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


_REFEL = {}

S3 = np.sqrt(3.0)
# reference triangle vertices (centred, unit edges), local vertex j <-> the
# triangle's j-th mesh vertex
TRI_V = np.array([[-0.5, -0.5 / S3], [0.5, -0.5 / S3], [0.0, 1.0 / S3]])
# Simpson's rule on [0, 1]: the edge quadrature of the electric field
SIMPSON_S = np.array([0.0, 0.5, 1.0])
SIMPSON_W = np.array([1.0, 4.0, 1.0]) / 6.0
IBX = 5


def basis(order, pts):
    """nodal basis values [P][N] and gradients [P][N][3] at reference points
    pts[P][3] (psi_l = sum_k coef[k, l] xi^a eta^b zeta^c)"""
    if order not in _REFEL:
        _REFEL[order] = refel(order)
    r = _REFEL[order]
    e, coef = r["exps"], r["coef"]
    pts = np.atleast_2d(pts)
    def mono(p, d=None):
        out = np.ones((len(pts), len(e)))
        for k, ex in enumerate(e):
            ex = list(ex)
            fac = 1.0
            if d is not None:
                fac = ex[d]
                ex[d] = max(ex[d] - 1, 0)
            out[:, k] = fac * pts[:, 0] ** ex[0] * pts[:, 1] ** ex[1] * pts[:, 2] ** ex[2]
        return out
    val = mono(pts) @ coef
    grad = np.stack([mono(pts, d) @ coef for d in range(3)], axis=2)
    return val, grad


def efield(F):
    """electric field from the Cartesian fluxes F[..][3][8] of the induction
    equation: E_x = F_z[B_y], E_y = F_x[B_z], E_z = F_y[B_x]"""
    return np.stack([F[..., 2, IBX + 1], F[..., 0, IBX + 2], F[..., 1, IBX]], axis=-1)


def emf_faces(U, F, n, t, gamma=5.0 / 3.0):
    """edge field E . t from K zones about an edge: the mean over the faces
    between consecutive zones (k -> k + 1 mod K, unit normals n[K][3] from
    zone k toward zone k + 1) of -(t x n) . F_B, F_B the B rows of the 1-D HLL
    flux of the two zones' states U[K][8] and Cartesian fluxes F[K][3][8]"""
    K = len(U)
    k2 = (np.arange(K) + 1) % K
    Fs = np.zeros((K, 8))
    _lib().rgo_prism_hll(K, np.ascontiguousarray(U), np.ascontiguousarray(U[k2]),
                         np.ascontiguousarray(F.reshape(K, 24)), np.ascontiguousarray(F[k2].reshape(K, 24)),
                         np.ascontiguousarray(n), gamma, Fs)
    tn = np.cross(t[None, :], n)
    return float(-(Fs[:, IBX:IBX + 3] * tn).sum(1).mean())


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

    def vertex_rings(self):
        """for every mesh vertex its (triangle, local vertex) pairs in
        counter-clockwise order seen from outside, starting at its lowest
        triangle (a triangle (v, a, b) is followed by the one with the
        directed edge v -> b)"""
        where, inc = {}, [[] for _ in range(len(self.vert))]
        for t, tri in enumerate(self.tri):
            for j in range(3):
                where[(tri[j], tri[(j + 1) % 3])] = (t, j)
                inc[tri[j]].append((t, j))
        rings = []
        for v in range(len(self.vert)):
            ring = [min(inc[v])]
            while True:
                t, j = ring[-1]
                nxt = where[(v, self.tri[t][(j + 2) % 3])]
                if nxt == ring[0]:
                    break
                ring.append(nxt)
            assert len(ring) == len(inc[v])
            rings.append(ring)
        return rings

    def edge_emfs(self, aU, aF, gamma=5.0 / 3.0):
        """line integrals of E along every edge from the predictor's time
        averages aU[z][N][8], aF[z][N][3][8] (Section VI; see the module
        notes).  Gam_ang[n_edges][n_rad + 1]: mesh edge e at radius r_kr, from
        its first triangle's local vertex e1 to e1 + 1; Gam_rad[n_vert][n_rad]:
        the radial edge at vertex v through shell k, outward."""
        order, nr = self.order, self.n_rad
        zones = np.arange(self.nz)
        x, _, _ = self.geometry(zones)
        cen, _ = self.frames(zones)
        E = self.edges()

        def at(z, xi):
            """state, flux, position and d x / d xi of zone z at reference point xi"""
            val, grad = basis(order, xi)
            return (val[0] @ aU[z], np.einsum("l,ldv->dv", val[0], aF[z]), val[0] @ x[z],
                    np.einsum("ld,lc->cd", grad[0], x[z]))

        Gang = np.zeros((len(E), nr + 1))
        for e, (t1, e1, t2, e2) in enumerate(E):
            d1 = TRI_V[(e1 + 1) % 3] - TRI_V[e1]
            d2 = TRI_V[(e2 + 1) % 3] - TRI_V[e2]
            for kr in range(nr + 1):
                G = 0.0
                for s, w in zip(SIMPSON_S, SIMPSON_W):
                    p1, p2 = TRI_V[e1] + s * d1, TRI_V[e2] + (1 - s) * d2
                    # zones: below (zeta = +1/2) and above (zeta = -1/2) the radius
                    side = []
                    for k, zeta in ((kr - 1, 0.5), (kr, -0.5)):
                        if 0 <= k < nr:
                            side.append([at(t1 * nr + k, np.array([p1[0], p1[1], zeta])),
                                         at(t2 * nr + k, np.array([p2[0], p2[1], zeta])), k])
                    # position and tangent from the first triangle's zone
                    (_, _, xp, jac), _, k0 = side[0][0], side[0][1], side[0][2]
                    dx = jac[:, :2] @ d1
                    dl = np.linalg.norm(dx)
                    tt = dx / dl
                    if len(side) == 2:
                        (a_lo, b_lo, klo), (a_hi, b_hi, khi) = side
                        # counter-clockwise about t: SW, SE, NE, NW with east = t1
                        # (left of the edge seen from outside) and north = outward
                        St = [b_lo, a_lo, a_hi, b_hi]
                        zs = [t2 * nr + klo, t1 * nr + klo, t1 * nr + khi, t2 * nr + khi]
                        Es = O.emf4(np.array([q[0] for q in St]), np.array([efield(q[1]) for q in St]),
                                    cen[zs], tt, gamma)
                    else:
                        a, b, _ = side[0]
                        rh = xp / np.linalg.norm(xp)
                        n = np.cross(tt, rh)
                        n /= np.linalg.norm(n)
                        Es = emf_faces(np.array([a[0], b[0]]), np.array([a[1], b[1]]),
                                       np.array([n, -n]), tt, gamma)
                    G += w * dl * Es
                Gang[e, kr] = G
        Grad = np.zeros((len(self.vert), nr))
        for v, ring in enumerate(self.vertex_rings()):
            vhat = self.vert[v] / np.linalg.norm(self.vert[v])
            n = []
            for t, j in ring:
                b = self.vert[self.tri[t][(j + 2) % 3]]
                c = np.cross(vhat, b)
                n.append(c / np.linalg.norm(c))
            n = np.array(n)
            for k in range(nr):
                G = 0.0
                for s, w in zip(SIMPSON_S, SIMPSON_W):
                    St = [at(t * nr + k, np.array([TRI_V[j][0], TRI_V[j][1], s - 0.5])) for t, j in ring]
                    jac = St[0][3]
                    dl = np.linalg.norm(jac[:, 2])
                    Es = emf_faces(np.array([q[0] for q in St]), np.array([q[1] for q in St]), n,
                                   jac[:, 2] / dl, gamma)
                    G += w * dl * Es
                Grad[v, k] = G
        return Gang, Grad

    def ct_update(self, PhiB, Gang, Grad, dt):
        """magnetic fluxes PhiB[n_faces] through the faces (numbered and
        directed as in face_fluxes) after dt of constrained transport: minus dt
        times the circulation of the edge integrals around each face, taken
        counter-clockwise about the face's direction"""
        nr, nrf = self.n_rad, self.ntri * (self.n_rad + 1)
        E = self.edges()
        tedge = {}
        for e, (t1, e1, t2, e2) in enumerate(E):
            tedge[(t1, e1)] = (e, 1.0)
            tedge[(t2, e2)] = (e, -1.0)
        out = np.array(PhiB, dtype=np.float64, copy=True)
        for t in range(self.ntri):
            for kf in range(nr + 1):
                circ = sum(sg * Gang[e, kf] for e, sg in (tedge[(t, j)] for j in range(3)))
                out[t * (nr + 1) + kf] -= dt * circ
        for e, (t1, e1, t2, e2) in enumerate(E):
            A, B = self.tri[t1][e1], self.tri[t1][(e1 + 1) % 3]
            for k in range(nr):
                circ = Gang[e, k] + Grad[B, k] - Gang[e, k + 1] - Grad[A, k]
                out[nrf + e * nr + k] -= dt * circ
        return out

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

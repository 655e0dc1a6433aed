"""Pins of the oracle's triangular-prism element and icosahedral mesh against
what the paper prints and what the mathematics fixes (CPU only)."""
import math

import numpy as np
import pytest

import tests.golden_io as G
from oracle import oracle as O
from oracle import prism as P
from oracle.prism import IBX

S3 = math.sqrt(3.0)


def _galerkin_is_R_kron_D(r, R):
    """The reduced full-Galerkin matrices of eq. (5.29) factor into the
    printed time matrix R and the nodal derivative matrices (the spaces are
    closed under differentiation), as eqs. (C.35)-(C.36) and (D.30)-(D.32)
    state: Kd0 = R[1:, :1] (x) D, Kd = R[1:, 1:] (x) D, Kt0 = 1 (x) I."""
    N, M = r["N"], r["M"]
    R = np.asarray(R)
    # rounding of the basis (Vandermonde condition number up to 323 at fourth
    # order) and of the quadrature sums, relative to the largest entry of D
    tol = 1e-13 * np.abs(r["D"]).max() * N
    for d in range(3):
        np.testing.assert_allclose(r["Kd0"][d], np.kron(R[1:, :1], r["D"][d]), rtol=0, atol=tol)
        np.testing.assert_allclose(r["Kd"][d], np.kron(R[1:, 1:], r["D"][d]), rtol=0, atol=tol)
    np.testing.assert_allclose(r["Kt0"], np.kron(np.ones((M - 1, 1)), np.eye(N)), rtol=0, atol=1e-12)


def test_second_order_update_matches_appendix_B():
    r = P.refel(2)
    rows = G.prism_order2_update()
    for i, (f, g, h) in enumerate(rows):
        np.testing.assert_allclose(r["D"][0][i], f, rtol=0, atol=1e-13)
        np.testing.assert_allclose(r["D"][1][i], g, rtol=0, atol=1e-13)
        np.testing.assert_allclose(r["D"][2][i], h, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r["tau"], [0.0, 0.5], rtol=0, atol=1e-15)
    _galerkin_is_R_kron_D(r, G.time_R()[2])


def test_second_order_basis_matches_B10_to_B15():
    """(B.10)-(B.15): psi_1 = 1/6 - xi/2 - eta/(2 sqrt 3) + zeta/3 - xi zeta - eta zeta/sqrt 3,
    psi_3 = 1/6 + eta/sqrt 3 + zeta/3 + 2 eta zeta/sqrt 3, psi_6 = 1/6 + eta/sqrt 3 - zeta/3 - 2 eta zeta/sqrt 3
    on the monomials (1, xi, eta, zeta, xi zeta, eta zeta) of eq. (5.12)."""
    r = P.refel(2)
    assert [tuple(e) for e in r["exps"]] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)]
    printed = {0: [1 / 6, -1 / 2, -1 / (2 * S3), 1 / 3, -1, -1 / S3],
               1: [1 / 6, 1 / 2, -1 / (2 * S3), 1 / 3, 1, -1 / S3],
               2: [1 / 6, 0, 1 / S3, 1 / 3, 0, 2 / S3],
               3: [1 / 6, -1 / 2, -1 / (2 * S3), -1 / 3, 1, 1 / S3],
               4: [1 / 6, 1 / 2, -1 / (2 * S3), -1 / 3, -1, 1 / S3],
               5: [1 / 6, 0, 1 / S3, -1 / 3, 0, -2 / S3]}
    for l, c in printed.items():
        np.testing.assert_allclose(r["coef"][:, l], c, rtol=0, atol=1e-13)


def test_third_order_element_matches_appendix_C():
    """Nodes (C.2)-(C.16) and monomials (5.13) as printed; the printed bases
    (C.19), (C.21), (C.25), (C.28), (C.29); the Galerkin system against the
    printed R of (C.18)."""
    r = P.refel(3)
    nodes, monos, basis = G.prism_basis()
    np.testing.assert_allclose(r["nodes"], nodes, rtol=0, atol=1e-15)
    assert [tuple(e) for e in r["exps"]] == monos
    for l1, coefs in basis.items():
        c = dict(zip([tuple(e) for e in r["exps"]], r["coef"][:, l1 - 1]))
        for e, v in c.items():
            assert abs(v - coefs.get(e, 0.0)) < 1e-12, (l1, e, v, coefs.get(e, 0.0))
    _galerkin_is_R_kron_D(r, G.time_R()[3])


def test_fourth_order_element_matches_appendix_D():
    r = P.refel(4)
    nodes, monos = G.prism_order4_nodes()
    np.testing.assert_allclose(r["nodes"], nodes, rtol=0, atol=1e-15)
    assert [tuple(e) for e in r["exps"]] == monos
    _galerkin_is_R_kron_D(r, G.time_R()[4])


@pytest.mark.parametrize("order", [2, 3, 4])
def test_derivative_matrices_differentiate_the_space_exactly(order):
    """D_d applied to the nodal values of every monomial of eqs. (5.12)-(5.14)
    gives the nodal values of its exact derivative, and psi_l(node_i) = delta_il
    (eq. 5.3)."""
    r = P.refel(order)
    X = r["nodes"]
    V = np.array([[np.prod(x ** np.array(e)) for e in r["exps"]] for x in X])
    np.testing.assert_allclose(V @ r["coef"], np.eye(r["N"]), rtol=0, atol=1e-12)
    for k, e in enumerate(r["exps"]):
        m = V[:, k]
        for d in range(3):
            if e[d] == 0:
                exact = np.zeros(len(X))
            else:
                ee = np.array(e); ee[d] -= 1
                exact = e[d] * np.prod(X ** ee, axis=1)
            np.testing.assert_allclose(r["D"][d] @ m, exact, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_predictor_exact_for_advected_polynomial_on_affine_prism(order):
    """On an affine prism a density polynomial of total degree <= p-1 (inside
    the space of eqs. 5.12-5.14) advected by uniform v with uniform p and B is
    reproduced exactly at every space-time node after p Picard iterations
    (ADER-CG, eqs. 5.20-5.29)."""
    r = P.refel(order)
    N, X0 = r["N"], r["nodes"]
    rng = np.random.default_rng(11)
    A = np.eye(3) * 0.1 + 0.02 * rng.normal(size=(3, 3))
    x0 = np.array([1.1, -0.2, 0.6])
    X = X0 @ A.T + x0
    J = np.full((1, N), np.linalg.det(A))
    h = [A[:, 0], A[:, 1], A[:, 2]]
    met = np.zeros((1, N, 3, 3))
    met[0, :, 0] = np.cross(h[1], h[2]); met[0, :, 1] = np.cross(h[2], h[0]); met[0, :, 2] = np.cross(h[0], h[1])
    v = np.array([0.6, -0.4, 0.3]); B = np.array([0.3, -0.1, 0.2]); p = 0.9; gam = 5 / 3
    exps = [(a, b, c) for a in range(order) for b in range(order - a) for c in range(order - a - b)]
    cf = 0.05 * rng.normal(size=len(exps)); cf[0] = 1.0

    def state(x):
        y = (x - x0) / 0.1
        rh = sum(c * y[:, 0] ** a * y[:, 1] ** b * y[:, 2] ** cc for c, (a, b, cc) in zip(cf, exps))
        U = np.zeros((len(x), 8))
        U[:, 0] = rh; U[:, 1:4] = rh[:, None] * v
        U[:, 4] = p / (gam - 1) + 0.5 * rh * (v @ v) + 0.5 * (B @ B)
        U[:, 5:8] = B
        return U

    dt = 0.02
    aU, aF, Ul = P.predict(order, J, met, state(X)[None], dt, gam, levels=True)
    for t in range(order):
        np.testing.assert_allclose(Ul[0, t] / J[0][:, None], state(X - v * r["tau"][t] * dt), rtol=0, atol=1e-11)
    # the time average of the state is the Gauss-weighted average of the levels
    ref = sum(r["wt"][t] * state(X - v * r["tau"][t] * dt) for t in range(1, order))
    np.testing.assert_allclose(aU[0], ref, rtol=0, atol=1e-11)


# ---------------------------------------------------------------- mesh
@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosahedral_mesh_topology(level):
    """20 4^L triangles, 10 4^L + 2 vertices on the unit sphere, every edge
    shared by exactly two triangles with opposite orientation (a closed
    oriented surface, V - E + F = 2), all triangles counter-clockwise seen
    from outside."""
    m = P.OraclePrismMesh(level, 1, order=2)
    V, T = m.vert, m.tri
    assert len(T) == 20 * 4 ** level and len(V) == 10 * 4 ** level + 2
    np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, rtol=0, atol=1e-15)
    directed = {}
    for a, b, c in T:
        for e in ((a, b), (b, c), (c, a)):
            assert e not in directed
            directed[e] = 1
    for (a, b) in directed:
        assert (b, a) in directed
    nE = len(directed) // 2
    assert len(V) - nE + len(T) == 2
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    assert np.all(np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0)


def test_icosahedral_edge_angles_match_section_IIa():
    """Mean central angle of an edge at levels 0, 1 and 4, as printed."""
    for level, deg, digits in G.icosahedral_angles():
        m = P.OraclePrismMesh(level, 1, order=2)
        V, T = m.vert, m.tri
        ang = []
        for i, j in ((0, 1), (1, 2), (2, 0)):
            ang.append(np.degrees(np.arccos(np.clip(np.einsum("ij,ij->i", V[T[:, i]], V[T[:, j]]), -1, 1))))
        assert round(float(np.mean(ang)), digits) == pytest.approx(deg, abs=1e-9), (level, np.mean(ang))
    np.testing.assert_allclose(G.icosahedral_angles()[0][1], 63.4)
    m = P.OraclePrismMesh(0, 1, order=2)
    V, T = m.vert, m.tri
    ang0 = np.degrees(np.arccos(V[T[0, 0]] @ V[T[0, 1]]))
    np.testing.assert_allclose(ang0, 90 - np.degrees(np.arctan(0.5)), rtol=0, atol=1e-12)


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("order", [2, 3, 4])
def test_zone_geometry_sphericity_and_radial_lines(order):
    """The map interpolates the sphere at its lattice nodes, which are the
    prism's nodes on the inner and outer faces, and is linear in radius
    along the vertical edges (Section II.b, Fig. 3)."""
    m = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.6, order=order)
    r = P.refel(order)
    zones = np.arange(m.nz)
    x, J, met = m.geometry(zones)
    t, k = m.zone_tri_shell(zones)
    r0, r1 = m.radius[k], m.radius[k + 1]
    zeta = r["nodes"][:, 2]
    rad = np.linalg.norm(x, axis=2)
    for i in range(r["N"]):
        expect = (0.5 - zeta[i]) * r0 + (0.5 + zeta[i]) * r1
        if abs(zeta[i]) == 0.5:
            np.testing.assert_allclose(rad[:, i], expect, rtol=1e-14, atol=0)
    # vertical-edge nodes lie on the radial line through the vertex
    vert_nodes = [i for i in range(r["N"]) if np.min(np.linalg.norm(r["nodes"][i, :2] - r["nodes"][:3, :2], axis=1)) < 1e-12]
    for i in vert_nodes:
        kv = int(np.argmin(np.linalg.norm(r["nodes"][i, :2] - r["nodes"][:3, :2], axis=1)))
        vdir = m.vert[m.tri[t, kv]]
        expect = ((0.5 - zeta[i]) * r0 + (0.5 + zeta[i]) * r1)[:, None] * vdir
        np.testing.assert_allclose(x[:, i], expect, rtol=0, atol=1e-14)
    assert np.all(J > 0)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_curl_metrics_have_zero_discrete_divergence(order):
    """sum_d D_d (J a^d)_n = 0 at every node (free-stream preservation of
    eq. 5.11 in curl form), and the metrics approach J times the inverse
    Jacobian as the zones shrink."""
    r = P.refel(order)
    m = P.OraclePrismMesh(2, 2, order=order)
    zones = np.arange(0, m.nz, 7)
    x, J, met = m.geometry(zones)
    for z in range(len(zones)):
        div = sum(r["D"][d] @ met[z, :, d, :] for d in range(3))
        assert np.abs(div).max() < 1e-13 * np.abs(met[z]).max()
    # against the cofactor of the map's Jacobian: halving the zones in every
    # direction shrinks the gap by 2^(p-1) (the interpolation error of the
    # curl form's vector potential), up to a margin
    gaps = []
    for level, n_rad in ((2, 4), (3, 8)):
        mm = P.OraclePrismMesh(level, n_rad, order=order)
        zz = np.arange(0, mm.nz, 97)
        xx, JJ, mt = mm.geometry(zz)
        gaps.append(_metric_gap(r, xx, JJ, mt))
    assert gaps[1] / gaps[0] < 1.25 * 0.5 ** (order - 1), gaps


def _metric_gap(r, x, J, met):
    """max relative difference between the curl-form metrics and J d xi/dx
    from the nodal interpolant of x (differentiated with D)"""
    worst = 0.0
    for z in range(len(x)):
        jac = np.stack([r["D"][d] @ x[z] for d in range(3)], axis=2)  # [i][n][d] = d x_n / d xi_d
        for i in range(r["N"]):
            cof = np.linalg.det(jac[i]) * np.linalg.inv(jac[i])           # [d][n] = J d xi_d / d x_n
            worst = max(worst, np.abs(cof - met[z, i]).max() / np.abs(cof).max())
    return worst


@pytest.mark.parametrize("order", [2, 3, 4])
def test_predictor_keeps_a_uniform_state_on_curved_zones(order):
    """Free stream: a uniform state stays uniform through the predictor on the
    curved zones, and the averaged flux is the physical flux of that state."""
    from oracle import oracle as O
    m = P.OraclePrismMesh(1, 2, order=order)
    zones = np.arange(0, m.nz, 5)
    U = np.array([1.1, 0.3, -0.2, 0.4, 2.5, 0.2, 0.1, -0.3])
    Ua = np.tile(U, (len(zones), m.N, 1))
    aU, aF = m.predict(zones, Ua, 0.05)
    # round-off of the metric sums only (a wrong metric term moves the state
    # by dt times the flux, about 1e-2 here)
    np.testing.assert_allclose(aU, Ua, rtol=0, atol=1e-12)
    F = O.flux(U)
    np.testing.assert_allclose(aF, np.broadcast_to(F, aF.shape), rtol=0, atol=1e-12)


# ---------------------------------------------------------------- face rules and traces
def _tri_exact(f, n=8):
    """(1/|T|) integral of f over the printed triangle (0,0), (1,0), (1/2, sqrt 3/2)
    by a collapsed Gauss-Legendre rule of numpy's (exact for polynomials of
    degree < 2n - 1)"""
    g, gw = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1); gw = 0.5 * gw
    A, B, Cc = np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.5, S3 / 2])
    tot = 0.0
    for s, ws in zip(g, gw):
        for t, wt in zip(g, gw):
            x = A + s * (B - A) + (1 - s) * t * (Cc - A)
            tot += ws * wt * (1 - s) * f(x[0], x[1])
    return 2 * tot


@pytest.mark.parametrize("rule,degree", [("A1", 2), ("A3", 2), ("A5", 3)])
def test_triangle_rules_of_appendix_A_are_exact(rule, degree):
    """The printed triangle rules integrate every monomial up to the degree
    their scheme's order needs (p - 1: second-order rule at least 1, third 2,
    fourth 3) exactly, with weights summing to one and points inside."""
    R = np.array(G.triangle_rules()[rule])
    x, y, w = R[:, 0], R[:, 1], R[:, 2]
    assert abs(w.sum() - 1) < 1e-15
    assert np.all(y > 0) and np.all(y < S3 * x) and np.all(y < S3 * (1 - x))
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            exact = _tri_exact(lambda u, v: u ** a * v ** b)
            assert abs((w * x ** a * y ** b).sum() - exact) < 1e-14, (rule, a, b)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_points_are_the_printed_rules_on_the_prism_faces(order):
    """The oracle's face points: the printed triangle rule on both triangle
    faces (shifted to the centred triangle) and the printed square rule on the
    three side faces (x along the edge, y along zeta)."""
    xi, w, nt, ns = P.face_points(order)
    tri = np.array(G.triangle_rules()[{2: "A1", 3: "A3", 4: "A5"}[order]])
    sq = np.array(G.square_rules()[{2: "A2", 3: "A4", 4: "A6"}[order]])
    assert (nt, ns) == (len(tri), len(sq)) and len(w) == 2 * nt + 3 * ns
    v1 = np.array([-0.5, -0.5 / S3])
    for f, zeta in ((0, 0.5), (1, -0.5)):
        blk = slice(f * nt, (f + 1) * nt)
        np.testing.assert_allclose(xi[blk, :2], tri[:, :2] + v1, rtol=0, atol=1e-15)
        np.testing.assert_allclose(xi[blk, 2], zeta, rtol=0, atol=0)
        np.testing.assert_allclose(w[blk], tri[:, 2], rtol=0, atol=1e-16)
    V = np.array([[-0.5, -0.5 / S3], [0.5, -0.5 / S3], [0.0, 1 / S3]])
    for k in range(3):
        blk = slice(2 * nt + k * ns, 2 * nt + (k + 1) * ns)
        along = V[k] + sq[:, :1] * (V[(k + 1) % 3] - V[k])
        np.testing.assert_allclose(xi[blk, :2], along, rtol=0, atol=1e-15)
        np.testing.assert_allclose(xi[blk, 2], sq[:, 1] - 0.5, rtol=0, atol=1e-15)
        np.testing.assert_allclose(w[blk], sq[:, 2], rtol=0, atol=1e-16)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_traces_reproduce_polynomials_of_the_space(order):
    """Nodal values of a monomial of the element's space, traced to the face
    points, give the monomial's values there (the nodal interpolant is exact)."""
    r = P.refel(order)
    xi, w, nt, ns = P.face_points(order)
    X = r["nodes"]
    rng = np.random.default_rng(order)
    aU = np.zeros((1, r["N"], 8)); aF = np.zeros((1, r["N"], 3, 8))
    want = np.zeros((len(w), 32))
    for k in range(32):
        e = r["exps"][rng.integers(len(r["exps"]))]
        c = rng.normal()
        vals = c * np.prod(X ** e, axis=1)
        (aU[0, :, k] if k < 8 else aF[0, :, (k - 8) // 8, (k - 8) % 8])[...] = vals
        want[:, k] = c * np.prod(xi ** e, axis=1)
    tr = P.traces(order, aU, aF)
    np.testing.assert_allclose(tr[0], want, rtol=0, atol=1e-12 * max(1, np.abs(want).max()))


def test_square_rule_A2_integrates_bilinear_functions():
    """(A.2), the second-order side-face rule, integrates 1, x, y and x y over
    the unit square exactly (all a second-order trace needs)."""
    R = np.array(G.square_rules()["A2"])
    x, y, w = R[:, 0], R[:, 1], R[:, 2]
    for f, exact in ((lambda a, b: 1 + 0 * a, 1.0), (lambda a, b: a, 0.5), (lambda a, b: b, 0.5),
                     (lambda a, b: a * b, 0.25)):
        assert abs((w * f(x, y)).sum() - exact) < 1e-15


# ---------------------------------------------------------------- face fluxes
def _zone_faces(m):
    """for every zone its five faces with the sign of the zone's outward normal:
    [(face, sign)] x 5 per zone"""
    nr, nrf = m.n_rad, m.ntri * (m.n_rad + 1)
    faces = [[] for _ in range(m.nz)]
    for t in range(m.ntri):
        for k in range(nr):
            z = t * nr + k
            faces[z].append((t * (nr + 1) + k + 1, +1))    # top: +r is outward
            faces[z].append((t * (nr + 1) + k, -1))        # bottom
    for e, (t1, e1, t2, e2) in enumerate(m.edges()):
        for k in range(nr):
            faces[t1 * nr + k].append((nrf + e * nr + k, +1))
            faces[t2 * nr + k].append((nrf + e * nr + k, -1))
    return faces


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_points_of_neighbours_coincide(order):
    """The two sides of every face see the same physical points: a radial
    face's triangle points from the zone below and above, a side face's points
    from the first triangle and the mirrored points of its neighbour."""
    m = P.OraclePrismMesh(1, 2, r_in=1.0, r_out=1.5, order=order)
    xi, w, nt, ns = P.face_points(order)
    xq, dA = m.face_geometry(np.arange(m.nz))
    nr = m.n_rad
    for t in range(m.ntri):
        np.testing.assert_allclose(xq[t * nr, :nt], xq[t * nr + 1, nt:2 * nt], rtol=0, atol=1e-14)
    xs = xi[2 * nt:2 * nt + ns]
    sx = xs[:, 0] + 0.5                                     # position along edge 0 (xi from -1/2 to 1/2)
    mirror = [int(np.argmin(np.abs(sx - (1 - sx[i])) + np.abs(xs[:, 2] - xs[i, 2]))) for i in range(ns)]
    for t1, e1, t2, e2 in m.edges():
        for k in range(nr):
            a = xq[t1 * nr + k, 2 * nt + e1 * ns + np.arange(ns)]
            b = xq[t2 * nr + k, 2 * nt + e2 * ns + np.array(mirror)]
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_face_area_vectors_close_each_zone(order):
    """The rule-weighted outward area vectors of a zone's five faces sum to
    zero: exactly where the face rules integrate the map's area vectors
    (orders 2, 3), and at fourth order (cubic map, (A.5) exact to degree 3)
    with a gap that shrinks with the zones."""
    gaps = []
    for level in (1, 2):
        m = P.OraclePrismMesh(level, 2, r_in=1.0, r_out=1.5, order=order)
        _, dA = m.face_geometry(np.arange(m.nz))
        gaps.append(np.abs(dA.sum(1)).max() / np.abs(dA).sum(1).max())
    if order < 4:
        assert max(gaps) < 1e-14
    else:
        assert gaps[1] < gaps[0] / 8 and gaps[1] < 1e-5, gaps


@pytest.mark.parametrize("order", [2, 3])
def test_face_fluxes_of_a_uniform_state_cancel(order):
    """A uniform state's face fluxes are F(U) . A_f, so every zone's net
    outward flux vanishes where the faces close exactly (free stream of the
    corrector)."""
    from oracle import oracle as O
    m = P.OraclePrismMesh(1, 2, r_in=1.0, r_out=1.5, order=order)
    U = np.array([1.1, 0.3, -0.2, 0.4, 2.5, 0.2, 0.1, -0.3])
    F = O.flux(U)
    Q = len(P.face_points(order)[1])
    tr = np.zeros((m.nz, Q, 32)); tr[:, :, :8] = U; tr[:, :, 8:] = F.reshape(24)
    Phi = m.face_fluxes(tr)
    scale = np.abs(Phi).max()
    for faces in _zone_faces(m):
        net = sum(s * Phi[f] for f, s in faces)
        assert np.abs(net).max() < 1e-13 * scale


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_volumes_fill_the_shell(order):
    """The zones' volumes sum to the volume the maps enclose, which approaches
    (4 pi / 3)(r_out^3 - r_in^3) at the rate of the map (flat facets at order 2,
    Section II.b's sphericity at orders 3 and 4); zones of one column scale as
    r_k^3 and a uniform state is left unchanged by the update."""
    exact = 4 * np.pi / 3 * (1.5 ** 3 - 1.0)
    errs = []
    for level in (1, 2):
        m = P.OraclePrismMesh(level, 3, r_in=1.0, r_out=1.5, order=order)
        vol = m.volumes(np.arange(m.nz))
        errs.append(abs(vol.sum() - exact) / exact)
        q = (1.5) ** (1 / 3)
        np.testing.assert_allclose(vol[1::3] / vol[0::3], q ** 3, rtol=1e-13)
    # flat facets: h^2; the quadratic and cubic maps: h^4 (measured 15-16 per halving)
    rate = {2: 3.5, 3: 12.0, 4: 12.0}[order]
    assert errs[0] / errs[1] > rate and errs[1] < {2: 5e-2, 3: 2e-4, 4: 1e-5}[order], errs


def test_prism_update_conserves_up_to_boundary_fluxes():
    """With any face fluxes, sum_z V_z (U1 - U) = -dt (outer minus inner
    boundary fluxes): interior faces cancel in pairs (Section VI)."""
    m = P.OraclePrismMesh(1, 3, order=3)
    rng = np.random.default_rng(2)
    nf = m.ntri * (m.n_rad + 1) + len(m.edges()) * m.n_rad
    Phi = rng.normal(size=(nf, 8))
    U = rng.normal(size=(m.nz, 8))
    dt = 0.01
    U1 = m.update(U, Phi, dt)
    vol = m.volumes(np.arange(m.nz))
    nr = m.n_rad
    outer = Phi[[t * (nr + 1) + nr for t in range(m.ntri)]].sum(0)
    inner = Phi[[t * (nr + 1) for t in range(m.ntri)]].sum(0)
    np.testing.assert_allclose((vol[:, None] * (U1 - U)).sum(0), -dt * (outer - inner), rtol=0, atol=1e-13)


# ---------------------------------------------------------------- divergence-free B
def divfree_inputs_linear(m, zones, B0, G):
    """the KKT inputs of the field B(x) = B0 + G x (G trace-free, so div B = 0):
    zone means, Taylor coefficients (degree 1: l0 G; higher: 0), the outward
    normal B at the face points and the face averages by each face's rule"""
    order = m.order
    nc = len(P.taylor_indices(order))
    xi, w, nt, ns = P.face_points(order)
    Q = len(w)
    cen, l0 = m.frames(zones)
    xq, dA = m.face_geometry(zones)
    nin, nout = P.divfree_sizes(order)
    Bin = np.zeros((len(zones), nin))
    ti = P.taylor_indices(order)
    for z in range(len(zones)):
        for c in range(3):
            Bin[z, c * (nc + 1)] = B0[c] + G[c] @ cen[z]
            for a, e in enumerate(ti):
                if sum(e) == 1:
                    Bin[z, c * (nc + 1) + 1 + a] = l0[z] * G[c][int(np.argmax(e))]
        Bx = B0[None] + xq[z] @ G.T
        an = np.linalg.norm(dA[z], axis=1)
        nrm = dA[z] / an[:, None]
        bn = (Bx * nrm).sum(1)
        Bin[z, 3 * (nc + 1):3 * (nc + 1) + Q] = bn
        faces = [np.arange(nt), np.arange(nt, 2 * nt)] + [2 * nt + k * ns + np.arange(ns) for k in range(3)]
        for f, q in enumerate(faces):
            Bin[z, 3 * (nc + 1) + Q + f] = (an[q] * bn[q]).sum() / an[q].sum()
    return Bin


@pytest.mark.parametrize("order", [2, 3, 4])
def test_divfree_reconstruction_reproduces_linear_divergence_free_fields(order):
    """Consistent inputs of a divergence-free linear field (in the space at
    every order) give that field back exactly at the nodes of curved zones
    (Section IV.b: the constraints and the least squares are all met by it)."""
    m = P.OraclePrismMesh(1, 2, r_in=1.0, r_out=1.5, order=order)
    rng = np.random.default_rng(17)
    G = rng.normal(size=(3, 3)); G -= np.eye(3) * np.trace(G) / 3
    B0 = rng.normal(size=3)
    zones = np.arange(0, m.nz, 7)
    out = m.divfree(zones, divfree_inputs_linear(m, zones, B0, G))
    x, _, _ = m.geometry(zones)
    N = m.N
    want = B0[None, None] + x @ G.T                 # [z][N][3]
    got = out[:, :3 * N].reshape(len(zones), 3, N).transpose(0, 2, 1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    cen, _ = m.frames(zones)
    np.testing.assert_allclose(out[:, 3 * N:], B0[None] + cen @ G.T, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- constrained transport on the prisms

_EPS = np.zeros((3, 3, 3))
_EPS[0, 1, 2] = _EPS[1, 2, 0] = _EPS[2, 0, 1] = 1.0
_EPS[0, 2, 1] = _EPS[2, 1, 0] = _EPS[1, 0, 2] = -1.0
_U0 = np.array([1.0, 0.3, -0.2, 0.1, 2.0, 0.4, 0.2, -0.3])


def test_vertex_rings_are_counter_clockwise_cycles():
    """Every vertex of level 2 has valence 5 (the 12 icosahedron vertices)
    or 6, consecutive triangles of its ring share the edge to the next
    vertex, and the ring turns counter-clockwise seen from outside."""
    m = P.OraclePrismMesh(2, 1, order=2)
    rings = m.vertex_rings()
    val = np.array([len(r) for r in rings])
    assert (val == 5).sum() == 12 and (val == 6).sum() == len(rings) - 12
    for v, ring in enumerate(rings):
        cen = [m.vert[m.tri[t]].mean(0) for t, _ in ring]
        for i, (t, j) in enumerate(ring):
            t2, j2 = ring[(i + 1) % len(ring)]
            assert m.tri[t][j] == v and m.tri[t2][j2] == v
            assert m.tri[t][(j + 2) % 3] == m.tri[t2][(j2 + 1) % 3]
            assert np.cross(cen[i] - m.vert[v], cen[(i + 1) % len(ring)] - m.vert[v]) @ m.vert[v] > 0


def test_ct_keeps_every_zones_net_flux_for_any_edge_integrals():
    """The circulations of the edge integrals around a zone's five faces
    cancel (each edge bounds two of them, run both ways), so the update
    keeps each zone's net outward magnetic flux for arbitrary integrals."""
    m = P.OraclePrismMesh(1, 3, order=3)
    F, S = m.zone_faces()
    rng = np.random.default_rng(2)
    nf = m.ntri * (m.n_rad + 1) + len(m.edges()) * m.n_rad
    Phi0 = rng.normal(size=nf)
    Phi1 = m.ct_update(Phi0, rng.normal(size=(len(m.edges()), m.n_rad + 1)),
                       rng.normal(size=(len(m.vert), m.n_rad)), 0.3)
    assert np.abs((S * (Phi1 - Phi0)[F]).sum(1)).max() < 1e-14
    assert np.abs(Phi1 - Phi0).max() > 0.1


def _uniform(m):
    Fl = O.flux(_U0)
    return (np.broadcast_to(_U0, (m.nz, m.N, 8)).copy(), np.broadcast_to(Fl, (m.nz, m.N, 3, 8)).copy(),
            P.efield(Fl))


@pytest.mark.parametrize("order", [2, 3, 4])
def test_edge_integrals_of_a_uniform_state_are_exact(order):
    """A uniform state has E = -v x B everywhere: every edge integral is
    E . (chord) (Simpson's rule is exact for the tangent of a curve of degree
    p - 1 <= 3), and no face flux changes."""
    m = P.OraclePrismMesh(1, 2, r_in=1.0, r_out=1.5, order=order)
    aU, aF, E = _uniform(m)
    Ga, Gr = m.edge_emfs(aU, aF)
    for e, (t1, e1, _, _) in enumerate(m.edges()):
        chord = m.vert[m.tri[t1][(e1 + 1) % 3]] - m.vert[m.tri[t1][e1]]
        np.testing.assert_allclose(Ga[e], m.radius * (E @ chord), rtol=0, atol=1e-15)
    np.testing.assert_allclose(Gr, (m.vert @ E)[:, None] * np.diff(m.radius)[None, :], rtol=0, atol=1e-15)
    nf = m.ntri * (m.n_rad + 1) + len(m.edges()) * m.n_rad
    assert np.abs(m.ct_update(np.zeros(nf), Ga, Gr, 1.0)).max() < 1e-15


@pytest.mark.parametrize("order", [2, 3])
def test_ct_obeys_stokes_for_a_linear_electric_field(order):
    """With a uniform state and the induction fluxes of E = G x (continuous,
    so every edge solver returns E . t), each face's flux changes by
    -dt (curl E) . A_f, A_f the face's vector area from the face rules (exact
    at orders 2 and 3, as Simpson's rule is for E . dx/ds on these edges)."""
    m = P.OraclePrismMesh(1, 2, r_in=1.0, r_out=1.5, order=order)
    aU, aF, _ = _uniform(m)
    G = np.random.default_rng(3).normal(size=(3, 3))
    x, _, _ = m.geometry(np.arange(m.nz))
    Ex = x @ G.T
    for d in range(3):
        for i in range(3):
            aF[:, :, d, IBX + i] = -np.einsum("k,znk->zn", _EPS[d, i], Ex)
    Ga, Gr = m.edge_emfs(aU, aF)
    dt = 0.25
    E = m.edges()
    nr, nrf = m.n_rad, m.ntri * (m.n_rad + 1)
    dPhi = m.ct_update(np.zeros(nrf + len(E) * nr), Ga, Gr, dt)
    _, dA = m.face_geometry(np.arange(m.nz))
    _, _, nt, ns = P.face_points(order)
    A = np.zeros((len(dPhi), 3))
    for t in range(m.ntri):
        for kf in range(nr + 1):
            A[t * (nr + 1) + kf] = dA[t * nr + kf - 1, :nt].sum(0) if kf > 0 else -dA[t * nr, nt:2 * nt].sum(0)
    for e, (t1, e1, _, _) in enumerate(E):
        for k in range(nr):
            A[nrf + e * nr + k] = dA[t1 * nr + k, 2 * nt + e1 * ns:2 * nt + (e1 + 1) * ns].sum(0)
    curl = np.einsum("ijk,kj->i", _EPS, G)
    np.testing.assert_allclose(dPhi, -dt * (A @ curl), rtol=0, atol=1e-14)


def test_k_face_edge_rule_with_three_zones_is_the_hexahedral_corner_rule():
    """The mean of the faces' 1-D HLL induction fluxes over K zones (the
    radial edges' rule) is, for K = 3, the hexahedral oracle's three-zone
    corner rule, computed there from the electric fields alone."""
    rng = np.random.default_rng(4)
    t = np.array([0.0, 0.0, 1.0])
    ang = np.array([0.3, 2.2, 4.1])
    n = np.stack([-np.sin(ang + 1.05), np.cos(ang + 1.05), 0 * ang], 1)
    for _ in range(5):
        U = np.array([_U0 * (1 + 0.3 * rng.uniform(-1, 1, 8)) for _ in range(3)])
        U[:, 4] += 1.0
        F = np.array([O.flux(u) for u in U])
        a = P.emf_faces(U, F, n, t)
        b = O.emf3(U, P.efield(F), n, t)
        assert abs(a - b) < 1e-14 * max(1.0, abs(b))


def _ring_frame(K):
    """K zones about the z axis counter-clockwise; the face between zone k
    and k + 1 lies at the angle between them, its unit normal pointing from
    k to k + 1 (the rotation direction about z)"""
    ang = 2 * np.pi * (np.arange(K) + 0.5) / K
    return np.stack([-np.sin(ang), np.cos(ang), 0 * ang], 1), np.array([0.0, 0.0, 1.0])


def _mhd_state(rho, v, p, B, gam=5.0 / 3.0):
    v, B = np.asarray(v, float), np.asarray(B, float)
    return np.array([rho, *(rho * v), p / (gam - 1) + 0.5 * rho * v @ v + 0.5 * B @ B, *B])


@pytest.mark.parametrize("K", [5, 6])
@pytest.mark.parametrize("phi", [0.0, 40.0, 100.0, 250.0])
def test_k_face_edge_rule_takes_the_upwind_fields_in_supersonic_flow(K, phi):
    """Flow faster than every fast speed across every face of a five- or
    six-zone edge: each face's HLL flux is its upwind zone's, so the edge
    field is the mean over the faces of the upwind zones' E . t."""
    n, t = _ring_frame(K)
    d = np.array([np.cos(np.deg2rad(phi)), np.sin(np.deg2rad(phi)), 0.0])
    if min(abs(n @ d)) < 0.2:
        d = np.array([np.cos(np.deg2rad(phi + 11)), np.sin(np.deg2rad(phi + 11)), 0.0])
    gen = np.random.default_rng(K * 1000 + int(phi))
    U = np.array([_mhd_state(gen.uniform(0.7, 1.3), 80.0 * d + 0.2 * gen.normal(size=3), gen.uniform(0.5, 1.5),
                             0.5 * gen.normal(size=3)) for _ in range(K)])
    F = np.array([O.flux(u) for u in U])
    Et = P.efield(F) @ t
    up = [k if n[k] @ d > 0 else (k + 1) % K for k in range(K)]
    want = np.mean(Et[up])
    assert abs(P.emf_faces(U, F, n, t) - want) < 1e-13 * np.abs(Et).max()


@pytest.mark.parametrize("K", [5, 6])
def test_k_face_edge_rule_is_invariant_under_relabelling_and_rotation(K):
    """The K-face mean does not depend on which zone of the ring comes first,
    and rotating the states, normals and tangent together leaves it alone."""
    n, t = _ring_frame(K)
    gen = np.random.default_rng(K)
    U = np.array([_mhd_state(gen.uniform(0.7, 1.3), gen.normal(size=3), gen.uniform(0.5, 1.5), gen.normal(size=3))
                  for _ in range(K)])
    F = np.array([O.flux(u) for u in U])
    a = P.emf_faces(U, F, n, t)
    for r in range(1, K):
        assert abs(P.emf_faces(np.roll(U, -r, 0), np.roll(F, -r, 0), np.roll(n, -r, 0), t) - a) < 1e-14 * max(1, abs(a))
    q, rr = np.linalg.qr(gen.normal(size=(3, 3)))
    q = q * np.sign(np.diag(rr))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    Ur = U.copy()
    Ur[:, 1:4] = U[:, 1:4] @ q.T
    Ur[:, 5:8] = U[:, 5:8] @ q.T
    Fr = np.array([O.flux(u) for u in Ur])
    assert abs(P.emf_faces(Ur, Fr, n @ q.T, q @ t) - a) < 1e-13 * max(1, abs(a))


# ---- polynomial fields for the divergence-free pin (dict: exponent triple -> coefficient)

def _pmul(p, q):
    out = {}
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            e = (e1[0] + e2[0], e1[1] + e2[1], e1[2] + e2[2])
            out[e] = out.get(e, 0.0) + c1 * c2
    return out


def _pderiv(p, d):
    out = {}
    for e, c in p.items():
        if e[d] > 0:
            f = list(e)
            f[d] -= 1
            out[tuple(f)] = out.get(tuple(f), 0.0) + c * e[d]
    return out


def _padd(p, q, s=1.0):
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, 0.0) + s * c
    return out


def _peval(p, x):
    return sum(c * x[..., 0] ** e[0] * x[..., 1] ** e[1] * x[..., 2] ** e[2] for e, c in p.items())


def _pshift(p, c, l0):
    """p(c + l0 X) as a polynomial in X"""
    out = {}
    for e, coef in p.items():
        term = {(0, 0, 0): coef}
        for d in range(3):
            lin = {(0, 0, 0): c[d]}
            unit = [0, 0, 0]
            unit[d] = 1
            lin[tuple(unit)] = l0
            for _ in range(e[d]):
                term = _pmul(term, lin)
        out = _padd(out, term)
    return out


def _zone_quadrature(order, x_nodes, n=6):
    """points [P][3] and weights J dxi [P] of one zone from its nodal map
    (the map lies in the element space, so the nodal interpolant and its
    gradient are exact): Gauss in zeta times a collapsed Gauss rule on the
    reference triangle"""
    g, gw = np.polynomial.legendre.leggauss(n)
    s, sw = 0.5 * (g + 1), 0.5 * gw
    A, B, Cv = P.TRI_V
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            u, v = s[i], (1 - s[i]) * s[j]
            xy = A + u * (B - A) + v * (Cv - A)
            for k in range(n):
                pts.append([xy[0], xy[1], s[k] - 0.5])
                wts.append(sw[i] * sw[j] * sw[k] * (1 - s[i]) * 2 * (S3 / 4))
    pts, wts = np.array(pts), np.array(wts)
    val, grad = P.basis(order, pts)
    x = val @ x_nodes
    jac = np.einsum("pld,lc->pcd", grad, x_nodes)
    return x, wts * np.abs(np.linalg.det(jac))


@pytest.mark.parametrize("order", [3, 4])
def test_divfree_reconstruction_reproduces_divergence_free_polynomials_of_degree_p_minus_1(order):
    """B = curl A for a random vector potential A of degree p is a
    divergence-free polynomial of degree p - 1, inside the reconstruction's
    space: with its own zone means, Taylor coefficients about the centroid,
    face-point normal components and face averages (by the faces' rules) as
    inputs, the reconstruction returns it exactly at the nodes of curved zones
    (Section IV.b: all constraints and least-squares rows are met by B).
    The zone moments come from an independent quadrature of the nodal map."""
    m = P.OraclePrismMesh(1, 2, r_in=1.0, r_out=1.5, order=order)
    rng = np.random.default_rng(40 + order)
    monos = [(a, b, c) for a in range(order + 1) for b in range(order + 1 - a) for c in range(order + 1 - a - b)]
    Apot = [{e: rng.normal() for e in monos} for _ in range(3)]
    Bpol = [_padd(_pderiv(Apot[2], 1), _pderiv(Apot[1], 2), -1.0),
            _padd(_pderiv(Apot[0], 2), _pderiv(Apot[2], 0), -1.0),
            _padd(_pderiv(Apot[1], 0), _pderiv(Apot[0], 1), -1.0)]
    div = _padd(_padd(_pderiv(Bpol[0], 0), _pderiv(Bpol[1], 1)), _pderiv(Bpol[2], 2))
    assert max(abs(c) for c in div.values()) < 1e-12
    zones = np.array([0, 5, 17, 33, m.nz - 1])
    cen, l0 = m.frames(zones)
    x, _, _ = m.geometry(zones)
    xq, dA = m.face_geometry(zones)
    _, _, nt, ns = P.face_points(order)
    te = P.taylor_indices(order)
    nc = len(te)
    nin, _ = P.divfree_sizes(order)
    Q = dA.shape[1]
    Bin = np.zeros((len(zones), nin))
    for i in range(len(zones)):
        xg, wg = _zone_quadrature(order, x[i])
        X = (xg - cen[i]) / l0[i]
        mom = {e: (wg * X[:, 0] ** e[0] * X[:, 1] ** e[1] * X[:, 2] ** e[2]).sum() / wg.sum() for e in te}
        for comp in range(3):
            bX = _pshift(Bpol[comp], cen[i], l0[i])
            # B = b_0 + sum b_a X^a = (b_0 + sum b_a <X^a>) + sum b_a (X^a - <X^a>)
            mean = bX.get((0, 0, 0), 0.0) + sum(bX.get(e, 0.0) * mom[e] for e in te)
            Bin[i, comp * (nc + 1)] = mean
            for a, e in enumerate(te):
                Bin[i, comp * (nc + 1) + 1 + a] = bX.get(e, 0.0)
        an = np.linalg.norm(dA[i], axis=1)
        nrm = dA[i] / an[:, None]
        Bq = np.stack([_peval(Bpol[c], xq[i]) for c in range(3)], 1)
        bn = (Bq * nrm).sum(1)
        Bin[i, 3 * (nc + 1):3 * (nc + 1) + Q] = bn
        faces = [np.arange(nt), np.arange(nt, 2 * nt)] + [2 * nt + k * ns + np.arange(ns) for k in range(3)]
        for f, q in enumerate(faces):
            Bin[i, 3 * (nc + 1) + Q + f] = (an[q] * bn[q]).sum() / an[q].sum()
    out = m.divfree(zones, Bin)
    N = m.N
    got = out[:, :3 * N].reshape(len(zones), 3, N).transpose(0, 2, 1)
    want = np.stack([_peval(Bpol[c], x) for c in range(3)], 2)
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(out[:, 3 * N:], Bin[:, [0, nc + 1, 2 * (nc + 1)]], rtol=0, atol=1e-11 * scale)

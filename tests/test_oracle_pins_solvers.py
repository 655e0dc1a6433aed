"""Pins of the oracle's Riemann solvers and WENO-AO internals.

Each check compares a piece of the oracle with something it does not
compute itself:

* the fast magnetosonic speed against the closed forms for B = 0, B along
  the normal and B across it, and against the largest characteristic speed
  of the MHD flux Jacobian (its eigenvalues, from central differences of the
  physical flux and numpy's eigenvalue routine);
* the HLL flux in the subsonic branch against values worked out by hand for
  states with known Davis speeds (Section II.c, Section VI step 5);
* the four-state edge electric field in genuinely two-dimensional data:
  supersonic diagonal flows pick exactly the upwind corner, and the result
  does not change when the four zones are relabelled or the whole
  configuration is rotated;
* the three-zone corner solver: equal states give E . t, supersonic flow
  gives the mean of the three faces' upwind electric fields, and it is
  invariant under relabelling and rotation;
* the WENO-AO smoothness indicators, nonlinear weights and blended
  coefficients (Section III, eqs. 3.1-3.4) on zone averages of a polynomial
  of the reconstruction degree, against the indicator integrated with numpy's
  polynomial derivatives over the zone and the small stencils solved with
  numpy's least squares.
"""
import numpy as np
import numpy.polynomial.polynomial as NP
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


def _state(rho, v, p, B, gam=5 / 3):
    v = np.asarray(v, float)
    B = np.asarray(B, float)
    return np.array([rho, *(rho * v), p / (gam - 1) + 0.5 * rho * v @ v + 0.5 * B @ B, *B])


def _efield(U):
    return -np.cross(U[1:4] / U[0], U[5:8])


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rotate_state(U, R):
    V = U.copy()
    V[1:4] = R @ U[1:4]
    V[5:8] = R @ U[5:8]
    return V


# ---------------------------------------------------------------- fast speed
def test_fast_speed_closed_forms():
    gam = 5 / 3
    n = np.array([0.48, -0.6, 0.64])
    rho, p = 1.3, 0.7
    a = np.sqrt(gam * p / rho)
    # no field: the sound speed
    assert abs(O.fast_speed(_state(rho, [0.1, 0.2, 0.3], p, [0, 0, 0]), n) - a) < 1e-15
    # field along the normal: the larger of the sound and Alfven speeds
    for bmag in (0.3, 2.5):
        U = _state(rho, [0.1, -0.2, 0.3], p, bmag * n)
        assert abs(O.fast_speed(U, n) - max(a, bmag / np.sqrt(rho))) < 1e-14
    # field across the normal: sqrt(a^2 + b^2)
    t = np.cross(n, [1.0, 0.0, 0.0])
    t /= np.linalg.norm(t)
    U = _state(rho, [0.1, -0.2, 0.3], p, 1.7 * t)
    assert abs(O.fast_speed(U, n) - np.sqrt(a * a + 1.7 ** 2 / rho)) < 1e-14


def _flux_jacobian(U, n, gam):
    """Jacobian of n . F(U) by central differences of the physical flux."""
    J = np.zeros((8, 8))
    for j in range(8):
        h = 1e-6 * max(1.0, abs(U[j]))
        Up, Um = U.copy(), U.copy()
        Up[j] += h
        Um[j] -= h
        J[:, j] = (O.flux(Up, gam).T @ n - O.flux(Um, gam).T @ n) / (2 * h)
    return J


@pytest.mark.parametrize("seed", range(6))
def test_fast_speed_is_the_largest_characteristic_speed(seed):
    """v_n +- c_f are the extreme eigenvalues of the flux Jacobian along n."""
    gen = np.random.default_rng(seed)
    gam = 5 / 3
    n = gen.normal(size=3)
    n /= np.linalg.norm(n)
    U = _state(gen.uniform(0.5, 2.0), gen.normal(size=3) * 0.5, gen.uniform(0.2, 2.0), gen.normal(size=3), gam)
    lam = np.linalg.eigvals(_flux_jacobian(U, n, gam)).real
    vn = U[1:4] @ n / U[0]
    cf = O.fast_speed(U, n, gam)
    assert abs(lam.max() - (vn + cf)) < 1e-6 * (abs(vn) + cf)
    assert abs(lam.min() - (vn - cf)) < 1e-6 * (abs(vn) + cf)


# ---------------------------------------------------------------- HLL subsonic branch
def test_hll_subsonic_hydro_hand_values():
    """Gas at rest on both sides with sound speed 1 (gamma = 5/3): S_L = -1,
    S_R = 1, so F* = (F_L + F_R)/2 - (U_R - U_L)/2 with F = (0, p, 0, 0, 0)."""
    n = np.array([1.0, 0.0, 0.0])
    UL = _state(1.0, [0, 0, 0], 0.6, [0, 0, 0])
    UR = _state(0.25, [0, 0, 0], 0.15, [0, 0, 0])
    Fs = O.hll(UL, UR, n)
    # rho: -(0.25 - 1)/2; m_x: (0.6 + 0.15)/2; E: -(0.225 - 0.9)/2
    want = np.array([0.375, 0.375, 0.0, 0.0, 0.3375, 0.0, 0.0, 0.0])
    np.testing.assert_allclose(Fs, want, rtol=0, atol=1e-15)


def test_hll_subsonic_magnetised_hand_values():
    """gamma = 2, B across the normal, fast speed 2 on both sides, v_x = +-0.5:
    S_L = -2.5, S_R = 2.5 and F* = (F_L + F_R)/2 - 1.25 (U_R - U_L); the
    fluxes for v = (v_x, 0, 0), B = (0, B_y, 0) are
    (rho v_x, rho v_x^2 + p + B_y^2/2, 0, 0, (E + p + B_y^2/2) v_x, 0, v_x B_y, 0)."""
    gam = 2.0
    n = np.array([1.0, 0.0, 0.0])
    sL = dict(rho=1.0, vx=0.5, p=0.5, By=np.sqrt(3.0))
    sR = dict(rho=4.0, vx=-0.5, p=2.0, By=np.sqrt(12.0))

    def cons(s):
        return _state(s["rho"], [s["vx"], 0, 0], s["p"], [0, s["By"], 0], gam)

    def flux(s):
        E = s["p"] / (gam - 1) + 0.5 * s["rho"] * s["vx"] ** 2 + 0.5 * s["By"] ** 2
        pt = s["p"] + 0.5 * s["By"] ** 2
        return np.array([s["rho"] * s["vx"], s["rho"] * s["vx"] ** 2 + pt, 0, 0, (E + pt) * s["vx"], 0,
                         s["vx"] * s["By"], 0])

    UL, UR = cons(sL), cons(sR)
    assert abs(O.fast_speed(UL, n, gam) - 2.0) < 1e-15 and abs(O.fast_speed(UR, n, gam) - 2.0) < 1e-15
    want = 0.5 * (flux(sL) + flux(sR)) - 1.25 * (UR - UL)
    np.testing.assert_allclose(O.hll(UL, UR, n, gam), want, rtol=0, atol=1e-14)
    # the mirror image: swapping the sides and the normal negates the flux
    np.testing.assert_allclose(O.hll(UR, UL, -n, gam), -want, rtol=0, atol=1e-14)


# ---------------------------------------------------------------- four-state edge field
_CEN4 = np.array([[-1.0, -0.9, 0.1], [1.1, -1.0, -0.05], [0.9, 1.05, 0.0], [-1.0, 1.0, 0.08]])


def _four_states(seed, drift=(0.0, 0.0, 0.0), scale=0.3):
    gen = np.random.default_rng(seed)
    U4 = np.array([_state(gen.uniform(0.6, 1.4), np.asarray(drift) + scale * gen.normal(size=3),
                          gen.uniform(0.5, 1.5), 0.7 * gen.normal(size=3)) for _ in range(4)])
    return U4, np.array([_efield(u) for u in U4])


@pytest.mark.parametrize("corner,direction", [(0, (1, 1)), (1, (-1, 1)), (2, (-1, -1)), (3, (1, -1))])
def test_emf4_supersonic_diagonal_flow_takes_the_upwind_corner(corner, direction):
    """Flow faster than every fast speed along both in-plane directions: the
    wave fan lies entirely downstream, so the edge sees the upwind zone's
    electric field alone (SW for flow toward NE, and so on)."""
    t = np.array([0.0, 0.0, 1.0])
    cen = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], float)
    drift = 25.0 * np.array([direction[0], direction[1], 0.0])
    U4, E4 = _four_states(7 + corner, drift=drift)
    Es = O.emf4(U4, E4, cen, t)
    assert abs(Es - E4[corner] @ t) < 1e-13 * np.abs(E4 @ t).max()


@pytest.mark.parametrize("seed", range(4))
def test_emf4_relabelling_and_rotation_invariance(seed):
    """The electric field along the edge is a property of the four zones, not
    of which one is called south-west, nor of the frame the data are given in
    (subsonic, genuinely two-dimensional data)."""
    t = np.array([0.02, -0.01, 1.0])
    t /= np.linalg.norm(t)
    U4, E4 = _four_states(100 + seed)
    Es = O.emf4(U4, E4, _CEN4, t)
    scale = np.abs(E4 @ t).max()
    for r in (1, 2, 3):
        Er = O.emf4(np.roll(U4, -r, 0), np.roll(E4, -r, 0), np.roll(_CEN4, -r, 0), t)
        assert abs(Er - Es) < 1e-14 * scale
    R = _rotation(seed)
    Erot = O.emf4(np.array([_rotate_state(u, R) for u in U4]), E4 @ R.T, _CEN4 @ R.T, R @ t)
    assert abs(Erot - Es) < 1e-14 * scale
    # and it is not a plain average: the four corner values differ from it
    assert np.abs(E4 @ t - Es).min() > 1e-3 * scale


# ---------------------------------------------------------------- three-zone corner field
def _three_zone_frame():
    """Three zones about the z axis at 90, 210 and 330 degrees; face k (from
    zone k to zone k+1) has the unit normal pointing from k to k+1."""
    ang = np.deg2rad([90.0, 210.0, 330.0])
    c = np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], 1)
    n = np.array([c[(k + 1) % 3] - c[k] for k in range(3)])
    return n / np.linalg.norm(n, axis=1)[:, None], np.array([0.0, 0.0, 1.0])


def test_emf3_equal_states_give_the_zone_field():
    n3, t = _three_zone_frame()
    U = _state(1.2, [0.3, -0.1, 0.2], 0.8, [0.4, 0.5, -0.3])
    E = _efield(U)
    assert abs(O.emf3(np.array([U] * 3), np.array([E] * 3), n3, t) - E @ t) < 1e-15


@pytest.mark.parametrize("phi", [0.0, 60.0, 180.0, 300.0, 15.0])
def test_emf3_supersonic_flow_takes_the_upwind_fields(phi):
    """Flow faster than the fast speeds across every face: each face's HLL
    flux is its upwind zone's n x E, whose projection gives that zone's
    E . t, and the corner value is the mean over the three faces."""
    n3, t = _three_zone_frame()
    d = np.array([np.cos(np.deg2rad(phi)), np.sin(np.deg2rad(phi)), 0.0])
    gen = np.random.default_rng(int(phi))
    U3 = np.array([_state(gen.uniform(0.7, 1.3), 60.0 * d + 0.2 * gen.normal(size=3), gen.uniform(0.5, 1.5),
                          0.5 * gen.normal(size=3)) for _ in range(3)])
    E3 = np.array([_efield(u) for u in U3])
    assert min(abs(n3 @ d)) > 0.25   # every face is crossed supersonically
    up = [k if n3[k] @ d > 0 else (k + 1) % 3 for k in range(3)]
    want = np.mean([E3[u] @ t for u in up])
    assert abs(O.emf3(U3, E3, n3, t) - want) < 1e-13 * np.abs(E3 @ t).max()


@pytest.mark.parametrize("seed", range(3))
def test_emf3_relabelling_and_rotation_invariance(seed):
    n3, t = _three_zone_frame()
    gen = np.random.default_rng(300 + seed)
    U3 = np.array([_state(gen.uniform(0.6, 1.4), 0.3 * gen.normal(size=3), gen.uniform(0.5, 1.5),
                          0.7 * gen.normal(size=3)) for _ in range(3)])
    E3 = np.array([_efield(u) for u in U3])
    Es = O.emf3(U3, E3, n3, t)
    scale = np.abs(E3 @ t).max()
    for r in (1, 2):
        assert abs(O.emf3(np.roll(U3, -r, 0), np.roll(E3, -r, 0), np.roll(n3, -r, 0), t) - Es) < 1e-14 * scale
    R = _rotation(10 + seed)
    Er = O.emf3(np.array([_rotate_state(u, R) for u in U3]), E3 @ R.T, n3 @ R.T, R @ t)
    assert abs(Er - Es) < 1e-14 * scale


# ---------------------------------------------------------------- WENO-AO internals
def _taylor_exponents(deg):
    """Multi-indices of degree 1..deg in the oracle's coefficient order (by
    degree, then the x exponent descending, then the y exponent descending)."""
    return [(a, b, d - a - b) for d in range(1, deg + 1) for a in range(d, -1, -1) for b in range(d - a, -1, -1)]


def _poly_coeffs(exps, vals, deg):
    c = np.zeros((deg + 1,) * 3)
    for e, v in zip(exps, vals):
        c[e] += v
    return c


@pytest.fixture(scope="module", params=[3, 4])
def weno_case(request):
    order = request.param
    m = O.OracleMesh(4, 6, 1.0, 2.0, n_ghost=3, order=order)
    return m


def _zone_avg(m, j, coef3, cen0, len0):
    x, w = m.cubature(j)
    X = (x - cen0) / len0
    return (w * NP.polyval3d(X[:, 0], X[:, 1], X[:, 2], coef3)).sum() / w.sum()


@pytest.mark.parametrize("which", ["regular", "cube_corner"])
@pytest.mark.parametrize("eps", [1e-4, 3e-2])
def test_weno_indicators_weights_and_blend_on_polynomial_data(weno_case, which, eps):
    """Zone averages of a polynomial of the reconstruction degree p-1 written
    in the zone's scaled coordinates X = (x - centroid)/|V|^(1/3).  The large
    stencil's least squares then reproduce it, so its smoothness indicator is
    the zone average of the sum over every multi-index 1 <= |a| <= p-1 of the
    squared derivative d^a q (numpy's polynomial derivatives, integrated with
    the zone's cubature); each small stencil is the least-squares linear fit
    of the neighbours' average differences at their centroids (numpy), with
    indicator |c|^2; the weights are gamma / (beta + eps)^2 normalised
    (gamma_hi = 0.85, the seven small stencils share 0.15) and the blend is
    (w_hi/gamma_hi)(P_hi - sum gamma_s P_s) + sum w_s P_s."""
    m = weno_case
    order = m.order
    deg = order - 1
    cen, vol, shell, stn = m.zones()
    _, nbr = m.zone_faces()
    g = m.n_ghost
    mid = (shell == g + 2)
    full = stn.max()
    cand = np.where(mid & (stn == full))[0] if which == "regular" else np.where(mid & (stn < full))[0]
    assert len(cand) > 0
    z = int(cand[len(cand) // 3])
    len0 = vol[z] ** (1.0 / 3.0)
    exps = _taylor_exponents(deg)
    gen = np.random.default_rng(order * 10 + (which == "regular"))
    U = np.zeros((8, m.nz))
    coeffs = {}
    for v in range(8):
        vals = gen.normal(size=len(exps)) * np.array([0.5 ** sum(e) for e in exps])
        c3 = _poly_coeffs(exps, vals, deg)
        c3[0, 0, 0] = gen.normal()
        coeffs[v] = (vals, c3)
        # zone averages of every zone that can enter zone z's stencils
        near = np.where(np.linalg.norm(cen - cen[z], axis=1) < 6 * len0)[0]
        for j in near:
            U[v, j] = _zone_avg(m, j, c3, cen[z], len0)
    det = m.weno_detail(U, z, weno_eps=eps)
    # central stencil and the six one-sided stencils, each dropping the
    # neighbour whose direction is opposite to one face's neighbour
    dirs = cen[nbr[z]] - cen[z]
    opp = [int(np.argmin(dirs @ dirs[lf])) for lf in range(6)]
    sets = [list(range(6))] + [[j for j in range(6) if j != opp[lf]] for lf in range(6)]
    Xn = (cen[nbr[z]] - cen[z]) / len0
    ghi, gs = 0.85, 0.15 / 7
    ders = [e for e in exps]   # every multi-index of order 1..deg, once
    xq, wq = m.cubature(z)
    Xq = (xq - cen[z]) / len0
    for v in range(8):
        vals, c3 = coeffs[v]
        bhi = 0.0
        for d in ders:
            dc = c3
            for ax in range(3):
                if d[ax]:
                    dc = NP.polyder(dc, d[ax], axis=ax)
            bhi += (wq * NP.polyval3d(Xq[:, 0], Xq[:, 1], Xq[:, 2], dc) ** 2).sum() / wq.sum()
        du = U[v, nbr[z]] - U[v, z]
        cs = [np.linalg.lstsq(Xn[s], du[s], rcond=None)[0] for s in sets]
        bs = np.array([c @ c for c in cs])
        # indicators: the large stencil's, then the small ones as a set
        assert abs(det["beta"][v, 0] - bhi) < 1e-9 * bhi
        np.testing.assert_allclose(np.sort(det["beta"][v, 1:]), np.sort(bs), rtol=1e-9)
        raw = np.array([ghi / (bhi + eps) ** 2] + [gs / (b + eps) ** 2 for b in bs])
        w = raw / raw.sum()
        assert abs(det["w"][v, 0] - w[0]) < 1e-9 * w[0]
        np.testing.assert_allclose(np.sort(det["w"][v, 1:]), np.sort(w[1:]), rtol=1e-9)
        # blended coefficients: large-stencil coefficients are the polynomial's own
        lin = gs * np.sum(cs, axis=0)
        nl = np.sum(w[1:, None] * np.array(cs), axis=0)
        want = w[0] / ghi * vals.copy()
        want[:3] += -w[0] / ghi * lin + nl
        np.testing.assert_allclose(det["coef"][v], want, rtol=0, atol=1e-9 * np.abs(vals).max())
        # the weights are genuinely nonlinear here
        assert abs(w[0] - ghi) > 1e-3


def test_weno_linear_weights_flag(weno_case):
    m = weno_case
    cen, vol, shell, stn = m.zones()
    z = int(np.where(shell == m.n_ghost + 2)[0][5])
    U = np.random.default_rng(3).normal(size=(8, m.nz))
    det = m.weno_detail(U, z, flags=O.FLAG_LINEAR_WEIGHTS)
    assert (det["w"][:, 0] == 0.85).all() and np.allclose(det["w"][:, 1:], 0.15 / 7, rtol=0, atol=1e-17)

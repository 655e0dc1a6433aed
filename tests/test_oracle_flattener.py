"""Pins of the oracle's flattener (CPU).

Section VII.a applies a flattener on its coarse meshes and defers its
definition to other work; the reading (oracle/scheme.c, flattener_eta) is a
compression detector: eta = min(1, max(0, -(l0 D + kappa c) / (kappa c))) with
D the discrete divergence of the zone averages' velocity, l0 = V^(1/3) and c
the smallest fast speed over the zone and its face neighbours; every
reconstruction coefficient of a zone is scaled by 1 - eta.

Checked: the flattener leaves uniform flow, expansion and a gas at rest
untouched (the step is bit-identical to the plain step there); in uniform
compression v = -alpha x its divergence is within a few per cent of the
exact -3 alpha, so eta follows the closed form; above 2 kappa c / l0 every
zone is flattened fully and a fully flattened uniformly compressing state
steps like a first-order one would (every coefficient zero); and the
per-zone values equal an independent evaluation of the definition from the
oracle's face geometry (numpy).
"""
import numpy as np
import pytest

import rg_inputs as RI
from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")

GAM = 5.0 / 3.0


def _state(m, v_of_x, rho=1.0, p=1.0, B=(0.2, -0.1, 0.3)):
    cen, vol, shell, _ = m.zones()
    v = v_of_x(cen)
    U = np.zeros((8, m.nz))
    U[0] = rho
    U[1:4] = rho * v.T
    U[5:8] = np.asarray(B, float)[:, None]
    U[4] = p / (GAM - 1) + 0.5 * rho * (v * v).sum(1) + 0.5 * np.sum(np.square(B))
    x, n, dA = m.face_quad()
    Bf = np.einsum("fqc,c,fq->f", n, np.asarray(B, float), dA) / dA.sum(1)
    return U, Bf


@pytest.fixture(scope="module")
def mesh():
    return O.OracleMesh(8, 6, order=3, n_ghost=2)


def _eta_numpy(m, U, kappa):
    """the definition evaluated with numpy from the oracle's face geometry"""
    cen, vol, shell, _ = m.zones()
    zf, nbr = m.zone_faces()
    _, _, area, fz = m.faces()
    x, n, dA = m.face_quad()
    S = np.einsum("fq,fqc->fc", dA, n)            # vector area of each face (owner's orientation)
    v = (U[1:4] / U[0]).T
    p = (GAM - 1) * (U[4] - 0.5 * (U[1:4] ** 2).sum(0) / U[0] - 0.5 * (U[5:8] ** 2).sum(0))
    cf = np.sqrt(np.maximum(GAM * p / U[0], 0) + (U[5:8] ** 2).sum(0) / U[0])
    g = m.n_ghost
    rec = (shell >= g - 1) & (shell <= g + m.n_rad)
    eta = np.zeros(m.nz)
    for z in np.where(rec)[0]:
        sg = np.where(fz[zf[z], 0] == z, 1.0, -1.0)
        D = np.sum(sg[:, None] * S[zf[z]] * 0.5 * (v[z] + v[nbr[z]])) / vol[z]
        c = min(cf[z], cf[nbr[z]].min())
        eta[z] = min(1.0, max(0.0, -(vol[z] ** (1 / 3) * D + kappa * c) / (kappa * c)))
    return eta, rec


def test_flattener_is_off_for_uniform_expanding_and_resting_flow(mesh):
    m = mesh
    for vf in (lambda x: np.tile([0.3, -0.2, 0.1], (len(x), 1)),     # uniform flow
               lambda x: 0.5 * x,                                   # expansion
               lambda x: np.zeros_like(x)):                        # at rest
        U, Bf = _state(m, vf)
        plain = m.step(U, Bf, 1e-3, gamma=GAM)
        flat = m.step(U, Bf, 1e-3, gamma=GAM, flattener=0.1)
        assert (m.last_eta == 0.0).all()
        assert np.array_equal(plain[0], flat[0]) and np.array_equal(plain[1], flat[1])


def test_flattener_in_uniform_compression_follows_the_closed_form():
    """v = -alpha x: div v = -3 alpha exactly, c = sqrt(gamma p / rho + B^2 / rho)
    is uniform, so eta = clamp((3 alpha l0 - kappa c) / (kappa c), 0, 1) up to
    the discrete divergence's error on the curved zones."""
    m = O.OracleMesh(16, 8, order=3, n_ghost=2)
    cen, vol, shell, _ = m.zones()
    kappa, p, rho, B = 0.1, 1.0, 1.0, np.array([0.2, -0.1, 0.3])
    c = np.sqrt(GAM * p / rho + B @ B / rho)
    g = m.n_ghost
    act = (shell >= g) & (shell < g + m.n_rad)
    l0 = vol ** (1 / 3)
    alpha = 1.5 * kappa * c / (3 * np.median(l0[act]))   # eta about 0.5 in the median zone
    U, Bf = _state(m, lambda x: -alpha * x, rho=rho, p=p, B=B)
    # ghost shells hold the same field (bc = 1), so every divergence sees it
    m.step(U, Bf, 1e-4, gamma=GAM, bc=1, flattener=kappa)
    want = np.clip((3 * alpha * l0 - kappa * c) / (kappa * c), 0, 1)
    # the divergence is exact for this linear field up to the face curvature
    err = np.abs(m.last_eta - want)[act]
    assert err.max() < 0.08 and np.median(err) < 0.02, (err.max(), np.median(err))
    assert 0.2 < np.median(m.last_eta[act]) < 0.8
    # strong compression: every reconstructed zone flattened fully
    U, Bf = _state(m, lambda x: -10 * alpha * x, rho=rho, p=p, B=B)
    m.step(U, Bf, 1e-5, gamma=GAM, bc=1, flattener=kappa)
    rec = (shell >= g - 1) & (shell <= g + m.n_rad)
    assert (m.last_eta[rec] == 1.0).all() and (m.last_eta[~rec] == 0.0).all()


def test_flattener_matches_its_definition_on_the_blast(mesh):
    from tests.test_oracle_fallback import blast_state
    m = mesh
    prob = RI.blast_problem(p_in=1000.0, radius=0.3)
    U, Bf = blast_state(m, prob)
    # let the blast develop so that the flow compresses somewhere
    for _ in range(3):
        U, Bf, _ = m.step(U, Bf, m.cfl_dt(U, 0.15, prob["gamma"]), gamma=prob["gamma"], fallback=True)
    # the step's continuative boundary fill: ghost shells copy the nearest interior shell
    K, g = m.ktot, m.n_ghost
    Uf = U.copy()
    for k in range(K):
        src = g if k < g else (g + m.n_rad - 1 if k >= g + m.n_rad else k)
        Uf[:, k::K] = U[:, src::K]
    global GAM
    old, GAM = GAM, prob["gamma"]
    try:
        want, rec = _eta_numpy(m, Uf, 0.1)
    finally:
        GAM = old
    m.step(U, Bf, 1e-5, gamma=prob["gamma"], flattener=0.1, fallback=True)
    assert np.abs(m.last_eta - want).max() < 1e-12
    assert (want[rec] > 0).sum() > 5 and (want[rec] == 0).sum() > 100

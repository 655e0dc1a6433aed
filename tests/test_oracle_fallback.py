"""Pins of the oracle's first-order fallback (positivity).

The paper leaves positivity to the ruggedised-WENO literature.  The step's
fallback is defined in the oracle: an interior zone whose high-order update
would leave a non-positive (or non-finite) density or pressure is flagged, and
every face and edge of a flagged zone is solved again with the same Riemann
solvers on the zones' conserved states at t^n, a flagged zone taking the
first-order finite-volume update of its own eight averages.  These tests pin
that definition against what fixes it from outside the fallback code: the
plain step's own output (which zones are flagged), the pinned HLL solver and
the face quadrature (the re-solved fluxes), the update formula, and the
invariants the update must keep (conservation, div B, positivity).
"""
import numpy as np
import pytest

import rg_inputs as RI
from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")

N_ANG = N_RAD = 8


def _pressure(U, gamma):
    m2 = (U[1:4] ** 2).sum(0)
    b2 = (U[5:8] ** 2).sum(0)
    return (gamma - 1.0) * (U[4] - 0.5 * m2 / U[0] - 0.5 * b2)


def blast_state(mesh, prob):
    """Zone averages of the blast: the uniform-B state of the wave initialiser
    (dB = 0) with the energy set from the piecewise-constant pressure."""
    U, Bf = mesh.init_alfven(prob)
    cen = mesh.zones()[0]
    p = RI.blast_pressure(prob, cen)
    U[4] = p / (prob["gamma"] - 1.0) + 0.5 * (U[1:4] ** 2).sum(0) / U[0] + 0.5 * (U[5:8] ** 2).sum(0)
    return U, Bf


@pytest.fixture(scope="module")
def case():
    m = O.OracleMesh(N_ANG, N_RAD, 1.0, 2.0, n_ghost=3, order=3)
    prob = RI.blast_problem(p_in=1000.0, radius=0.3)
    gam = prob["gamma"]
    U0, B0 = blast_state(m, prob)
    # three steps with the fallback spread the blast; in the next one the
    # second round of the check flags a zone the first round passed
    U1, B1 = U0, B0
    for _ in range(3):
        U1, B1, _ = m.step(U1, B1, m.cfl_dt(U1, 0.3, gam), gamma=gam, fallback=True)
    dt = m.cfl_dt(U1, 0.3, gam)
    plain = m.step(U1, B1, dt, gamma=gam, debug=True)
    fb = m.step(U1, B1, dt, gamma=gam, debug=True, fallback=True)
    wave = RI.alfven_problem()
    Uw, Bw = m.init_alfven(wave)
    dtw = m.cfl_dt(Uw, 0.3, wave["gamma"])
    first = m.step(Uw, Bw, dtw, gamma=wave["gamma"], debug=True, fallback=True)
    first_plain = m.step(Uw, Bw, dtw, gamma=wave["gamma"], debug=True)
    return dict(m=m, gam=gam, dt=dt, U0=U0, B0=B0, U1=U1, B1=B1, plain=plain, fb=fb, first=first,
                first_plain=first_plain)


def _interior(m):
    shell = m.zones()[2]
    return (shell >= m.n_ghost) & (shell < m.n_ghost + m.n_rad)


def test_flags_start_from_the_zones_the_plain_step_leaves_non_positive(case):
    """Round one flags exactly the zones the plain step leaves non-positive;
    later rounds add only face neighbours of flagged zones, and the check ends
    with every unflagged interior zone positive."""
    m, gam = case["m"], case["gam"]
    Up = case["plain"][0]
    act = _interior(m)
    with np.errstate(invalid="ignore"):
        bad = act & ~((Up[0] > 0) & (_pressure(Up, gam) > 0))
    flags = case["fb"][4].astype(bool)
    assert bad.sum() > 0, "the case must exercise the fallback"
    assert (flags >= bad).all() and not (flags & ~act).any()
    _, nbr = m.zone_faces()
    added = np.where(flags & ~bad)[0]
    assert len(added) > 0, "the case must exercise a second round"
    for z in added:
        assert flags[nbr[z]].any()
    Uo = case["fb"][0]
    assert ((Uo[0] > 0) & (_pressure(Uo, gam) > 0))[act & ~flags].all()


def test_nothing_flagged_means_the_plain_step_bit_for_bit(case):
    Uf, Bfo, phif, gamf, flags = case["first"]
    Up, Bp, phip, gamp = case["first_plain"]
    assert flags.sum() == 0
    np.testing.assert_array_equal(Uf, Up)
    np.testing.assert_array_equal(Bfo, Bp)
    np.testing.assert_array_equal(phif, phip)
    np.testing.assert_array_equal(gamf, gamp)


def test_fallback_changes_only_faces_and_edges_of_flagged_zones(case):
    m = case["m"]
    flags = case["fb"][4].astype(bool)
    zf, _ = m.zone_faces()
    fe, _ = m.face_edges()
    fmask = np.zeros(m.nf, bool)
    fmask[zf[flags].ravel()] = True
    emask = np.zeros(m.ne, bool)
    emask[fe[fmask].ravel()] = True
    phip, gamp = case["plain"][2], case["plain"][3]
    phif, gamf = case["fb"][2], case["fb"][3]
    np.testing.assert_array_equal(phif[~fmask], phip[~fmask])
    np.testing.assert_array_equal(gamf[~emask], gamp[~emask])
    assert (np.abs(phif[fmask] - phip[fmask]).max(1) > 0).all()
    assert (gamf[emask] != gamp[emask]).mean() > 0.5


def test_refluxed_faces_are_hll_of_the_zone_states_over_the_face_quadrature(case):
    """Phi_f = sum_q dA_q HLL(U_L, U_R; n_q) with U the zones' eight averages."""
    m, gam = case["m"], case["gam"]
    U1 = case["U1"]
    flags = case["fb"][4].astype(bool)
    zf, _ = m.zone_faces()
    _, _, _, fz = m.faces()
    _, qn, qdA = m.face_quad()
    act = _interior(m)   # ghost zones are refilled by the step
    faces = np.unique(zf[flags].ravel())
    faces = [f for f in faces if act[fz[f, 0]] and act[fz[f, 1]]]
    assert len(faces) > 0
    phif = case["fb"][2]
    for f in faces:
        UL, UR = U1[:, fz[f, 0]], U1[:, fz[f, 1]]
        ref = sum(qdA[f, q] * O.hll(UL, UR, qn[f, q], gam) for q in range(qn.shape[1]))
        np.testing.assert_allclose(phif[f], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_flagged_zones_take_the_first_order_update_of_their_own_averages(case):
    """A flagged zone's eight averages, its B included, are advanced from its
    own values at t^n by the face fluxes (the first-order finite-volume
    scheme); unflagged zones start B from the reconstruction's mean."""
    m, dt = case["m"], case["dt"]
    U1 = case["U1"]
    Uo, _, phi, _, flags = case["fb"]
    _, vol, _, _ = m.zones()
    zf, _ = m.zone_faces()
    _, _, _, fz = m.faces()
    for z in np.where(flags)[0]:
        sg = np.where(fz[zf[z], 0] == z, 1.0, -1.0)
        ref = U1[:, z] - dt / vol[z] * (sg[:, None] * phi[zf[z]]).sum(0)
        np.testing.assert_allclose(Uo[:, z], ref, rtol=1e-13, atol=1e-13 * np.abs(U1[:, z]).max())


def test_fallback_step_is_conservative_divergence_free_and_positive(case):
    m, gam, dt = case["m"], case["gam"], case["dt"]
    U1 = case["U1"]
    Uo, Bo, phi, _, flags = case["fb"]
    _, vol, _, _ = m.zones()
    zf, _ = m.zone_faces()
    _, _, area, fz = m.faces()
    act = _interior(m)
    sg = np.where(fz[zf][:, :, 0] == np.arange(m.nz)[:, None], 1.0, -1.0)
    div = np.abs((sg * area[zf] * Bo[zf]).sum(1)) / (area[zf] * np.abs(Bo[zf])).sum(1)
    assert div[act].max() < 1e-13
    bnd = np.zeros(8)
    for z in np.where(act)[0]:
        for lf in range(6):
            f = zf[z, lf]
            other = fz[f, 1] if fz[f, 0] == z else fz[f, 0]
            if not act[other]:
                bnd -= dt * (1 if fz[f, 0] == z else -1) * phi[f]
    dsum = ((Uo - U1)[:, act] * vol[act]).sum(1)
    np.testing.assert_allclose(dsum[:5], bnd[:5], rtol=0, atol=1e-13 * np.abs(U1[:5, act] * vol[act]).sum(1).max())
    # the flagged zones come out positive (they did not without the fallback)
    f = flags.astype(bool)
    assert (Uo[0, f] > 0).all() and (_pressure(Uo, gam)[f] > 0).all()

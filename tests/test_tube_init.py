"""Initial states of the spherical MHD shock tubes (Section VIII.c), on the CPU.

Brio-Wu and Ryu-Jones as the section sets them up: a jump in the fluid
state at r = 4.5, a toroidal field B_phi = (sin theta / 2) T(r) from the
tapered radial vector potential A_r, and a radial field
B_r = B_r0 sin(theta) (4.5 / r)^2.  Pins of the oracle's initial state:

* the discrete divergence of its face B vanishes to round-off;
* the outward flux through a whole sphere is the closed form
  B_r0 r0^2 * integral of sin(theta) over the sphere = pi^2 B_r0 r0^2
  (the face rule is converged to about 4e-7 relative at 4 zones per cube edge;
  a wrong sign or a missing r0^2 misses it by O(1));
* away from the taper, every face value agrees with the average of the
  pointwise B . n over the face (its own 3 x 3 rule), so both the orientation
  of the radial flux and the sign of the potential's curl are right;
* zones entirely on one side of r = 4.5 hold that side's density exactly.

The library's own initialisation (rg_init_tube, on a host-only geometry)
agrees with the oracle's: face B to round-off (the two edge and face rules
are the same), zone averages away from the jump to the difference of the two
zone cubatures (measured 5.8e-5 relative).
"""
import numpy as np
import pytest

import rg_inputs as RI
from oracle import oracle as O

PROBLEMS = {"brio_wu": RI.brio_wu_problem, "ryu_jones": RI.ryu_jones_problem}
N_ANG, N_RAD, ORDER = 4, 12, 4


@pytest.fixture(scope="module", params=sorted(PROBLEMS))
def case(request):
    prob = PROBLEMS[request.param](N_RAD)
    m = O.OracleMesh(N_ANG, N_RAD, prob["r_in"], prob["r_out"], n_ghost=3, order=ORDER)
    U, Bf = m.init_tube(prob)
    return request.param, prob, m, U, Bf


def _pointwise_B(prob, X):
    r = np.linalg.norm(X, axis=-1)
    s = np.hypot(X[..., 0], X[..., 1])
    st = s / r
    h = np.tanh((r - prob["rm"]) / prob["delta"])
    T = prob["left"][6] * (1 - h) + prob["right"][6] * (1 + h)
    er = X / r[..., None]
    ep = np.stack([-X[..., 1] / s, X[..., 0] / s, np.zeros_like(s)], -1)
    return (prob["Br0"] * st * (prob["r0"] / r) ** 2)[..., None] * er + (0.5 * st * T)[..., None] * ep


def test_tube_face_B_is_divergence_free(case):
    _, _, m, _, Bf = case
    zf, _ = m.zone_faces()
    _, _, area, fz = m.faces()
    sg = np.where(fz[zf][:, :, 0] == np.arange(m.nz)[:, None], 1.0, -1.0)
    div = np.abs((sg * (Bf * area)[zf]).sum(1))
    assert div.max() < 1e-13 * (np.abs(Bf) * area).max()


def test_tube_flux_through_a_sphere_is_the_closed_form(case):
    _, prob, m, _, Bf = case
    _, _, shell, _ = m.zones()
    zf, _ = m.zone_faces()
    fc, fn, area, _ = m.faces()
    for k in (3, 3 + N_RAD // 2, 3 + N_RAD):      # the inner boundary, mid-shell, the outer boundary
        f = np.unique(zf[shell == k, 4])
        assert len(f) == 6 * N_ANG * N_ANG
        outward = np.sign(np.einsum("fc,fc->f", fn[f], fc[f]))
        total = (Bf[f] * area[f] * outward).sum()
        exact = np.pi ** 2 * prob["Br0"] * prob["r0"] ** 2
        assert abs(total - exact) < 1e-5 * exact


def test_tube_face_values_match_the_pointwise_field_away_from_the_taper(case):
    _, prob, m, _, Bf = case
    fc, _, _, _ = m.faces()
    x, n, dA = m.face_quad()
    Bq = np.einsum("fqc,fqc,fq->f", _pointwise_B(prob, x), n, dA) / dA.sum(1)
    far = np.abs(np.linalg.norm(fc, axis=1) - prob["rm"]) > 6 * prob["delta"]
    assert far.sum() > m.nf // 2
    assert np.abs(Bq - Bf)[far].max() < 1e-3 * np.abs(Bf).max()


def test_tube_density_is_the_side_state_off_the_jump(case):
    _, prob, m, U, _ = case
    _, _, shell, _ = m.zones()
    g = 3
    radius = prob["r_in"] * (prob["r_out"] / prob["r_in"]) ** ((np.arange(N_RAD + 2 * g + 1) - g) / N_RAD)
    lo, hi = radius[shell], radius[shell + 1]
    inside, outside = hi <= prob["rm"], lo > prob["rm"]
    assert inside.any() and outside.any()
    assert np.all(U[0, inside] == prob["left"][0]) and np.all(U[0, outside] == prob["right"][0])
    cut = ~(inside | outside)
    assert np.all((U[0, cut] > min(prob["left"][0], prob["right"][0]) - 1e-14)
                  & (U[0, cut] < max(prob["left"][0], prob["right"][0]) + 1e-14))


def test_library_tube_init_matches_the_oracle(case):
    import paper_1905_02504_amd as R
    from tests.parity_util import Mapping
    _, prob, m, Uo, Bo = case
    lib = R.ShellMHD(N_ANG, N_RAD, ORDER, r_in=prob["r_in"], r_out=prob["r_out"], n_ghost=3, device=False)
    mp = Mapping(lib, m)
    Ul, Bl = lib.init_tube(prob)
    Um, Bm = mp.U(Uo), mp.Bf(Bo)
    assert np.abs(Bl - Bm).max() < 1e-12 * np.abs(Bm).max()
    cen, _ = lib.zone_data()
    far = np.abs(np.linalg.norm(cen, axis=1) - prob["rm"]) > 0.25
    scale = np.maximum(np.abs(Um).max(1, keepdims=True), 1.0)   # Brio-Wu's momenta are 0 on both sides
    assert (np.abs(Ul - Um)[:, far] / scale).max() < 1e-3
    lib.close()


def test_library_tube_init_rejects_a_theta_field():
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    prob = dict(RI.brio_wu_problem(N_RAD))
    prob["left"] = prob["left"][:5] + (0.5,) + prob["left"][6:]
    lib = R.ShellMHD(N_ANG, N_RAD, ORDER, r_in=prob["r_in"], r_out=prob["r_out"], n_ghost=3, device=False)
    with pytest.raises(N.RGError, match="B_theta"):
        lib.init_tube(prob)
    lib.close()

"""Checks at the benchmark's full size, in the launch configuration it times
(fourth order, 6 x 128 x 128 angular x 128 radial = 12,582,912 zones).

The oracle cannot run this mesh, so these check properties that hold at any
size and that an indexing, tiling or launch-shape mistake anywhere on the
mesh would break:

* a uniform flowing state is a fixed point of the step (free stream);
* the benchmark's state (Alfven wave + 1 % noise) after one step: div B at
  round-off and the totals of rho, momentum and energy changed by exactly
  the fluxes through the two radial boundaries;
* the mesh is invariant under the 90 degree rotation about the z axis (a
  symmetry of the cube), so rotating the initial data rotates the result:
  every zone's update is compared with its image's.

Tolerances, from measurements at N = 32, 64, 128 per cube edge.  Free
stream: the zones are 0.012 across at |x| = 1..2, so their geometry carries
round-off of about eps |x| / h relative, which the divergence-free map
amplifies; the reconstruction's zone B then departs from the uniform field by
5e-12, 2.2e-11, 1.05e-10 (growing as 1/h^2), the fluid variables by at most
1.9e-12 at N = 128.  Rotation: on smooth data the two sides' reconstructions
in the MinMod of eq. (4.11) differ only by the truncation error, so a
rounding-level difference between the two runs can flip its choice; the
results then differ at the truncation level, 5.2e-7, 3.4e-8, 2.2e-9 (falling
as h^4), not at round-off.  An indexing or orientation mistake gives
differences of the order of the data's variation across a zone (1e-2 here).
"""
import numpy as np
import pytest

import rg_inputs as RI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_ANG = N_RAD = 128
ORDER = 4


@pytest.fixture(scope="module")
def lib():
    import paper_1905_02504_amd as R
    print(f"[fullsize] building 6x{N_ANG}^2x{N_RAD}, order {ORDER}", flush=True)
    sh = R.ShellMHD(N_ANG, N_RAD, ORDER, n_ghost=3)
    yield sh
    sh.close()


def _rel(x, ref):
    rms = torch.sqrt(torch.mean(ref * ref, dim=1, keepdim=True))
    return ((x - ref).abs() / torch.maximum(ref.abs(), rms)).max().item()


def test_uniform_flow_is_preserved(lib):
    prob = dict(RI.alfven_problem())
    prob["dB"] = 0.0
    U_h, Bf_h = lib.init_alfven(prob)          # uniform B along the seeded axis, v = 0
    v = np.array([0.3, -0.2, 0.1])
    U_h[1:4] = U_h[0] * v[:, None]
    U_h[4] += 0.5 * U_h[0] * (v @ v)
    U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
    dt = lib.cfl_dt(U, 0.3, prob["gamma"])
    print(f"[fullsize] free stream, dt {dt:.3e}", flush=True)
    U1, Bf1, _ = lib.step(U, Bf, dt, gamma=prob["gamma"])
    inter = torch.from_numpy(lib.interior()).cuda()
    e_fluid = _rel(U1[:5, inter], U[:5, inter])
    e_zb = _rel(U1[5:, inter], U[5:, inter])
    e_b = ((Bf1 - Bf).abs().max() / Bf.abs().max()).item()
    print(f"[fullsize] free stream: rho, m, E {e_fluid:.2e}; zone B {e_zb:.2e}; face B {e_b:.2e}", flush=True)
    assert e_fluid < 2e-11 and e_b < 1e-11
    assert e_zb < 1e-9


def _outflow(lib, Phi):
    ncol = lib.info["n_columns"]
    rad = Phi[:, :ncol * (lib.K + 1)].reshape(8, ncol, lib.K + 1)
    return (rad[:, :, lib.g + lib.n_rad].sum(1) - rad[:, :, lib.g].sum(1)).cpu().numpy()


def test_bench_state_step_conserves_and_keeps_div_b(lib):
    prob = RI.alfven_problem()
    gam = prob["gamma"]
    U_h, Bf_h = lib.init_alfven(prob, noise=RI.white_noise(lib.nz), noise_amp=0.01)
    U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
    del U_h, Bf_h
    dt = lib.cfl_dt(U, 0.3, gam)
    d0 = lib.diag(U, Bf, gam)
    U1, Bf1, _ = lib.step(U, Bf, dt, gamma=gam)
    d1 = lib.diag(U1, Bf1, gam)
    expected = np.array(d0["sums"]) - dt * _outflow(lib, lib.fluxes()[0])
    err = np.abs(np.array(d1["sums"]) - expected)[:5] / np.abs(np.array(d0["sums"]))[:5].clip(min=1.0)
    print(f"[fullsize] bench state: div B {d1['div_rel_max']:.2e}, conservation {err.max():.2e}", flush=True)
    assert d1["div_rel_max"] < 1e-13
    assert err.max() < 1e-12


def test_cube_rotation_equivariance(lib):
    from scipy.spatial import cKDTree
    prob = RI.alfven_problem()
    gam = prob["gamma"]
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    prob_r = dict(prob)
    prob_r["frame"] = prob["frame"] @ Rz.T          # each row (e1, e2, a) rotated
    cen, _ = lib.zone_data()
    print("[fullsize] matching zones under the rotation", flush=True)
    _, perm = cKDTree(cen).query(cen @ Rz.T)        # zone perm[z] is the image of zone z
    assert len(np.unique(perm)) == len(perm)
    out = []
    dt = None
    for p in (prob, prob_r):
        U_h, Bf_h = lib.init_alfven(p)
        U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
        del U_h, Bf_h
        if dt is None:
            dt = lib.cfl_dt(U, 0.3, gam)
        U1, _, _ = lib.step(U, Bf, dt, gamma=gam)
        out.append(U1)
        del U, Bf
    U1, U1r = out
    Rt = torch.from_numpy(Rz).cuda()
    img = U1.clone()
    img[1:4] = Rt @ U1[1:4]
    img[5:8] = Rt @ U1[5:8]
    p_t = torch.from_numpy(perm).cuda()
    ref = torch.empty_like(img)
    ref[:, p_t] = img                                # ref at the image zone
    sel = torch.from_numpy(lib.interior()).cuda()    # the rotation keeps every shell
    e = _rel(U1r[:, sel], ref[:, sel])
    print(f"[fullsize] rotation: max relative difference {e:.2e}", flush=True)
    assert e < 2e-8

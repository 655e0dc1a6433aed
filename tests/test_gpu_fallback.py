"""Parity of the step's first-order fallback with the oracle.

Inputs: the magnetised blast (p = 1000 inside a ball of radius 0.3 at 1.5 a,
p = 0.1 and |B| = 10/sqrt(4 pi) outside, gamma = 1.4) on 6 x 8^3 zones, made
by the oracle (for third order after three oracle steps with the fallback, a
state whose check needs a second round).  On the same input both sides take
the plain step and the step with the fallback; the state (1e-12 relative per
zone and variable), the per-zone flags (exactly) and the face fluxes and edge
electric fields must agree.  The intermediate fluxes get 3e-10: next to a
10^4 pressure jump the fourth-order reconstruction turns the different
summation orders of the two sides into flux differences of a few 1e-11
relative to the flux's rms (measured 3e-11 and 9e-11 on the plain step),
while the updated state stays within 1e-12.
"""
import sys

import numpy as np
import pytest

import rg_inputs as RI
from oracle import oracle as O
from tests.parity_util import Mapping, rel_err
from tests.test_oracle_fallback import blast_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_STAGE = 3e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("order,presteps", [(3, 3), (4, 0)])
def test_fallback_parity_blast(order, presteps):
    import paper_1905_02504_amd as R
    say(f"[fallback] order {order}, 6x8^3 blast, {presteps} oracle steps first")
    om = O.OracleMesh(8, 8, order=order, n_ghost=3)
    lib = R.ShellMHD(8, 8, order, n_ghost=3, device=True)
    mp = Mapping(lib, om)
    prob = RI.blast_problem(p_in=1000.0, radius=0.3)
    gam = prob["gamma"]
    U1, B1 = blast_state(om, prob)
    for _ in range(presteps):
        U1, B1, _ = om.step(U1, B1, om.cfl_dt(U1, 0.3, gam), gamma=gam, fallback=True)
    dt = om.cfl_dt(U1, 0.3, gam)
    inter = lib.interior()
    for fb in (False, True):
        ref = om.step(U1, B1, dt, gamma=gam, debug=True, fallback=fb)
        U = torch.from_numpy(mp.U(U1)).cuda()
        Bf = torch.from_numpy(mp.Bf(B1)).cuda()
        say(f"[fallback] GPU step, fallback={fb}")
        Ug, Bg, _ = lib.step(U, Bf, dt, gamma=gam, fallback=fb)
        Phi, Gam = lib.fluxes()
        flags = lib.fallback_zones()
        torch.cuda.synchronize()
        Ug = Ug.cpu().numpy(); Bg = Bg.cpu().numpy(); Phi = Phi.cpu().numpy(); Gam = Gam.cpu().numpy()
        flags = flags.cpu().numpy()
        computed_f = np.abs(Phi).sum(0) > 0
        computed_e = Gam != 0
        res = {"U": rel_err(Ug[:, inter], mp.U(ref[0])[:, inter]).max(),
               "Bf": rel_err(Bg, mp.Bf(ref[1])).max(),
               "Phi": rel_err(Phi[:, computed_f], mp.Phi(ref[2])[:, computed_f]).max(),
               "Gam": rel_err(Gam[computed_e], mp.Gam(ref[3])[computed_e]).max()}
        say(f"[fallback] fallback={fb} errors {res}")
        assert res["U"] < TOL and res["Bf"] < TOL, res
        assert res["Phi"] < TOL_STAGE and res["Gam"] < TOL_STAGE, res
        if fb:
            fz = ref[4][mp.z]
            say(f"[fallback] flagged zones: GPU {int(flags.sum())}, oracle {int(fz.sum())}")
            assert fz.sum() > 0
            np.testing.assert_array_equal(flags, fz)
            # zones newly flagged per round (rg_step_fallback_counts) against
            # the round in which the oracle flagged each zone
            counts = lib.fallback_counts()
            want = np.bincount(om.last_fallback_round, minlength=5)[1:5].tolist()
            say(f"[fallback] per-round counts: GPU {counts}, oracle {want}")
            assert counts == want
        else:
            assert flags.sum() == 0
            assert lib.fallback_counts() == [0, 0, 0, 0]


@pytest.mark.parametrize("order", [3, 4])
def test_fallback_parity_blast_three_way_split_mesh(order):
    """The blast on 6 x 6^2 x 6 zones (6 = 3 x 2: a 3 x 3 first split and one
    bisection per cube face), its initial state by the oracle's cubature of
    the pressure step (radius 0.35 at 1.5 a), one step with the fallback
    against the oracle."""
    import paper_1905_02504_amd as R
    say(f"[fallback] order {order}, 6x6^3 blast")
    om = O.OracleMesh(6, 6, order=order, n_ghost=3)
    lib = R.ShellMHD(6, 6, order, n_ghost=3, device=True)
    mp = Mapping(lib, om)
    prob = RI.blast_problem(p_in=1000.0, radius=0.35)
    gam = prob["gamma"]
    U0, B0 = om.init_blast(prob)
    dt = om.cfl_dt(U0, 0.15, gam)
    ref = om.step(U0, B0, dt, gamma=gam, fallback=True)
    dt_lib = lib.cfl_dt(torch.from_numpy(mp.U(U0)).cuda(), 0.15, gam)
    Ug, Bg, _ = lib.step(torch.from_numpy(mp.U(U0)).cuda(), torch.from_numpy(mp.Bf(B0)).cuda(), dt, gamma=gam,
                         fallback=True)
    flags = lib.fallback_zones().cpu().numpy()
    inter = lib.interior()
    eU = rel_err(Ug.cpu().numpy()[:, inter], mp.U(ref[0])[:, inter]).max()
    eB = rel_err(Bg.cpu().numpy(), mp.Bf(ref[1])).max()
    say(f"[fallback] errors U {eU:.2e} Bf {eB:.2e} dt {abs(dt_lib - dt) / dt:.2e}, flagged GPU {int(flags.sum())} "
        f"oracle {int(ref[2].sum())}")
    assert eU < TOL and eB < TOL and abs(dt_lib - dt) < 1e-12 * dt
    np.testing.assert_array_equal(flags, ref[2][mp.z])


@pytest.mark.parametrize("order", [3, 4])
def test_flattener_parity_blast(order):
    """The flattener (kappa 0.1) on the 6 x 8^3 blast after three oracle steps
    (the blast front compresses): one step with the flattener and the
    fallback against the oracle."""
    import paper_1905_02504_amd as R
    say(f"[flattener] order {order}, 6x8^3 blast")
    om = O.OracleMesh(8, 8, order=order, n_ghost=3)
    lib = R.ShellMHD(8, 8, order, n_ghost=3, device=True)
    mp = Mapping(lib, om)
    prob = RI.blast_problem(p_in=1000.0, radius=0.3)
    gam = prob["gamma"]
    U1, B1 = blast_state(om, prob)
    for _ in range(3):
        U1, B1, _ = om.step(U1, B1, om.cfl_dt(U1, 0.15, gam), gamma=gam, fallback=True)
    dt = om.cfl_dt(U1, 0.15, gam)
    ref = om.step(U1, B1, dt, gamma=gam, fallback=True, flattener=0.1)
    eta = om.last_eta
    Ug, Bg, _ = lib.step(torch.from_numpy(mp.U(U1)).cuda(), torch.from_numpy(mp.Bf(B1)).cuda(), dt, gamma=gam,
                         fallback=True, flattener=0.1)
    flags = lib.fallback_zones().cpu().numpy()
    inter = lib.interior()
    eU = rel_err(Ug.cpu().numpy()[:, inter], mp.U(ref[0])[:, inter]).max()
    eB = rel_err(Bg.cpu().numpy(), mp.Bf(ref[1])).max()
    say(f"[flattener] zones flattened {(eta > 0).sum()} (fully {(eta == 1).sum()}); errors U {eU:.2e} Bf {eB:.2e}; "
        f"fallback GPU {int(flags.sum())} oracle {int(ref[2].sum())}")
    assert (eta > 0).sum() > 5
    assert eU < TOL and eB < TOL
    np.testing.assert_array_equal(flags, ref[2][mp.z])


def test_adjoint_refuses_the_flattener():
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    lib = R.ShellMHD(4, 3, 3, n_ghost=2, device=True)
    U, Bf = lib.init_alfven(RI.alfven_problem())
    U = torch.from_numpy(U).cuda()
    Bf = torch.from_numpy(Bf).cuda()
    gU, gB = torch.zeros_like(U), torch.zeros_like(Bf)
    p = N.rg_step_params(5.0 / 3.0, 1e-3, 0.0, 0, 0, 0.0, 0, 0.1)
    with pytest.raises(N.RGError, match="flattener"):
        N.rg_step_adjoint(lib._geom, p, U.data_ptr(), Bf.data_ptr(), U.data_ptr(), Bf.data_ptr(),
                          gU.data_ptr(), gB.data_ptr(), 0)


def test_adjoint_refuses_the_fallback():
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    say("[fallback] adjoint with the fallback on")
    lib = R.ShellMHD(4, 3, 3, n_ghost=2, device=True)
    U, Bf = lib.init_alfven(RI.alfven_problem())
    U = torch.from_numpy(U).cuda()
    Bf = torch.from_numpy(Bf).cuda()
    gU, gB = torch.zeros_like(U), torch.zeros_like(Bf)
    p = N.rg_step_params(5.0 / 3.0, 1e-3, 0.0, 0, 0, 0.0, 1)
    with pytest.raises(N.RGError, match="fallback"):
        N.rg_step_adjoint(lib._geom, p, U.data_ptr(), Bf.data_ptr(), U.data_ptr(), Bf.data_ptr(),
                          gU.data_ptr(), gB.data_ptr(), 0)


@pytest.mark.parametrize("order", [3, 4])
def test_weno_order_indicator_parity(order):
    """rg_step_weno_order after a step on the blast equals the oracle's
    indicator zone by zone (FP32 output of FP64 weights: 1e-6 absolute)."""
    import paper_1905_02504_amd as R
    say(f"[weno-order] order {order}, 6x8^3 blast")
    om = O.OracleMesh(8, 8, order=order, n_ghost=3)
    lib = R.ShellMHD(8, 8, order, n_ghost=3, device=True)
    mp = Mapping(lib, om)
    prob = RI.blast_problem(p_in=1000.0, radius=0.3)
    U0, B0 = blast_state(om, prob)
    ref = om.weno_order(U0, B0)
    lib.step(torch.from_numpy(mp.U(U0)).cuda(), torch.from_numpy(mp.Bf(B0)).cuda(),
             om.cfl_dt(U0, 0.3, prob["gamma"]), gamma=prob["gamma"])
    got = lib.weno_order().cpu().numpy().astype(np.float64)
    err = np.abs(got - ref[mp.z]).max()
    say(f"[weno-order] max difference {err:.2e}; zones below 1e-3: GPU {(got < 1e-3).sum()}, "
        f"oracle {(ref < 1e-3).sum()}")
    assert err < 1e-6

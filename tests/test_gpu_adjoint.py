"""Adjoint of the step (rg_step_adjoint) against finite differences.

The adjoint is the vector-Jacobian product of one step with dt held fixed.
For seeded output gradients (gU1, gBf1) and seeded input directions
(dU, dBf) it must satisfy

    <gU, dU> + <gBf, dBf>  =  <gU1, J dU> + <gBf1, J dBf>

where the right side is taken by central differences (h = 1e-6 and 1e-7,
FP64) of (a) the library's own step and (b) the oracle's step, on the same
inputs.  Bar: 1e-6 relative.  The loss-based check runs the differentiable rollout
(torch.autograd) through several steps, one checkpoint per step.

The step is piecewise smooth: MinMod (eq. 4.11), the HLL branch and the
signal-speed maxima switch branches at ties, and the adjoint differentiates
the branch taken.  A difference quotient is only a check where no decision
flips within +-h.  On smooth data MinMod ties are dense (the two sides'
reconstructions agree up to truncation error, and a face's central
quadrature point sits next to the face mean), so these checks use rough
states: an Alfven wave with 20% seeded per-zone noise in every primitive
variable and in face B, which keeps every decision far from its tie.
"""
import sys

import numpy as np
import pytest

import rg_inputs as RI
from tests.parity_util import roughen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = 1e-6
TOL = 1e-6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_state(lib, order, problem, om=None):
    if problem == "rough":
        prob = RI.alfven_problem()
        U_h, Bf_h = lib.init_alfven(prob)
        U_h, Bf_h = roughen(U_h, Bf_h, prob["gamma"])
    elif problem == "alfven":
        prob = RI.alfven_problem()
        U_h, Bf_h = lib.init_alfven(prob, noise=RI.white_noise(lib.nz), noise_amp=0.01)
    else:
        from tests.parity_util import Mapping
        prob = RI.harmonic_problem()
        Uo, Bfo = om.init_harmonic(prob)
        mp = Mapping(lib, om)
        U_h, Bf_h = mp.U(Uo), mp.Bf(Bfo)
    return torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda(), prob["gamma"]


def seeded(shape, seed):
    return torch.from_numpy(np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)).cuda()


def directions(U, Bf, seed):
    """input direction scaled per variable by the state's rms"""
    dU = seeded(U.shape, seed) * U.pow(2).mean(1, keepdim=True).sqrt()
    dB = seeded(Bf.shape, seed + 1) * Bf.pow(2).mean().sqrt()
    return dU.contiguous(), dB.contiguous()


def fd_dot(lib, U, Bf, dU, dB, gU1, gB1, dt, gam, bc, h=H):
    Up, Bp, _ = lib.step((U + h * dU).contiguous(), (Bf + h * dB).contiguous(), dt, gamma=gam, bc=bc)
    Um, Bm, _ = lib.step((U - h * dU).contiguous(), (Bf - h * dB).contiguous(), dt, gamma=gam, bc=bc)
    return float(((Up - Um) / (2 * h) * gU1).sum() + ((Bp - Bm) / (2 * h) * gB1).sum())


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def fd_check(a, quotient):
    """Relative difference of the adjoint's directional derivative a from the
    central quotients at h and h / 10.  A decision that flips within +-h spoils
    the quotient that straddles it (rarely both); a wrong adjoint misses both,
    since the two quotients then agree with each other and not with a."""
    return min(rel(a, quotient(H)), rel(a, quotient(H / 10)))


@pytest.mark.parametrize("order,problem,bc,ndir", [(3, "rough", 0, 32), (4, "rough", 0, 32),
                                                   (3, "rough", 1, 8), (4, "rough", 1, 8)])
def test_adjoint_matches_central_differences(order, problem, bc, ndir):
    import paper_1905_02504_amd as R
    from oracle import oracle as O
    say(f"[adjoint] FD order={order} {problem} bc={bc} directions={ndir}")
    n_ang, n_rad = 4, 6
    lib = R.ShellMHD(n_ang, n_rad, order, n_ghost=order - 1)
    om = O.OracleMesh(n_ang, n_rad, order=order, n_ghost=order - 1) if problem == "harmonic" else None
    U, Bf, gam = make_state(lib, order, problem, om)
    dt = lib.cfl_dt(U, 0.4, gam)
    gU1 = seeded(U.shape, 7).contiguous()
    gB1 = seeded(Bf.shape, 8).contiguous()
    gU, gB = lib.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam, bc=bc)
    gU2, gB2 = lib.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam, bc=bc)
    torch.cuda.synchronize()
    assert torch.equal(gU, gU2) and torch.equal(gB, gB2), "adjoint is not deterministic"
    worst = 0.0
    for d in range(ndir):
        dU, dB = directions(U, Bf, 1000 + 2 * d)
        a = float((gU * dU).sum() + (gB * dB).sum())
        worst = max(worst, fd_check(a, lambda h: fd_dot(lib, U, Bf, dU, dB, gU1, gB1, dt, gam, bc, h)))
    say(f"[adjoint] worst relative difference {worst:.2e}")
    assert worst < TOL
    if bc == 0:
        # continuative boundaries overwrite the ghost shells: no gradient there
        inter = torch.from_numpy(lib.interior()).cuda()
        assert float(gU[:, ~inter].abs().max()) == 0.0


def test_adjoint_separate_inputs():
    """zone-state-only and face-B-only directions, each against differences"""
    import paper_1905_02504_amd as R
    lib = R.ShellMHD(4, 5, 3, n_ghost=2)
    U, Bf, gam = make_state(lib, 3, "rough")
    dt = lib.cfl_dt(U, 0.4, gam)
    gU1 = seeded(U.shape, 17).contiguous()
    gB1 = seeded(Bf.shape, 18).contiguous()
    gU, gB = lib.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam)
    dU, dB = directions(U, Bf, 77)
    zU, zB = torch.zeros_like(dU), torch.zeros_like(dB)
    for u, b in ((dU, zB), (zU, dB)):
        a = float((gU * u).sum() + (gB * b).sum())
        f = fd_dot(lib, U, Bf, u, b, gU1, gB1, dt, gam, 0)
        say(f"[adjoint] separate input: adjoint {a:.12e} FD {f:.12e}")
        assert fd_check(a, lambda h: fd_dot(lib, U, Bf, u, b, gU1, gB1, dt, gam, 0, h)) < TOL


def test_adjoint_against_oracle_differences():
    """The same identity with the right side from the oracle's own step."""
    import paper_1905_02504_amd as R
    from oracle import oracle as O
    from tests.parity_util import Mapping
    order, n_ang, n_rad = 3, 8, 8
    say("[adjoint] oracle FD, order 3, 6x8x8x8")
    om = O.OracleMesh(n_ang, n_rad, order=order, n_ghost=order - 1)
    lib = R.ShellMHD(n_ang, n_rad, order, n_ghost=order - 1)
    mp = Mapping(lib, om)
    U_l, Bf_l, gam = make_state(lib, order, "rough")
    U_l = U_l.cpu().numpy()
    Bf_l = Bf_l.cpu().numpy()
    # the same state in the oracle's numbering and face orientation
    Uo = np.zeros_like(U_l)
    Uo[:, mp.z] = U_l
    Bfo = np.zeros_like(Bf_l)
    Bfo[mp.f] = mp.fs * Bf_l
    dt = om.cfl_dt(Uo, 0.4, gam)
    U = torch.from_numpy(mp.U(Uo)).cuda()
    Bf = torch.from_numpy(mp.Bf(Bfo)).cuda()
    rng = np.random.default_rng(5)
    gU1_h = rng.uniform(-1, 1, size=(8, lib.nz))
    gB1_h = rng.uniform(-1, 1, size=lib.nf)
    gU, gB = lib.step_adjoint(U, Bf, torch.from_numpy(gU1_h).cuda(), torch.from_numpy(gB1_h).cuda(), dt, gamma=gam)
    gU = gU.cpu().numpy()
    gB = gB.cpu().numpy()
    for d in range(3):
        r = np.random.default_rng(300 + d)
        dUo = r.uniform(-1, 1, size=Uo.shape) * np.sqrt((Uo ** 2).mean(1, keepdims=True))
        dBo = r.uniform(-1, 1, size=Bfo.shape) * np.sqrt((Bfo ** 2).mean())
        def oracle_fd(h):
            Up, Bp = om.step(Uo + h * dUo, Bfo + h * dBo, dt, gamma=gam)
            Um, Bm = om.step(Uo - h * dUo, Bfo - h * dBo, dt, gamma=gam)
            return float((mp.U((Up - Um) / (2 * h)) * gU1_h).sum() + (mp.Bf((Bp - Bm) / (2 * h)) * gB1_h).sum())
        a = float((gU * mp.U(dUo)).sum() + (gB * mp.Bf(dBo)).sum())
        err = fd_check(a, oracle_fd)
        say(f"[adjoint] direction {d}: adjoint {a:.12e}, relative difference from the oracle's quotient {err:.2e}")
        assert err < TOL


def _oracle_twin(n_ang, n_rad, order):
    """library and oracle on the same mesh, a rough state in both numberings"""
    import paper_1905_02504_amd as R
    from oracle import oracle as O
    from tests.parity_util import Mapping
    om = O.OracleMesh(n_ang, n_rad, order=order, n_ghost=order - 1)
    lib = R.ShellMHD(n_ang, n_rad, order, n_ghost=order - 1)
    mp = Mapping(lib, om)
    U_l, Bf_l, gam = make_state(lib, order, "rough")
    U_l = U_l.cpu().numpy()
    Bf_l = Bf_l.cpu().numpy()
    Uo = np.zeros_like(U_l)
    Uo[:, mp.z] = U_l
    Bfo = np.zeros_like(Bf_l)
    Bfo[mp.f] = mp.fs * Bf_l
    return om, lib, mp, Uo, Bfo, gam


CS_H = 1e-30       # complex-step size
CS_TOL = 1e-9      # adjoint against the oracle's exact directional derivative


@pytest.mark.parametrize("order", [3, 4])
def test_adjoint_against_oracle_complex_step(order):
    """<gU, dU> + <gBf, dBf> from the library's adjoint against the oracle's
    own derivative of its step: the complex step (C99 complex state through
    the whole oracle step, branches on real parts; oracle/sreal.h), which
    is exact to rounding, so the bar is 1e-9 relative, for 32 seeded global
    directions on 6 x 8^3 zones."""
    say(f"[adjoint] oracle complex step, order {order}, 6x8x8x8, 32 directions")
    om, lib, mp, Uo, Bfo, gam = _oracle_twin(8, 8, order)
    dt = om.cfl_dt(Uo, 0.4, gam)
    U = torch.from_numpy(mp.U(Uo)).cuda()
    Bf = torch.from_numpy(mp.Bf(Bfo)).cuda()
    rng = np.random.default_rng(15)
    gU1_h = rng.uniform(-1, 1, size=(8, lib.nz))
    gB1_h = rng.uniform(-1, 1, size=lib.nf)
    gU, gB = lib.step_adjoint(U, Bf, torch.from_numpy(gU1_h).cuda(), torch.from_numpy(gB1_h).cuda(), dt, gamma=gam)
    gU = gU.cpu().numpy()
    gB = gB.cpu().numpy()
    worst = 0.0
    for d in range(32):
        r = np.random.default_rng(900 + d)
        dUo = r.uniform(-1, 1, size=Uo.shape) * np.sqrt((Uo ** 2).mean(1, keepdims=True))
        dBo = r.uniform(-1, 1, size=Bfo.shape) * np.sqrt((Bfo ** 2).mean())
        Uc, Bc = om.step_complex(Uo + 1j * CS_H * dUo, Bfo + 1j * CS_H * dBo, dt, gamma=gam)
        b = float((mp.U(Uc.imag / CS_H) * gU1_h).sum() + (mp.Bf(Bc.imag / CS_H) * gB1_h).sum())
        a = float((gU * mp.U(dUo)).sum() + (gB * mp.Bf(dBo)).sum())
        err = rel(a, b)
        worst = max(worst, err)
        if d % 8 == 0 or err > CS_TOL:
            say(f"[adjoint] direction {d}: adjoint {a:.15e}, oracle complex step {b:.15e}, relative {err:.2e}")
    say(f"[adjoint] worst relative difference over 32 directions {worst:.2e}")
    assert worst < CS_TOL


def test_rollout_gradient_against_oracle_complex_step():
    """The differentiation workload's loss (the outer four shells' |V|
    [(rho - rho*)^2 + (|B|^2 - b*)^2] after 4 third-order steps, dt fixed)
    on 6 x 8^3 zones: the library's autograd gradient (one checkpoint per
    step, rg_step_adjoint in backward) against the oracle's complex-step
    derivative of the same 4-step loss, along 8 seeded global directions in
    the initial conserved variables and face B; bar 1e-9 of sum |g d|."""
    say("[adjoint] rollout against the oracle's complex step, order 3, 6x8x8x8, 4 steps")
    om, lib, mp, Uo, Bfo, gam = _oracle_twin(8, 8, 3)
    dt = om.cfl_dt(Uo, 0.4, gam)
    rho_t_l, b_t_l = RI.loss_targets(lib.nz)
    _, vol_l = lib.zone_data()
    k = lib.shells()
    outer_l = (k >= lib.g + lib.n_rad - 4) & (k < lib.g + lib.n_rad)
    U = torch.from_numpy(mp.U(Uo)).cuda().requires_grad_(True)
    Bf = torch.from_numpy(mp.Bf(Bfo)).cuda().requires_grad_(True)
    U4, _ = lib.rollout(U, Bf, dt, 4, gamma=gam)
    lo = tuple(torch.from_numpy(x).cuda() for x in (rho_t_l, b_t_l, np.abs(vol_l))) + \
        (torch.from_numpy(outer_l).cuda(),)
    loss_outer_shells(U4, *lo).backward()
    gU, gB = U.grad.cpu().numpy(), Bf.grad.cpu().numpy()
    # the loss on the oracle's numbering
    rho_t, b_t, vol = (np.zeros(om.nz) for _ in range(3))
    rho_t[mp.z], b_t[mp.z], vol[mp.z] = rho_t_l, b_t_l, np.abs(vol_l)
    outer = np.zeros(om.nz, bool)
    outer[mp.z] = outer_l
    worst = 0.0
    for d in range(8):
        r = np.random.default_rng(950 + d)
        dUo = r.uniform(-1, 1, size=Uo.shape) * np.sqrt((Uo ** 2).mean(1, keepdims=True))
        dBo = r.uniform(-1, 1, size=Bfo.shape) * np.sqrt((Bfo ** 2).mean())
        Uc, Bc = Uo + 1j * CS_H * dUo, Bfo + 1j * CS_H * dBo
        for _ in range(4):
            Uc, Bc = om.step_complex(Uc, Bc, dt, gamma=gam)
        Lc = (vol[outer] * ((Uc[0, outer] - rho_t[outer]) ** 2 + ((Uc[5:8, outer] ** 2).sum(0) - b_t[outer]) ** 2)).sum()
        b = Lc.imag / CS_H
        terms = np.abs(gU * mp.U(dUo)).sum() + np.abs(gB * mp.Bf(dBo)).sum()
        a = float((gU * mp.U(dUo)).sum() + (gB * mp.Bf(dBo)).sum())
        err = abs(a - b) / terms
        worst = max(worst, err)
        say(f"[adjoint] rollout direction {d}: autograd {a:.15e}, oracle complex step {b:.15e}, "
            f"difference / sum |terms| {err:.2e}")
    assert worst < CS_TOL


def loss_outer_shells(U, rho_t, b_t, vol, outer):
    """sum over the outer four interior shells of |V| [(rho - rho*)^2 + (|B|^2 - b*)^2]"""
    rho = U[0, outer]
    b2 = (U[5:8, outer] ** 2).sum(0)
    return (vol[outer] * ((rho - rho_t[outer]) ** 2 + (b2 - b_t[outer]) ** 2)).sum()


def loss_difference(Ua, Ub, rho_t, b_t, vol, outer):
    """L(Ua) - L(Ub) written as sums of products of differences, so that no
    digits are lost to the cancellation of two nearly equal losses"""
    ra, rb = Ua[0, outer], Ub[0, outer]
    Ba, Bb = Ua[5:8, outer], Ub[5:8, outer]
    b2a, b2b = (Ba ** 2).sum(0), (Bb ** 2).sum(0)
    db2 = ((Ba - Bb) * (Ba + Bb)).sum(0)
    return (vol[outer] * ((ra - rb) * (ra + rb - 2 * rho_t[outer]) + db2 * (b2a + b2b - 2 * b_t[outer]))).sum()


def rollout_case(n_ang, n_rad):
    import paper_1905_02504_amd as R
    lib = R.ShellMHD(n_ang, n_rad, 3, n_ghost=2)
    U0, B0, gam = make_state(lib, 3, "rough")
    dt = lib.cfl_dt(U0, 0.4, gam)
    rho_t, b_t = (torch.from_numpy(x).cuda() for x in RI.loss_targets(lib.nz))
    _, vol = lib.zone_data()
    vol = torch.from_numpy(np.abs(vol)).cuda()
    k = lib.shells()
    outer = torch.from_numpy((k >= lib.g + lib.n_rad - 4) & (k < lib.g + lib.n_rad)).cuda()
    U = U0.clone().requires_grad_(True)
    Bf = B0.clone().requires_grad_(True)
    U4, _ = lib.rollout(U, Bf, dt, 4, gamma=gam)
    loss_outer_shells(U4, rho_t, b_t, vol, outer).backward()
    return lib, U0, B0, gam, dt, (rho_t, b_t, vol, outer), U.grad, Bf.grad


def rollout_fd(lib, U0, B0, gam, dt, lo, dU, dB, h):
    with torch.no_grad():
        Up, _ = lib.rollout((U0 + h * dU).contiguous(), (B0 + h * dB).contiguous(), dt, 4, gamma=gam)
        Um, _ = lib.rollout((U0 - h * dU).contiguous(), (B0 - h * dB).contiguous(), dt, 4, gamma=gam)
        return float(loss_difference(Up, Um, *lo)) / (2 * h)


def test_rollout_gradient_small():
    """4 differentiable third-order steps on 6 x 4 x 4 x 6 zones: autograd
    gradient of the outer-shell loss against central differences (h = 1e-6)."""
    say("[adjoint] rollout, order 3, 6x4x4x6, 4 steps")
    lib, U0, B0, gam, dt, lo, gU, gB = rollout_case(4, 6)
    assert torch.isfinite(gU).all() and torch.isfinite(gB).all()
    worst = 0.0
    for d in range(8):
        dU, dB = directions(U0, B0, 500 + 2 * d)
        a = float((gU * dU).sum() + (gB * dB).sum())
        worst = max(worst, fd_check(a, lambda h: rollout_fd(lib, U0, B0, gam, dt, lo, dU, dB, h)))
    say(f"[adjoint] worst relative difference {worst:.2e}")
    assert worst < TOL


def test_rollout_gradient_third_order_6x32cubed_4_steps():
    """4 differentiable third-order steps on 6 x 32 x 32 x 32 zones (rough
    Alfven state, dt fixed from the initial state).

    (a) The autograd gradient equals the hand-chained adjoints bit for bit
    (one checkpoint per step, forward recomputed).  (b) 32 seeded directional
    derivatives against central differences of the loss: 16 in the initial
    conserved variables and 16 in the vector potential (edge line integrals
    of A, mapped to face B by rg_stokes; their gradient is rg_stokes_T of the
    face-B gradient).  Each direction is confined to a ball of zones / edges
    around a seeded point of the outer shells: at this size a step takes
    millions of MinMod and HLL decisions, and a global direction flips some
    of them within +-h.  The quotients use h = 1e-7 and 1e-8 with the loss
    difference formed without cancellation, and the difference is measured
    against sum |g * d|, the size of the terms of the inner product."""
    say("[adjoint] rollout, order 3, 6x32^3, 4 steps")
    lib, U0, B0, gam, dt, lo, gU, gB = rollout_case(32, 32)
    assert torch.isfinite(gU).all() and torch.isfinite(gB).all()
    rho_t, b_t, vol, outer = lo
    # (a) hand-chained adjoints
    states = [(U0, B0)]
    with torch.no_grad():
        for _ in range(4):
            U1, B1, _ = lib.step(*states[-1], dt, gamma=gam)
            states.append((U1, B1))
        U4 = states[-1][0].clone().requires_grad_(True)
        with torch.enable_grad():
            loss_outer_shells(U4, rho_t, b_t, vol, outer).backward()
        gUn, gBn = U4.grad.contiguous(), torch.zeros_like(B0)
        for n in range(3, -1, -1):
            gUn, gBn = lib.step_adjoint(states[n][0], states[n][1], gUn, gBn, dt, gamma=gam)
    assert torch.equal(gUn, gU) and torch.equal(gBn, gB)
    # (b) localised directions against differences
    gA = lib.stokes_T(gB.contiguous())
    zc, _ = lib.zone_data()
    em, _ = lib.edge_data()
    k = lib.shells()
    outer_h = ((k >= lib.g + lib.n_rad - 4) & (k < lib.g + lib.n_rad))
    rng = np.random.default_rng(600)
    centres = zc[rng.choice(np.where(outer_h)[0], 32, replace=False)]
    brms = B0.pow(2).mean().sqrt()
    worst = 0.0
    for d in range(32):
        x0 = centres[d]
        if d < 16:
            near = torch.from_numpy(np.linalg.norm(zc - x0, axis=1) < 0.15).cuda()
            dU, _ = directions(U0, B0, 700 + 2 * d)
            dU = (dU * near).contiguous()
            dB = torch.zeros_like(B0)
            a = float((gU * dU).sum())
            terms = float((gU * dU).abs().sum())
        else:
            near = torch.from_numpy(np.linalg.norm(em - x0, axis=1) < 0.15).cuda()
            dA = (seeded((lib.ne,), 700 + 2 * d) * near).contiguous()
            dB = lib.stokes(dA)
            scale = float(brms / dB.pow(2).mean().sqrt())
            dA = (dA * scale).contiguous()
            dB = (dB * scale).contiguous()
            dU = torch.zeros_like(U0)
            a = float((gA * dA).sum())
            terms = float((gB * dB).abs().sum())
        fd = [rollout_fd(lib, U0, B0, gam, dt, lo, dU, dB, h) for h in (1e-7, 1e-8)]
        err = min(abs(a - f) for f in fd) / terms
        say(f"[adjoint] rollout direction {d} ({'U' if d < 16 else 'A'}): autograd {a:.12e} "
            f"FD {fd[0]:.12e} / {fd[1]:.12e}, difference / sum |terms| {err:.2e}")
        worst = max(worst, err)
    assert worst < TOL

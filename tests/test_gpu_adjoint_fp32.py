"""Adjoint of the FP32 form (rg_step_adjoint on an RG_MODE_FP32 geometry).

The FP32 form computes the reconstruction, the face nodal B, the predictor
and the traces in FP32; its adjoint recomputes that forward, reverses the
predictor in FP32 and everything else in FP64.  On rough states (as for the
FP64 adjoint: every MinMod, HLL and speed decision far from its tie):

* its gradients agree with the FP64 adjoint's on the same inputs to the
  FP32 rounding of the form (relative L2 difference of the zone-state and
  face-B gradients);
* its directional derivatives agree with central differences of the FP64
  step (the differences are taken in FP64, as the form approximates it);
* it is deterministic;
* on the differentiation workload (third order, 6 x 32^3, 4 checkpointed
  steps, the outer-shell loss) the FP32 rollout's gradient agrees with the
  FP64 rollout's.
"""
import numpy as np
import pytest

import rg_inputs as RI
from tests.test_gpu_adjoint import (directions, fd_dot, loss_outer_shells, make_state, say, seeded)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# bars from the measured differences (6 x 4^2 x 6: 3.8e-8 against the FP64
# adjoint, 3.3e-7 against FP64 differences; the rollout: 4.9e-6) with margin;
# the differences bar is the adjoint's 1e-6
TOL_ADJ = 1e-6       # FP32 adjoint vs FP64 adjoint of one step, relative L2
TOL_FD = 1e-6        # directional derivative vs FP64 central differences, relative
TOL_ROLLOUT = 2e-5   # FP32 rollout gradient vs FP64, relative L2 (4 steps of FP32 forward)


def libs(n_ang, n_rad, order):
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    g = order - 1
    return (R.ShellMHD(n_ang, n_rad, order, n_ghost=g),
            R.ShellMHD(n_ang, n_rad, order, n_ghost=g, mode=N.RG_MODE_FP32))


def l2rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("order", [3, 4])
def test_fp32_adjoint_against_fp64_adjoint_and_differences(order):
    say(f"[adjoint32] order {order}, 6x4^2x6")
    lib64, lib32 = libs(4, 6, order)
    U, Bf, gam = make_state(lib64, order, "rough")
    dt = lib64.cfl_dt(U, 0.4, gam)
    gU1 = seeded(U.shape, 7).contiguous()
    gB1 = seeded(Bf.shape, 8).contiguous()
    gU64, gB64 = lib64.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam)
    gU32, gB32 = lib32.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam)
    gU32b, gB32b = lib32.step_adjoint(U, Bf, gU1, gB1, dt, gamma=gam)
    torch.cuda.synchronize()
    assert torch.equal(gU32, gU32b) and torch.equal(gB32, gB32b), "FP32 adjoint is not deterministic"
    eu, eb = l2rel(gU32, gU64), l2rel(gB32, gB64)
    say(f"[adjoint32] vs FP64 adjoint: zone state {eu:.2e}, face B {eb:.2e}")
    assert eu < TOL_ADJ and eb < TOL_ADJ
    worst = 0.0
    for d in range(8):
        dU, dB = directions(U, Bf, 1000 + 2 * d)
        a = float((gU32 * dU).sum() + (gB32 * dB).sum())
        f = fd_dot(lib64, U, Bf, dU, dB, gU1, gB1, dt, gam, 0)
        worst = max(worst, abs(a - f) / abs(f))
    say(f"[adjoint32] vs FP64 central differences: worst {worst:.2e}")
    assert worst < TOL_FD


def test_fp32_rollout_gradient_third_order_6x32cubed_4_steps():
    say("[adjoint32] rollout, order 3, 6x32^3, 4 steps, FP32 and FP64")
    lib64, lib32 = libs(32, 32, 3)
    U0, B0, gam = make_state(lib64, 3, "rough")
    dt = lib64.cfl_dt(U0, 0.4, gam)
    rho_t, b_t = (torch.from_numpy(x).cuda() for x in RI.loss_targets(lib64.nz))
    _, vol = lib64.zone_data()
    vol = torch.from_numpy(np.abs(vol)).cuda()
    k = lib64.shells()
    outer = torch.from_numpy((k >= lib64.g + lib64.n_rad - 4) & (k < lib64.g + lib64.n_rad)).cuda()
    grads = []
    for lib in (lib64, lib32):
        U = U0.clone().requires_grad_(True)
        Bf = B0.clone().requires_grad_(True)
        U4, _ = lib.rollout(U, Bf, dt, 4, gamma=gam)
        loss_outer_shells(U4, rho_t, b_t, vol, outer).backward()
        grads.append((U.grad, Bf.grad))
    (gU64, gB64), (gU32, gB32) = grads
    eu, eb = l2rel(gU32, gU64), l2rel(gB32, gB64)
    say(f"[adjoint32] rollout gradient vs FP64: zone state {eu:.2e}, face B {eb:.2e}")
    assert eu < TOL_ROLLOUT and eb < TOL_ROLLOUT

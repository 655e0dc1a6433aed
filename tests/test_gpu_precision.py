"""Reduced-precision form (RG_MODE_FP32) against the FP64 library on the same
inputs: relative L1 error per conserved variable after one step, and div B,
which constrained transport keeps at round-off in either precision."""
import numpy as np
import pytest

import rg_inputs as RI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_L1 = 1e-6
TOL_DIV = 1e-13


def _div_rel_max(lib, om, Bf):
    """max relative div B over interior zones, through the oracle's connectivity"""
    from tests.parity_util import Mapping
    from tests.test_gpu_parity import div_rel_max
    return div_rel_max(om, Mapping(lib, om), Bf)


def run_pair(order, n_ang, n_rad, problem, cfl, bc):
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    print(f"[precision] order={order} N={n_ang} Nr={n_rad} {problem}", flush=True)
    g = order - 1
    lib64 = R.ShellMHD(n_ang, n_rad, order, n_ghost=g, mode=N.RG_MODE_FP64)
    lib32 = R.ShellMHD(n_ang, n_rad, order, n_ghost=g, mode=N.RG_MODE_FP32)
    from oracle import oracle as O
    om = O.OracleMesh(n_ang, n_rad, order=order, n_ghost=g)
    prob = RI.alfven_problem() if problem == "alfven" else RI.harmonic_problem()
    if problem == "alfven":
        U_h, Bf_h = lib64.init_alfven(prob, noise=RI.white_noise(lib64.nz), noise_amp=0.01)
    else:
        from tests.parity_util import Mapping
        mp = Mapping(lib64, om)
        Uo, Bfo = om.init_harmonic(prob)
        U_h, Bf_h = mp.U(Uo), mp.Bf(Bfo)
    U = torch.from_numpy(U_h).cuda()
    Bf = torch.from_numpy(Bf_h).cuda()
    gam = prob["gamma"]
    dt = lib64.cfl_dt(U, cfl, gam)
    U64, B64, _ = lib64.step(U, Bf, dt, gamma=gam, bc=bc)
    U32, B32, _ = lib32.step(U, Bf, dt, gamma=gam, bc=bc)
    torch.cuda.synchronize()
    inter = lib64.interior()
    U64 = U64.cpu().numpy()[:, inter]; U32 = U32.cpu().numpy()[:, inter]
    l1 = np.abs(U32 - U64).sum(1) / np.abs(U64).sum(1)
    B64 = B64.cpu().numpy(); B32 = B32.cpu().numpy()
    l1b = np.abs(B32 - B64).sum() / np.abs(B64).sum()
    div = _div_rel_max(lib32, om, B32)
    print(f"[precision] rel L1 per variable {np.array2string(l1, precision=2)}, Bf {l1b:.2e}, div B {div:.2e}",
          flush=True)
    return l1, l1b, div


@pytest.mark.parametrize("order", [3, 4])
def test_fp32_form_small_harmonic(order):
    l1, l1b, div = run_pair(order, 8, 8, "harmonic", 0.4, 0)
    assert l1.max() < TOL_L1 and l1b < TOL_L1 and div < TOL_DIV


def test_fp32_form_alfven_fourth_order():
    l1, l1b, div = run_pair(4, 16, 16, "alfven", 0.3, 0)
    assert l1.max() < TOL_L1 and l1b < TOL_L1 and div < TOL_DIV

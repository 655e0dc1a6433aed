"""Reduced-precision forms against the FP64 library on the same inputs:
relative L1 error per conserved variable after one step, and div B, which
constrained transport keeps at round-off in any precision.  RG_MODE_FP32 is
the FP32 form; RG_MODE_BF16 is that form with the predictor's flux
derivatives on the BF16 matrix cores (each FP32 value split exactly into
three BF16 parts), held to the same bar."""
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


def run_pair(order, n_ang, n_rad, problem, cfl, bc, mode="fp32"):
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    print(f"[precision] order={order} N={n_ang} Nr={n_rad} {problem} {mode}", flush=True)
    g = order - 1
    lib64 = R.ShellMHD(n_ang, n_rad, order, n_ghost=g, mode=N.RG_MODE_FP64)
    lib32 = R.ShellMHD(n_ang, n_rad, order, n_ghost=g,
                       mode=N.RG_MODE_BF16 if mode == "bf16" else N.RG_MODE_FP32)
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


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
@pytest.mark.parametrize("order", [3, 4])
def test_reduced_form_small_harmonic(order, mode):
    l1, l1b, div = run_pair(order, 8, 8, "harmonic", 0.4, 0, mode)
    assert l1.max() < TOL_L1 and l1b < TOL_L1 and div < TOL_DIV


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_reduced_form_alfven_fourth_order(mode):
    l1, l1b, div = run_pair(4, 16, 16, "alfven", 0.3, 0, mode)
    assert l1.max() < TOL_L1 and l1b < TOL_L1 and div < TOL_DIV


@pytest.mark.parametrize("order", [3, 4])
def test_bf16_derivatives_match_fp32_form(order):
    """The BF16 matrix-core derivative against the FP32 form's VALU one on the
    same inputs: both sum exact products in FP32 and differ only in the order
    of the sums, so the states after one step agree to a few FP32 units
    relative to each variable's scale (the FP32 form itself sits about 1e-7
    from the FP64 scheme)."""
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    print(f"[precision] bf16 vs fp32 form, order {order}, 6x12^2x12, Alfven wave + 1% noise", flush=True)
    g = order - 1
    a = R.ShellMHD(12, 12, order, n_ghost=g, mode=N.RG_MODE_FP32)
    b = R.ShellMHD(12, 12, order, n_ghost=g, mode=N.RG_MODE_BF16)
    prob = RI.alfven_problem()
    U_h, Bf_h = a.init_alfven(prob, noise=RI.white_noise(a.nz), noise_amp=0.01)
    U = torch.from_numpy(U_h).cuda()
    Bf = torch.from_numpy(Bf_h).cuda()
    gam = prob["gamma"]
    dt = a.cfl_dt(U, 0.3, gam)
    Ua, Ba, _ = a.step(U, Bf, dt, gamma=gam)
    Ub, Bb, _ = b.step(U, Bf, dt, gamma=gam)
    inter = a.interior()
    Ua = Ua.cpu().numpy()[:, inter]; Ub = Ub.cpu().numpy()[:, inter]
    scale = np.abs(Ua).max(1, keepdims=True)
    err = (np.abs(Ub - Ua) / scale).max(1)
    errb = float((Bb - Ba).abs().max() / Ba.abs().max())
    print(f"[precision] max |bf16 - fp32| / scale per variable {np.array2string(err, precision=2)}, Bf {errb:.2e}",
          flush=True)
    assert err.max() < 1e-5 and errb < 1e-5


def test_bf16_form_has_no_adjoint():
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    print("[precision] the adjoint refuses the BF16 form", flush=True)
    lib = R.ShellMHD(4, 3, 3, n_ghost=2, mode=N.RG_MODE_BF16)
    U, Bf = lib.init_alfven(RI.alfven_problem())
    U = torch.from_numpy(U).cuda()
    Bf = torch.from_numpy(Bf).cuda()
    gU, gB = torch.zeros_like(U), torch.zeros_like(Bf)
    p = N.rg_step_params(5.0 / 3.0, 1e-3, 0.0, 0, 0, 0.0, 0, 0.0)
    with pytest.raises(N.RGError, match="BF16"):
        N.rg_step_adjoint(lib._geom, p, U.data_ptr(), Bf.data_ptr(), U.data_ptr(), Bf.data_ptr(),
                          gU.data_ptr(), gB.data_ptr(), 0)

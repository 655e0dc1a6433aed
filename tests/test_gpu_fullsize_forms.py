"""The reduced-precision forms at the benchmark's full size, in the launch
configuration it times (fourth order, 6 x 128 x 128 angular x 128 radial =
12,582,912 zones): one step of the benchmark state (Alfven wave + 1 % noise)
in the FP32 form and in the BF16 form against the FP64 scheme's step on the
same input and dt.  Properties that hold at any size: div B at round-off
(constrained transport stays FP64), the totals of rho, momentum and energy
changed by exactly the fluxes through the two radial boundaries (the update
stays FP64), and the relative L1 difference from the FP64 step per variable
within the forms' FP32 accuracy (1e-6; measured about 1e-7).  The FP64
geometry is closed before a reduced form's is built: the two sets of work
buffers do not fit in HBM together."""
import numpy as np
import pytest

import rg_inputs as RI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_ANG = N_RAD = 128
ORDER = 4


def _outflow(lib, Phi):
    ncol = lib.info["n_columns"]
    rad = Phi[:, :ncol * (lib.K + 1)].reshape(8, ncol, lib.K + 1)
    return (rad[:, :, lib.g + lib.n_rad].sum(1) - rad[:, :, lib.g].sum(1)).cpu().numpy()


@pytest.fixture(scope="module")
def fp64_step():
    import paper_1905_02504_amd as R
    print(f"[fullsize-forms] FP64 reference, 6x{N_ANG}^2x{N_RAD}, order {ORDER}", flush=True)
    sh = R.ShellMHD(N_ANG, N_RAD, ORDER, n_ghost=3)
    prob = RI.alfven_problem()
    U_h, Bf_h = sh.init_alfven(prob, noise=RI.white_noise(sh.nz), noise_amp=0.01)
    U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
    dt = sh.cfl_dt(U, 0.3, prob["gamma"])
    U1, _, _ = sh.step(U, Bf, dt, gamma=prob["gamma"])
    inter = sh.interior()
    ref = U1[:, torch.from_numpy(inter).cuda()].cpu().numpy()
    del U, Bf, U1
    sh.close()
    return U_h, Bf_h, dt, ref, inter, prob["gamma"]


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_reduced_form_full_size_step(fp64_step, mode):
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    U_h, Bf_h, dt, ref, inter, gam = fp64_step
    print(f"[fullsize-forms] {mode} form", flush=True)
    sh = R.ShellMHD(N_ANG, N_RAD, ORDER, n_ghost=3, mode=N.RG_MODE_BF16 if mode == "bf16" else N.RG_MODE_FP32)
    try:
        U, Bf = torch.from_numpy(U_h).cuda(), torch.from_numpy(Bf_h).cuda()
        d0 = sh.diag(U, Bf, gam)
        U1, Bf1, _ = sh.step(U, Bf, dt, gamma=gam)
        d1 = sh.diag(U1, Bf1, gam)
        expected = np.array(d0["sums"]) - dt * _outflow(sh, sh.fluxes()[0])
        cons = (np.abs(np.array(d1["sums"]) - expected)[:5] / np.abs(np.array(d0["sums"]))[:5].clip(min=1.0)).max()
        got = U1[:, torch.from_numpy(inter).cuda()].cpu().numpy()
        l1 = np.abs(got - ref).sum(1) / np.abs(ref).sum(1)
        print(f"[fullsize-forms] {mode}: div B {d1['div_rel_max']:.2e}, conservation {cons:.2e}, "
              f"rel L1 vs FP64 {np.array2string(l1, precision=2)}", flush=True)
        assert d1["div_rel_max"] < 1e-13
        assert cons < 1e-12
        assert l1.max() < 1e-6
    finally:
        sh.close()

"""Design order of accuracy on the circularly polarised Alfven wave.

The wave is an exact solution of ideal MHD (it translates along its axis at
the Alfven speed), so the error of the full scheme after a fixed time
measures its order.  Meshes 6 x N x N x N for N = 16, 32, 64; the same final
time T = 20 dt_64 reached in 5, 10 and 20 steps (dt halves with the mesh
spacing); ghost shells hold the exact solution at the start of every step
(fixed radial boundaries).  Error: volume-weighted L1 over the interior zones,
summed over the eight conserved variables.
"""
import numpy as np
import pytest

import rg_inputs as RI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CFL = 0.3


def ghost_masks(lib):
    k = lib.shells()
    zg = ~((k >= lib.g) & (k < lib.g + lib.n_rad))
    nrf = lib.info["n_radial_faces"]
    f = np.arange(lib.nf)
    kf = np.where(f < nrf, f % (lib.K + 1), (f - nrf) % lib.K)
    fg = np.where(f < nrf, (kf < lib.g) | (kf > lib.g + lib.n_rad), (kf < lib.g) | (kf > lib.g + lib.n_rad - 1))
    return torch.from_numpy(zg).cuda(), torch.from_numpy(fg).cuda()


def run(order, n, steps, dt):
    import paper_1905_02504_amd as R
    lib = R.ShellMHD(n, n, order, n_ghost=max(3, order - 1))
    prob = RI.alfven_problem()
    gam = prob["gamma"]
    zg, fg = ghost_masks(lib)
    U_h, Bf_h = lib.init_alfven(prob, t=0.0)
    U = torch.from_numpy(U_h).cuda()
    Bf = torch.from_numpy(Bf_h).cuda()
    for s in range(steps):
        if s > 0:
            Ue, Be = lib.init_alfven(prob, t=s * dt)
            U[:, zg] = torch.from_numpy(Ue).cuda()[:, zg]
            Bf[fg] = torch.from_numpy(Be).cuda()[fg]
        U, Bf, _ = lib.step(U, Bf, dt, gamma=gam, bc=1)
    Ue, _ = lib.init_alfven(prob, t=steps * dt)
    _, vol = lib.zone_data()
    inter = lib.interior()
    err = (np.abs(U.cpu().numpy()[:, inter] - Ue[:, inter]) * np.abs(vol[inter])).sum() / np.abs(vol[inter]).sum()
    lib.close()
    return err


@pytest.mark.parametrize("order", [3, 4])
def test_alfven_wave_converges_at_design_order(order):
    import paper_1905_02504_amd as R
    # dt on the finest mesh from its initial state, then 2x and 4x on the coarser ones
    lib = R.ShellMHD(64, 64, order, n_ghost=max(3, order - 1))
    prob = RI.alfven_problem()
    U_h, _ = lib.init_alfven(prob)
    dt64 = lib.cfl_dt(torch.from_numpy(U_h).cuda(), CFL, prob["gamma"])
    lib.close()
    errs = {}
    for n, steps in ((16, 5), (32, 10), (64, 20)):
        errs[n] = run(order, n, steps, dt64 * 20 / steps)
        print(f"[convergence] order {order} N={n} steps={steps} L1 error {errs[n]:.4e}", flush=True)
    o1 = np.log2(errs[16] / errs[32])
    o2 = np.log2(errs[32] / errs[64])
    print(f"[convergence] order {order}: observed {o1:.2f} (16->32), {o2:.2f} (32->64)", flush=True)
    assert o2 > order - 0.5

"""rg_cfl_dt_noalloc, the allocation-free variant of rg_cfl_dt, through the
C-ABI: the same timestep bit for bit on two calls in a row, the second on a
smaller mesh, and a third back on the first (the shared device array keeps
the last call's partial minima, which no later call may read)."""
import sys

import numpy as np
import pytest

import rg_inputs as RI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(n_ang, n_rad, order, seed):
    import paper_1905_02504_amd as R
    lib = R.ShellMHD(n_ang, n_rad, order, n_ghost=order - 1, device=True)
    noise = np.random.default_rng(seed).uniform(-1, 1, size=(2, lib.nz))
    U, Bf = lib.init_alfven(RI.alfven_problem(), noise=noise, noise_amp=0.2)
    return lib, torch.from_numpy(U).cuda()


def test_cfl_dt_noalloc_matches_cfl_dt():
    from paper_1905_02504_amd import _native as N
    big = _case(16, 16, 4, 1)     # 24,576 interior zones: 96 block minima
    small = _case(4, 5, 3, 2)     # 480 interior zones: 2 block minima
    stream = torch.cuda.current_stream().cuda_stream
    for name, (lib, U) in (("big", big), ("small", small), ("big again", big)):
        say(f"[noalloc] {name}: {lib.nz} zones")
        for cfl in (0.4, 0.13):
            ref = N.rg_cfl_dt(lib._geom, U.data_ptr(), 5.0 / 3.0, cfl, stream)
            got = N.rg_cfl_dt_noalloc(lib._geom, U.data_ptr(), 5.0 / 3.0, cfl, stream)
            say(f"[noalloc] cfl {cfl}: rg_cfl_dt {ref!r}, rg_cfl_dt_noalloc {got!r}")
            assert got == ref and ref > 0

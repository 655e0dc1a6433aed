"""Conditioning of the per-column reconstruction systems (CPU).

rg_geom_conditioning reports, per column, the 2-norm condition number of the
large-stencil least-squares matrix (Section III, eq. 3.4 rows) and the 1-norm
condition number of the divergence-free KKT matrix (Section IV.b).  The
first is checked against numpy's SVD of the same matrix as the oracle builds
it (zone cubature, its own code); the report then explains the one parity
case whose two sides differ by more than 1e-12: on thin zones the oracle
alone moves by far more than on regular ones when its inputs change by one
ulp.
"""
import numpy as np
import pytest

import rg_inputs as RI
from oracle import oracle as O
from tests.parity_util import Mapping, rel_err

pytestmark = pytest.mark.filterwarnings("ignore")


def _lib():
    import paper_1905_02504_amd as R
    return R


@pytest.mark.parametrize("order,n_ang,n_rad", [(3, 4, 6), (4, 4, 8), (4, 2, 70)])
def test_least_squares_condition_matches_numpy_svd(order, n_ang, n_rad):
    R = _lib()
    lib = R.ShellMHD(n_ang, n_rad, order, n_ghost=order - 1, device=False)
    om = O.OracleMesh(n_ang, n_rad, order=order, n_ghost=order - 1)
    mp = Mapping(lib, om)
    lsq, kkt = lib.conditioning()
    assert lsq.shape == (6 * n_ang * n_ang,) and (lsq >= 1).all() and (kkt >= 1).all()
    cen, vol, shell, stn = om.zones()
    K = lib.K
    g = om.n_ghost
    # zones of interior shells in a few columns, the library's column of each
    zlib = np.arange(lib.nz)
    for zl in zlib[(zlib % K == g + 1)][:: max(1, 6 * n_ang * n_ang // 7)]:
        zo = mp.z[zl]
        s = np.linalg.svd(om.weno_rows(zo), compute_uv=False)
        assert abs(lsq[zl // K] - s[0] / s[-1]) < 1e-6 * (s[0] / s[-1]), (zl, lsq[zl // K], s[0] / s[-1])


def _ulp_sensitivity(order, n_ang, n_rad):
    om = O.OracleMesh(n_ang, n_rad, order=order, n_ghost=order - 1)
    prob = RI.harmonic_problem()
    U, Bf = om.init_harmonic(prob)
    dt = om.cfl_dt(U, 0.4, prob["gamma"])
    U1, _ = om.step(U, Bf, dt, gamma=prob["gamma"])
    gen = np.random.default_rng(5)
    Up = U * (1 + np.finfo(float).eps * gen.choice([-1, 1], size=U.shape))
    Bp = Bf * (1 + np.finfo(float).eps * gen.choice([-1, 1], size=Bf.shape))
    U2, _ = om.step(Up, Bp, dt, gamma=prob["gamma"])
    _, _, shell, _ = om.zones()
    act = (shell >= om.n_ghost) & (shell < om.n_ghost + om.n_rad)
    return rel_err(U2[:, act], U1[:, act]).max()


@pytest.mark.slow
def test_thin_zones_amplify_rounding():
    """Fourth order, two columns per cube edge, 70 shells (zones about 70
    times wider than deep) against 4 columns and 8 shells: the condition
    numbers differ by three orders of magnitude, and a one-ulp change of the
    oracle's inputs moves its output about a hundred times more."""
    R = _lib()
    thin = R.ShellMHD(2, 70, 4, n_ghost=3, device=False).conditioning()
    reg = R.ShellMHD(4, 8, 4, n_ghost=3, device=False).conditioning()
    assert thin[0].max() > 1e3 * reg[0].max() and thin[1].max() > 1e3 * reg[1].max()
    d_thin = _ulp_sensitivity(4, 2, 70)
    d_reg = _ulp_sensitivity(4, 4, 8)
    assert d_reg < 1e-13 and d_thin > 20 * d_reg, (d_thin, d_reg)

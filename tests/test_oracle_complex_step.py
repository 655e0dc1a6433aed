"""The oracle's complex-step directional derivative (CPU).

The step's state-dependent arithmetic compiled with C99 complex numbers
(oracle/scheme_cx.c, oracle/sreal.h) gives, for state U + i h dU and face B
Bf + i h dB, the step's directional derivative along (dU, dB) as the
imaginary part over h, exact to rounding, with every branch taken by the
real parts.  Checked: its real part is the real oracle's step; its
derivative agrees with central differences of the real oracle; and it is
linear in the direction (the derivative along a + 2b is the derivative
along a plus twice that along b), which it would not be if an imaginary
part leaked into a branch decision or the two solves of a real system with
a complex right-hand side were mixed up.
"""
import numpy as np
import pytest

import rg_inputs as RI
from oracle import oracle as O
from tests.parity_util import roughen

pytestmark = pytest.mark.filterwarnings("ignore")

H = 1e-30


@pytest.fixture(scope="module", params=[3, 4])
def case(request):
    order = request.param
    m = O.OracleMesh(4, 4, order=order, n_ghost=order - 1)
    prob = RI.alfven_problem()
    U, Bf = m.init_alfven(prob)
    # a rough state, whose branch decisions sit far from their ties (on
    # smooth data MinMod ties are dense and central differences cross them)
    U, Bf = roughen(U, Bf, prob["gamma"])
    return m, U, Bf, m.cfl_dt(U, 0.3, prob["gamma"]), prob["gamma"]


def _dir(m, seed):
    gen = np.random.default_rng(seed)
    return gen.normal(size=(8, m.nz)), gen.normal(size=m.nf)


def test_real_part_is_the_real_step(case):
    m, U, Bf, dt, gam = case
    dU, dB = _dir(m, 1)
    Ur, Br = m.step(U, Bf, dt, gamma=gam)
    Uc, Bc = m.step_complex(U + 1j * H * dU, Bf + 1j * H * dB, dt, gamma=gam)
    scale = np.abs(Ur).max(1, keepdims=True)
    assert (np.abs(Uc.real - Ur) / scale).max() < 1e-15
    assert np.abs(Bc.real - Br).max() < 1e-15 * np.abs(Br).max()


def test_derivative_matches_central_differences(case):
    m, U, Bf, dt, gam = case
    dU, dB = _dir(m, 2)
    Uc, Bc = m.step_complex(U + 1j * H * dU, Bf + 1j * H * dB, dt, gamma=gam)
    gU, gB = Uc.imag / H, Bc.imag / H
    # central quotients at h and h / 10: a quotient whose interval straddles a
    # MinMod tie or an HLL branch switch is spoilt, the other is not
    eU, eB = [], []
    for h in (1e-6, 1e-7):
        Up, Bp = m.step(U + h * dU, Bf + h * dB, dt, gamma=gam)
        Um, Bm = m.step(U - h * dU, Bf - h * dB, dt, gamma=gam)
        eU.append(np.abs(gU - (Up - Um) / (2 * h)))
        eB.append(np.abs(gB - (Bp - Bm) / (2 * h)))
    assert np.abs(gU).max() > 1e-3
    assert np.minimum(*eU).max() < 1e-6 * np.abs(gU).max()
    assert np.minimum(*eB).max() < 1e-6 * np.abs(gB).max()


def test_derivative_is_linear_in_the_direction(case):
    m, U, Bf, dt, gam = case
    a, b = _dir(m, 3), _dir(m, 4)

    def deriv(d):
        Uc, Bc = m.step_complex(U + 1j * H * d[0], Bf + 1j * H * d[1], dt, gamma=gam)
        return Uc.imag / H, Bc.imag / H

    ga, gb = deriv(a), deriv(b)
    gab = deriv((a[0] + 2 * b[0], a[1] + 2 * b[1]))
    for k in range(2):
        want = ga[k] + 2 * gb[k]
        assert np.abs(gab[k] - want).max() < 1e-12 * np.abs(want).max()

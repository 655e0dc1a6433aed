"""Pins of the 1-D references used by the spherical shock-tube checks (CPU).

The exact planar Riemann solver reproduces the star state of Sod's problem
tabulated in Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics" (test 1: p* = 0.30313, u* = 0.92745, rho*_L = 0.42632,
rho*_R = 0.26557), and the finite-volume scheme in planar mode converges to
that exact solution.

The equatorial MHD scheme is pinned by what ideal MHD fixes for it:
* with no field and no rotation it is the spherical Euler scheme;
* in planar mode a small transverse pulse on a uniform normal field is an
  Alfven wave: it travels at B_n / sqrt(rho) unchanged (L1 convergence,
  about 1.5 orders with the minmod limiter, to the translated pulse);
* a uniform gas at rest threaded by B_r = C / r^2 is an equilibrium (the
  field's pressure gradient balances its tension) and stays at rest to
  round-off, the scheme being balanced for it;
* so is a toroidal field B_phi = K / r (magnetic pressure and hoop stress
  cancel), which the scheme keeps to its truncation error: the spurious
  velocity falls at second order.
A dropped term or a wrong sign in any of these parts fails one of them.
"""
import numpy as np

from tests.radial_reference import exact_sod, mhd_equator, spherical_euler


def test_exact_solver_star_state_of_sod():
    # just left and right of the contact (u* t = 0.185 at t = 0.2)
    q = exact_sod(np.array([0.9, 0.95]), 1.0, 1.0, 0.0, 0.125, 0.1, 0.0, 1.4)
    np.testing.assert_allclose(q[2], [0.30313, 0.30313], atol=1e-5)
    np.testing.assert_allclose(q[1], [0.92745, 0.92745], atol=1e-5)
    np.testing.assert_allclose(q[0], [0.42632, 0.26557], atol=1e-5)
    # undisturbed states beyond the waves
    np.testing.assert_allclose(exact_sod(np.array([-2.0, 2.0]), 1.0, 1.0, 0.0, 0.125, 0.1, 0.0, 1.4).T,
                               [[1.0, 0.0, 1.0], [0.125, 0.0, 0.1]])


def test_planar_scheme_converges_to_the_exact_solution():
    err = []
    for n in (250, 500):
        rc, q = spherical_euler(0.0, 1.0, n, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, 0.2, planar=True)
        ex = exact_sod((rc - 0.5) / 0.2, 1.0, 1.0, 0.0, 0.125, 0.1, 0.0, 1.4)
        err.append(np.abs(q - ex).mean(axis=1))
    assert (err[1] < err[0]).all()
    assert err[1][0] < 4e-3


def test_mhd_equator_without_field_is_the_euler_scheme():
    args = (2.0, 3.0, 400, 2.5)
    _, q_e = spherical_euler(*args, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, 0.2)
    _, q_m = mhd_equator(*args, (1.0, 1.0, 0.0, 0.0, 0.0), (0.125, 0.1, 0.0, 0.0, 0.0), 0.0, 1.4, 0.2)
    rho, vr, vp, p, bp = q_m
    np.testing.assert_allclose(np.array([rho, vr, p]), q_e, rtol=0, atol=1e-10)
    assert np.abs(vp).max() == 0.0 and np.abs(bp).max() == 0.0


def test_mhd_equator_planar_alfven_pulse_travels_at_the_alfven_speed():
    rho0, B0, eps, w, x0, t = 4.0, 2.0, 1e-3, 0.05, 0.3, 0.2
    vA = B0 / np.sqrt(rho0)
    pulse = lambda x: eps * np.exp(-((x - x0) / w) ** 2)

    def init(x):
        b = pulse(x)
        return np.full_like(x, rho0), np.ones_like(x), 0 * x, -b / np.sqrt(rho0), b

    err = []
    for n in (200, 400):
        rc, q = mhd_equator(0.0, 1.0, n, 0.0, None, None, B0, 5.0 / 3.0, t, planar=True, init=init)
        ex = pulse(rc - vA * t)
        err.append(np.abs(q[4] - ex).mean() / eps)     # L1 (minmod clips the peak in max norm)
        np.testing.assert_allclose(q[2], -q[4] / np.sqrt(rho0), atol=0.05 * eps)
    # measured 3.9e-3 and 1.4e-3; a pulse going the wrong way or standing still is off by O(1)
    assert err[1] < 3e-3 and err[0] / err[1] > 2.5


def test_mhd_equator_radial_field_equilibrium_stays_at_rest():
    init = lambda r: (np.ones_like(r), np.ones_like(r), 0 * r, 0 * r, 0 * r)
    _, q = mhd_equator(4.0, 6.0, 200, 0.0, None, None, 3.0 * 4.5 ** 2, 2.0, 0.1, init=init)
    assert np.abs(q[1]).max() < 1e-12 and np.abs(q[2]).max() == 0.0
    assert np.abs(q[3] - 1.0).max() < 1e-12 and np.abs(q[0] - 1.0).max() < 1e-12


def test_mhd_equator_toroidal_field_equilibrium_to_second_order():
    K = 5.0
    init = lambda r: (np.ones_like(r), np.ones_like(r), 0 * r, 0 * r, K / r)
    vmax = []
    for n in (100, 200):
        _, q = mhd_equator(4.0, 6.0, n, 0.0, None, None, 1.0, 2.0, 0.05, init=init)
        inner = slice(n // 5, -n // 5)     # away from the zero-gradient ends
        vmax.append(np.abs(q[1][inner]).max())
    assert vmax[0] < 1e-3 and vmax[0] / vmax[1] > 3.0

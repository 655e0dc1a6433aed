"""Pins of the 1-D reference used by the spherical shock-tube check (CPU).

The exact planar Riemann solver reproduces the star state of Sod's problem
tabulated in Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics" (test 1: p* = 0.30313, u* = 0.92745, rho*_L = 0.42632,
rho*_R = 0.26557), and the finite-volume scheme in planar mode converges to
that exact solution.
"""
import numpy as np

from tests.radial_reference import exact_sod, spherical_euler


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

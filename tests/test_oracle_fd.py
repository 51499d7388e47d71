"""Pins of the oracle's forward-difference Jacobian and of ROS4 driven by it (the paper's ROS4
set-up, Section 5: first-order forward differences, one source-term evaluation per column)."""
import numpy as np
import scipy.linalg

from oracle import oracle as O
from paper_1608_05794_amd import synth


def test_fd_jacobian_approximates_analytic(oracle_mech):
    # the analytic Jacobian is pinned against Richardson-extrapolated central differences elsewhere;
    # a one-sided difference with the CVODE increment rule must agree with it to O(sqrt(eps))
    # relative to the row scale (a dropped term, a wrong sign or a transposed column is O(1))
    for name, recipe in (("M13", "small"), ("M53", "mid")):
        m = oracle_mech(name)
        y, P = synth.reactor_states(m.n_species, 6, recipe, seed=11)
        J = m.jac(y, P)
        Jf = m.jac_fd(y, P, h=1e-9)
        scale = np.abs(J).max(axis=2, keepdims=True)
        assert np.all(np.abs(J - Jf) <= 1e-4 * scale), name
        # column order: the largest entry of every column sits in the same row
        assert np.array_equal(np.abs(J).argmax(axis=1), np.abs(Jf).argmax(axis=1))


def test_fd_jacobian_of_linear_system_is_exact():
    # for y' = A y the forward difference equals A up to rounding, so the FD-driven ROS4 matches the
    # exact-Jacobian ROS4 step for step and the closed-form solution to the requested tolerance
    rng = np.random.default_rng(3)
    N = 6
    Q = scipy.linalg.qr(rng.standard_normal((N, N)))[0]
    A = Q @ np.diag(-np.logspace(0, 4, N)) @ Q.T
    y0 = rng.standard_normal(N)
    exact = scipy.linalg.expm(A * 1e-2) @ y0
    ra = O.integrate_linear(A, y0, 1e-2, "ros4", rtol=1e-9, atol=1e-12)
    rf = O.integrate_linear(A, y0, 1e-2, "ros4", rtol=1e-9, atol=1e-12, jacobian="fd")
    assert ra["status"] == rf["status"] == 0
    assert ra["n_accept"] == rf["n_accept"] and ra["n_reject"] == rf["n_reject"]
    np.testing.assert_allclose(rf["y"], ra["y"], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(rf["y"], exact, rtol=1e-6, atol=1e-9)


def test_fd_ros4_integration_agrees_with_analytic(oracle_mech):
    # both drive the same ODE to rtol 1e-8: the end states agree in units of the error weights
    m = oracle_mech("M13")
    y, P = synth.reactor_states(m.n_species, 8, "small", seed=7)
    ra = m.integrate(y, P, 1e-5)
    rf = m.integrate(y, P, 1e-5, jacobian="fd")
    assert np.all(ra["status"] == 0) and np.all(rf["status"] == 0)
    w = np.abs(rf["y"] - ra["y"]) / (np.abs(ra["y"]) + 1e-12 / 1e-8)
    assert w.max() <= 1e-6

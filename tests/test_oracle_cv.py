"""Pins of the oracle's constant-volume form (Section 3: c_v and the internal energies in place of
c_p and the enthalpies; the density is fixed)."""
import numpy as np
import pytest

from paper_1608_05794_amd import synth

R = 8.314462618


def _density(m, y, P):
    W = np.asarray(m.W)
    S = (y[1:] / W[:, None]).sum(axis=0)
    return P / (R * y[0] * S)


def _internal_energy(m, y):
    """Mass-specific internal energy sum_k Y_k (H_k - R T) / W_k from the NASA-7 tables."""
    W = np.asarray(m.W)
    out = np.zeros(y.shape[1])
    for r in range(y.shape[1]):
        T = y[0, r]
        cp, h, s = m.thermo(T)
        out[r] = (y[1:, r] * R * T * (h - 1.0) / W).sum()
    return out


def _cv(m, y):
    W = np.asarray(m.W)
    out = np.zeros(y.shape[1])
    for r in range(y.shape[1]):
        cp, h, s = m.thermo(y[0, r])
        out[r] = (y[1:, r] * R * (cp - 1.0) / W).sum()
    return out


@pytest.mark.parametrize("name,recipe", [("M13", "small"), ("M53", "mid")])
def test_cv_source_term_conserves_internal_energy(oracle_mech, name, recipe):
    # closed rigid adiabatic reactor: du/dt = sum_k (U_k / W_k) dY_k/dt + c_v dT/dt = 0
    m = oracle_mech(name)
    y, P = synth.reactor_states(m.n_species, 6, recipe, seed=31)
    rho = _density(m, y, P)
    f = m.rhs(y, rho, reactor="cv")
    W = np.asarray(m.W)
    for r in range(y.shape[1]):
        T = y[0, r]
        cp, h, s = m.thermo(T)
        U = R * T * (h - 1.0)
        terms = np.concatenate([U / W * f[1:, r], [_cv(m, y[:, r:r + 1])[0] * f[0, r]]])
        assert abs(terms.sum()) <= 1e-12 * np.abs(terms).sum()
    # mass is conserved and the species rates are those of the constant-pressure form at the same state
    assert np.all(np.abs(f[1:].sum(axis=0)) <= 1e-12 * np.abs(f[1:]).sum(axis=0))
    fp = m.rhs(y, P)
    np.testing.assert_allclose(f[1:], fp[1:], rtol=1e-12, atol=1e-300)
    # and the temperature rates differ exactly by the energy form: rho c_v f_T^v - rho c_p f_T^p = R T sum wdot
    assert not np.allclose(f[0], fp[0])


def test_cv_jacobian_vs_central_differences(oracle_mech):
    from .test_oracle_jac import fd_jacobian

    class CV:
        def __init__(self, m):
            self.m = m

        def rhs(self, y, rho):
            return self.m.rhs(y, rho, reactor="cv")

    for name, recipe in (("M13", "small"), ("M53", "mid")):
        m = oracle_mech(name)
        y, P = synth.reactor_states(m.n_species, 2, recipe, seed=41)
        rho = _density(m, y, P)
        J = m.jac(y, rho, reactor="cv")
        for r in range(y.shape[1]):
            Jfd = fd_jacobian(CV(m), y[:, r].copy(), rho[r])
            yscale = np.maximum(np.abs(y[:, r]), 1e-9)
            contrib = np.abs(J[r]) * yscale[None, :]
            rowscale = contrib.max(axis=1, keepdims=True) + 1e-300
            err = np.abs(J[r] - Jfd) * yscale[None, :] / rowscale
            assert err.max() < 2e-7, (name, r, np.unravel_index(err.argmax(), err.shape), err.max())


@pytest.mark.parametrize("method", ["ros4", "rkf45"])
def test_cv_integration_conserves_energy_and_mass(oracle_mech, method):
    m = oracle_mech("M13")
    y, P = synth.reactor_states(m.n_species, 6, "small", seed=51)
    rho = _density(m, y, P)
    te = 1e-5 if method == "ros4" else 2e-12
    res = m.integrate(y, rho, te, method, reactor="cv")
    assert np.all(res["status"] == 0)
    u0, u1 = _internal_energy(m, y), _internal_energy(m, res["y"])
    # the energy drift stays at the level of the error control (rtol 1e-8 on T and on each Y)
    cv = _cv(m, res["y"])
    assert np.all(np.abs(u1 - u0) <= 1e-7 * cv * res["y"][0] + 1e-9 * np.abs(u0))
    np.testing.assert_allclose(res["y"][1:].sum(axis=0), y[1:].sum(axis=0), rtol=1e-9)
    # a rigid reactor that heats up raises its pressure by the ideal-gas law; it does not stay at P0
    W = np.asarray(m.W)
    P1 = rho * R * res["y"][0] * (res["y"][1:] / W[:, None]).sum(axis=0)
    assert np.all(np.isfinite(P1)) and not np.allclose(P1, P, rtol=1e-6)

"""Pins of the oracle's thermodynamics and source term (Section 3).

Nothing here re-implements the oracle's formulas: the checks are conservation
laws that any correct source term satisfies, values the generator was built
from, derivative identities, and closed-form solutions of tiny mechanisms.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_05794_amd import synth

from . import mechs_for_tests as TM

R = synth.R_GAS


@pytest.mark.parametrize("name", ["M13", "M53", "M111"])
def test_thermo_matches_construction_data(name, mech_path):
    """H(298.15) and S(298.15) reproduce the drawn formation data; cp follows the smooth model."""
    mech = synth.make_mechanism(name)
    m = O.Mechanism(mech_path(name))
    cp, h, s = m.thermo(298.15)
    for k, sp in enumerate(mech.species):
        assert abs(h[k] * R * 298.15 - sp.hf298) < 1.5e3          # J/mol, fit residual
        assert abs(s[k] * R - sp.s298) < 1.5                      # J/(mol K)
    for T in (300.0, 700.0, 1500.0, 4000.0):
        cp, _, _ = m.thermo(T)
        for k, sp in enumerate(mech.species):
            ref, _, _ = synth._smooth_thermo(sp.model[0], sp.model[1], sp.hf298, sp.s298, np.array([T]))
            assert abs(cp[k] - ref[0]) < 0.5


@pytest.mark.parametrize("name", ["M13", "M53"])
def test_thermo_derivative_identities(name, oracle_mech):
    """dH/dT = cp and dS/dT = cp/T on both ranges; cp > 0 on [100, 8000] K; continuity at Tmid."""
    m = oracle_mech(name)
    for T in (400.0, 850.0, 1300.0, 3000.0):
        d = 1e-4 * T
        _, hp, sp = m.thermo(T + d)
        _, hm, sm = m.thermo(T - d)
        cp, _, _ = m.thermo(T)
        dH = ((T + d) * hp - (T - d) * hm) / (2 * d)          # d(H/R)/dT
        dS = (sp - sm) / (2 * d)
        assert np.allclose(dH, cp, rtol=1e-7, atol=1e-7)
        assert np.allclose(dS * T, cp, rtol=1e-7, atol=1e-7)
    for T in np.linspace(100.0, 8000.0, 80):
        assert np.all(m.thermo(T)[0] > 0)
    lo = m.thermo(1000.0 - 1e-9)
    hi = m.thermo(1000.0)
    for a, b in zip(lo, hi):
        assert np.allclose(a, b, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("name,recipe", [("M13", "small"), ("M53", "mid"), ("M111", "divergent")])
def test_rhs_conservation(name, recipe, oracle_mech):
    """Mass, elements and enthalpy are conserved by the source term (Eqs. ydot, tdot)."""
    m = oracle_mech(name)
    y, P = synth.reactor_states(m.n_species, 64, recipe, seed=11)
    f = m.rhs(y, P)
    W = m.W[:, None]
    scale = np.abs(f[1:]).sum(axis=0)
    assert np.all(np.abs(f[1:].sum(axis=0)) <= 1e-13 * scale)
    E = m.comp.T.astype(float)
    mol = f[1:] / W
    assert np.all(np.abs(E @ mol) <= 1e-13 * (E @ np.abs(mol)))
    for r in range(8):
        qf, qr, rho, cp_mass, hRT = m.rates(y[:, r], P[r])
        T = y[0, r]
        H = R * T * hRT                                      # J/mol
        terms = H * f[1:, r] / m.W[:, 0] if m.W.ndim == 2 else H * f[1:, r] / m.W
        # cp dT/dt + sum_k (H_k/W_k) dY_k/dt = 0 (adiabatic, isobaric)
        assert abs(cp_mass * f[0, r] + terms.sum()) <= 1e-12 * np.abs(terms).sum()


def _closed_form_YA(y, P, mech, keff_f, keff_r, t):
    """Y_A(t) for A <=> B with constant effective first-order rates."""
    YA0, YB0 = y[1, 0], y[2, 0]
    eq = keff_r * (YA0 + YB0) / (keff_f + keff_r)
    return eq + (YA0 - eq) * math.exp(-(keff_f + keff_r) * t)


@pytest.mark.parametrize("method", ["ros4", "rkf45"])
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_isomerization_closed_form(kind, method, tmp_path):
    """A <=> B (elementary, third-body, Lindemann, Troe at its centre) against the exact exponential relaxation."""
    T, P = 1000.0, 2.0e5
    A = 1.0e3                      # kf = A T / 2 with beta = 1, Ea = R T ln 2 (order-1 rate, 1/s)
    a7A, a7B = 5.0, 5.7            # Kc = exp(0.7)
    y, Pa = TM.isomer_state(T=T, P=P)
    base = TM.isomer_mechanism(0, A=A, T=T)
    rho, C = TM.concentrations(base, y, P)
    M = C[0] + C[1] + 2.5 * C[2]   # efficiencies 1, 1, 2.5
    kinf = A * T / 2.0
    if kind == 0:
        mech = TM.isomer_mechanism(0, A=A, T=T, a7A=a7A, a7B=a7B)
        keff = kinf
    elif kind == 1:
        # third-body: rate constant in m^3/(mol s); scale A so that [M] k is O(1e5)
        mech = TM.isomer_mechanism(1, A=A / M, T=T, a7A=a7A, a7B=a7B)
        keff = kinf / M * M
    elif kind == 2:
        Pr = 3.0
        k0 = Pr * kinf / M
        mech = TM.isomer_mechanism(2, A=A, T=T, a7A=a7A, a7B=a7B, low=(k0, 0.0, 0.0))
        keff = kinf * Pr / (1.0 + Pr)
    else:
        # Troe with Fcent = 0.5 exactly (a = 0.5, T3 -> 0, T1 -> inf, T2 -> inf) and Pr at the centre,
        # log10 Pr = 0.4 + 0.67 log10 Fcent, where the broadening factor equals Fcent.
        Fc = 0.5
        Pr = 10.0 ** (0.4 + 0.67 * math.log10(Fc))
        k0 = Pr * kinf / M
        mech = TM.isomer_mechanism(3, A=A, T=T, a7A=a7A, a7B=a7B, low=(k0, 0.0, 0.0), troe=(0.5, 1e-30, 1e30, 1e30))
        keff = kinf * Pr / (1.0 + Pr) * Fc
    path = TM.write(mech, tmp_path / "iso.ckm")
    m = O.Mechanism(path)
    Kc = math.exp(a7B - a7A)
    kf, kr = keff, keff / Kc
    # the source term at t = 0 already has the closed-form rate
    f = m.rhs(y, Pa)
    dYA = -kf * y[1, 0] + kr * y[2, 0]
    assert f[1, 0] == pytest.approx(dYA, rel=1e-12)
    assert abs(f[0, 0]) < 1e-9
    t_end = 1.5 / (kf + kr)
    res = m.integrate(y, Pa, t_end, method, rtol=1e-11, atol=1e-15)
    assert res["status"][0] == 0
    YA = res["y"][1, 0]
    assert YA == pytest.approx(_closed_form_YA(y, P, mech, kf, kr, t_end), rel=2e-9)
    assert res["y"][0, 0] == pytest.approx(T, rel=1e-12)


# Troe broadening (Gilbert, Luther & Troe 1983, the standard fall-off form the paper defers to):
# log10 F = log10 Fc / (1 + f^2), f = x / (n - 0.14 x), x = log10 Pr + c, c = -0.4 - 0.67 log10 Fc,
# n = 0.75 - 1.27 log10 Fc, Fc = (1 - a) exp(-T/T***) + a exp(-T/T*) + exp(-T**/T).
# Points where F is known without evaluating that expression: x = 0 (f = 0, F = Fc), x = n / 1.14
# (f = +1, F = sqrt(Fc)) and x = -n / 0.86 (f = -1, F = sqrt(Fc)); and parameter sets in which
# exactly one Fc term is non-zero and equals 1/2.  A wrong 0.14, 1.27, 0.67, 0.4 or 0.75, or a
# swapped role of T***, T* or T**, moves F away from these values.
_LN2 = math.log(2.0)
_TROE_ISOLATED = {
    # (a, T***, T*, T**) at T = 1000 K; each gives Fc = 1/2 from a single term
    "T***": (0.0, 1000.0 / _LN2, 1e30, 1e30),
    "T*": (1.0, 1e30, 1000.0 / _LN2, 1e30),
    "T**": (0.0, 1e-30, 1e30, 1000.0 * _LN2),
}


@pytest.mark.parametrize("term", sorted(_TROE_ISOLATED))
@pytest.mark.parametrize("point", ["centre", "f=+1", "f=-1"])
def test_troe_broadening_closed_forms(term, point, tmp_path):
    T, P = 1000.0, 2.0e5
    A = 1.0e3
    a7A, a7B = 5.0, 5.7
    y, Pa = TM.isomer_state(T=T, P=P)
    base = TM.isomer_mechanism(0, A=A, T=T)
    rho, C = TM.concentrations(base, y, P)
    M = C[0] + C[1] + 2.5 * C[2]
    kinf = A * T / 2.0
    Fc = 0.5
    L = math.log10(Fc)
    c, n = -0.4 - 0.67 * L, 0.75 - 1.27 * L
    x = {"centre": 0.0, "f=+1": n / 1.14, "f=-1": -n / 0.86}[point]
    F = Fc if point == "centre" else math.sqrt(Fc)
    Pr = 10.0 ** (x - c)
    k0 = Pr * kinf / M
    mech = TM.isomer_mechanism(3, A=A, T=T, a7A=a7A, a7B=a7B, low=(k0, 0.0, 0.0), troe=_TROE_ISOLATED[term])
    m = O.Mechanism(TM.write(mech, tmp_path / "troe.ckm"))
    kf = kinf * Pr / (1.0 + Pr) * F
    kr = kf / math.exp(a7B - a7A)
    f = m.rhs(y, Pa)
    assert f[1, 0] == pytest.approx(-kf * y[1, 0] + kr * y[2, 0], rel=1e-12)
    assert f[2, 0] == pytest.approx(kf * y[1, 0] - kr * y[2, 0], rel=1e-12)


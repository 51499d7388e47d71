"""Hand-built tiny mechanisms whose dynamics have closed forms.

Species A and B are isomers (same composition and molar mass) with identical
NASA coefficients a1..a6 and different a7: H_A = H_B, so dT/dt = 0 and the
density stays constant, and the equilibrium constant is exp(a7_B - a7_A).
A bath species with a third-body efficiency different from 1 keeps [M]
constant but not equal to the total concentration.
"""
import math

import numpy as np

from paper_1608_05794_amd import synth

R = synth.R_GAS


def _species(name, comp, a7):
    a = np.array([3.5, 1e-4, 0.0, 0.0, 0.0, -1000.0, a7])
    W = sum(synth.ELEMENT_W[e] * c for e, c in comp.items())
    return synth.Species(name, dict(comp), W, a.copy(), a.copy())


def isomer_mechanism(kind, A=1.0e3, beta=1.0, Ea=None, T=1000.0, a7A=5.0, a7B=5.7, low=None, troe=None,
                     bath_eff=2.5):
    """A <=> B (kind 0), A + M <=> B + M (kind 1), A (+M) <=> B (+M) (kind 2 Lindemann, 3 Troe).

    With beta = 1 and Ea = R T ln 2 the forward rate constant at T is A*T/2 exactly.
    """
    if Ea is None:
        Ea = R * T * math.log(2.0)
    sp = [_species("A", {"H": 1, "O": 1, "N": 1}, a7A), _species("B", {"H": 1, "O": 1, "N": 1}, a7B),
          _species("N2", {"N": 2}, 10.0)]
    # the bath must be thermally inert too: give it the same a1..a6 shape (its H does not matter,
    # it has no production rate)
    eff = [(2, bath_eff)] if kind >= 1 else []
    r = synth.Reaction(kind, 1, [(0, 1)], [(1, 1)], (A, beta, Ea), low=low or (), troe=troe or (), eff=eff)
    return synth.Mechanism(["H", "O", "N"], sp, [r])


def write(mech, path):
    synth.write_mechanism(mech, str(path))
    return str(path)


def isomer_state(YA=0.3, YB=0.1, T=1000.0, P=2.0e5):
    y = np.array([[T], [YA], [YB], [1.0 - YA - YB]])
    return y, np.array([P])


def concentrations(mech, y, P):
    T = y[0, 0]
    Y = y[1:, 0]
    W = np.array([s.W for s in mech.species])
    rho = P / (R * T * np.sum(Y / W))
    return rho, rho * Y / W

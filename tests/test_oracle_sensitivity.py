"""How far rounding alone moves an integration: the oracle against itself with y0 perturbed by one ulp.

This calibrates the integration parity bar.  Species within a few decades of atol = 1e-12 are only
controlled to atol by the step-size controller, so their plain relative error after a long stiff
integration is set by rounding amplification and exceeds 1e-6 even oracle-against-oracle; measured
in the solver's own error weights (atol + rtol |y|) the difference stays far below 1e-6.
"""
import numpy as np

from paper_1608_05794_amd import synth

from .parity_util import state_rel_error, weighted_error


def test_one_ulp_sensitivity(oracle_mech):
    m = oracle_mech("M53")
    y, P = synth.reactor_states(m.n_species, 67, "mid", seed=1002)
    y, P = y[:, :24].copy(), P[:24].copy()
    a = m.integrate(y, P, 2e-6, "ros4")
    flip = np.random.default_rng(0).choice([-1.0, 1.0], size=y.shape)
    b = m.integrate(y * (1.0 + 2.220446049250313e-16 * flip), P, 2e-6, "ros4")
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    eT, eY = state_rel_error(a["y"], b["y"])
    ew = weighted_error(a["y"], b["y"])
    print(f"oracle vs oracle (1 ulp): rel T {eT:.2e}, rel Y(>1e-12) {eY:.2e}, weighted {ew:.2e}")
    assert eY > 1e-6          # the plain relative bar is not attainable near atol
    assert ew < 1e-7 and eT < 1e-9

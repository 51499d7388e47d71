"""The library's step-size controller against a closed form (Algorithm 1 under the stated
controller), not only against the oracle: with negligible source terms (A <=> B with a rate
constant of order 1e-300) the starting step takes the published fallback result 1e-6 s, every
error estimate is negligible, each accepted step grows h by the upper bound 5, and the run ends
after the first m with 1e-6 (5^m - 1) / 4 >= t_end, the last step clipped onto t_end."""
import math

import numpy as np
import pytest
import torch

from . import mechs_for_tests as TM

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method,kernel", [("ros4", "wave"), ("ros4", "lane"), ("rkf45", "wave"), ("rkf45", "lane")])
def test_step_counts_of_a_quiescent_mixture(method, kernel, tmp_path):
    from paper_1608_05794_amd import ck
    g = ck.Mechanism(TM.write(TM.isomer_mechanism(0, A=1e-300), tmp_path / "quiescent.mech"))
    y1, P1 = TM.isomer_state()
    n = 130                                   # three wavefronts, a ragged last one
    y0 = np.repeat(y1, n, axis=1)
    P0 = np.repeat(P1, n)
    for t_end in (1e-5, 1e-3, 3e-2):
        m = math.ceil(math.log(4.0 * t_end / 1e-6 + 1.0, 5.0))
        print(f"[controller] {method} {kernel}: {n} reactors to {t_end:g} s, expect {m} steps", flush=True)
        y = torch.as_tensor(y0, device="cuda")
        t = torch.zeros(n, dtype=torch.float64, device="cuda")
        h = torch.zeros(n, dtype=torch.float64, device="cuda")
        r = ck.integrate(g, y, torch.as_tensor(P0, device="cuda"), t_end, method=method, kernel=kernel, t=t, h=h)
        torch.cuda.synchronize()
        assert np.all(r["status"].cpu().numpy() == 0)
        assert np.all(r["n_accept"].cpu().numpy() == m) and np.all(r["n_reject"].cpu().numpy() == 0)
        assert np.all(t.cpu().numpy() == t_end)
        assert np.array_equal(r["y"].cpu().numpy(), y0)

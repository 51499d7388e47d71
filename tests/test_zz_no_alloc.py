"""The allocation-free ROS4 entry point (ck_integrate_ros4_noalloc) against the allocating one
(ck_integrate_ros4 with a library-owned workspace), through the C ABI: two calls in a row on each
mechanism, the second with a smaller batch (the fixed device array keeps the previous call's
contents).  Bitwise for the single-wavefront kernel (13 and 53 species); to the integration
tolerance for the four-wavefront workgroup kernels, half-row and tile forms (111 species,
reaction sums ordered by LDS atomics across wavefronts)."""
import numpy as np
import pytest
import torch

from paper_1608_05794_amd import synth

from .parity_util import weighted_error

pytestmark = pytest.mark.gpu

CASES = [("M13", "small", (300, 77), 1e-6, "wave"), ("M53", "mid", (260, 65), 1e-7, "wave"),
         ("M111", "divergent", (40, 9), 2e-10, "group"), ("M111", "divergent", (40, 9), 2e-10, "tile")]


@pytest.mark.parametrize("name,recipe,sizes,t_end,kernel", CASES)
def test_noalloc_equals_allocating_entry_point(mech_path, name, recipe, sizes, t_end, kernel):
    from paper_1608_05794_amd import ck
    g = ck.Mechanism(mech_path(name))
    for call, n in enumerate(sizes):
        y0, P0 = synth.reactor_states(g.n_species, n, recipe, seed=9100 + call)
        print(f"[noalloc {name}] call {call}: {n} reactors to {t_end:g} s ({kernel})", flush=True)
        y = torch.as_tensor(y0, device="cuda")
        P = torch.as_tensor(P0, device="cuda")
        ref = ck.integrate(g, y, P, t_end, kernel=kernel)
        yy = y.clone()
        got = ck.integrate_noalloc(g, yy, P, t_end, kernel=kernel)
        torch.cuda.synchronize()
        assert torch.equal(got["status"], ref["status"]) and bool((ref["status"] == 0).all().item())
        if kernel == "wave":
            assert torch.equal(got["y"], ref["y"])
            assert torch.equal(got["n_accept"], ref["n_accept"]) and torch.equal(got["n_reject"], ref["n_reject"])
        else:
            a, b = got["y"].cpu().numpy(), ref["y"].cpu().numpy()
            assert np.max(np.abs(a[0] - b[0]) / b[0]) <= 1e-6 and weighted_error(a, b) <= 1e-6


def test_noalloc_rejects_oversized_workspace(mech_path):
    """The one-reactor-per-lane kernel needs scratch linear in n: beyond the fixed array the call is
    refused with CK_ETOOBIG before anything runs."""
    from paper_1608_05794_amd import ck
    g = ck.Mechanism(mech_path("M53"))
    n = 4096
    assert g.workspace_bytes(n, kernel="lane") > 64 << 20
    y0, P0 = synth.reactor_states(g.n_species, n, "mid", seed=9200)
    y = torch.as_tensor(y0, device="cuda")
    P = torch.as_tensor(P0, device="cuda")
    with pytest.raises(ck.CkError, match="-7"):
        ck.integrate_noalloc(g, y, P, 1e-9, kernel="lane")
    assert torch.equal(y, torch.as_tensor(y0, device="cuda"))

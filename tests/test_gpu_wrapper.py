"""The binding on strided state views: a reactor-contiguous slice of a wider array (leading
dimension larger than the reactor count) gives the same results as a compact copy."""
import numpy as np
import pytest
import torch

from paper_1608_05794_amd import synth

pytestmark = pytest.mark.gpu


def test_sliced_state_views(mech_path):
    from paper_1608_05794_amd import ck
    g = ck.Mechanism(mech_path("M13"))
    y0, P0 = synth.reactor_states(g.n_species, 10, "small", seed=31)
    wide = torch.as_tensor(y0, device="cuda")                 # [N, 10]
    P = torch.as_tensor(P0, device="cuda")
    view = wide[:, 3:7]                                      # strides (10, 1): ld = 10, n = 4
    compact = view.contiguous()
    print("[wrapper] M13, view of 4 reactors with ld 10", flush=True)
    a = ck.integrate(g, view, P[3:7], 1e-7, method="ros4")   # copy of a strided view
    b = ck.integrate(g, compact, P[3:7], 1e-7, method="ros4")
    torch.cuda.synchronize()
    assert torch.equal(a["y"], b["y"]) and torch.equal(a["status"], b["status"])
    # in place on the view: only its columns change, and they equal the compact result
    before = wide.clone()
    c = ck.integrate(g, view, P[3:7], 1e-7, method="ros4", inplace=True)
    torch.cuda.synchronize()
    assert torch.equal(wide[:, 3:7], b["y"])
    assert torch.equal(wide[:, :3], before[:, :3]) and torch.equal(wide[:, 7:], before[:, 7:])
    assert torch.equal(c["status"], b["status"])
    # Jacobian and source term of the view
    wide.copy_(before)
    Ja = ck.jac(g, wide[:, 3:7], P[3:7])
    Jb = ck.jac(g, before[:, 3:7].contiguous(), P[3:7])
    fa = ck.rhs(g, wide[:, 3:7].contiguous(), P[3:7])
    fb = ck.rhs(g, before[:, 3:7].contiguous(), P[3:7])
    fc = ck.rhs(g, wide[:, 3:7], P[3:7])                     # a strided view without an output
    fd = torch.zeros_like(wide)
    ck.rhs(g, wide, P, out=fd)                               # an output with the state's strides
    torch.cuda.synchronize()
    assert Ja.shape == (g.N * g.N, 4) and torch.equal(Ja, Jb) and torch.equal(fa, fb)
    assert fc.shape == (g.N, 4) and torch.equal(fc, fb) and torch.equal(fd[:, 3:7], fb)
    assert np.all(a["status"].cpu().numpy() == 0)

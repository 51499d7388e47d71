"""Graph-driven step loop (ck_integrate_graph): bounded launches captured in a HIP graph and replayed
until every reactor is done give the same results as the same launches issued one by one from the
host, and as one unbounded call."""
import numpy as np
import pytest
import torch

from paper_1608_05794_amd import synth

pytestmark = pytest.mark.gpu

RECIPE = {"M13": "small", "M53": "mid", "M111": "divergent"}


def _host_loop(ck, g, y, p, t_end, method, launch_steps, launches, **opts):
    """The same bounded launches, one host-synchronised call each."""
    n = y.shape[1]
    yy = y.clone()
    t = torch.zeros(n, dtype=torch.float64, device="cuda")
    h = torch.zeros(n, dtype=torch.float64, device="cuda")
    na = torch.zeros(n, dtype=torch.int64, device="cuda")
    nr = torch.zeros(n, dtype=torch.int64, device="cuda")
    st = None
    for _ in range(launches):
        r = ck.integrate(g, yy, p, t_end, method=method, t=t, h=h, inplace=True, max_steps=launch_steps, **opts)
        na += r["n_accept"]
        nr += r["n_reject"]
        st = r["status"]
        torch.cuda.synchronize()
    return yy, st, na, nr, t, h


@pytest.mark.parametrize("name,method,n,t_end,ls,K", [("M53", "ros4", 200, 1e-7, 37, 3),
                                                      ("M13", "ros4", 300, 1e-6, 25, 4),
                                                      ("M13", "rkf45", 150, 1e-10, 40, 2)])
def test_graph_equals_host_loop_at_every_replay(mech_path, name, method, n, t_end, ls, K):
    from paper_1608_05794_amd import ck
    g = ck.Mechanism(mech_path(name))
    y0, P0 = synth.reactor_states(g.n_species, n, RECIPE[name], seed=4242)
    y = torch.as_tensor(y0, device="cuda")
    p = torch.as_tensor(P0, device="cuda")
    for reps in (1, 2, 3):
        print(f"[graph] {name} {method} {n} reactors, {ls} steps x {K} launches x {reps} replays", flush=True)
        gr = ck.integrate_graph(g, y, p, t_end, method=method, launch_steps=ls, launches_per_graph=K,
                                max_steps=reps * K * ls)
        hy, hst, hna, hnr, ht, hh = _host_loop(ck, g, y, p, t_end, method, ls, reps * K)
        # the graph stops replaying once every reactor is done; later host launches change nothing
        assert gr["replays"] <= reps
        assert torch.equal(gr["y"], hy) and torch.equal(gr["status"], hst)
        assert torch.equal(gr["n_accept"].to(torch.int64), hna) and torch.equal(gr["n_reject"].to(torch.int64), hnr)
        assert torch.equal(gr["t"], ht) and torch.equal(gr["h"], hh)
    # run to completion: equals one unbounded call
    gr = ck.integrate_graph(g, y, p, t_end, method=method, launch_steps=ls, launches_per_graph=K)
    one = ck.integrate(g, y, p, t_end, method=method)
    torch.cuda.synchronize()
    assert np.all(one["status"].cpu().numpy() == 0)
    assert torch.equal(gr["status"], one["status"]) and torch.equal(gr["y"], one["y"])
    assert torch.equal(gr["n_accept"], one["n_accept"]) and torch.equal(gr["n_reject"], one["n_reject"])
    steps = (one["n_accept"] + one["n_reject"]).max().item()
    assert gr["replays"] == -(-steps // (ls * K))
    print(f"[graph] {name} {method}: {gr['replays']} replays for at most {steps} attempted steps", flush=True)


def test_graph_group_kernel_within_tolerance(mech_path):
    """111 species (four-wavefront workgroup kernel, summation order varies): to tolerance."""
    from paper_1608_05794_amd import ck

    from .parity_util import weighted_error
    g = ck.Mechanism(mech_path("M111"))
    y0, P0 = synth.reactor_states(g.n_species, 64, "divergent", seed=4343)
    y = torch.as_tensor(y0, device="cuda")
    p = torch.as_tensor(P0, device="cuda")
    gr = ck.integrate_graph(g, y, p, 2e-10, launch_steps=60, launches_per_graph=4)
    one = ck.integrate(g, y, p, 2e-10)
    torch.cuda.synchronize()
    assert torch.equal(gr["status"], one["status"]) and np.all(one["status"].cpu().numpy() == 0)
    ya, yb = gr["y"].cpu().numpy(), one["y"].cpu().numpy()
    assert np.max(np.abs(ya[0] - yb[0]) / yb[0]) <= 1e-6 and weighted_error(ya, yb) <= 1e-6


def test_graph_freezes_failed_reactors(mech_path):
    """A reactor with a non-finite state ends NONFINITE and stays so across later launches, while the
    others finish."""
    from paper_1608_05794_amd import ck
    g = ck.Mechanism(mech_path("M13"))
    y0, P0 = synth.reactor_states(g.n_species, 64, "small", seed=4444)
    y0[3, 5] = np.nan
    y = torch.as_tensor(y0, device="cuda")
    p = torch.as_tensor(P0, device="cuda")
    gr = ck.integrate_graph(g, y, p, 1e-7, launch_steps=20, launches_per_graph=2)
    torch.cuda.synchronize()
    st = gr["status"].cpu().numpy()
    assert st[5] == 3 and np.all(np.delete(st, 5) == 0)
    assert gr["n_accept"][5].item() == 0 and gr["n_reject"][5].item() == 0

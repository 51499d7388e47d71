"""Parity at the full workload sizes (the two non-default 111-species forms at a quarter of it), in
the launch configuration the benchmark times: the whole batch
on the device through bounded launches of the persistent kernel that resume from (t, h), with the
library workspace passed explicitly; a seeded sample of reactors (plus the first and the last, the
ragged end of the work queue) integrated one by one by the oracle.  End times are shortened so the
batch finishes in well under a minute; every sampled reactor still takes hundreds to thousands of
attempted steps.  Bar: identical statuses, |dT|/T <= 1e-6 and weighted error <= 1e-6."""
import numpy as np
import pytest
import torch

from paper_1608_05794_amd import synth

from .parity_util import state_rel_error, weighted_error

pytestmark = pytest.mark.gpu

CASES = [
    # mechanism, species, state recipe, seed, reactors, t_end, kernel, precision, attempted steps per launch
    ("M53", 53, "mid", 1002, 131072, 1e-9, "wave", "fp64", 500),
    ("M53", 53, "mid", 1002, 131072, 1e-10, "wave", "fp32_refine", 500),
    # the tile form is the default for N > 64 and runs the full 111-species batch; the half-row form
    # and the refined tile form run a quarter of it (65536 reactors: still 256 per compute unit
    # through the persistent queue, with its ragged end)
    ("M111", 111, "divergent", 1003, 65536, 1e-12, "group", "fp64", 200),
    ("M111", 111, "divergent", 1003, 262144, 1e-12, "tile", "fp64", 200),
    ("M111", 111, "divergent", 1003, 65536, 1e-12, "tile", "fp32_refine", 200),
]


def _launches(ck, g, y, P, t_end, kernel, precision, launch_steps, tag):
    n = y.shape[1]
    dev = y.device
    te = torch.full((n,), t_end, dtype=torch.float64, device=dev)
    t = torch.zeros(n, dtype=torch.float64, device=dev)
    h = torch.zeros(n, dtype=torch.float64, device=dev)
    ws = torch.empty(g.workspace_bytes(n, kernel=kernel, precision=precision), dtype=torch.uint8, device=dev)
    steps = torch.zeros(n, dtype=torch.int64, device=dev)
    for launch in range(1, 100):
        r = ck.integrate(g, y, P, te, t=t, h=h, workspace=ws, inplace=True, kernel=kernel, precision=precision,
                         max_steps=launch_steps)
        steps += r["n_accept"] + r["n_reject"]
        left = int((r["status"] == 1).sum().item())
        print(f"[{tag}] launch {launch}: {left} reactors unfinished", flush=True)
        if left == 0:
            break
    return r["status"], t, steps


@pytest.mark.parametrize("mech,ns,recipe,seed,n,t_end,kernel,precision,launch_steps", CASES,
                         ids=[f"{c[0]}-{c[4]}-{c[6]}-{c[7]}" for c in CASES])
def test_full_batch_sampled_parity(oracle_mech, mech, ns, recipe, seed, n, t_end, kernel, precision, launch_steps):
    from paper_1608_05794_amd import ck
    tag = f"{mech} x {n} {kernel} {precision} to {t_end:g} s"
    g = ck.Mechanism(synth.mechanism_file(mech))
    y0, P0 = synth.reactor_states(ns, n, recipe, seed=seed)
    y = torch.as_tensor(y0, device="cuda")
    P = torch.as_tensor(P0, device="cuda")
    status, t, steps = _launches(ck, g, y, P, t_end, kernel, precision, launch_steps, tag)
    torch.cuda.synchronize()
    assert int((status == 0).sum().item()) == n
    assert torch.all(t == t_end)
    idx = np.concatenate([[0, n - 1], np.random.default_rng(seed + 7).choice(np.arange(1, n - 1), 30, replace=False)])
    om = oracle_mech(mech)
    orc = om.integrate(np.ascontiguousarray(y0[:, idx]), np.ascontiguousarray(P0[idx]), t_end, "ros4")
    yg = y.cpu().numpy()[:, idx]
    assert np.all(orc["status"] == 0)
    eT, eY = state_rel_error(yg, orc["y"])
    ew = weighted_error(yg, orc["y"])
    sg = steps.cpu().numpy()[idx]
    so = orc["n_accept"] + orc["n_reject"]
    print(f"[{tag}] sample of {len(idx)}: weighted {ew:.2e} rel T {eT:.2e} rel Y(>1e-12) {eY:.2e}; mean steps "
          f"{sg.mean():.0f} (oracle {so.mean():.0f}), batch mean {steps.double().mean().item():.0f}", flush=True)
    assert eT <= 1e-6 and ew <= 1e-6

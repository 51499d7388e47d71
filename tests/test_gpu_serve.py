"""Continuous batching: every request's result is the same served in a mix as integrated alone."""
import numpy as np
import pytest
import torch

from paper_1608_05794_amd import synth

pytestmark = pytest.mark.gpu


def test_alone_equals_mix(mech_path):
    """Every request served in a mix of mechanisms, sizes and end times equals its integration alone:
    bitwise for the single-wavefront kernels (13 and 53 species); for 111 species the four-wavefront
    workgroup kernel sums reaction contributions in a timing-dependent order, so the bar there is
    the integration tolerance (|dT|/T <= 1e-6 and the weighted difference <= 1e-6) with equal
    statuses."""
    from paper_1608_05794_amd import ck, serve

    from .parity_util import weighted_error
    mechs = {k: ck.Mechanism(mech_path(k)) for k in ("M13", "M53", "M111")}
    species = {k: m.n_species for k, m in mechs.items()}
    reqs = serve.poisson_requests(15, rate=200.0, seed=77, mech_weights=(("M13", 0.4), ("M53", 0.4), ("M111", 0.2)),
                                  n_range=(1, 300), t_range=(1e-9, 2e-8), species=species)
    for r in reqs:
        if r.mech == "M111":
            r.t_end *= 0.05          # 111 species: a few hundred to a few thousand steps
    assert any(r.mech == "M111" for r in reqs)
    srv = serve.Server(mechs, capacity={"M13": 2048, "M53": 2048, "M111": 1024}, hbm_budget=4e9, launch_steps=37)
    done = srv.run(reqs, time_limit=300)
    assert len(done) == len(reqs) and not srv.rejected
    assert srv.iterations > 1
    for r in done:
        g = mechs[r.mech]
        alone = ck.integrate(g, torch.as_tensor(r.y0, device="cuda"), torch.as_tensor(r.P, device="cuda"),
                             r.t_end, method="ros4")
        torch.cuda.synchronize()
        ya = alone["y"].cpu().numpy()
        assert np.array_equal(alone["status"].cpu().numpy(), r.result["status"])
        if r.mech == "M111":
            eT = np.max(np.abs(ya[0] - r.result["y"][0]) / ya[0])
            ew = weighted_error(r.result["y"], ya)
            print(f"[serve M111 request {r.rid}: {r.n} reactors] rel T {eT:.2e} weighted {ew:.2e}", flush=True)
            assert eT <= 1e-6 and ew <= 1e-6, r.rid
        else:
            assert np.array_equal(ya, r.result["y"]), r.rid
            assert np.array_equal((alone["n_accept"] + alone["n_reject"]).cpu().numpy(), r.result["steps"])
        assert r.completed >= r.admitted >= r.arrival - 1e-9
    s = serve.latency_summary(done, 200.0, max(r.completed for r in done))
    print(f"[serve] {s}", flush=True)
    assert s["p50_s"] <= s["p99_s"]


def test_admission_respects_budget(mech_path):
    from paper_1608_05794_amd import ck, serve
    mechs = {"M13": ck.Mechanism(mech_path("M13"))}
    reqs = serve.poisson_requests(6, rate=1e6, seed=78, mech_weights=(("M13", 1.0),), n_range=(200, 200),
                                  t_range=(1e-9, 1e-9), species={"M13": 13})
    reqs.append(serve.Request(99, "M13", reqs[0].y0.repeat(3, axis=1), reqs[0].P.repeat(3), 1e-9, reqs[-1].arrival))
    # a budget that sizes the pool at 448 slots: room for exactly two 200-reactor requests at a time
    fixed = mechs["M13"].workspace_bytes(1)
    budget = fixed + 480 * serve.Pool.slot_bytes(mechs["M13"].N)
    srv = serve.Server(mechs, hbm_budget=budget, launch_steps=10)
    assert srv.pools["M13"].cap == 448 and srv.allocated <= budget
    peak = []
    orig = serve.Pool.admit

    def spy(self, req):
        ok = orig(self, req)
        peak.append(len(self.active))
        return ok
    serve.Pool.admit = spy
    try:
        done = srv.run(reqs, time_limit=120)
    finally:
        serve.Pool.admit = orig
    # six requests served two at a time; the 600-reactor one can never fit and is rejected on arrival
    assert len(done) == 6 and max(peak) <= 2
    assert [r.rid for r in srv.rejected] == [99] and srv.backlog() == 0


def test_autotuner_returns_a_working_configuration(mech_path):
    from paper_1608_05794_amd import ck, tune
    g = ck.Mechanism(mech_path("M13"))
    y0, P = synth.reactor_states(g.n_species, 512, "small", seed=5)
    y, p = torch.as_tensor(y0, device="cuda"), torch.as_tensor(P, device="cuda")
    best, table = tune.tune(g, y, p, 1e-6, steps=5)
    assert table and all(v > 0 for _, v in table)
    assert best["kernel"] in ("wave", "group", "tile", "lane")
    # the chosen options integrate to the same result as the default launch (kernel choice aside)
    r = ck.integrate(g, y, p, 1e-7, **best)
    torch.cuda.synchronize()
    assert np.all(r["status"].cpu().numpy() == 0)
    assert np.array_equal(y.cpu().numpy(), y0)   # the tuner leaves the sample untouched

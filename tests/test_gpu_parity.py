"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars (the library's reading of the target tolerances):
  - source term: max_k |f_gpu - f_oracle| / D_k <= 1e-12, D_k the gross
    production + destruction scale of component k (near partial equilibrium
    the net rates cancel, so a plain relative error is meaningless there);
  - Jacobian: row-scaled contribution error <= 1e-10;
  - integration (rtol 1e-8, atol 1e-12): identical statuses, |dT|/T <= 1e-6,
    and |dy_i| <= 1e-6 (|y_i| + atol/rtol) for every component: the difference
    measured in the solver's own error weights.  The plain relative error of
    every Y > 1e-12 is printed too; for species within a few decades of atol it
    is set by rounding amplification (the oracle against itself with a one-ulp
    perturbation of y0 shows the same size, see test_oracle_sensitivity.py).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1608_05794_amd import synth

from .parity_util import jac_scaled_error, rhs_scale, state_rel_error, weighted_error

pytestmark = pytest.mark.gpu

RECIPE = {"M13": "small", "M53": "mid", "M111": "divergent", "M70": "divergent", "M35X": "mid", "M63": "mid",
          "M127": "divergent"}


@pytest.fixture(scope="module")
def ck():
    from paper_1608_05794_amd import ck as CK
    assert torch.cuda.is_available()
    return CK


@pytest.fixture(scope="module")
def gmech(ck, mech_path):
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = ck.Mechanism(mech_path(name))
        return cache[name]
    return get


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("kernel", ["wave", "lane"])
@pytest.mark.parametrize("name,n", [("M13", 200), ("M53", 131), ("M111", 70)])
def test_rhs_parity(ck, gmech, oracle_mech, name, n, kernel):
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=101)
    f = ck.rhs(g, dev(y), dev(P), kernel=kernel).cpu().numpy()
    fo = om.rhs(y, P)
    D = rhs_scale(om, y, P)
    err = np.abs(f - fo) / D
    print(f"[rhs {name} {kernel}] max scaled error {err.max():.3e}", flush=True)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("kernel", ["lane", "wave"])
@pytest.mark.parametrize("name,n", [("M13", 70), ("M53", 66), ("M70", 37), ("M111", 9)])
def test_jacobian_parity(ck, gmech, oracle_mech, name, n, kernel):
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=202)
    J = ck.jac(g, dev(y), dev(P), kernel=kernel).cpu().numpy()          # [N*N, n]
    J = J.T.reshape(n, om.N, om.N)
    Jo = om.jac(y, P)
    err = jac_scaled_error(J, Jo, y)
    print(f"[jac {name} {kernel}] max scaled error {err:.3e}", flush=True)
    assert err <= 1e-10


def _report_and_check(tag, res, orc):
    eT, eY = state_rel_error(res["y"], orc["y"])
    ew = weighted_error(res["y"], orc["y"])
    steps = res["n_accept"] + res["n_reject"]
    same = np.mean(steps == orc["n_accept"] + orc["n_reject"])
    print(f"[{tag}] weighted {ew:.2e}  rel T {eT:.2e}  rel Y(>1e-12) {eY:.2e}  identical step counts {same:.3f}  "
          f"mean steps {steps.mean():.0f}", flush=True)
    assert eT <= 1e-6 and ew <= 1e-6


def _integrate_both(ck, g, om, y, P, t_end, method, kernel, **kw):
    res = ck.integrate(g, dev(y), dev(P), t_end, method=method, kernel=kernel, **kw)
    torch.cuda.synchronize()
    orc = om.integrate(y, P, t_end, method, **{k: v for k, v in kw.items() if k in ("rtol", "atol", "max_steps",
                                                                                    "h0", "h_fixed", "jacobian", "reactor")})
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()}, orc


@pytest.mark.parametrize("kernel", ["wave", "lane"])
def test_ros4_parity_small(ck, gmech, oracle_mech, kernel):
    """Small configuration: M13, P = 1 atm, 1024 reactors, ROS4 to 1e-4 s at rtol 1e-8, atol 1e-12."""
    g, om = gmech("M13"), oracle_mech("M13")
    n = 1024 if kernel == "wave" else 128
    y, P = synth.reactor_states(om.n_species, n, "small", seed=1001)
    res, orc = _integrate_both(ck, g, om, y, P, 1e-4, "ros4", kernel)
    assert np.array_equal(res["status"], orc["status"])
    assert np.all(orc["status"] == 0)
    _report_and_check(f"ros4 M13 {kernel}", res, orc)


@pytest.mark.parametrize("kernel", ["wave", "lane"])
def test_ros4_parity_mid_sample(ck, gmech, oracle_mech, kernel):
    """M53 (mid configuration states), a ragged batch of 67 reactors over a shorter horizon."""
    g, om = gmech("M53"), oracle_mech("M53")
    y, P = synth.reactor_states(om.n_species, 67, "mid", seed=1002)
    # the lane kernel is latency-bound on one wavefront: give it a budget of attempted steps
    kw = {} if kernel == "wave" else {"max_steps": 400}
    res, orc = _integrate_both(ck, g, om, y, P, 2e-6, "ros4", kernel, **kw)
    assert np.array_equal(res["status"], orc["status"])
    _report_and_check(f"ros4 M53 {kernel}", res, orc)


@pytest.mark.parametrize("kernel", ["wave", "lane"])
def test_rkf45_parity(ck, gmech, oracle_mech, kernel):
    """RKF45 on the small mechanism over a stability-bound horizon (explicit steps ~ 1/rho(J))."""
    g, om = gmech("M13"), oracle_mech("M13")
    y, P = synth.reactor_states(om.n_species, 130, "small", seed=1003)
    res, orc = _integrate_both(ck, g, om, y, P, 2e-12, "rkf45", kernel)
    assert np.array_equal(res["status"], orc["status"])
    assert np.all(orc["status"] == 0)
    _report_and_check(f"rkf45 M13 {kernel}", res, orc)


def test_rkf45_parity_m111_two_slots(ck, gmech, oracle_mech):
    """N > 64: the wavefront RKF45 keeps two state components per lane."""
    g, om = gmech("M111"), oracle_mech("M111")
    y, P = synth.reactor_states(om.n_species, 20, "divergent", seed=1004)
    res, orc = _integrate_both(ck, g, om, y, P, 1e-13, "rkf45", "wave")
    assert np.array_equal(res["status"], orc["status"])
    _report_and_check(f"rkf45 M111 wave", res, orc)


def test_ros4_m111_lane(ck, gmech, oracle_mech):
    """N = 112 through the lane kernel."""
    g, om = gmech("M111"), oracle_mech("M111")
    y, P = synth.reactor_states(om.n_species, 5, "divergent", seed=1005)
    # a fixed budget of 12 attempted steps (the lane kernel is latency-bound at this batch size)
    res, orc = _integrate_both(ck, g, om, y, P, 1e-3, "ros4", "lane", max_steps=12)
    assert np.array_equal(res["status"], orc["status"]) and np.all(res["status"] == 1)
    _report_and_check(f"ros4 M111 lane", res, orc)


@pytest.mark.parametrize("name,n,te", [("M13", 300, 1e-4), ("M53", 67, 2e-6), ("M111", 24, 2e-7)])
def test_ros4_group_parity(ck, gmech, oracle_mech, name, n, te):
    """Workgroup kernel: one wavefront per reactor for N <= 64, four for N = 112 (rows over thread pairs)."""
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=1009)
    res, orc = _integrate_both(ck, g, om, y, P, te, "ros4", "group")
    assert np.array_equal(res["status"], orc["status"])
    _report_and_check(f"ros4 group {name}", res, orc)


@pytest.mark.parametrize("name,n,te", [("M111", 24, 2e-7), ("M70", 70, 1e-7)])
def test_ros4_tile_parity(ck, gmech, oracle_mech, name, n, te):
    """Tile form (N > 64): iteration matrix in 16x16 matrix-core tiles, blocked Gauss-Jordan inverse
    with FP64 MFMA rank-16 updates.  M70 (N = 71) pads to five tile rows (nine padding rows and
    columns, uneven tile-row ownership across the four wavefronts)."""
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=1013)
    print(f"[ros4 tile {name}] {n} reactors to {te:g} s", flush=True)
    res, orc = _integrate_both(ck, g, om, y, P, te, "ros4", "tile", max_steps=60000)
    assert np.array_equal(res["status"], orc["status"]) and np.all(orc["status"] == 0)
    _report_and_check(f"ros4 tile {name}", res, orc)


def test_ros4_tile_resume_and_fixed_step(ck, gmech, oracle_mech):
    """Tile form: fixed-step mode against the oracle (no controller, so every step is compared), and a
    run split into bounded launches resuming from (t, h) against one call, to tolerance (its reaction
    sums are ordered by LDS atomics across four wavefronts)."""
    g, om = gmech("M111"), oracle_mech("M111")
    y, P = synth.reactor_states(om.n_species, 33, "divergent", seed=1014)
    res, orc = _integrate_both(ck, g, om, y, P, 4e-14, "ros4", "tile", h_fixed=1e-15)
    assert np.all(np.isfinite(orc["y"]))
    assert np.all(res["status"] == 0) and np.all(orc["status"] == 0)
    assert np.array_equal(res["n_accept"], orc["n_accept"])
    _report_and_check("ros4 tile M111 fixed step", res, orc)
    whole = ck.integrate(g, dev(y), dev(P), 1e-10, kernel="tile", max_steps=60000)
    yy, t, h = dev(y), torch.zeros(33, dtype=torch.float64, device="cuda"), torch.zeros(33, dtype=torch.float64,
                                                                                        device="cuda")
    for _ in range(200):
        r = ck.integrate(g, yy, dev(P), 1e-10, kernel="tile", t=t, h=h, inplace=True, max_steps=97)
        if not bool((r["status"] == 1).any().item()):
            break
    torch.cuda.synchronize()
    assert torch.equal(r["status"], whole["status"]) and np.all(whole["status"].cpu().numpy() == 0)
    a, b = yy.cpu().numpy(), whole["y"].cpu().numpy()
    assert np.max(np.abs(a[0] - b[0]) / b[0]) <= 1e-6 and weighted_error(a, b) <= 1e-6


def test_ros4_second_window_recomputes_rates(ck, gmech, oracle_mech):
    """35 species, 900 reactions (duplicates included): the per-reaction scalars of the first Jacobian
    window (3 rows per 64 reactions, 45 rows) exceed the 40-row parking slice of N' = 40, so the
    wavefront kernel's second window evaluates the rate constants again instead of reading them."""
    g, om = gmech("M35X"), oracle_mech("M35X")
    assert 3 * ((om.n_reactions + 63) // 64) > (om.N + 7) // 8 * 8
    y, P = synth.reactor_states(om.n_species, 24, "mid", seed=1012)
    f = ck.rhs(g, dev(y), dev(P), kernel="wave").cpu().numpy()
    assert (np.abs(f - om.rhs(y, P)) / rhs_scale(om, y, P)).max() <= 1e-12
    res, orc = _integrate_both(ck, g, om, y, P, 1e-8, "ros4", "wave")
    assert np.array_equal(res["status"], orc["status"]) and np.all(orc["status"] == 0)
    _report_and_check("ros4 M35X wave (second window recomputes)", res, orc)


@pytest.mark.parametrize("method,kernel", [("ros4", "wave"), ("ros4", "lane"), ("ros4", "group"),
                                           ("rkf45", "wave"), ("rkf45", "lane")])
def test_edge_cases(ck, gmech, oracle_mech, method, kernel):
    g, om = gmech("M13"), oracle_mech("M13")
    y, P = synth.reactor_states(om.n_species, 65, "small", seed=1006)
    te = 1e-9 if method == "ros4" else 1e-13
    # n = 0 is a no-op
    empty = ck.integrate(g, dev(y[:, :0]), dev(P[:0]), te, method=method, kernel=kernel)
    assert empty["status"].numel() == 0
    # non-finite state -> NONFINITE, others unaffected; max_steps -> MAX_STEPS; tiny h0 -> H_UNDERFLOW
    bad = y.copy()
    bad[2, 3] = np.nan
    res, orc = _integrate_both(ck, g, om, bad, P, te, method, kernel)
    assert res["status"][3] == 3 and np.array_equal(res["status"], orc["status"])
    res, orc = _integrate_both(ck, g, om, y, P, 1e-5, method, kernel, max_steps=7)
    assert np.all(res["status"] == 1) and np.all(res["n_accept"] + res["n_reject"] == 7)
    res, orc = _integrate_both(ck, g, om, y, P, 1e-5, method, kernel, h0=1e-32)
    assert np.all(res["status"] == 2) and np.array_equal(res["status"], orc["status"])
    # fixed-step mode: exactly the requested number of steps, same values as the oracle
    res, orc = _integrate_both(ck, g, om, y, P, 1.6e-14, method, kernel, h_fixed=1e-15)
    assert np.all(res["n_accept"] == orc["n_accept"])
    assert weighted_error(res["y"], orc["y"]) <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_tile_edge_cases(ck, gmech, oracle_mech, precision):
    """Tile form (N = 112): an empty batch, a single reactor (one workgroup for one reactor, most of
    the grid idle), a non-finite state among finite ones, the attempted-step cap and a step below the
    h floor, each with the oracle's statuses."""
    g, om = gmech("M111"), oracle_mech("M111")
    y, P = synth.reactor_states(om.n_species, 5, "divergent", seed=1016)
    te = 2e-12
    kw = dict(precision=precision)
    print(f"[tile edge cases {precision}]", flush=True)
    empty = ck.integrate(g, dev(y[:, :0]), dev(P[:0]), te, kernel="tile", **kw)
    assert empty["status"].numel() == 0
    res, orc = _integrate_both(ck, g, om, y[:, :1], P[:1], te, "ros4", "tile", **kw)
    assert np.array_equal(res["status"], orc["status"]) and res["status"][0] == 0
    _report_and_check(f"tile one reactor {precision}", res, orc)
    bad = y.copy()
    bad[5, 2] = np.inf
    res, orc = _integrate_both(ck, g, om, bad, P, te, "ros4", "tile", **kw)
    assert res["status"][2] == 3 and np.array_equal(res["status"], orc["status"])
    res, orc = _integrate_both(ck, g, om, y, P, 1e-6, "ros4", "tile", max_steps=9, **kw)
    assert np.all(res["status"] == 1) and np.all(res["n_accept"] + res["n_reject"] == 9)
    res, orc = _integrate_both(ck, g, om, y, P, 1e-6, "ros4", "tile", h0=1e-32, **kw)
    assert np.all(res["status"] == 2) and np.array_equal(res["status"], orc["status"])


@pytest.mark.parametrize("kernel", ["wave", "lane", "group"])
def test_resume_and_batch_independence(ck, gmech, kernel):
    """(t, h, y) resume is bitwise; a reactor's result does not depend on its batch (Section 4: scalar and
    SIMD results agree)."""
    g = gmech("M13")
    y, P = synth.reactor_states(g.n_species, 96, "small", seed=1007)
    te = 5e-8
    full = ck.integrate(g, dev(y), dev(P), te, kernel=kernel)
    t = torch.zeros(96, dtype=torch.float64, device="cuda")
    h = torch.zeros(96, dtype=torch.float64, device="cuda")
    part = ck.integrate(g, dev(y), dev(P), te, t=t, h=h, kernel=kernel, max_steps=30)
    rest = ck.integrate(g, part["y"], dev(P), te, t=t, h=h, kernel=kernel)
    assert torch.equal(rest["y"], full["y"])
    assert torch.equal(rest["n_accept"] + part["n_accept"], full["n_accept"])
    idx = [5, 64, 95]
    alone = ck.integrate(g, dev(y[:, idx]), dev(P[idx]), te, kernel=kernel)
    assert torch.equal(alone["y"], full["y"][:, idx])


@pytest.mark.parametrize("name,kernel", [("M53", "wave"), ("M111", "group")])
def test_concurrent_streams_without_workspace(ck, gmech, name, kernel):
    """Two batches integrated at once on two streams, both with the library-owned workspace, give
    what each gives alone: the persistent kernels' queue counters and parking areas are per stream.
    One workgroup per CU each, so the two grids are resident together; t is not passed, so a reactor
    taken twice from a shared queue would be integrated twice (on M111 that moves each reactor's
    weighted error by 4 to 16).  The single-wavefront kernels are compared bit for bit; the
    four-wavefront GROUP form adds reaction contributions from its wavefronts with LDS atomics in a
    timing-dependent order, so it is compared to rounding: over the 1200-9800 stiff steps of this
    workload rounding alone moves the weighted error to ~1e-6 (the oracle against itself with y0
    perturbed by one ulp reaches 4.5e-7 on 70 of these reactors), so the bar is 1e-5, five decades
    under what a shared queue or parking area produces."""
    g = gmech(name)
    ya, Pa = synth.reactor_states(g.n_species, 700, RECIPE[name], seed=1010)
    yb, Pb = synth.reactor_states(g.n_species, 450, RECIPE[name], seed=1011)
    te = 2e-8
    alone_a = ck.integrate(g, dev(ya), dev(Pa), te, kernel=kernel, blocks_per_cu=1)
    alone_b = ck.integrate(g, dev(yb), dev(Pb), te, kernel=kernel, blocks_per_cu=1)
    da, pa, db, pb = dev(ya), dev(Pa), dev(yb), dev(Pb)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(2):
        with torch.cuda.stream(sa):
            ra = ck.integrate(g, da, pa, te, kernel=kernel, blocks_per_cu=1, stream=sa)
        with torch.cuda.stream(sb):
            rb = ck.integrate(g, db, pb, te, kernel=kernel, blocks_per_cu=1, stream=sb)
        torch.cuda.synchronize()
        for r, alone in ((ra, alone_a), (rb, alone_b)):
            assert torch.equal(r["status"], alone["status"])
            if g.N <= 64:
                assert torch.equal(r["n_accept"], alone["n_accept"])
                assert torch.equal(r["y"], alone["y"])
            else:
                yr, ya_ = r["y"].cpu().numpy(), alone["y"].cpu().numpy()
                eT, _ = state_rel_error(yr, ya_)
                ew = weighted_error(yr, ya_)
                print(f"[streams {name} {kernel}] weighted {ew:.2e} rel T {eT:.2e}", flush=True)
                assert eT <= 1e-6 and ew <= 1e-5


@pytest.mark.parametrize("name,n,te,kernel", [("M13", 512, 1e-4, "wave"), ("M53", 67, 2e-6, "wave"),
                                              ("M70", 40, 1e-7, "tile"), ("M111", 24, 2e-7, "tile")])
def test_ros4_fp32_refined(ck, gmech, oracle_mech, name, n, te, kernel):
    """FP32 factorisation with FP64 residual refinement (<= 3 sweeps; FP32 LU in the wavefront kernel,
    FP32 matrix-core Gauss-Jordan in the tile kernel for N > 64); RHS, Jacobian, error norm and control
    stay FP64.  Compared against the all-FP64 oracle; step counts and FP64 refactorings reported."""
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=1008)
    fb = torch.zeros(n, dtype=torch.int32, device="cuda")
    print(f"[ros4 fp32+refine {name}] {n} reactors to {te:g} s ({kernel})", flush=True)
    res, orc = _integrate_both(ck, g, om, y, P, te, "ros4", kernel, precision="fp32_refine", refine_sweeps=3,
                               n_fallback=fb, max_steps=60000)
    assert np.array_equal(res["status"], orc["status"]) and np.all(orc["status"] == 0)
    dacc = (res["n_accept"] - orc["n_accept"]).mean()
    drej = (res["n_reject"] - orc["n_reject"]).mean()
    nfb = int(fb.sum().item())
    steps = int((res["n_accept"] + res["n_reject"]).sum())
    print(f"[ros4 fp32+refine {name}] mean extra accepted {dacc:.2f}, mean extra rejected {drej:.2f}, "
          f"FP64 refactorings {nfb} of {steps} steps", flush=True)
    _report_and_check(f"ros4 fp32+refine {name}", res, orc)


@pytest.mark.parametrize("name,n,te,kernel", [("M53", 40, 2e-7, "wave"), ("M111", 12, 2e-8, "tile")])
def test_ros4_fp32_fallback_path(ck, gmech, oracle_mech, name, n, te, kernel):
    """The FP64 refactoring path of the refined mode, forced from the host: with one refinement sweep a
    solve rarely reaches the 2^-48 stopping test, so most steps are redone in FP64 and counted; the
    result still meets the FP64 parity bar."""
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=1015)
    fb = torch.zeros(n, dtype=torch.int32, device="cuda")
    print(f"[ros4 fp32 fallback {name}] {n} reactors to {te:g} s ({kernel})", flush=True)
    res, orc = _integrate_both(ck, g, om, y, P, te, "ros4", kernel, precision="fp32_refine", refine_sweeps=1,
                               n_fallback=fb, max_steps=60000)
    assert np.array_equal(res["status"], orc["status"]) and np.all(orc["status"] == 0)
    steps = res["n_accept"] + res["n_reject"]
    nfb = fb.cpu().numpy()
    print(f"[ros4 fp32 fallback {name}] FP64 refactorings {nfb.sum()} of {steps.sum()} steps", flush=True)
    assert nfb.sum() > 0 and np.all(nfb <= steps)
    _report_and_check(f"ros4 fp32 fallback {name}", res, orc)


@pytest.mark.parametrize("name,n,te", [("M13", 256, 1e-5), ("M53", 40, 5e-7)])
def test_ros4_fd_jacobian_parity(ck, gmech, oracle_mech, name, n, te):
    """ROS4 with the forward-difference Jacobian (one source-term evaluation per column, CVODE
    increments) against the oracle's forward-difference ROS4."""
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=1010)
    res, orc = _integrate_both(ck, g, om, y, P, te, "ros4", "wave", jacobian="fd")
    assert np.array_equal(res["status"], orc["status"])
    _report_and_check(f"ros4 fd-jacobian {name}", res, orc)


def test_fd_jacobian_option_rejected_where_unsupported(ck, gmech):
    g = gmech("M111")
    y, P = synth.reactor_states(g.n_species, 2, "divergent", seed=3)
    with pytest.raises(ck.CkError):
        ck.integrate(g, dev(y), dev(P), 1e-9, kernel="auto", jacobian="fd")
    g13 = gmech("M13")
    y, P = synth.reactor_states(g13.n_species, 2, "small", seed=3)
    with pytest.raises(ck.CkError):
        ck.integrate(g13, dev(y), dev(P), 1e-9, kernel="lane", jacobian="fd")
    with pytest.raises(ck.CkError):
        ck.integrate(g13, dev(y), dev(P), 1e-9, kernel="wave", jacobian="fd", precision="fp32_refine")


# ---- constant-volume form (Section 3): fixed density, c_v and internal energies ----------------

def _density(om, y, P):
    S = (y[1:] / np.asarray(om.W)[:, None]).sum(axis=0)
    return P / (synth.R_GAS * y[0] * S)


@pytest.mark.parametrize("name,n", [("M13", 200), ("M53", 131), ("M111", 70)])
def test_rhs_cv_parity(ck, gmech, oracle_mech, name, n):
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=111)
    rho = _density(om, y, P)
    f = ck.rhs(g, dev(y), dev(rho), reactor="cv").cpu().numpy()
    fo = om.rhs(y, rho, reactor="cv")
    # the pressure of the same state gives the same concentrations, hence the same gross rates;
    # the temperature row is scaled by sum_k |U_k| G_k / (rho c_v) instead
    D = rhs_scale(om, y, P)
    W = np.asarray(om.W)
    nu = np.abs(om.stoich()).astype(float)
    for r in range(n):
        qf, qr, _, _, hRT = om.rates(y[:, r], P[r])
        G = nu @ (np.abs(qf) + np.abs(qr))
        cp, _, _ = om.thermo(y[0, r])
        cv = (y[1:, r] * synth.R_GAS * (cp - 1.0) / W).sum()
        U = synth.R_GAS * y[0, r] * (hRT - 1.0)
        D[0, r] = np.sum(np.abs(U) * G) / (rho[r] * cv)
    err = np.abs(f - fo) / D
    print(f"[rhs cv {name}] max scaled error {err.max():.3e}", flush=True)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("name,n", [("M13", 70), ("M53", 66)])
def test_jacobian_cv_parity(ck, gmech, oracle_mech, name, n):
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=212)
    rho = _density(om, y, P)
    J = ck.jac(g, dev(y), dev(rho), reactor="cv").cpu().numpy().T.reshape(n, om.N, om.N)
    Jo = om.jac(y, rho, reactor="cv")
    err = jac_scaled_error(J, Jo, y)
    print(f"[jac cv {name}] max scaled error {err:.3e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("name,n,te", [("M13", 256, 1e-5), ("M53", 40, 1e-6)])
def test_ros4_cv_parity(ck, gmech, oracle_mech, name, n, te):
    g, om = gmech(name), oracle_mech(name)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=1011)
    rho = _density(om, y, P)
    res, orc = _integrate_both(ck, g, om, y, rho, te, "ros4", "wave", reactor="cv")
    assert np.array_equal(res["status"], orc["status"])
    _report_and_check(f"ros4 cv {name}", res, orc)


def test_rkf45_cv_parity(ck, gmech, oracle_mech):
    g, om = gmech("M13"), oracle_mech("M13")
    y, P = synth.reactor_states(om.n_species, 128, "small", seed=1012)
    rho = _density(om, y, P)
    res, orc = _integrate_both(ck, g, om, y, rho, 2e-12, "rkf45", "wave", reactor="cv")
    assert np.array_equal(res["status"], orc["status"])
    _report_and_check("rkf45 cv M13", res, orc)


def test_cv_rejected_where_unsupported(ck, gmech):
    g = gmech("M13")
    y, P = synth.reactor_states(g.n_species, 2, "small", seed=3)
    with pytest.raises(ck.CkError):
        ck.integrate(g, dev(y), dev(P), 1e-9, kernel="lane", reactor="cv")
    with pytest.raises(ck.CkError):
        ck.rhs(g, dev(y), dev(P), kernel="lane", reactor="cv")
    g111 = gmech("M111")
    y, P = synth.reactor_states(g111.n_species, 2, "divergent", seed=3)
    with pytest.raises(ck.CkError):
        ck.integrate(g111, dev(y), dev(P), 1e-9, reactor="cv")


@pytest.mark.parametrize("name,kernel,n,te", [("M63", "wave", 24, 1e-7), ("M127", "tile", 12, 1e-9),
                                             ("M127", "group", 12, 1e-9)])
def test_largest_sizes(ck, gmech, oracle_mech, name, kernel, n, te):
    """The largest state of each kernel family: N = 64 fills every lane of the wavefront kernel with
    a matrix row (no padding column), N = 128 gives the workgroup kernels eight tile rows (two per
    wavefront) and a 128-row Gauss-Jordan.  Source term, analytic Jacobian and ROS4 against the
    oracle, in FP64 and (wavefront and tile forms) with the FP32 factorisation refined in FP64;
    RKF45 (one reactor per wavefront at both sizes) over a short horizon."""
    g, om = gmech(name), oracle_mech(name)
    assert om.N in (64, 128)
    y, P = synth.reactor_states(om.n_species, n, RECIPE[name], seed=303)
    print(f"[largest {name} N={om.N}] {kernel}: {n} reactors to {te:g} s", flush=True)
    f = ck.rhs(g, dev(y), dev(P), kernel="wave").cpu().numpy()
    err = np.abs(f - om.rhs(y, P)) / rhs_scale(om, y, P)
    J = ck.jac(g, dev(y), dev(P), kernel="wave").cpu().numpy().T.reshape(n, om.N, om.N)
    ej = jac_scaled_error(J, om.jac(y, P), y)
    print(f"  rhs scaled error {err.max():.3e}, jacobian scaled error {ej:.3e}", flush=True)
    assert err.max() <= 1e-12 and ej <= 1e-10
    for prec in (("fp64",) if kernel == "group" else ("fp64", "fp32_refine")):
        res, orc = _integrate_both(ck, g, om, y, P, te, "ros4", kernel, precision=prec)
        assert np.all(res["status"] == 0) and np.all(orc["status"] == 0)
        _report_and_check(f"largest {name} {kernel} {prec}", res, orc)
    if kernel != "group":
        # the explicit pair on the same states, over a horizon its stability bound allows
        res, orc = _integrate_both(ck, g, om, y, P, 1e-12 if om.N == 64 else 1e-14, "rkf45", "wave")
        assert np.all(res["status"] == 0) and np.all(orc["status"] == 0)
        _report_and_check(f"largest {name} rkf45", res, orc)

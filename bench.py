"""Throughput benchmark of the batched reactor integration on one MI355X.

Workload (mid configuration): synthetic 53-species / 325-reaction mechanism
(30 third-body, 25 Troe), 131072 constant-pressure reactors with
T0 ~ U(900, 1800) K, P ~ U(1, 20) atm, Y0 ~ Dirichlet(0.5), integrated with
ROS4 to t = 1e-3 s at rtol 1e-8, atol 1e-12, FP64.  One "step" integrates the
whole batch from its initial state (about two minutes on one MI355X); inputs
are resident in HBM before the timed region.  --steps and --warmup are upper
limits: the run keeps to a wall-clock budget (--budget-s, counted from process
start), times at least one step and as many more as fit, and reports the
numbers it actually ran.  A warm-up pass is one bounded launch (a few attempted
steps per reactor over the whole batch).  Also reported: source-term (RHS)
evaluations per second over distinct state batches, the roofline of the
dominant kernel, and the CPU oracle on a bounded sample of the same workload.

Prints one JSON line (rank 0).  Only one GPU is used; --gpus > 1 exits.
"""
import argparse
import json
import os
import sys
import time

T_PROCESS_START = time.time()   # the wall budget of the headline leg counts from here

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reactors/s integrated (ROS4, rtol 1e-8), RHS evals/s, p50/p99 solve latency"
KERNEL_NAMES = {"wave": "integrate_wave_kernel<Ros4Adapter>", "auto": "integrate_wave_kernel<Ros4Adapter>",
                "group": "coop_kernel<4, Ros4CoopHalf>", "tile": "coop_kernel<4, Ros4CoopTile>",
                "lane": "integrate_lane_kernel<0>"}
PEAK_FP64_VECTOR = 78.6e12         # FLOP/s, MI355X FP64 vector (VALU)
# HBM traffic of the integrator kernel from two rocprofv3 --pmc runs of the default command (one
# with FETCH_SIZE, one with WRITE_SIZE; KiB per dispatch averaged over its launches), each scaled
# by what the counter reads for a device-to-device copy of 1 GiB (FETCH_SIZE reads half the bytes,
# WRITE_SIZE all of them).  Valid only for the default workload and for kernel sources whose hash
# matches; otherwise the traffic is reported as null.
TRAFFIC_REF = {
    "sources": ["paper_1608_05794_amd/csrc/k_wave.hip", "paper_1608_05794_amd/csrc/kinetics.h",
                "paper_1608_05794_amd/csrc/ck_internal.h", "paper_1608_05794_amd/csrc/launch.h",
                "paper_1608_05794_amd/csrc/mech.hip"],
    "sha256": "45bf3512875cebbad468a548f6952454bb4ab27ef01445e2dea2656d3ee155d1",
    "args": {"mech": "M53", "reactors": 131072, "t_end": 1e-3, "kernel": "wave", "precision": "fp64",
             "launch_steps": 2000},
    "fetch_kib_per_launch": 7323296.37, "fetch_factor": 1048576.0 / 524302.31,
    "write_kib_per_launch": 832079207.05, "write_factor": 1.0,
}
TRANSCENDENTAL_FLOPS = 20           # FP64 operations charged per exp / log / log10 / exp10


def algorithmic_flops(info):
    """Algorithmic FP64 operations per RHS, per Jacobian and per ROS4 / RKF45 step.

    info: dict with n_species, slot counts and reaction classes (see mech_structure).
    Counting: FMA = 2, other arithmetic = 1, each exp/log/log10/exp10 = TRANSCENDENTAL_FLOPS.
    """
    ns = info["n_species"]
    N = ns + 1
    T = TRANSCENDENTAL_FLOPS
    rhs = 2 * T + 3 * ns                      # ln T, 1/T, powers; mixture sums
    rhs += ns * (2 * 4 + 2 * 5 + 2 * 5 + 6)   # cp, H, S polynomials, C_k, g_k, cp sum
    rhs += ns * 6                              # Ydot, Tdot terms
    jac_extra = 0
    for slots, kind, neff in info["reactions"]:
        r = 2 * 2 + T                          # ln kf, kf
        r += 2 * slots + 4 + T                 # ln Kc, kr
        r += 2 * slots                         # mass-action products
        r += 3 + 2 * slots                     # q, scatter
        jr = 2 * slots * slots + 4 * slots + 8 # d prod / dC per slot pair, dT terms
        if kind >= 1:
            r += 2 * neff + 1                  # [M]
            jr += 2 * neff + 4
        if kind >= 2:
            r += 8 + T                         # k0 / kinf, Pr, c
            jr += 12
        if kind == 3:
            r += 30 + 5 * T                    # Fcent (3 exp), 2 log10, exp10
            jr += 30
        rhs += r
        jac_extra += jr
    jac = rhs + jac_extra + 6 * ns * ns + 20 * ns      # chain rule: row transform, column sums
    lu = (2 * N ** 3) // 3
    solve = 2 * N * N
    ros4 = jac + 2 * rhs + N * N + lu + 4 * solve + 24 * N
    rkf45 = 6 * rhs + 40 * N
    return dict(rhs=rhs, jac=jac, lu=lu, ros4_step=ros4, rkf45_step=rkf45, h0=2 * rhs)


def mech_structure(path):
    """Reaction classes and slot counts read from the mechanism file."""
    reactions = []
    ns = 0
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if not f:
                continue
            if f[0] == "SPECIES":
                ns = int(f[1])
            elif f[0] == "R":
                kind, nr = int(f[1]), int(f[3])
                npr = int(f[4 + 2 * nr])
                rest = f[5 + 2 * nr + 2 * npr:]
                skip = 3 + (3 if kind >= 2 else 0) + (4 if kind == 3 else 0)
                neff = int(rest[skip]) if kind >= 1 else 0
                reactions.append((nr + npr, kind, neff))
    return dict(n_species=ns, reactions=reactions)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--mech", default="M53")
    ap.add_argument("--reactors", type=int, default=131072)
    ap.add_argument("--t-end", type=float, default=1e-3)
    ap.add_argument("--kernel", default="wave", choices=["wave", "lane", "group", "tile", "auto"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refine"])
    ap.add_argument("--launch-steps", type=int, default=2000,
                    help="attempted steps per reactor per kernel launch; launches resume from (t, h)")
    ap.add_argument("--max-steps", type=int, default=1_000_000, help="attempted steps per reactor in total")
    ap.add_argument("--rhs-evals", type=int, default=100, help="RHS evaluations per reactor in the RHS leg")
    ap.add_argument("--rhs-batches", type=int, default=8, help="distinct state batches cycled in the RHS leg")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: 8 per host thread)")
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget of the headline run, from process start: timed steps stop once "
                         "another would not fit before the RHS and CPU legs (at least one step is timed)")
    ap.add_argument("--warmup-launch-steps", type=int, default=16,
                    help="attempted steps per reactor of one warm-up pass (a single bounded launch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--suite", default="integrate", choices=["integrate", "batching", "precision", "serving", "methods", "peaks"],
                    help="integrate: the headline line; batching / precision / serving: the three production "
                         "forms; methods: small configuration with both integrators, transfers, analytic vs "
                         "forward-difference Jacobian; peaks: achievable GEMM, FMA and copy rates (one "
                         "JSON line each, bounded workloads)")
    ap.add_argument("--batching-reactors", type=int, default=32768, help="batching suite: reactors (first of the batch)")
    ap.add_argument("--batching-t-end", type=float, default=1e-13, help="batching suite: common end time (s)")
    ap.add_argument("--serve-requests", type=int, default=32, help="serving suite: arrivals served")
    ap.add_argument("--serve-t-scale", type=float, default=1e-3, help="serving suite: factor on drawn end times")
    ap.add_argument("--serve-time-limit", type=float, default=150.0, help="serving suite: wall time limit (s)")
    ap.add_argument("--serve-launch-steps", type=int, default=400, help="serving suite: attempted steps per launch")
    ap.add_argument("--serve-precision", default="fp64", choices=["fp64", "fp32_refine"],
                    help="serving suite: linear-solve precision of the pools that support it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device three times (counter calibration) and exit")
    return ap.parse_args()


def measured_traffic(a):
    """HBM bytes per launch of the integrator kernel (see TRAFFIC_REF), or None."""
    import hashlib
    ref = TRAFFIC_REF
    if any(getattr(a, k) != v for k, v in ref["args"].items()):
        return None
    digests = []
    for f in ref["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            digests.append(hashlib.sha256(fh.read()).hexdigest())
    if hashlib.sha256("".join(digests).encode()).hexdigest() != ref["sha256"]:
        return None
    return (ref["fetch_kib_per_launch"] * 1024 * ref["fetch_factor"] +
            ref["write_kib_per_launch"] * 1024 * ref["write_factor"])


def host_threads():
    """Host threads for the oracle: the CPUs this process may run on, capped by OMP_NUM_THREADS when it
    is set (a GPU host may expose more cores than its share)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def cpu_baseline(path, y, P, t_end, sample):
    """The CPU oracle (one reactor per OpenMP task, dynamic schedule) on a bounded sample."""
    from oracle import oracle as O
    cores = host_threads()
    sample = sample or 8 * cores
    sample = min(sample, y.shape[1])
    m = O.Mechanism(path)
    ys, Ps = np.ascontiguousarray(y[:, :sample]), np.ascontiguousarray(P[:sample])
    t0 = time.perf_counter()
    res = m.integrate(ys, Ps, t_end, "ros4", nthreads=cores)
    dt = time.perf_counter() - t0
    return dict(value=sample / dt, unit="reactors/s", cores=cores, kind="oracle",
                sample=f"first {sample} reactors of the workload, ROS4 to {t_end:g} s, {dt:.1f} s wall",
                mean_steps=float(np.mean(res["n_accept"] + res["n_reject"])))


def _states(synth, torch, mech, n, seed):
    recipe = {"M13": "small", "M53": "mid", "M111": "divergent"}[mech]
    y0, P = synth.reactor_states({"M13": 13, "M53": 53, "M111": 111}[mech], n, recipe, seed=seed)
    dev = torch.device("cuda", 0)
    return torch.as_tensor(y0, device=dev), torch.as_tensor(P, device=dev)


def _timed_integrate(ck, torch, g, y, P, t_end, **opts):
    """One integrate call on a copy of y; returns (result, seconds) with HIP events on the current stream."""
    yy = y.clone()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    r = ck.integrate(g, yy, P, t_end, inplace=True, **opts)
    e1.record(stream)
    torch.cuda.synchronize()
    return r, e0.elapsed_time(e1) / 1e3


def _bounded_loop(ck, torch, g, y, P, t_end, launch_steps, log=None, **opts):
    """Integrate a copy of y to t_end in bounded launches resuming from (t, h), host-synchronised per
    launch (the host reads the statuses to decide whether to launch again).  Returns (result with
    summed step counts, seconds from the first launch to the last status read, launches)."""
    n = y.shape[1]
    yy = y.clone()
    t = torch.zeros(n, dtype=torch.float64, device=y.device)
    h = torch.zeros_like(t)
    steps = torch.zeros(n, dtype=torch.int64, device=y.device)
    ws = torch.empty(g.workspace_bytes(n, **opts), dtype=torch.uint8, device=y.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launches = 0
    while True:
        r = ck.integrate(g, yy, P, t_end, t=t, h=h, workspace=ws, inplace=True, max_steps=launch_steps, **opts)
        steps += r["n_accept"] + r["n_reject"]
        launches += 1
        left = int((r["status"] == 1).sum().item())
        if log:
            log(f"  launch {launches}: {time.perf_counter() - t0:.1f} s, {left} reactors unfinished")
        if left == 0:
            break
    torch.cuda.synchronize()
    r["steps"] = steps
    return r, time.perf_counter() - t0, launches


def suite_batching(a):
    """Batching against divergence (Section 4, Algorithm 2; Section 5.2, Eq. waste) on the 111-species
    half-hot / half-cold states: every reactor integrated to a common end time, so adaptive step counts
    diverge.  Timed: the persistent work-queue workgroup kernel in bounded launches driven from the
    host and replayed from a HIP graph (ck_integrate_graph), against the one-reactor-per-lane kernel
    (lockstep 64-lane wavefronts), whose waste is measured from its own step counts; the lane kernel
    again with the reactors ordered by initial temperature (a stiffness proxy), which groups similar
    step counts into a wavefront.  Bounded so the lane kernel finishes in about a minute: the first
    --batching-reactors states of the 262144-reactor batch to --batching-t-end.  Also the launch
    configuration chosen by the autotuner and the Eq. waste CDFs of a sample integrated further."""
    import torch

    from paper_1608_05794_amd import ck, metrics, synth, tune
    n, te = a.batching_reactors, a.batching_t_end
    out = {"suite": "batching", "data": "synthetic", "dtype": "f64",
           "workload": f"M111 (111 species, 784 reactions), first {n} of the 262144 half-hot / half-cold states "
                       f"(seed 1003), ROS4 to a common t_end = {te:g} s, rtol 1e-8, atol 1e-12"}
    g = ck.Mechanism(synth.mechanism_file("M111"))
    y0, P0 = synth.reactor_states(111, 262144, "divergent", seed=1003)
    y = torch.as_tensor(np.ascontiguousarray(y0[:, :n]), device="cuda")
    P = torch.as_tensor(np.ascontiguousarray(P0[:n]), device="cuda")
    log = lambda m: print(m, file=sys.stderr, flush=True)

    def row(r, dt, **kw):
        s = r["steps"] if "steps" in r else r["n_accept"] + r["n_reject"]
        s = s.to(torch.float64)
        st = torch.bincount(r["status"].to(torch.int64), minlength=4).tolist()
        return dict(seconds=dt, reactors_per_s=n / dt, reactor_steps_per_s=float(s.sum().item()) / dt,
                    mean_steps=float(s.mean().item()), max_steps=float(s.max().item()), status_histogram=st, **kw)

    # persistent workgroup kernel (tile form): host loop of bounded launches, then the graph-driven
    # loop; the half-row Gauss-Jordan form of the same kernel for comparison
    _bounded_loop(ck, torch, g, y[:, :256], P[:256], te, 200, kernel="tile")           # warm-up
    r, dt, nl = _bounded_loop(ck, torch, g, y, P, te, 200, log=log, kernel="tile")
    out["persistent_host_loop"] = row(r, dt, launches=nl, launch_steps=200, kernel="tile")
    ref = r
    log(f"batching persistent host loop: {dt:.2f} s, {nl} launches")
    _bounded_loop(ck, torch, g, y[:, :256], P[:256], te, 200, kernel="group")          # warm-up
    r, dt, nl = _bounded_loop(ck, torch, g, y, P, te, 200, log=log, kernel="group")
    out["persistent_half_row_host_loop"] = row(r, dt, launches=nl, launch_steps=200, kernel="group")
    gws = torch.empty(g.graph_workspace_bytes(n, kernel="tile"), dtype=torch.uint8, device="cuda")
    ck.integrate_graph(g, y[:, :256], P[:256], te, launch_steps=200, launches_per_graph=4, kernel="tile",
                       workspace=gws)                                                # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr = ck.integrate_graph(g, y, P, te, launch_steps=200, launches_per_graph=4, kernel="tile", workspace=gws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gr["steps"] = gr["n_accept"] + gr["n_reject"]
    out["persistent_graph_loop"] = row(gr, dt, replays=gr["replays"], launches_per_graph=4, launch_steps=200)
    out["persistent_graph_loop"]["statuses_equal_host_loop"] = bool(torch.equal(gr["status"], ref["status"]))
    log(f"batching persistent graph loop: {dt:.2f} s, {gr['replays']} replays")

    # one reactor per lane (lockstep 64-lane wavefronts), in bounded launches of 100 attempted steps
    # resuming from (t, h); the lockstep waste from its own step counts
    for tag, order in (("lane", None), ("lane_sorted_by_T0", torch.argsort(y[0]))):
        yy, pp = (y, P) if order is None else (y[:, order].contiguous(), P[order].contiguous())
        _timed_integrate(ck, torch, g, yy, pp, te, kernel="lane", max_steps=1)     # scratch allocation, code load
        r, dt, nl = _bounded_loop(ck, torch, g, yy, pp, te, 100, log=log, kernel="lane")
        s = r["steps"].cpu().numpy()
        w = metrics.waste(s, 64)
        out[tag] = row(r, dt, launches=nl, launch_steps=100, mean_waste_64=float(w.mean()),
                       lane_efficiency_64=metrics.lane_efficiency(s, 64),
                       waste_cdf_64={str(k): v for k, v in metrics.waste_cdf(s, widths=(64,))[64].items()})
        log(f"batching {tag}: {dt:.2f} s, mean waste {w.mean():.3f}")
    out["speedup_persistent_over_lane"] = out["persistent_host_loop"]["reactors_per_s"] / out["lane"]["reactors_per_s"]
    out["speedup_graph_over_host_loop"] = (out["persistent_graph_loop"]["reactors_per_s"] /
                                           out["persistent_host_loop"]["reactors_per_s"])

    # short launches (a serving-like loop of a few attempted steps per launch): the host loop
    # synchronises and reads the statuses after every launch, the graph loop once per replay
    ns_, te_s, ls, lpg = 4096, 1e-5, 8, 16
    gs = ck.Mechanism(synth.mechanism_file("M13"))
    ys, Ps = _states(synth, torch, "M13", ns_, 1001)
    short = {"workload": f"M13 x {ns_} reactors (small states, seed 1001), ROS4 to {te_s:g} s, "
                         f"{ls} attempted steps per launch, wavefront kernel"}
    _bounded_loop(ck, torch, gs, ys[:, :256], Ps[:256], te_s, ls, kernel="wave")        # warm-up
    r, dt, nl = _bounded_loop(ck, torch, gs, ys, Ps, te_s, ls, kernel="wave")
    short["host_loop"] = dict(seconds=dt, reactors_per_s=ns_ / dt, launches=nl)
    gws_s = torch.empty(gs.graph_workspace_bytes(ns_, kernel="wave"), dtype=torch.uint8, device="cuda")
    ck.integrate_graph(gs, ys[:, :256], Ps[:256], te_s, launch_steps=ls, launches_per_graph=lpg, kernel="wave",
                       workspace=gws_s)                                               # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr = ck.integrate_graph(gs, ys, Ps, te_s, launch_steps=ls, launches_per_graph=lpg, kernel="wave", workspace=gws_s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    short["graph_loop"] = dict(seconds=dt, reactors_per_s=ns_ / dt, replays=gr["replays"], launches_per_graph=lpg)
    short["statuses_equal"] = bool(torch.equal(gr["status"], r["status"]))
    short["states_equal"] = bool(torch.equal(gr["y"], r["y"]))
    short["speedup_graph_over_host_loop"] = short["host_loop"]["seconds"] / short["graph_loop"]["seconds"]
    out["short_launches"] = short
    log(f"batching short launches: host loop {short['host_loop']['seconds']:.3f} s ({nl} launches), graph loop "
        f"{dt:.3f} s ({gr['replays']} replays)")

    # launch configuration chosen by the autotuner on a 16384-reactor sample of each workload
    for mech, seed in (("M53", 1002), ("M111", 1003)):
        gm = ck.Mechanism(synth.mechanism_file(mech))
        ys, Ps = _states(synth, torch, mech, 16384, seed)
        best, table = tune.tune(gm, ys, Ps, 1e-3, steps=12)
        out[f"autotune_{mech}"] = {"best": {k: best[k] for k in ("kernel", "blocks_per_cu")},
                                   "table": [[c["kernel"], c["blocks_per_cu"], v] for c, v in table]}
        log(f"autotune {mech}: {best}")
    # Eq. waste CDFs for widths 4..64 from a sample integrated further (to 1e-9 s)
    ys, Ps = _states(synth, torch, "M111", 2048, 1003)
    r, dt = _timed_integrate(ck, torch, g, ys, Ps, 1e-9, kernel="tile")
    st = (r["n_accept"] + r["n_reject"]).cpu().numpy()
    out["waste_sample"] = {
        "reactors": 2048, "t_end": 1e-9, "mean_steps": float(st.mean()), "max_steps": int(st.max()),
        "mean_waste_by_width": {w: float(metrics.waste(st, w).mean()) for w in (4, 8, 16, 32, 64)},
        "lane_efficiency_64": metrics.lane_efficiency(st, 64),
        "waste_cdf": {str(w): v for w, v in metrics.waste_cdf(st).items()}}
    return out


def suite_precision(a):
    """FP32 factorisation with FP64 refinement against the all-FP64 solver, at 53 species (wavefront
    kernel, FP32 LU) and 111 species (tile workgroup kernel, FP32 matrix-core Gauss-Jordan): step
    counts, FP64 refactorings (steps whose refinement stagnated), the largest relative differences of
    T and Y (Y > 1e-12) between the two over the batch, and throughput."""
    import torch

    from paper_1608_05794_amd import ck, synth
    out = {"suite": "precision", "data": "synthetic", "dtype": "f64 (FP32 factorisation in fp32_refine)"}
    for mech, n, te, kernel, seed in (("M53", 16384, 1e-5, "wave", 1002), ("M111", 16384, 2e-10, "tile", 1003)):
        g = ck.Mechanism(synth.mechanism_file(mech))
        y, P = _states(synth, torch, mech, n, seed)
        res = {}
        for prec in ("fp64", "fp32_refine"):
            fb = torch.zeros(n, dtype=torch.int32, device="cuda")
            kw = dict(n_fallback=fb) if prec != "fp64" else {}
            _timed_integrate(ck, torch, g, y[:, :256].contiguous(), P[:256].contiguous(), te, kernel=kernel,
                             precision=prec, max_steps=4, **({} if prec == "fp64" else
                                                             dict(n_fallback=fb[:256])))   # warm-up
            r, dt = _timed_integrate(ck, torch, g, y, P, te, kernel=kernel, precision=prec, **kw)
            res[prec] = (r, dt, int(fb.sum().item()))
            print(f"precision {mech} {prec}: {dt:.1f} s", file=sys.stderr, flush=True)
        r64, r32 = res["fp64"][0], res["fp32_refine"][0]
        T64, T32 = r64["y"][0], r32["y"][0]
        Y64, Y32 = r64["y"][1:], r32["y"][1:]
        mask = Y64.abs() > 1e-12
        relY = ((Y32 - Y64).abs() / Y64.abs().clamp_min(1e-300))[mask]
        row = {"workload": f"{mech} x {n} reactors, ROS4 to {te:g} s, rtol 1e-8, atol 1e-12, kernel {kernel}"}
        for prec, (r, dt, nfb) in res.items():
            na, nr = int(r["n_accept"].sum().item()), int(r["n_reject"].sum().item())
            row[prec] = {"accepted": na, "rejected": nr, "seconds": dt, "reactor_steps_per_s": (na + nr) / dt,
                         "status_ok": int((r["status"] == 0).sum().item())}
            if prec != "fp64":
                row[prec]["fp64_refactorings"] = nfb
        row["fp32_vs_fp64"] = {"max_rel_T": float(((T32 - T64).abs() / T64).max().item()),
                               "max_rel_Y_above_1e-12": float(relY.max().item()),
                               "median_rel_Y_above_1e-12": float(relY.median().item()),
                               "identical_step_counts": float(((r64["n_accept"] + r64["n_reject"]) ==
                                                               (r32["n_accept"] + r32["n_reject"])).float().mean())}
        row["speed_ratio_fp32_over_fp64"] = row["fp32_refine"]["reactor_steps_per_s"] / row["fp64"]["reactor_steps_per_s"]
        out[mech] = row
    return out


def suite_serving(a):
    """Continuous batching on the configured request stream: Poisson arrivals at 2000 requests/s,
    mechanisms of 13 / 53 / 111 species with weights 0.3 / 0.5 / 0.2, reactor counts log-uniform in
    1..65536 and end times log-uniform in 1e-6..1e-3 s, states as in the other configurations,
    admitted into device-resident slot pools sized from a 200 GB HBM budget.  Bounded: the first
    --serve-requests arrivals of the stream, end times multiplied by --serve-t-scale, and a wall
    time limit; requests unfinished at the limit are reported as backlog.  Reports offered and
    served load and completed-request latency p50 / p99 (arrival to completion)."""
    import torch

    from paper_1608_05794_amd import ck, serve, synth
    mechs = {m: ck.Mechanism(synth.mechanism_file(m)) for m in ("M13", "M53", "M111")}
    species = {m: g.n_species for m, g in mechs.items()}
    reqs = serve.poisson_requests(a.serve_requests, 2000.0, seed=5000, n_range=(1, 65536), t_range=(1e-6, 1e-3),
                                  species=species)
    for r in reqs:
        r.t_end *= a.serve_t_scale
    pool_opts = {}
    if a.serve_precision != "fp64":
        pool_opts = {m: {"precision": a.serve_precision} for m in ("M13", "M53", "M111")}
    srv = serve.Server(mechs, hbm_budget=200e9, launch_steps=a.serve_launch_steps, pool_opts=pool_opts)
    by_mech = {m: sum(1 for r in reqs if r.mech == m) for m in mechs}
    t0 = time.perf_counter()
    done = srv.run(reqs, time_limit=a.serve_time_limit, log=lambda m: print(m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    summ = serve.latency_summary(done, 2000.0, el, arrived=reqs)
    lat = {m: [r.completed - r.arrival for r in done if r.mech == m] for m in mechs}
    steps = {m: float(np.mean(np.concatenate([r.result["steps"] for r in done if r.mech == m])))
             for m in mechs if any(r.mech == m for r in done)}
    return {"suite": "serving", "data": "synthetic", "dtype": "f64",
            "stream": f"first {len(reqs)} arrivals (seed 5000) of Poisson 2000/s, mechanisms 0.3/0.5/0.2 over "
                      f"13/53/111 species, reactors log-uniform 1-65536, t_end log-uniform 1e-6-1e-3 s "
                      f"x {a.serve_t_scale:g}, 200 GB budget",
            "requests": len(reqs), "requests_by_mechanism": by_mech, "reactors_offered": sum(r.n for r in reqs),
            "elapsed_s": el, "time_limit_s": a.serve_time_limit, "iterations": srv.iterations,
            "backlog_at_end": srv.backlog(), "max_backlog": srv.max_backlog, "rejected": len(srv.rejected),
            "pool_capacity": {m: p.cap for m, p in srv.pools.items()}, "allocated_bytes": srv.allocated,
            "precision": a.serve_precision, "launch_steps": a.serve_launch_steps,
            "p50_s_by_mechanism": {m: float(np.percentile(v, 50)) for m, v in lat.items() if v},
            "mean_attempted_steps_by_mechanism": steps, **summ}


def _median_time(ck, torch, g, y, P, t_end, warmup=3, runs=5, **opts):
    """Median over `runs` timed integrations (HIP events) after `warmup` untimed ones."""
    for _ in range(warmup):
        _timed_integrate(ck, torch, g, y, P, t_end, **opts)
    times, r = [], None
    for _ in range(runs):
        r, dt = _timed_integrate(ck, torch, g, y, P, t_end, **opts)
        times.append(dt)
    return r, float(np.median(times))


def cpu_baseline_rate(path, y, P, t_end, n, threads, **kw):
    """CPU baseline leg of the suites: the oracle (ROS4) timed on the first n reactors with `threads`
    host threads."""
    from oracle import oracle as O
    m = O.Mechanism(path)
    ys, Ps = np.ascontiguousarray(y[:, :n]), np.ascontiguousarray(P[:n])
    t0 = time.perf_counter()
    res = m.integrate(ys, Ps, t_end, "ros4", nthreads=threads, **kw)
    dt = time.perf_counter() - t0
    return {"kind": "oracle", "reactors": n, "cores": threads, "seconds": dt, "value": n / dt, "unit": "reactors/s",
            "mean_steps": float(np.mean(res["n_accept"] + res["n_reject"]))}


def deep_vs_shallow(ck, torch, synth, n=32768, reps=5):
    """Source term and analytic Jacobian evaluations per second at 13, 53 and 111 species, deep
    vectorisation (one reactor per wavefront for N <= 64, per four-wavefront group above) against
    shallow (one reactor per lane): median of `reps` launches on distinct seeded states, timed with
    HIP events on the launch stream."""
    res = {"reactors": n, "unit": "evaluations/s"}
    for name, ns in (("M13", 13), ("M53", 53), ("M111", 111)):
        g = ck.Mechanism(synth.mechanism_file(name))
        y0, P0 = synth.reactor_states(ns, n, "mid", seed=1003)
        y, P = torch.as_tensor(y0, device="cuda"), torch.as_tensor(P0, device="cuda")
        row = {}
        for op in ("rhs", "jacobian"):
            for fam, kern in (("deep", "wave"), ("shallow", "lane")):
                fn = (lambda: ck.rhs(g, y, P, kernel=kern)) if op == "rhs" else (lambda: ck.jac(g, y, P, kernel=kern))
                fn()
                times = []
                for _ in range(reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    out = fn()
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1) / 1e3)
                    del out
                row[f"{op}_{fam}"] = n / float(np.median(times))
            row[f"{op}_deep_over_shallow"] = row[f"{op}_deep"] / row[f"{op}_shallow"]
        print(f"methods deep vs shallow {name}: {row}", file=sys.stderr, flush=True)
        res[name] = row
        g.close()
    return res


def suite_methods(a):
    """The small configuration (13 species x 1024 reactors to 1e-4 s) with ROS4 and RKF45, a stiffness
    census of its initial states, its CPU baseline (the oracle on all host cores and on one); the rate
    with host-to-device and device-to-host transfers included; and ROS4 with the analytic Jacobian
    against forward differences (53 species), with the one-core CPU baseline of the 53-species
    workload."""
    import torch

    from paper_1608_05794_amd import ck, synth
    cores = len(os.sched_getaffinity(0))
    out = {"suite": "methods", "data": "synthetic", "dtype": "f64", "host_cores": cores}
    stat = lambda r: torch.bincount(r["status"].to(torch.int64), minlength=4).tolist()
    steps = lambda r: (r["n_accept"] + r["n_reject"]).to(torch.float64)

    # small configuration: ROS4 and RKF45 (RKF45 capped: its steps follow the stiffness, see census)
    path = synth.mechanism_file("M13")
    g = ck.Mechanism(path)
    n, te = 1024, 1e-4
    y0, P0 = synth.reactor_states(13, n, "small", seed=1001)
    y, P = torch.as_tensor(y0, device="cuda"), torch.as_tensor(P0, device="cuda")
    small = {"workload": f"M13 x {n} reactors to {te:g} s, rtol 1e-8, atol 1e-12"}
    for method, cap in (("ros4", 1_000_000), ("rkf45", 100_000)):
        r, dt = _median_time(ck, torch, g, y, P, te, method=method, kernel="wave", max_steps=cap)
        s = steps(r)
        small[method] = {"seconds_median_of_5": dt, "reactors_per_s": n / dt,
                         "reactor_steps_per_s": float(s.sum().item()) / dt, "mean_steps": float(s.mean().item()),
                         "max_steps_cap": cap, "status_histogram": stat(r)}
        print(f"methods small {method}: {dt * 1e3:.2f} ms, status {stat(r)}", file=sys.stderr, flush=True)
    # stiffness census: spectral radius of J at the initial states; explicit RKF45 needs about
    # t_end * rho / 3 steps (stability-bound)
    J = ck.jac(g, y, P).cpu().numpy().T.reshape(n, 14, 14)
    rho = np.abs(np.linalg.eigvals(J)).max(axis=1)
    small["stiffness_census"] = {"rho_percentiles_10_50_90": [float(v) for v in np.percentile(rho, [10, 50, 90])],
                                 "rkf45_steps_estimate_median": float(np.median(rho) * te / 3)}
    small["cpu_baseline"] = {"all_cores": cpu_baseline_rate(path, y0, P0, te, n, cores),
                             "one_core": cpu_baseline_rate(path, y0, P0, te, 128, 1)}
    # transfers included: pinned host state in, integrate, state / status / counters out
    hy = torch.empty(y0.shape, dtype=torch.float64, pin_memory=True)
    hy.copy_(torch.as_tensor(y0))
    hP = torch.empty(P0.shape, dtype=torch.float64, pin_memory=True)
    hP.copy_(torch.as_tensor(P0))
    oy = torch.empty(y0.shape, dtype=torch.float64, pin_memory=True)
    ost = torch.empty(n, dtype=torch.int32, pin_memory=True)
    times = []
    for i in range(8):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dy, dP = hy.to("cuda", non_blocking=True), hP.to("cuda", non_blocking=True)
        r = ck.integrate(g, dy, dP, te, method="ros4", kernel="wave", inplace=True)
        oy.copy_(r["y"], non_blocking=True)
        ost.copy_(r["status"], non_blocking=True)
        torch.cuda.synchronize()
        if i >= 3:
            times.append(time.perf_counter() - t0)
    small["ros4_with_transfers"] = {"seconds_median_of_5": float(np.median(times)),
                                    "reactors_per_s": n / float(np.median(times))}
    out["small"] = small

    # analytic Jacobian against forward differences (the paper's own set-up), 53 species
    path = synth.mechanism_file("M53")
    g = ck.Mechanism(path)
    n, te = 8192, 1e-7
    y0, P0 = synth.reactor_states(53, n, "mid", seed=1002)
    y, P = torch.as_tensor(y0, device="cuda"), torch.as_tensor(P0, device="cuda")
    jac = {"workload": f"M53 x {n} reactors, ROS4 to {te:g} s, rtol 1e-8, atol 1e-12"}
    for kind in ("analytic", "fd"):
        r, dt = _median_time(ck, torch, g, y, P, te, warmup=1, runs=3, kernel="wave", jacobian=kind)
        s = steps(r)
        jac[kind] = {"seconds_median_of_3": dt, "reactors_per_s": n / dt,
                     "reactor_steps_per_s": float(s.sum().item()) / dt, "mean_steps": float(s.mean().item()),
                     "status_histogram": stat(r)}
        print(f"methods jacobian {kind}: {dt:.2f} s", file=sys.stderr, flush=True)
    jac["analytic_speedup"] = jac["fd"]["seconds_median_of_3"] / jac["analytic"]["seconds_median_of_3"]
    out["jacobian"] = jac
    out["deep_vs_shallow"] = deep_vs_shallow(ck, torch, synth)
    # CPU baseline on one core for the headline workload's states (ROS4 to 1e-3 s)
    y0, P0 = synth.reactor_states(53, 4, "mid", seed=1002)
    out["cpu_baseline_one_core_M53_1e-3"] = cpu_baseline_rate(path, y0, P0, 1e-3, 4, 1)
    return out


def suite_peaks(a):
    """Achievable rates on this GPU, for context beside the published peaks the roofline uses: FP64
    GEMM (the library path, matrix units), an elementwise FP64 FMA over resident data (vector units,
    memory-bound by construction), and a device-to-device copy of 1 GiB (STREAM-like)."""
    import torch
    dev = torch.device("cuda", 0)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    out = {"suite": "peaks", "published": {"fp64_vector_tflops": 78.6, "fp64_matrix_tflops": 78.6, "hbm_tbps": 8.0}}
    n = 8192
    A = torch.randn(n, n, dtype=torch.float64, device=dev)
    B = torch.randn(n, n, dtype=torch.float64, device=dev)
    C = torch.empty_like(A)
    dt = timed(lambda: torch.matmul(A, B, out=C), 5)
    out["fp64_gemm_tflops"] = 2.0 * n ** 3 / dt / 1e12
    del A, B, C
    m = (1 << 30) // 8
    x = torch.ones(m, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    dt = timed(lambda: y.copy_(x), 10)
    out["copy_gbps"] = 2.0 * m * 8 / dt / 1e9
    # y = x + x * x: the three operands alias one tensor, so HBM sees one read and one write stream
    dt = timed(lambda: torch.addcmul(x, x, x, value=1.0, out=y), 10)
    out["fp64_fma_elementwise"] = {"tflops": 2.0 * m / dt / 1e12, "gbps": 2.0 * m * 8 / dt / 1e9}
    return out


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the reactors are independent and the library runs on a single "
              "device, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if a.suite != "integrate":
        fn = {"batching": suite_batching, "precision": suite_precision, "serving": suite_serving,
              "methods": suite_methods, "peaks": suite_peaks}[a.suite]
        print(json.dumps(fn(a)), flush=True)
        return

    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                          "dispatches": 3}), flush=True)
        return

    from paper_1608_05794_amd import ck, synth

    path = synth.mechanism_file(a.mech)
    g = ck.Mechanism(path)
    recipe = {"M13": "small", "M53": "mid", "M111": "divergent"}[a.mech]
    seed = {"M13": 1001, "M53": 1002, "M111": 1003}[a.mech]
    y0, P = synth.reactor_states(g.n_species, a.reactors, recipe, seed=seed)
    dev = torch.device("cuda", 0)
    y0d = torch.as_tensor(y0, device=dev)
    Pd = torch.as_tensor(P, device=dev)
    ted = torch.full((a.reactors,), a.t_end, dtype=torch.float64, device=dev)
    yw = torch.empty_like(y0d)
    ws = torch.empty(g.workspace_bytes(a.reactors, kernel=a.kernel, precision=a.precision), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream()
    info = mech_structure(path)
    fl = algorithmic_flops(info)

    tt = torch.zeros(a.reactors, dtype=torch.float64, device=dev)
    hh = torch.zeros(a.reactors, dtype=torch.float64, device=dev)
    acc_steps = torch.zeros(a.reactors, dtype=torch.int64, device=dev)

    def one_step(tag):
        """Integrate the whole batch from its initial state: a loop of bounded launches of the
        persistent kernel, each resuming every unfinished reactor from its (t, h)."""
        yw.copy_(y0d)
        tt.zero_()
        hh.zero_()
        acc_steps.zero_()
        launches, kern = 0, 0.0
        while True:
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            r = ck.integrate(g, yw, Pd, ted, method="ros4", t=tt, h=hh, workspace=ws, inplace=True,
                             kernel=a.kernel, precision=a.precision, max_steps=a.launch_steps)
            ev1.record(stream)
            acc_steps.add_(r["n_accept"] + r["n_reject"])
            torch.cuda.synchronize()
            launches += 1
            kern += ev0.elapsed_time(ev1) / 1e3
            left = int((r["status"] == 1).sum().item())
            print(f"{tag} launch {launches}: {ev0.elapsed_time(ev1) / 1e3:.2f} s, {left} reactors unfinished",
                  file=sys.stderr, flush=True)
            if left == 0 or launches * a.launch_steps >= a.max_steps:
                return r, kern, launches

    def elapsed():
        return time.time() - T_PROCESS_START

    # Warm-up passes (untimed): one bounded launch each over the whole batch from its initial state,
    # which loads the code objects and touches the workspace without a full two-minute integration.
    warm = 0
    for i in range(a.warmup):
        yw.copy_(y0d)
        tt.zero_()
        hh.zero_()
        ck.integrate(g, yw, Pd, ted, method="ros4", t=tt, h=hh, workspace=ws, inplace=True, kernel=a.kernel,
                     precision=a.precision, max_steps=a.warmup_launch_steps)
        torch.cuda.synchronize()
        warm += 1
    print(f"warm-up: {warm} passes of {a.warmup_launch_steps} attempted steps, {elapsed():.1f} s since start",
          file=sys.stderr, flush=True)

    # Timed steps: at least one; another only if it fits the budget with the RHS and CPU legs after it.
    reserve_s = 15.0 + (0.0 if a.no_cpu_baseline else 45.0)
    kern_s, walls, launches_l = [], [], []
    t0 = time.perf_counter()
    for i in range(a.steps):
        if walls and elapsed() + max(walls) + reserve_s > a.budget_s:
            print(f"budget: stopping after {len(walls)} timed steps ({elapsed():.1f} s since start, "
                  f"budget {a.budget_s:.0f} s)", file=sys.stderr, flush=True)
            break
        s0 = time.perf_counter()
        r, kern, launches = one_step(f"step {i}")
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - s0)
        kern_s.append(kern)
        launches_l.append(launches)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing_end_s = elapsed()
    n_steps = len(walls)
    steps = acc_steps.to(torch.float64)
    status = torch.bincount(r["status"].to(torch.int64), minlength=4).tolist()
    total_steps = float(steps.sum().item())
    kernel_s = sum(kern_s) / n_steps
    launches = launches_l[-1]
    flops_launch = total_steps * fl["ros4_step"] + a.reactors * fl["h0"]
    achieved = flops_launch / kernel_s

    # RHS leg: distinct state batches, cycled so consecutive evaluations never reuse cached state
    nb = max(1, a.rhs_batches)
    batches = [torch.as_tensor(synth.rhs_states(g.n_species, a.reactors, 20000 + k)[0], device=dev) for k in range(nb)]
    out = torch.empty_like(batches[0])
    ck.rhs(g, batches[0], Pd, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(a.rhs_evals):
        ck.rhs(g, batches[k % nb], Pd, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    rhs_s = e0.elapsed_time(e1) / 1e3
    rhs_rate = a.rhs_evals * a.reactors / rhs_s
    # the same leg with one reactor per lane (shallow vectorisation, Section 4) for comparison
    ck.rhs(g, batches[0], Pd, out=out, kernel="lane")
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(a.rhs_evals):
        ck.rhs(g, batches[k % nb], Pd, out=out, kernel="lane")
    e1.record(stream)
    torch.cuda.synchronize()
    rhs_rate_lane = a.rhs_evals * a.reactors / (e0.elapsed_time(e1) / 1e3)

    res = {
        "metric": METRIC,
        "value": a.reactors * n_steps / wall,
        "unit": "reactors/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": warm,
        "ms_per_step": 1e3 * wall / n_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.mech} x {a.reactors} reactors, ROS4 to {a.t_end:g} s, rtol 1e-8, atol 1e-12",
                   "mechanism": f"{a.mech} ({info['n_species']} species, {len(info['reactions'])} reactions)",
                   "reactors": a.reactors, "t_end": a.t_end, "kernel": a.kernel, "precision": a.precision,
                   "step": "integrate the whole batch from its initial state to t_end",
                   "warmup_pass": f"one launch of {a.warmup_launch_steps} attempted steps per reactor",
                   "steps_requested": a.steps, "warmup_requested": a.warmup, "budget_s": a.budget_s},
        "rhs_evals_per_s": rhs_rate,
        "rhs_evals_per_s_lane_kernel": rhs_rate_lane,
        "mean_steps_per_reactor": total_steps / a.reactors,
        "launches_per_step": launches,
        "step_seconds": walls,
        "wall_s_since_start_at_end_of_timing": timing_end_s,
        "status_counts": {"ok": status[0], "max_steps": status[1], "h_underflow": status[2], "nonfinite": status[3]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": measured_traffic(a),
                     "traffic_unit": "bytes per launch",
                     "kernel": (KERNEL_NAMES[a.kernel].replace("Adapter", "Adapter32").replace("CoopTile", "CoopTile32")
                                if a.precision != "fp64" else KERNEL_NAMES[a.kernel]),
                     "launches": launches,
                     "avg_launch_ms": 1e3 * kernel_s / launches,
                     "flops_per_step_of_batch": flops_launch, "kernel_s": kernel_s,
                     "flops_per_step": fl["ros4_step"]},
    }
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(path, y0, P, a.t_end, a.cpu_sample)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

"""Throughput benchmark of the batched reactor integration on one MI355X.

Workload (mid configuration): synthetic 53-species / 325-reaction mechanism
(30 third-body, 25 Troe), 131072 constant-pressure reactors with
T0 ~ U(900, 1800) K, P ~ U(1, 20) atm, Y0 ~ Dirichlet(0.5), integrated with
ROS4 to t = 1e-3 s at rtol 1e-8, atol 1e-12, FP64.  One "step" integrates the
whole batch from its initial state; inputs are resident in HBM before the
timed region.  Also reported: source-term (RHS) evaluations per second over
distinct state batches, the roofline of the dominant kernel, and the CPU
oracle on a bounded sample of the same workload.

Prints one JSON line (rank 0).  Only one GPU is used; --gpus > 1 exits.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reactors/s integrated (ROS4, rtol 1e-8), RHS evals/s, p50/p99 solve latency"
KERNEL_NAMES = {"wave": "integrate_wave_kernel<Ros4Adapter>", "auto": "integrate_wave_kernel<Ros4Adapter>",
                "group": "coop_kernel<Ros4Coop>", "lane": "integrate_lane_kernel<0>"}
PEAK_FP64_VECTOR = 78.6e12          # FLOP/s, MI355X FP64 vector (VALU)
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
    ap.add_argument("--kernel", default="wave", choices=["wave", "lane", "group", "auto"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refine"])
    ap.add_argument("--launch-steps", type=int, default=2000,
                    help="attempted steps per reactor per kernel launch; launches resume from (t, h)")
    ap.add_argument("--max-steps", type=int, default=1_000_000, help="attempted steps per reactor in total")
    ap.add_argument("--rhs-evals", type=int, default=100, help="RHS evaluations per reactor in the RHS leg")
    ap.add_argument("--rhs-batches", type=int, default=8, help="distinct state batches cycled in the RHS leg")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: 8 per host core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device three times (counter calibration) and exit")
    return ap.parse_args()


def cpu_baseline(path, y, P, t_end, sample):
    """The CPU oracle (one reactor per OpenMP task, dynamic schedule) on a bounded sample."""
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0))
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


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: reactors are independent and this build runs on a single "
              "MI355X; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch

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

    for i in range(a.warmup):
        one_step(f"warmup {i}")
    torch.cuda.synchronize()
    kern_s = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        r, kern, launches = one_step(f"step {i}")
        kern_s.append(kern)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = acc_steps.to(torch.float64)
    status = torch.bincount(r["status"].to(torch.int64), minlength=4).tolist()
    total_steps = float(steps.sum().item())
    kernel_s = sum(kern_s) / len(kern_s)
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

    res = {
        "metric": METRIC,
        "value": a.reactors * a.steps / wall,
        "unit": "reactors/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.mech} x {a.reactors} reactors, ROS4 to {a.t_end:g} s, rtol 1e-8, atol 1e-12",
                   "mechanism": f"{a.mech} ({info['n_species']} species, {len(info['reactions'])} reactions)",
                   "reactors": a.reactors, "t_end": a.t_end, "kernel": a.kernel, "precision": a.precision},
        "rhs_evals_per_s": rhs_rate,
        "mean_steps_per_reactor": total_steps / a.reactors,
        "launches_per_step": launches,
        "status_counts": {"ok": status[0], "max_steps": status[1], "h_underflow": status[2], "nonfinite": status[3]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": None,
                     "kernel": KERNEL_NAMES[a.kernel].replace("Adapter", "Adapter32" if a.precision != "fp64" else "Adapter"),
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

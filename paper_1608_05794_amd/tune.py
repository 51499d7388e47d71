"""Launch-configuration autotuner for the batched integrators.

For a mechanism and a sample of reactor states, time a bounded integration (a fixed budget of
attempted steps per reactor) for every candidate launch configuration -- kernel family and
resident workgroups per compute unit -- and return the fastest.  The throughput unit is
attempted reactor-steps per second, which does not depend on how far the sample gets.  All work
runs in the library's kernels; this module only chooses among their launch options.
"""
from __future__ import annotations

import time

import torch

from . import ck


def candidates(n_state, method="ros4", precision="fp64", max_blocks_per_cu=8):
    """Launch configurations worth timing for a state size N (T plus species)."""
    out = []
    wave_ok = (method == "ros4" and n_state <= 64) or (method == "rkf45" and precision == "fp64" and n_state <= 128)
    if wave_ok:
        for b in range(max_blocks_per_cu, 0, -1):
            out.append({"kernel": "wave", "blocks_per_cu": b})
    if method == "ros4" and precision == "fp64" and 64 < n_state <= 128:
        for b in (2, 1):
            out.append({"kernel": "tile", "blocks_per_cu": b})
    if method == "ros4" and precision == "fp64" and n_state <= 128:
        for b in (2, 1):
            out.append({"kernel": "group", "blocks_per_cu": b})
    if precision == "fp64":
        out.append({"kernel": "lane", "blocks_per_cu": 0})
    return out


def tune(mech: ck.Mechanism, y, p, t_end, method="ros4", steps=20, configs=None, **opts):
    """Time each configuration on (y, p) for `steps` attempted steps per reactor.

    y: [N, n] float64 device tensor (not modified); p: [n] device tensor.  Returns
    (best_opts, table) with table = [(config, reactor_steps_per_s)] in the order timed."""
    configs = configs if configs is not None else candidates(mech.N, method, opts.get("precision", "fp64"))
    table = []
    for cfg in configs:
        o = dict(opts, **cfg)
        try:
            yy = y.clone()
            ck.integrate(mech, yy, p, t_end, method=method, inplace=True, max_steps=2, **o)   # warm-up
            yy.copy_(y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ck.integrate(mech, yy, p, t_end, method=method, inplace=True, max_steps=steps, **o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        except ck.CkError:
            continue
        done = float((r["n_accept"] + r["n_reject"]).sum().item())
        table.append((cfg, done / dt if dt > 0 else 0.0))
    if not table:
        raise ck.CkError("no launch configuration supports this mechanism and options")
    best = max(table, key=lambda e: e[1])[0]
    return dict(opts, **best), table

"""Diagnostics of batched integration (Section 5.2).

waste(): the SIMD waste of Eq. waste for work units of P consecutive reactors,
W_j = 1 - sum_i N_i / (P max_i N_i), N_i the attempted steps of reactor i.
For the one-reactor-per-lane kernel a work unit is a 64-lane wavefront; for the
one-reactor-per-wavefront queue kernel every unit holds a single reactor and
the waste is zero by construction.
"""
import numpy as np


def waste(steps, width):
    """Waste of each complete group of `width` consecutive reactors (a trailing partial group is dropped)."""
    steps = np.asarray(steps, dtype=np.float64)
    n = (len(steps) // width) * width
    if n == 0:
        return np.zeros(0)
    g = steps[:n].reshape(-1, width)
    mx = g.max(axis=1)
    out = np.zeros(len(g))
    nz = mx > 0
    out[nz] = 1.0 - g[nz].sum(axis=1) / (width * mx[nz])
    return out


def waste_cdf(steps, widths=(4, 8, 16, 32, 64), thresholds=(0.01, 0.1, 0.25, 0.5)):
    """Fraction of work units with waste below each threshold, per width (the paper's waste CDFs)."""
    out = {}
    for w in widths:
        v = waste(steps, w)
        out[w] = {t: float(np.mean(v < t)) if len(v) else float("nan") for t in thresholds}
    return out


def lane_efficiency(steps, width=64):
    """Useful lane-steps over issued lane-steps for groups of `width` reactors run in lockstep."""
    steps = np.asarray(steps, dtype=np.float64)
    n = (len(steps) // width) * width
    g = steps[:n].reshape(-1, width)
    issued = width * g.max(axis=1).sum()
    return float(g.sum() / issued) if issued else 1.0

"""Writes tests/golden/truth_*.json: reference end states of seeded workload samples, computed by
the CPU oracle alone at tolerances three decades tighter than the library is run at.

Where several results are correct (an adaptive integration to rtol 1e-8: an accept/reject decision
can flip between two FP64 implementations at err ~ 1, and the step sequences then part), the
integrated parity tests compare each result with a tighter solution of the same initial value
problem (Section 2, Eq. ode; Algorithm 1).  The oracle's ROS4 (Appendix C) at rtol 1e-11,
atol 1e-15 serves as that solution; the same integration at rtol 1e-10, atol 1e-14 is stored beside
it, and their difference bounds how far the reference itself is from the exact solution (on the
M53 sample it is about 1e-13 in T and 4e-8 in Y, against 1e-11 and 2e-5 for rtol 1e-8).

Cases (states from synth.reactor_states, as the benchmark draws them; the sample is the first and
the last reactor of the batch plus seeded others):
  m53_mid_1e-3          53 species, 131072 'mid' states (seed 1002), t_end 1e-3 s  (headline)
  m111_divergent_2e-9   111 species, 262144 half-hot / half-cold states (seed 1003), t_end 2e-9 s
  m111_divergent_2e-12  the same states to 2e-12 s (short enough for the explicit RKF45 pair)

Run:  python tests/golden/make_truth.py [case ...]   (minutes on a few cores; imports only the
oracle and the input generator)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                       # noqa: E402
from paper_1608_05794_amd import synth               # noqa: E402

CASES = {
    "m53_mid_1e-3": dict(mech="M53", recipe="mid", seed=1002, n=131072, t_end=1e-3, extra=6),
    "m111_divergent_2e-9": dict(mech="M111", recipe="divergent", seed=1003, n=262144, t_end=2e-9, extra=6),
    "m111_divergent_2e-12": dict(mech="M111", recipe="divergent", seed=1003, n=262144, t_end=2e-12, extra=6),
}
TIGHT = (1e-11, 1e-15)
CHECK = (1e-10, 1e-14)


def sample_indices(n, extra, seed=77):
    """First and last reactor plus `extra` distinct seeded others, in increasing order."""
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(1, n - 1), size=extra, replace=False)
    return sorted({0, n - 1, *map(int, mid)})


def mech_sha256(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def make(name, directory):
    c = CASES[name]
    path = synth.mechanism_file(c["mech"], directory)
    m = O.Mechanism(path)
    y, P = synth.reactor_states(m.n_species, c["n"], c["recipe"], seed=c["seed"])
    idx = sample_indices(c["n"], c["extra"])
    ys, Ps = np.ascontiguousarray(y[:, idx]), np.ascontiguousarray(P[idx])
    out = dict(case=name, mechanism=c["mech"], mechanism_sha256=mech_sha256(path), recipe=c["recipe"],
               seed=c["seed"], batch=c["n"], t_end=c["t_end"], indices=idx, method="ros4")
    runs = {}
    for rtol, atol in (CHECK, TIGHT):
        t0 = time.time()
        r = m.integrate(ys, Ps, c["t_end"], "ros4", rtol=rtol, atol=atol, max_steps=5_000_000)
        print(f"{name}: rtol {rtol:g}: {time.time() - t0:.1f} s, steps {r['n_accept'] + r['n_reject']}",
              flush=True)
        assert np.all(r["status"] == 0), r["status"]
        runs[rtol] = r
    ref, chk = runs[TIGHT[0]], runs[CHECK[0]]
    out.update(rtol=TIGHT[0], atol=TIGHT[1], y=ref["y"].T.tolist(),
               steps=(ref["n_accept"] + ref["n_reject"]).tolist(),
               check_rtol=CHECK[0], check_atol=CHECK[1], y_check=chk["y"].T.tolist())
    dst = os.path.join(HERE, f"truth_{name}.json")
    with open(dst, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", dst, flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    d = os.environ.get("CK_MECH_DIR") or os.path.join(ROOT, "_mech")
    for nm in names:
        make(nm, d)

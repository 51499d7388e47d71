"""Host-side logic: the waste metric (Eq. waste) and the serving slot bookkeeping."""
import numpy as np

from paper_1608_05794_amd import metrics


def test_waste_closed_forms():
    # equal step counts waste nothing
    assert np.all(metrics.waste([7] * 64, 4) == 0.0)
    # one busy lane among P idle-ish lanes: W = 1 - (N + (P-1) M) / (P N)
    s = [100, 1, 1, 1]
    assert np.isclose(metrics.waste(s, 4)[0], 1 - 103 / 400)
    # groups are consecutive and a trailing partial group is dropped
    w = metrics.waste([1, 3, 2, 2, 5], 2)
    assert np.allclose(w, [1 - 4 / 6, 0.0])
    # wider groups never waste less on the same data (max over a superset)
    rng = np.random.default_rng(0)
    st = rng.integers(1, 1000, size=4096)
    means = [metrics.waste(st, p).mean() for p in (4, 8, 16, 32, 64)]
    assert all(a <= b + 1e-12 for a, b in zip(means, means[1:]))
    # lane efficiency is one minus the max-weighted mean waste
    g = st.reshape(-1, 64).astype(float)
    W = metrics.waste(st, 64)
    assert np.isclose(metrics.lane_efficiency(st, 64), 1 - np.sum(W * g.max(1)) / g.max(1).sum())


def test_slot_bookkeeping():
    from paper_1608_05794_amd import serve
    p = serve.Pool.__new__(serve.Pool)
    p.cap, p.free, p.active, p.hwm = 100, [(0, 100)], {}, 0
    a = p.alloc(30)
    b = p.alloc(50)
    assert a == (0, 30) and b == (30, 80) and p.alloc(30) is None
    p.release(*a)
    assert p.free == [(0, 30), (80, 100)]
    p.release(*b)
    assert p.free == [(0, 100)]


def test_tuner_candidates():
    from paper_1608_05794_amd import tune
    c53 = tune.candidates(54)
    assert {"kernel": "wave", "blocks_per_cu": 8} in c53 and {"kernel": "lane", "blocks_per_cu": 0} in c53
    c112 = tune.candidates(112)
    assert all(c["kernel"] != "wave" for c in c112) and any(c["kernel"] == "group" for c in c112)
    assert all(c["kernel"] == "wave" for c in tune.candidates(54, precision="fp32_refine"))
    assert tune.candidates(200) == [{"kernel": "lane", "blocks_per_cu": 0}]

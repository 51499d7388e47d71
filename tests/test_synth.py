"""Synthetic mechanism generator: balance, rank, connectivity, thermo sanity."""
import filecmp

import numpy as np
import pytest

from paper_1608_05794_amd import synth

SHAPES = {"M13": (13, 27, 4, 2), "M53": (53, 325, 30, 25), "M111": (111, 784, 60, 40)}


@pytest.mark.parametrize("name", ["M13", "M53", "M111"])
def test_mechanism_shape_and_balance(name):
    m = synth.make_mechanism(name)
    nsp, nrxn, ntb, ntroe = SHAPES[name]
    assert m.n_species == nsp and m.n_reactions == nrxn
    types = [r.type for r in m.reactions]
    assert types.count(1) == ntb and types.count(3) == ntroe
    nu = synth.stoich_matrix(m)
    E = synth.element_matrix(m)
    # every reaction is element balanced
    assert np.all(E @ nu == 0)
    # molar masses are the element sums
    W_e = np.array([synth.ELEMENT_W[e] for e in m.elements])
    assert np.allclose([s.W for s in m.species], W_e @ E, rtol=0, atol=1e-15)
    # the reactions span every element-conserving composition change
    assert np.linalg.matrix_rank(nu) == nsp - np.linalg.matrix_rank(E)
    # every species takes part
    assert np.all(np.abs(nu).sum(axis=1) > 0)
    for r in m.reactions:
        assert r.rev == 1
        assert all(1 <= v <= 2 for _, v in r.reac + r.prod)


def test_seeded_reproducible(tmp_path):
    a, b = tmp_path / "a.ckm", tmp_path / "b.ckm"
    synth.write_mechanism(synth.make_mechanism("M53"), str(a))
    synth.write_mechanism(synth.make_mechanism("M53"), str(b))
    assert filecmp.cmp(a, b, shallow=False)


@pytest.mark.parametrize("recipe", ["small", "mid", "divergent"])
def test_states(recipe):
    y, P = synth.reactor_states(53, 1000, recipe, seed=5)
    assert y.shape == (54, 1000) and P.shape == (1000,)
    assert np.allclose(y[1:].sum(axis=0), 1.0, atol=1e-14)
    assert np.all(y[1:] > 0)
    if recipe == "divergent":
        hot = y[0] >= 1400
        assert hot.sum() == 500 and np.all((y[0] <= 900) | hot)
        # interleaved: both kinds appear in most 64-wide groups
        g = hot[:960].reshape(-1, 64)
        assert np.mean(g.any(axis=1) & (~g).any(axis=1)) > 0.9
    y2, _ = synth.reactor_states(53, 1000, recipe, seed=5)
    assert np.array_equal(y, y2)

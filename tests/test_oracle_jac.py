"""Pin of the oracle's analytic Jacobian: Richardson-extrapolated central differences of its source term."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_05794_amd import synth

from . import mechs_for_tests as TM


def fd_jacobian(m, y_col, P):
    """Central differences with one Richardson step (error O(h^4)), column by column."""
    N = y_col.shape[0]
    J = np.zeros((N, N))
    for j in range(N):
        h = 1e-3 * abs(y_col[j]) if j > 0 else 1e-2
        h = max(h, 1e-9)

        def D(hh):
            yp = y_col.copy()
            ym = y_col.copy()
            yp[j] += hh
            ym[j] -= hh
            both = m.rhs(np.stack([yp, ym], 1), np.array([P, P]))
            return (both[:, 0] - both[:, 1]) / (2 * hh)
        J[:, j] = (4.0 * D(h / 2) - D(h)) / 3.0
    return J


def _check(m, y, P, tol):
    J = m.jac(y, P)
    for r in range(y.shape[1]):
        Jfd = fd_jacobian(m, y[:, r].copy(), P[r])
        # entries compared against the row's largest derivative contribution scaled by the column size,
        # i.e. |dJ_ij| * |y_j| <= tol * max_j |J_ij y_j|
        yscale = np.maximum(np.abs(y[:, r]), 1e-9)
        contrib = np.abs(J[r]) * yscale[None, :]
        rowscale = contrib.max(axis=1, keepdims=True) + 1e-300
        err = np.abs(J[r] - Jfd) * yscale[None, :] / rowscale
        assert err.max() < tol, (r, np.unravel_index(err.argmax(), err.shape), err.max())


@pytest.mark.parametrize("name,recipe,n", [("M13", "small", 6), ("M53", "mid", 3), ("M111", "divergent", 2)])
def test_jacobian_vs_central_differences(name, recipe, n, oracle_mech):
    m = oracle_mech(name)
    y, P = synth.reactor_states(m.n_species, n, recipe, seed=21)
    _check(m, y, P, 2e-7)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_jacobian_falloff_paths(kind, tmp_path):
    """Third-body and fall-off derivative paths, including the temperature dependence of Fcent."""
    low = (2.0e4, -0.7, 3.0e4) if kind >= 2 else None
    troe = (0.6, 300.0, 2500.0, 6000.0) if kind == 3 else None
    mech = TM.isomer_mechanism(kind, A=3.0e5, beta=0.8, Ea=4.0e4, low=low, troe=troe)
    # make the two isomers thermally different so that T and the reverse rate respond
    mech.species[1].a_low[5] -= 3000.0
    mech.species[1].a_high[5] -= 3000.0
    m = O.Mechanism(TM.write(mech, tmp_path / "m.ckm"))
    y = np.array([[1100.0, 1400.0], [0.3, 0.05], [0.2, 0.4], [0.5, 0.55]])
    P = np.array([1.5e5, 8.0e5])
    _check(m, y, P, 1e-8)

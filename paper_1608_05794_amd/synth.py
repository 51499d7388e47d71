"""Seeded synthetic inputs: reaction mechanisms and reactor states.

This module only *constructs* inputs.  It evaluates none of the kinetics
(no rates, no source terms, no integration); both the GPU library and the
CPU oracle read what it writes.

Mechanism shapes follow the paper's model table (Section 5, "Details of the
chemical kinetic models"): a small H/O/N set of 13 species and 27 reactions,
a GRI-sized 53/325 set and a USC-sized 111/784 set, all reversible, with
third-body and pressure fall-off (Troe) reactions (Section 3, Eq. wdot and
the text around it).  Real mechanisms are not shipped, so species, reactions
and parameters are drawn from seeded distributions:

* species: distinct small formulas over the element set, always including the
  element atoms and homonuclear diatomics;
* reactions: element-balanced templates A+B=C+D, A+B=C, 2A=B+C; third-body
  and Troe reactions are combinations A+B(+M)=AB(+M); each is written in the
  direction that is favoured at 1200 K by the drawn formation data, so that
  reverse rates are not orders of magnitude above forward rates;
* Arrhenius parameters (Eq. kfor): A log-uniform 1e6..1e14 in CHEMKIN cgs
  units for the reaction order, converted to SI; beta uniform -1..2;
  Ea uniform 0..2e5 J/mol;
* thermodynamics (Eq. tfits, two-range NASA-7): cp(T) from a smooth
  Einstein-mode model, fitted on [200,1000] and [1000,6000] K with cp, dcp/dT,
  H and S continuous at 1000 K.

File format (text, one record per line, SI units, Ea in J/mol):

    CKMECH 1
    CONST <R> <p0>
    ELEMENTS <n>            then n lines: E <name> <W kg/mol>
    SPECIES <n>             then n lines:
        S <name> <W> <ncomp> (<elem> <count>)* <Tlow> <Tmid> <Thigh> <a_low x7> <a_high x7>
    REACTIONS <n>           then n lines:
        R <type> <rev> <nr> (<sp> <nu>)* <np> (<sp> <nu>)* <A> <beta> <Ea>
          [<A0> <beta0> <Ea0>]        (type 2 Lindemann, 3 Troe)
          [<a> <T3> <T1> <T2>]        (type 3 Troe)
          <neff> (<sp> <alpha>)*      (efficiencies, types 1-3; 0 for type 0)
    END

Reaction types: 0 elementary, 1 third-body, 2 Lindemann fall-off, 3 Troe
fall-off.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

R_GAS = 8.314462618          # J/(mol K)
P0 = 101325.0                # Pa
ATM = 101325.0

ELEMENT_W = {"H": 1.008e-3, "C": 12.011e-3, "N": 14.007e-3, "O": 15.999e-3}

T_LOW, T_MID, T_HIGH = 200.0, 1000.0, 6000.0
T_REF = 298.15


@dataclass
class Species:
    name: str
    comp: dict                 # element -> count
    W: float
    a_low: np.ndarray          # 7 NASA coefficients on [T_LOW, T_MID]
    a_high: np.ndarray         # 7 NASA coefficients on [T_MID, T_HIGH]
    hf298: float = 0.0         # J/mol (construction data, kept for tests)
    s298: float = 0.0          # J/(mol K)
    model: tuple = ()          # (c0, thetas) of the smooth cp model


@dataclass
class Reaction:
    type: int                  # 0 elementary, 1 third-body, 2 Lindemann, 3 Troe
    rev: int
    reac: list                 # [(species index, nu)]
    prod: list
    arr: tuple                 # (A [SI], beta, Ea [J/mol])
    low: tuple = ()            # fall-off low-pressure Arrhenius (A0, beta0, Ea0)
    troe: tuple = ()           # (a, T3, T1, T2)
    eff: list = field(default_factory=list)   # [(species index, alpha)]


@dataclass
class Mechanism:
    elements: list
    species: list
    reactions: list

    @property
    def n_species(self):
        return len(self.species)

    @property
    def n_reactions(self):
        return len(self.reactions)


# Mechanism recipes (species count, reaction count, third-body, Troe, elements, seed)
MECHS = {
    "M13": dict(nsp=13, nrxn=27, n_tb=4, n_troe=2, elements="HON", max_atoms=7, max_c=2, seed=13),
    "M53": dict(nsp=53, nrxn=325, n_tb=30, n_troe=25, elements="CHON", max_atoms=7, max_c=2, seed=53),
    "M111": dict(nsp=111, nrxn=784, n_tb=60, n_troe=40, elements="CHON", max_atoms=9, max_c=3, seed=111),
    # test-only: many reactions per species (duplicates allowed), so the wavefront kernel's
    # per-reaction scalars of the first Jacobian window do not fit its parking slice and the
    # second window recomputes them
    "M35X": dict(nsp=35, nrxn=900, n_tb=20, n_troe=10, elements="CHON", max_atoms=7, max_c=2, seed=35, dup=True),
    # test-only: N = 71 is not a multiple of 8 or 16, so the N > 64 kernels carry padding rows
    # and columns (and the tile form has five tile rows: uneven ownership over four wavefronts)
    "M70": dict(nsp=70, nrxn=420, n_tb=36, n_troe=24, elements="CHON", max_atoms=8, max_c=3, seed=70),
    # test-only: the largest sizes of each kernel family, N = 64 (one reactor per wavefront, every
    # lane a matrix row) and N = 128 (the four-wavefront workgroup kernels: eight tile rows)
    "M63": dict(nsp=63, nrxn=380, n_tb=34, n_troe=26, elements="CHON", max_atoms=8, max_c=3, seed=63),
    "M127": dict(nsp=127, nrxn=900, n_tb=64, n_troe=40, elements="CHON", max_atoms=9, max_c=3, seed=127),
}


# --------------------------------------------------------------------------------------
# species
# --------------------------------------------------------------------------------------
def _formula_name(comp, elements):
    s = ""
    for e in elements:
        c = comp.get(e, 0)
        if c == 1:
            s += e
        elif c > 1:
            s += f"{e}{c}"
    return s


def _draw_species(rng, elements, nsp, max_atoms, max_c):
    forced = []
    for e in elements:
        forced.append({e: 1})
    for e in elements:
        forced.append({e: 2})
    comps = []
    seen = set()
    for c in forced:
        key = tuple(c.get(e, 0) for e in elements)
        seen.add(key)
        comps.append(c)
    # every other candidate formula
    ranges = [range(0, (max_c if e == "C" else 3) + 1) for e in elements]
    cand = []
    for key in np.ndindex(*[len(r) for r in ranges]):
        tot = sum(key)
        if tot < 1 or tot > max_atoms or key in seen:
            continue
        cand.append(key)
    order = rng.permutation(len(cand))
    for i in order:
        if len(comps) >= nsp:
            break
        key = cand[i]
        seen.add(key)
        comps.append({e: int(k) for e, k in zip(elements, key) if k})
    if len(comps) < nsp:
        raise ValueError("element set too small for the requested species count")
    return comps[:nsp]


def _einstein_cp(x):
    # x = theta/T; cp contribution of one harmonic mode in units of R
    ex = np.exp(-x)
    return x * x * ex / (1.0 - ex) ** 2


def _einstein_h(theta, T):
    # vibrational energy of one mode / R  (K)
    return theta / np.expm1(theta / T)


def _einstein_s(theta, T):
    x = theta / T
    return x / np.expm1(x) - np.log(-np.expm1(-x))


def _smooth_thermo(c0, thetas, hf, s298, T):
    """cp/R, H/R (K), S/R of the smooth model at temperatures T (array)."""
    T = np.asarray(T, dtype=np.float64)
    cp = c0 + np.zeros_like(T) + sum(_einstein_cp(th / T) for th in thetas)
    h = hf / R_GAS + c0 * (T - T_REF) + sum(_einstein_h(th, T) - _einstein_h(th, T_REF) for th in thetas)
    s = s298 / R_GAS + c0 * np.log(T / T_REF) + sum(_einstein_s(th, T) - _einstein_s(th, T_REF) for th in thetas)
    return cp, h, s


def _nasa_fit(c0, thetas, hf, s298):
    """Constrained least-squares NASA-7 fit of the smooth model (14 unknowns).

    Rows: cp/R, H/(R T_s) and S/R samples on each range; equality constraints
    at T_MID for cp, dcp/dT, H and S.  The columns are the NASA-7 basis, i.e.
    the meaning the file format gives to the coefficients.
    """
    def rows(T):
        one = np.ones_like(T)
        z = np.zeros_like(T)
        cp = np.stack([one, T, T**2, T**3, T**4, z, z], 1)
        h = np.stack([one, T / 2, T**2 / 3, T**3 / 4, T**4 / 5, 1 / T, z], 1)     # H/(R T)
        s = np.stack([np.log(T), T, T**2 / 2, T**3 / 3, T**4 / 4, z, one], 1)
        return cp, h, s

    blocks, rhs = [], []
    for lo, hi, off in ((T_LOW, T_MID, 0), (T_MID, T_HIGH, 7)):
        T = np.linspace(lo, hi, 60)
        cp_t, h_t, s_t = _smooth_thermo(c0, thetas, hf, s298, T)
        bc, bh, bs = rows(T)
        for b, y, w in ((bc, cp_t, 1.0), (bh, h_t / T, 1.0), (bs, s_t, 1.0)):
            m = np.zeros((len(T), 14))
            m[:, off:off + 7] = b * w
            blocks.append(m)
            rhs.append(y * w)
    A = np.concatenate(blocks)
    b = np.concatenate(rhs)
    # column scaling for conditioning
    scale = np.array([1.0, 1e-3, 1e-6, 1e-9, 1e-12, 1e4, 1.0] * 2)
    A = A / scale   # A @ (x*scale) with x' = x*scale  ->  x = x'/scale ... handled below
    # constraints at T_MID
    Tm = np.array([T_MID])
    bc, bh, bs = rows(Tm)
    dcp = np.array([[0.0, 1.0, 2 * T_MID, 3 * T_MID**2, 4 * T_MID**3, 0.0, 0.0]])
    C = np.zeros((4, 14))
    for r, vec in enumerate((bc, dcp, bh, bs)):
        C[r, 0:7] = vec[0]
        C[r, 7:14] = -vec[0]
    C = C / scale
    # KKT system
    K = np.zeros((18, 18))
    K[:14, :14] = A.T @ A
    K[:14, 14:] = C.T
    K[14:, :14] = C
    f = np.zeros(18)
    f[:14] = A.T @ b
    sol = np.linalg.solve(K, f)
    x = sol[:14] / scale
    return x[:7].copy(), x[7:].copy()


def _make_species(rng, elements, comps, hf_range, s_range):
    out = []
    for comp in comps:
        n_atoms = sum(comp.values())
        if n_atoms == 1:
            c0, nvib = 2.5, 0
        elif n_atoms == 2:
            c0, nvib = 3.5, 1
        else:
            c0, nvib = 4.0, 3 * n_atoms - 6
        thetas = tuple(float(t) for t in rng.uniform(500.0, 3000.0, size=nvib))
        hf = float(rng.uniform(*hf_range))
        s298 = float(rng.uniform(*s_range))
        a_lo, a_hi = _nasa_fit(c0, thetas, hf, s298)
        W = sum(ELEMENT_W[e] * c for e, c in comp.items())
        out.append(Species(_formula_name(comp, elements), dict(comp), W, a_lo, a_hi, hf, s298, (c0, thetas)))
    return out


# --------------------------------------------------------------------------------------
# reactions
# --------------------------------------------------------------------------------------
def _candidates(comps, elements):
    vec = [tuple(c.get(e, 0) for e in elements) for c in comps]
    index = {v: i for i, v in enumerate(vec)}
    n = len(vec)
    exch, comb = set(), set()
    for a in range(n):
        for b in range(a, n):
            tot = tuple(x + y for x, y in zip(vec[a], vec[b]))
            c = index.get(tot)
            if c is not None:
                comb.add(((a, b), (c,)))
            for c in range(n):
                rest = tuple(x - y for x, y in zip(tot, vec[c]))
                if min(rest) < 0:
                    continue
                d = index.get(rest)
                if d is None or d < c:
                    continue
                if (c, d) == (a, b):
                    continue
                key = tuple(sorted([(a, b), (c, d)]))
                exch.add(key)
    return sorted(exch), sorted(comb)


def _stoich(side):
    out = {}
    for s in side:
        out[s] = out.get(s, 0) + 1
    return sorted(out.items())


def _arrhenius(rng, order):
    A_cgs = 10.0 ** rng.uniform(6.0, 14.0)
    beta = float(rng.uniform(-1.0, 2.0))
    Ea = float(rng.uniform(0.0, 2.0e5))
    return (A_cgs * (1e-6) ** (order - 1), beta, Ea)


def _orient(species, left, right, t_ref=1200.0):
    # Drawn formation data only (no NASA evaluation): favoured direction at t_ref.
    dg = 0.0
    for s in right:
        dg += species[s].hf298 - t_ref * species[s].s298
    for s in left:
        dg -= species[s].hf298 - t_ref * species[s].s298
    return (left, right) if dg <= 0.0 else (right, left)


def _build_reactions(rng, species, elements, nrxn, n_tb, n_troe, dup=False):
    comps = [s.comp for s in species]
    exch, comb = _candidates(comps, elements)
    nsp = len(species)
    if len(comb) < n_tb + n_troe:
        raise ValueError("not enough combination candidates for fall-off/third-body reactions")
    comb_idx = rng.permutation(len(comb))
    fall = [comb[i] for i in comb_idx[: n_tb + n_troe]]
    used = set(fall)
    pool = [r for r in exch + comb if r not in used]
    pool = [pool[i] for i in rng.permutation(len(pool))]
    n_elem = nrxn - n_tb - n_troe
    chosen = []
    covered = set()
    for left, right in fall:
        covered.update(left)
        covered.update(right)
    # first cover every species, then fill at random
    for r in pool:
        if len(chosen) >= n_elem:
            break
        sp = set(r[0]) | set(r[1])
        if not sp <= covered:
            chosen.append(r)
            covered |= sp
    for r in pool:
        if len(chosen) >= n_elem:
            break
        if r not in chosen:
            chosen.append(r)
    if dup:
        # duplicate reactions (same stoichiometry, own rate expression), as real mechanisms have
        k = 0
        while len(chosen) < n_elem and pool:
            chosen.append(pool[k % len(pool)])
            k += 1
    if len(chosen) < n_elem or len(covered) < nsp:
        raise ValueError("candidate pool too small")
    reactions = []
    kinds = [1] * n_tb + [3] * n_troe
    for kind, (left, right) in zip(kinds, fall):
        left, right = _orient(species, left, right)
        reac, prod = _stoich(left), _stoich(right)
        order = sum(nu for _, nu in reac)
        neff = int(rng.integers(0, 4))
        eff_sp = rng.choice(nsp, size=neff, replace=False)
        eff = [(int(s), float(rng.uniform(0.3, 5.0))) for s in sorted(eff_sp)]
        if kind == 1:
            reactions.append(Reaction(1, 1, reac, prod, _arrhenius(rng, order + 1), eff=eff))
        else:
            hi = _arrhenius(rng, order)
            lo = _arrhenius(rng, order + 1)
            troe = (float(rng.uniform(0.0, 1.0)), float(10 ** rng.uniform(1.0, 3.0)),
                    float(10 ** rng.uniform(math.log10(500.0), math.log10(5000.0))),
                    float(10 ** rng.uniform(math.log10(2000.0), 4.0)))
            reactions.append(Reaction(3, 1, reac, prod, hi, low=lo, troe=troe, eff=eff))
    for left, right in chosen:
        left, right = _orient(species, left, right)
        reac, prod = _stoich(left), _stoich(right)
        order = sum(nu for _, nu in reac)
        reactions.append(Reaction(0, 1, reac, prod, _arrhenius(rng, order)))
    # interleave types in a seeded order
    perm = rng.permutation(len(reactions))
    return [reactions[i] for i in perm]


def stoich_matrix(mech):
    """Net stoichiometric matrix nu'' - nu' (species x reactions), integers."""
    nu = np.zeros((mech.n_species, mech.n_reactions), dtype=np.int64)
    for i, r in enumerate(mech.reactions):
        for s, v in r.reac:
            nu[s, i] -= v
        for s, v in r.prod:
            nu[s, i] += v
    return nu


def element_matrix(mech):
    E = np.zeros((len(mech.elements), mech.n_species), dtype=np.int64)
    for k, s in enumerate(mech.species):
        for e, c in s.comp.items():
            E[mech.elements.index(e), k] = c
    return E


def make_mechanism(name="M13", seed=None, hf_range=(-150e3, 150e3), s_range=(150.0, 350.0)):
    p = dict(MECHS[name])
    dup = p.pop("dup", False)
    seed = p.pop("seed") if seed is None else seed
    elements = list(p["elements"])
    for attempt in range(50):
        rng = np.random.default_rng([seed, attempt])
        comps = _draw_species(rng, elements, p["nsp"], p["max_atoms"], p["max_c"])
        species = _make_species(rng, elements, comps, hf_range, s_range)
        try:
            reactions = _build_reactions(rng, species, elements, p["nrxn"], p["n_tb"], p["n_troe"], dup)
        except ValueError:
            continue
        mech = Mechanism(elements, species, reactions)
        nu = stoich_matrix(mech)
        E = element_matrix(mech)
        if np.linalg.matrix_rank(nu) == mech.n_species - np.linalg.matrix_rank(E):
            return mech
    raise RuntimeError("could not draw a mechanism with full stoichiometric rank")


def write_mechanism(mech, path):
    lines = ["CKMECH 1", f"CONST {R_GAS!r} {P0!r}", f"ELEMENTS {len(mech.elements)}"]
    for e in mech.elements:
        lines.append(f"E {e} {ELEMENT_W[e]!r}")
    lines.append(f"SPECIES {mech.n_species}")
    for s in mech.species:
        comp = " ".join(f"{mech.elements.index(e)} {c}" for e, c in sorted(s.comp.items(), key=lambda t: mech.elements.index(t[0])))
        a = " ".join(repr(float(v)) for v in list(s.a_low) + list(s.a_high))
        lines.append(f"S {s.name} {s.W!r} {len(s.comp)} {comp} {T_LOW!r} {T_MID!r} {T_HIGH!r} {a}")
    lines.append(f"REACTIONS {mech.n_reactions}")
    for r in mech.reactions:
        f = [f"R {r.type} {r.rev} {len(r.reac)}"]
        f += [f"{s} {v}" for s, v in r.reac]
        f.append(str(len(r.prod)))
        f += [f"{s} {v}" for s, v in r.prod]
        f.append(" ".join(repr(float(v)) for v in r.arr))
        if r.type in (2, 3):
            f.append(" ".join(repr(float(v)) for v in r.low))
        if r.type == 3:
            f.append(" ".join(repr(float(v)) for v in r.troe))
        if r.type != 0:
            f.append(str(len(r.eff)))
            f += [f"{s} {a!r}" for s, a in r.eff]
        lines.append(" ".join(f))
    lines.append("END")
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    os.replace(tmp, path)


def mechanism_file(name, directory=None):
    """Path of the named synthetic mechanism, generated on first use."""
    if directory is None:
        directory = os.environ.get("CK_MECH_DIR", os.path.join(os.path.dirname(os.path.abspath(__file__)), "_mech"))
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, f"{name}.ckm")
    if not os.path.exists(path):
        write_mechanism(make_mechanism(name), path)
    return path


# --------------------------------------------------------------------------------------
# reactor states
# --------------------------------------------------------------------------------------
# Workload recipes; each draws T0, P and Y0 from seeded distributions.
STATE_RECIPES = {
    # small: 1 atm, T0 U(1000,1500), Y0 Dirichlet(1)
    "small": dict(T=((1000.0, 1500.0),), P=(1.0, 1.0), alpha=1.0),
    # mid: T0 U(900,1800), P U(1,20) atm, Y0 Dirichlet(0.5)
    "mid": dict(T=((900.0, 1800.0),), P=(1.0, 20.0), alpha=0.5),
    # batching: half hot U(1400,1800), half cold U(600,900), interleaved by a seeded permutation
    "divergent": dict(T=((1400.0, 1800.0), (600.0, 900.0)), P=(1.0, 20.0), alpha=0.5),
}


def reactor_states(nsp, n, recipe="mid", seed=1002):
    """Return (y, P): y is SoA float64 [N][n] with row 0 = T and rows 1.. = Y_k; P [n] in Pa."""
    spec = STATE_RECIPES[recipe]
    rng = np.random.default_rng(seed)
    bands = spec["T"]
    if len(bands) == 1:
        T = rng.uniform(bands[0][0], bands[0][1], size=n)
    else:
        half = n // 2
        T = np.concatenate([rng.uniform(*bands[0], size=half), rng.uniform(*bands[1], size=n - half)])
        T = T[rng.permutation(n)]
    lo, hi = spec["P"]
    P = ATM * (rng.uniform(lo, hi, size=n) if hi > lo else np.full(n, lo))
    Y = rng.dirichlet(np.full(nsp, spec["alpha"]), size=n)
    y = np.empty((nsp + 1, n), dtype=np.float64)
    y[0] = T
    y[1:] = Y.T
    return np.ascontiguousarray(y), P.astype(np.float64)


def rhs_states(nsp, n, seed):
    """States for RHS-only throughput batches (same distribution as 'mid')."""
    return reactor_states(nsp, n, "mid", seed)


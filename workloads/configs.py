"""The five benchmark workloads as seeded synthetic inputs, plus scaled-down
variants of the same recipes for tests.

Recipes (shared by the oracle and the GPU path; see also the module doc of
``workloads.trees``):

* ``c1``: 4096 identical cells, full binary branch tree of 15 branches x 5
  compartments (75 unknowns); a ~ U(0.5, 2), c ~ U(0.1, 1), rhs ~ N(0, 1);
  seed 0; one solve.
* ``c2``: 65,536 random cells, seed 1.  Per cell a branch budget
  B ~ U{16..256}; tips split with probability 1/2 per round while the count
  stays <= B; branch length min(Geom(1/12), 64); a = 10**U(-2,2) r_b**2 with
  r_b ~ U(0.2, 2) per branch; c = sigma_c_m/dt, sigma_c_m ~ U(0.1, 1),
  dt = 0.025; rhs ~ N(0, 1).
* ``c3``: 200,000 cells, seed 2, sizes 50/500/5000/20000 compartments drawn
  with weights 0.4/0.3/0.2/0.1 (size-targeted growth), values as c2; the time
  loop draws I^k_i = 0.1 Z(seed 3, k, i) on each side from its own
  Philox4x32-10 generator.
* ``c4``: the c2 cells and sigma_c_m draws at dt in {0.001, 0.025, 1.0}.
* ``c5``: 16,384 cells of 1000 compartments, seed 4; values as c2 (dt 0.025);
  I_i ~ N(0, 0.1**2) constant; target_c ~ N(0, 1); 100 steps.

``scale`` < 1 keeps the recipe and shrinks the number of cells.
"""
from __future__ import annotations

import numpy as np

from .trees import CableSystem, Forest, cable_values, full_binary_forest, grow_random_forest

C1_CELLS = 4096
C2_CELLS = 65536
C3_CELLS = 200_000
C5_CELLS = 16_384
C3_SIZES = np.array([50, 500, 5000, 20000], dtype=np.int64)
C3_WEIGHTS = np.array([0.4, 0.3, 0.2, 0.1])


def _rngs(seed: int, k: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(k)]


def c1(ncells: int = C1_CELLS, seed: int = 0) -> CableSystem:
    f = full_binary_forest(ncells, 4, 5)
    rng = np.random.Generator(np.random.PCG64(seed))
    s = cable_values(f, rng, a_kind="uniform")
    s.meta["name"] = "c1"
    return s


def c2_forest(ncells: int = C2_CELLS, seed: int = 1) -> tuple[Forest, np.random.Generator]:
    rt, rv = _rngs(seed, 2)
    budget = rt.integers(16, 257, size=ncells)
    f = grow_random_forest(rt, ncells, max_branches=budget)
    return f, rv


def c2(ncells: int = C2_CELLS, seed: int = 1, dt: float = 0.025) -> CableSystem:
    f, rv = c2_forest(ncells, seed)
    s = cable_values(f, rv, a_kind="cable", dt=dt)
    s.meta["name"] = "c2"
    return s


def c4(dts=(0.001, 0.025, 1.0), ncells: int = C2_CELLS, seed: int = 1) -> dict:
    """The c2 morphology and draws, assembled at several time steps."""
    f, rv = c2_forest(ncells, seed)
    base = cable_values(f, rv, a_kind="cable", dt=0.025)
    out = {}
    for dt in dts:
        c = base.meta["sigma_cm"] / dt
        diag = c + base.a + np.bincount(f.parent[f.parent >= 0], weights=base.a[f.parent >= 0],
                                        minlength=f.n)
        out[dt] = CableSystem(f, base.a, c, diag, base.upper, base.rhs,
                              {"a_kind": "cable", "dt": dt, "name": "c4"})
    return out


def c3_sizes(ncells: int = C3_CELLS, seed: int = 2) -> np.ndarray:
    rt = _rngs(seed, 3)[2]
    return C3_SIZES[rt.choice(4, size=ncells, p=C3_WEIGHTS)]


def c3(ncells: int = C3_CELLS, seed: int = 2) -> CableSystem:
    rt, rv, _ = _rngs(seed, 3)
    sizes = c3_sizes(ncells, seed)
    f = grow_random_forest(rt, ncells, target_size=sizes)
    s = cable_values(f, rv, a_kind="cable", dt=0.025, rhs=False)
    s.meta.update(name="c3", sizes=sizes, noise_seed=3, noise_sigma=0.1)
    return s


def c5(ncells: int = C5_CELLS, seed: int = 4, size: int = 1000) -> CableSystem:
    rt, rv, rx = _rngs(seed, 3)
    f = grow_random_forest(rt, ncells, target_size=np.full(ncells, size, dtype=np.int64))
    s = cable_values(f, rv, a_kind="cable", dt=0.025, rhs=False)
    s.meta.update(name="c5", I=0.1 * rx.standard_normal(f.n), target=rx.standard_normal(ncells),
                  steps=100, checkpoint_every=10)
    return s


def random_system(n_cells: int, seed: int, *, small: bool = True) -> CableSystem:
    """Small random forests (branch budget U{1..24}) for tests."""
    rt, rv = _rngs(seed, 2)
    budget = rt.integers(1, 25 if small else 257, size=n_cells)
    f = grow_random_forest(rt, n_cells, max_branches=budget, mean_len=4.0 if small else 12.0,
                           max_len=16 if small else 64)
    return cable_values(f, rv, a_kind="cable", dt=0.025)

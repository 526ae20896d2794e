"""The paper-style tree generator (levels, split probability, lengths
shrinking away from the soma): closed forms at p = 0 and p = 1, the
numbering every generator promises, and a cell-lane replay on such trees
against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from workloads import cable_values, grow_level_forest

from test_cell_lanes import _check


def lens(levels, len0=40, decay=0.8):
    return [max(1, int(round(len0 * decay ** l))) for l in range(levels)]


def test_full_binary_at_p1_and_chain_at_p0():
    f = grow_level_forest(np.random.default_rng(0), 5, levels=6, p_split=1.0)
    L = lens(6)
    assert f.n == 5 * sum(2 ** l * L[l] for l in range(6))
    assert len(f.branch_offsets) - 1 == 5 * (2 ** 6 - 1)
    g = grow_level_forest(np.random.default_rng(0), 7, levels=6, p_split=0.0)
    assert g.n == 7 * sum(L)
    # one chain per cell: every compartment but the root hangs off its predecessor
    roots = g.cell_offsets[:-1]
    inner = np.setdiff1d(np.arange(g.n), roots)
    assert np.all(g.parent[inner] == inner - 1) and np.all(g.parent[roots] == -1)


@pytest.mark.parametrize("p", [0.25, 0.6])
def test_numbering_and_level_lengths(p):
    f = grow_level_forest(np.random.default_rng(3), 40, levels=7, p_split=p)
    i = np.arange(f.n)
    assert np.all(f.parent < i)
    bo = f.branch_offsets
    starts = bo[:-1]
    inner = np.setdiff1d(i, starts)
    assert np.all(f.parent[inner] == inner - 1)  # branches are consecutive
    assert np.all(np.isin(f.cell_offsets[:-1], starts))
    # branch length is a function of its level: level = number of branch ancestors
    L = lens(7)
    bid = np.searchsorted(bo, i, side="right") - 1
    lev = np.zeros(len(starts), dtype=np.int64)
    for b in range(len(starts)):
        pa = f.parent[starts[b]]
        lev[b] = 0 if pa < 0 else lev[bid[pa]] + 1
    assert np.all(np.diff(bo) == np.array(L)[lev])
    # every branch ends at a tip or has one or two children, all one level deeper
    nch = np.bincount(bid[f.parent[starts[lev > 0]]], minlength=len(starts))
    assert set(np.unique(nch[lev < 6])) <= {1, 2} and np.all(nch[lev == 6] == 0)


def test_cell_lane_replay_on_level_trees():
    f = grow_level_forest(np.random.default_rng(5), 70, levels=8, p_split=0.5)
    s = cable_values(f, np.random.default_rng(6), a_kind="cable", rhs=False)
    _check(f, s.diag, s.upper)
    # and the oracle itself is exact on one such cell against dense LU
    c0 = f.subset(np.array([0]))
    A = np.zeros((c0.n, c0.n))
    d = s.diag[: c0.n]
    u = s.upper[: c0.n]
    A[np.arange(c0.n), np.arange(c0.n)] = d
    for k in range(1, c0.n):
        A[k, c0.parent[k]] = A[c0.parent[k], k] = u[k]
    rhs = np.random.default_rng(7).standard_normal(c0.n)
    assert np.allclose(oracle.solve(c0, d, u, rhs), np.linalg.solve(A, rhs), rtol=1e-12, atol=1e-13)

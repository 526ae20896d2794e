"""Setup tables (paper §4-§6): the library's C++ builder against the plain
Python builder in the oracle, bit for bit, plus invariants that pin the
Python builder itself (identity numbering, re-root optimality by brute force,
bijections, level structure, packing limits, the Fig 4.1 toy).  CPU only: the
library is loaded but no device call is made (host_only plans)."""
import itertools
from collections import deque

import numpy as np
import pytest

from oracle import tables as otab
from workloads import Forest, configs, full_binary_forest

OPTION_SETS = [
    dict(),
    dict(split_branches=1),
    dict(rebalance_root=1),
    dict(rebalance_root=1, split_branches=1),
    dict(cell_order=1, max_group_unknowns=900),
    dict(group_width=128, max_group_unknowns=0),
    dict(rebalance_root=1, split_branches=1, cell_order=1, group_width=256, max_group_unknowns=3000),
    dict(split_branches=2),
    dict(level_balance=1, max_group_unknowns=0),
    dict(split_branches=2, level_balance=1, cell_order=1, max_group_unknowns=6000),
    dict(rebalance_root=1, split_branches=2, level_balance=1, group_width=128, max_group_unknowns=0),
]


def lib_tables(f, branch_offsets="user", **opts):
    from paper_1810_12742_amd import Plan
    mg = opts.pop("max_group_unknowns", 2048)
    bo = f.branch_offsets if branch_offsets == "user" else branch_offsets
    p = Plan(f.parent, f.cell_offsets, bo, host_only=True, max_group_unknowns=mg, **opts)
    # the paper's tables; the flow kernel's step schedule is checked by its replay test
    t = {k: v for k, v in p.tables().items() if not k.startswith(("flow_", "cell_", "res_", "seq_"))}
    p.close()
    return t


def py_tables(f, branch_offsets="user", **opts):
    mg = opts.pop("max_group_unknowns", 2048)
    bo = f.branch_offsets if branch_offsets == "user" else branch_offsets
    return otab.build(f.parent, f.cell_offsets, bo, max_group_unknowns=mg, **opts)


def assert_same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), k


FORESTS = {
    "c1": lambda: configs.c1(64).forest,
    "c2": lambda: configs.c2(96).forest,
    "small": lambda: configs.random_system(200, seed=11).forest,
    "c3": lambda: configs.c3(60).forest,
}


@pytest.mark.parametrize("name", list(FORESTS))
@pytest.mark.parametrize("opts", OPTION_SETS, ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()) or "default")
def test_library_tables_match_python_builder(name, opts):
    f = FORESTS[name]()
    assert_same(lib_tables(f, **dict(opts)), py_tables(f, **dict(opts)))


@pytest.mark.parametrize("opts", OPTION_SETS[:4])
def test_maximal_chain_branches_match(opts):
    f = configs.random_system(150, seed=4).forest
    assert_same(lib_tables(f, branch_offsets=None, **dict(opts)), py_tables(f, branch_offsets=None, **dict(opts)))


def _random_numbered_tree(rng, n):
    """A tree with parent[i] < i but not breadth-first numbered."""
    par = [-1] + [int(rng.integers(0, i)) for i in range(1, n)]
    return par


def test_arbitrary_parent_numbering_matches():
    rng = np.random.default_rng(3)
    parents = [_random_numbered_tree(rng, int(rng.integers(1, 40))) for _ in range(60)]
    sizes = [len(p) for p in parents]
    off = np.zeros(len(parents) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    par = np.concatenate([np.where(np.array(p) >= 0, np.array(p) + o, -1) for p, o in zip(parents, off[:-1])])
    f = Forest(par.astype(np.int32), off, np.arange(off[-1] + 1))
    for opts in OPTION_SETS[:4]:
        assert_same(lib_tables(f, branch_offsets=None, **dict(opts)), py_tables(f, branch_offsets=None, **dict(opts)))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_breadth_first_inputs_keep_identity_numbering(name):
    """Configs 1-2 are breadth-first numbered: without options the plan
    numbering is the identity and plan branches are the user branches."""
    f = FORESTS[name]()
    t = py_tables(f)
    assert np.array_equal(t["node_plan"], np.arange(f.n))
    br = t["branches"]
    assert np.array_equal(br[:, 2], f.branch_offsets[:-1])
    assert np.array_equal(br[:, 4], np.diff(f.branch_offsets))
    assert (br[:, 3] == 1).all()


def _check_invariants(f, t, T, balanced=False):
    n = f.n
    node_plan = t["node_plan"]
    br = t["branches"]
    # bijection inside each cell
    for c in range(f.ncells):
        lo, hi = f.cell_offsets[c], f.cell_offsets[c + 1]
        assert sorted(node_plan[lo:hi]) == list(range(lo, hi))
    # branch pieces cover every compartment exactly once, in tree-edge steps
    seen = np.zeros(n, dtype=int)
    for gid in range(br.shape[0]):
        cell, lvl, first, d, ln, pb, g, rank = br[gid]
        nodes = first + d * np.arange(ln)
        seen[nodes] += 1
        if pb >= 0:
            # a child runs at a deeper level than its parent; one deeper unless
            # level balancing moved its subtree
            assert br[pb, 0] == cell
            assert br[pb, 1] < lvl if balanced else br[pb, 1] == lvl - 1
        else:
            assert lvl == 0
    assert (seen == 1).all()
    # plan parent before child, u_src is the stored edge
    user_of = np.empty(n, dtype=np.int64)
    user_of[node_plan] = np.arange(n)
    par = f.parent
    for k in range(n):
        s = t["u_src"][k]
        i = user_of[k]
        if s < 0:
            continue
        assert s == i or par[s] == i
    # packing: per group and level at most T branches unless the group is one cell
    gofs, gcells = t["group_offsets"], t["group_cells"]
    assert sorted(gcells) == list(range(f.ncells))
    for g in range(len(gofs) - 1):
        cells = set(gcells[gofs[g]:gofs[g + 1]])
        m = np.isin(br[:, 0], list(cells))
        if len(cells) > 1:
            cnt = np.bincount(br[m, 1])
            assert cnt.max() <= T
    # lanes: per segment descending length
    lanes, seg = t["lanes"], t["seg_offsets"]
    assert sorted(lanes) == list(range(br.shape[0]))
    for s in range(len(seg) - 1):
        ln = br[lanes[seg[s]:seg[s + 1]], 4]
        assert (np.diff(ln) <= 0).all()


@pytest.mark.parametrize("opts", OPTION_SETS)
def test_table_invariants(opts):
    f = configs.random_system(120, seed=8).forest
    o = dict(opts)
    T = o.get("group_width", 64)
    _check_invariants(f, py_tables(f, **o), T, balanced=bool(o.get("level_balance")))


def _eccentricity(adj, v):
    dist = {v: 0}
    q = deque([v])
    while q:
        a = q.popleft()
        for b in adj[a]:
            if b not in dist:
                dist[b] = dist[a] + 1
                q.append(b)
    return max(dist.values())


def test_reroot_picks_tree_centre_bruteforce():
    """Re-rooting (§6) minimises the depth of the compartment tree: the new root
    has minimum eccentricity, the smaller user index on a tie."""
    s = configs.random_system(150, seed=13)
    f = s.forest
    t = py_tables(f, branch_offsets=None, rebalance_root=1)
    br = t["branches"]
    roots = br[br[:, 5] < 0]
    for c in range(f.ncells):
        lo, hi = f.cell_offsets[c], f.cell_offsets[c + 1]
        adj = {i: [] for i in range(lo, hi)}
        for i in range(lo + 1, hi):
            adj[i].append(int(f.parent[i]))
            adj[int(f.parent[i])].append(i)
        ecc = {i: _eccentricity(adj, i) for i in range(lo, hi)}
        best = min(ecc.values())
        want = min(i for i in ecc if ecc[i] == best)
        got = roots[roots[:, 0] == c][0, 2]
        assert got == want, (c, got, want)


def test_split_keeps_floor_average_and_bounds_lengths():
    f = configs.c2(64).forest
    t0 = py_tables(f)
    t1 = py_tables(f, split_branches=1)
    assert t1["branches"].shape[0] > t0["branches"].shape[0]
    assert t1["branches"][:, 4].sum() == f.n
    # level-0 branches never exceed the floor of the level-0 average of the input
    roots = t0["branches"][t0["branches"][:, 1] == 0, 4]
    cap = roots.sum() // len(roots)
    r1 = t1["branches"][t1["branches"][:, 1] == 0, 4]
    assert r1.max() <= max(cap, roots.min())


def test_fig41_toy_sort():
    """Fig 4.1: one block, 16 sub-matrices of up to five steps; after the
    per-level sort, lanes hold branches by descending length."""
    rng = np.random.default_rng(41)
    lens = rng.integers(1, 6, size=16)
    # a root branch with 16 children of the given lengths
    parents = [-1]
    first_child_parent = 0
    for ln in lens:
        start = len(parents)
        parents.append(first_child_parent)
        parents.extend(range(start, start + ln - 1))
    f = Forest(np.array(parents, dtype=np.int32), np.array([0, len(parents)], dtype=np.int64),
               np.arange(len(parents) + 1))
    t = py_tables(f, branch_offsets=None, group_width=64)
    br, lanes, seg = t["branches"], t["lanes"], t["seg_offsets"]
    lvl1 = br[lanes[seg[1]:seg[2]], 4]
    assert list(lvl1) == sorted(lens, reverse=True)


@pytest.mark.parametrize("case,code", [
    ("bad_first_offset", "BAD_OFFSETS"),
    ("empty_cell", "BAD_OFFSETS"),
    ("root_parent", "BAD_PARENT"),
    ("parent_after_child", "BAD_PARENT"),
    ("cross_cell_parent", "BAD_PARENT"),
    ("branch_not_chain", "BAD_BRANCHES"),
    ("branch_crosses_cell", "BAD_BRANCHES"),
    ("bad_group_width", "OPTION"),
])
def test_validation_errors(case, code):
    from paper_1810_12742_amd import HinesError, Plan
    f = full_binary_forest(3, 2, 3)
    par = f.parent.copy()
    off = f.cell_offsets.copy()
    bo = f.branch_offsets.copy()
    kw = {}
    if case == "bad_first_offset":
        off[0] = 1
    elif case == "empty_cell":
        off = np.array([0, 0, 9, 18, 27])
    elif case == "root_parent":
        par[9] = 3
    elif case == "parent_after_child":
        par[4] = 5
    elif case == "cross_cell_parent":
        par[10] = 2
    elif case == "branch_not_chain":
        bo = np.array([0, 5, 9, 12, 15, 18, 21, 24, 27])
    elif case == "branch_crosses_cell":
        bo = np.array([0, 3, 6, 10, 12, 15, 18, 21, 24, 27])
    elif case == "bad_group_width":
        kw["group_width"] = 100
    with pytest.raises(HinesError) as ei:
        Plan(par, off, bo, host_only=True, **kw)
    assert ei.value.code == code
    with pytest.raises(otab.SetupError) as ej:
        otab.build(par, off, bo, **kw)
    assert ej.value.code == code


def test_empty_forest():
    from paper_1810_12742_amd import Plan
    p = Plan(np.zeros(0, dtype=np.int32), np.zeros(1, dtype=np.int64), None, host_only=True)
    assert p.info["n"] == 0 and p.info["ngroups"] == 0
    t = p.tables()
    assert all(len(v) <= 1 for k, v in t.items() if k not in ("group_seg_offsets", "seg_offsets", "group_offsets"))


def test_single_compartment_cells():
    f = Forest(np.full(5, -1, dtype=np.int32), np.arange(6, dtype=np.int64), np.arange(6, dtype=np.int64))
    assert_same(lib_tables(f), py_tables(f))


def test_library_exports_every_declared_symbol():
    """Every function declared in include/hines.h is exported by libhines.so."""
    import ctypes
    import os
    import re
    from paper_1810_12742_amd import library_path, load
    load()
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hines.h")).read()
    names = sorted(set(re.findall(r"\b(hines_[a-z_0-9]+)\s*\(", hdr)))
    assert "hines_solve" in names and "hines_setup" in names
    lib = ctypes.CDLL(library_path())
    for nm in names:
        assert hasattr(lib, nm), nm


def test_setup_time_is_linear():
    """§6: the setup is linear in the number of neurons."""
    import time
    from paper_1810_12742_amd import Plan
    times = []
    for ncells in (2048, 8192):
        f = configs.c2(ncells).forest
        t0 = time.perf_counter()
        Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=True, split_branches=1).close()
        times.append((time.perf_counter() - t0) / f.n)
    assert times[1] < 2.5 * times[0]


def _forest_from_cells(cells):
    """Concatenate per-cell (parent list, branch starts) pairs into a Forest."""
    par, off, bo = [], [0], []
    for p, starts in cells:
        o = off[-1]
        par.extend(v + o if v >= 0 else -1 for v in p)
        bo.extend(s + o for s in starts)
        off.append(o + len(p))
    bo.append(off[-1])
    return Forest(np.array(par, dtype=np.int32), np.array(off, dtype=np.int64), np.array(bo, dtype=np.int64))


def _chain(parent_of_first, start, length):
    """Parents of a run of `length` compartments starting at `start`."""
    return [parent_of_first] + list(range(start, start + length - 1))


def test_split_rule_below_level_zero_hand_derived():
    """S5 worked by hand on two cells (section 6: the average is taken over the
    branches of one level of all cells, after the levels above were cut).

    Cell A: root branch of 2 (0-1), children of 6 (2-7) and 2 (8-9).
    Cell B: root branch of 4 (10-13), one child of 4 (14-17).
    Level 0: S = 6, m = 2, average 3: B's root (4 > 3) keeps 3; its tail
      (compartment 13) moves to level 1 and adopts B's child (now level 2).
    Level 1: A's 6, A's 2, B's tail 1: S = 9, m = 3, average 3: A's 6 keeps
      2-4, its tail 5-7 moves to level 2.
    Level 2: A's tail 3, B's child 4: S = 7, m = 2, floor 3: B's child keeps
      14-16, its tail 17 moves to level 3.
    Level 3: B's tail alone (1 = average): unchanged."""
    a = _chain(-1, 0, 2) + _chain(1, 2, 6) + _chain(1, 8, 2)
    b = _chain(-1, 0, 4) + _chain(3, 4, 4)
    f = _forest_from_cells([(a, [0, 2, 8]), (b, [0, 4])])
    t = py_tables(f, split_branches=1)
    br = t["branches"]
    got = sorted((int(r[0]), int(r[1]), int(r[2]), int(r[4])) for r in br)  # cell, level, first, len
    want = sorted([
        (0, 0, 0, 2), (0, 1, 2, 3), (0, 1, 8, 2), (0, 2, 5, 3),
        (1, 0, 10, 3), (1, 1, 13, 1), (1, 2, 14, 3), (1, 3, 17, 1),
    ])
    assert got == want
    # parents: each tail hangs under its kept piece, adopted children under the tail
    by_first = {int(r[2]): k for k, r in enumerate(br)}
    assert br[by_first[5], 5] == by_first[2]
    assert br[by_first[13], 5] == by_first[10]
    assert br[by_first[14], 5] == by_first[13]
    assert br[by_first[17], 5] == by_first[14]
    assert_same(lib_tables(f, split_branches=1), t)


def _star_cell(nkids):
    """A root compartment with nkids single-compartment child branches."""
    return ([-1] + [0] * nkids, list(range(nkids + 1)))


def test_packing_is_greedy_by_level_width():
    """S7 (section 4): a cell joins the open group whenever every level's
    branch count stays within the group width; only a cell that does not fit
    opens a new group.  Level-1 widths 40, 30, 20, 14, 50 with T = 64:
    {40}, {30, 20, 14} (64 fits exactly), {50}."""
    f = _forest_from_cells([_star_cell(k) for k in (40, 30, 20, 14, 50)])
    t = py_tables(f, branch_offsets=None, group_width=64, max_group_unknowns=0)
    assert list(t["group_offsets"]) == [0, 1, 4, 5]
    assert list(t["group_cells"]) == [0, 1, 2, 3, 4]
    assert_same(lib_tables(f, branch_offsets=None, group_width=64, max_group_unknowns=0), t)


def test_packing_is_greedy_by_compartment_cap():
    """S7 with a compartment cap of 10: sizes 4, 4, 4, 2, 7, 3 pack as
    {4, 4}, {4, 2}, {7, 3}; a cell that fits (the 3 after the 7) joins the
    open group instead of a later or a new one."""
    sizes = [4, 4, 4, 2, 7, 3]
    f = _forest_from_cells([(_chain(-1, 0, s), [0]) for s in sizes])
    t = py_tables(f, max_group_unknowns=10)
    assert list(t["group_offsets"]) == [0, 2, 4, 6]
    assert_same(lib_tables(f, max_group_unknowns=10), t)
    # descending sizes (cell_order 1) visit 7, 4, 4, 4, 3, 2: the open group
    # takes each cell that fits, giving {7}, {4, 4}, {4, 3, 2}
    t1 = py_tables(f, max_group_unknowns=10, cell_order=1)
    assert list(t1["group_cells"]) == [4, 0, 1, 2, 5, 3]
    assert list(t1["group_offsets"]) == [0, 1, 3, 6]
    assert_same(lib_tables(f, max_group_unknowns=10, cell_order=1), t1)


def test_split_per_group_averages_hand_derived():
    """S5' (the outlook, §8: per-block averages from an intermediate packing).
    The cells of the S5 example (A: 2 + {6, 2}; B: 4 + 4) packed with a cap of
    10 compartments form two groups, {A} and {B}.  Inside {A}: level 0 holds A's
    root alone (average 2, nothing to cut); level 1 holds 6 and 2 (S = 8, m = 2,
    average 4): the 6 keeps 4 (2-5), its tail 6-7 moves to level 2.  Inside {B}
    every level holds one branch: nothing is cut.  (The averages over all
    cells cut B's root instead.)"""
    a = _chain(-1, 0, 2) + _chain(1, 2, 6) + _chain(1, 8, 2)
    b = _chain(-1, 0, 4) + _chain(3, 4, 4)
    f = _forest_from_cells([(a, [0, 2, 8]), (b, [0, 4])])
    t = py_tables(f, split_branches=2, max_group_unknowns=10)
    got = sorted((int(r[0]), int(r[1]), int(r[2]), int(r[4])) for r in t["branches"])
    want = sorted([(0, 0, 0, 2), (0, 1, 2, 4), (0, 1, 8, 2), (0, 2, 6, 2), (1, 0, 10, 4), (1, 1, 14, 4)])
    assert got == want
    assert list(t["group_offsets"]) == [0, 1, 2]
    assert_same(lib_tables(f, split_branches=2, max_group_unknowns=10), t)
    # with one group (no cap) the per-group and the global averages agree
    assert_same(py_tables(f, split_branches=2, max_group_unknowns=0), py_tables(f, split_branches=1, max_group_unknowns=0))


def test_level_balance_moves_smallest_subtrees_down():
    """S7' (the outlook, §8: subtrees may move one level down to even out the
    level widths of a block).  The open group holds P, a root with 50 leaf
    branches on level 1.  Q is a root with 20 children on level 1, the first
    ten with one child each (level 2), the last ten leaves.  With T = 64, Q
    overflows level 1 by 6: the six leaf children of smallest breadth-first
    rank (Q's branches 11-16) move to level 2 and Q joins P's group
    (64 branches on level 1, 16 on level 2).  Without balancing Q opens a
    second group."""
    p_cell = _star_cell(50)
    q_par = [-1] + [0] * 20 + list(range(1, 11))
    q_cell = (q_par, list(range(31)))
    f = _forest_from_cells([p_cell, q_cell])
    t0 = py_tables(f, branch_offsets=None, group_width=64, max_group_unknowns=0)
    assert list(t0["group_offsets"]) == [0, 1, 2]
    t = py_tables(f, branch_offsets=None, group_width=64, max_group_unknowns=0, level_balance=1)
    assert list(t["group_offsets"]) == [0, 2]
    br = t["branches"]
    q = br[br[:, 0] == 1]
    moved = sorted(int(r[7]) for r in q if r[1] == 2 and f.parent[int(r[2])] == 51)  # children of Q's root on level 2
    assert moved == list(range(11, 17))
    assert np.bincount(br[:, 1]).tolist() == [2, 64, 16]
    # every branch stays deeper than its parent; lanes of a level run by length
    for r in br:
        if r[5] >= 0:
            assert r[1] > br[r[5], 1]
    assert_same(lib_tables(f, branch_offsets=None, group_width=64, max_group_unknowns=0, level_balance=1), t)

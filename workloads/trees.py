"""Seeded synthetic neuron-shaped forests and cable-equation coefficients.

This module only *draws inputs*: morphologies (a parent array, a user branch
layout and per-cell offsets) and the coefficient values of the implicit-Euler
cable system (paper §1, the discrete system following the cable equation).
It contains no step of the Hines solve.  Both the FP64 oracle and the GPU
library consume exactly the arrays produced here.

Numbering produced by every generator (paper §2): branches of a cell are
numbered breadth first from the root branch, children of one branch in the
order they were created, and the compartments of a branch are consecutive,
ordered by distance to the root.  Hence ``parent[i] < i`` and, inside a branch,
``parent[i] == i - 1``.  The root of each cell is its first compartment and
has ``parent == -1``.

Matrix convention (paper §1): ``a[i] > 0`` is the conductance of the edge
between compartment ``i`` and ``parent[i]`` (``a[root] = 0``), ``c[i] > 0`` is
sigma_i c_m,i / dt.  Then ``diag[i] = c[i] + a[i] + sum_{k: parent[k]=i} a[k]``,
``upper[i] = -a[i]`` is the signed off-diagonal entry A[i, parent[i]], and the
matrix is symmetric and strictly diagonally dominant.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Forest:
    parent: np.ndarray          # int32[n]; -1 at each cell root
    cell_offsets: np.ndarray    # int64[ncells + 1]
    branch_offsets: np.ndarray  # int64[nbranches + 1]; the user branch layout
    branch_radius: np.ndarray | None = None  # float64[nbranches] (random trees only)

    @property
    def n(self) -> int:
        return int(self.parent.shape[0])

    @property
    def ncells(self) -> int:
        return int(self.cell_offsets.shape[0] - 1)

    @property
    def nbranches(self) -> int:
        return int(self.branch_offsets.shape[0] - 1)

    def subset(self, cells) -> "Forest":
        """The forest made of the listed cells (ascending), renumbered densely."""
        cells = np.asarray(cells, dtype=np.int64)
        lo = self.cell_offsets[cells]
        hi = self.cell_offsets[cells + 1]
        sizes = hi - lo
        new_off = np.zeros(len(cells) + 1, dtype=np.int64)
        np.cumsum(sizes, out=new_off[1:])
        idx = _ranges(lo, sizes)
        shift = np.repeat(new_off[:-1] - lo, sizes)
        par = self.parent[idx].astype(np.int64)
        par = np.where(par >= 0, par + shift, -1).astype(np.int32)
        # branches whose first compartment lies in a chosen cell
        bo = self.branch_offsets[:-1]
        cell_of_branch = np.searchsorted(self.cell_offsets, bo, side="right") - 1
        keep = np.isin(cell_of_branch, cells)
        starts = bo[keep]
        cmap = np.full(self.ncells, -1, dtype=np.int64)
        cmap[cells] = np.arange(len(cells))
        starts = starts - self.cell_offsets[cell_of_branch[keep]] + new_off[cmap[cell_of_branch[keep]]]
        order = np.argsort(starts, kind="stable")
        new_bo = np.concatenate([starts[order], [new_off[-1]]]).astype(np.int64)
        rad = None if self.branch_radius is None else self.branch_radius[keep][order]
        return Forest(par, new_off, new_bo, rad)


@dataclass
class CableSystem:
    forest: Forest
    a: np.ndarray      # float64[n]: edge conductance to the parent (0 at roots)
    c: np.ndarray      # float64[n]: sigma c_m / dt
    diag: np.ndarray   # float64[n]
    upper: np.ndarray  # float64[n]: -a (A[i, parent[i]]); 0 at roots
    rhs: np.ndarray    # float64[n]
    meta: dict = field(default_factory=dict)


def _ranges(starts: np.ndarray, lengths: np.ndarray) -> np.ndarray:
    """Concatenation of arange(s, s + l) for each (s, l)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    offs = np.zeros(len(lengths), dtype=np.int64)
    np.cumsum(lengths[:-1], out=offs[1:])
    out = np.arange(total, dtype=np.int64)
    out -= np.repeat(offs - np.asarray(starts, dtype=np.int64), lengths)
    return out


def _layout(cell_of_branch, parent_branch, length, ncells) -> Forest:
    """Compartment arrays for branches given in final (cell-major BFS) order.

    ``parent_branch`` indexes the same order; roots have -1.
    """
    nb = len(length)
    boff = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(length, out=boff[1:])
    n = int(boff[-1])
    parent = np.arange(-1, n - 1, dtype=np.int64)
    first = boff[:-1]
    is_root = parent_branch < 0
    attach = np.where(is_root, -1, boff[np.maximum(parent_branch, 0) + 1] - 1)
    parent[first] = attach
    cell_sizes = np.bincount(cell_of_branch, weights=length, minlength=ncells).astype(np.int64)
    coff = np.zeros(ncells + 1, dtype=np.int64)
    np.cumsum(cell_sizes, out=coff[1:])
    return Forest(parent.astype(np.int32), coff, boff)


def full_binary_forest(ncells: int, branch_depth: int = 4, comp_per_branch: int = 5) -> Forest:
    """Identical cells, each a full binary branch tree of ``2**branch_depth - 1``
    branches (children of branch b are 2b+1 and 2b+2, already breadth first),
    every branch ``comp_per_branch`` compartments long."""
    nbr = (1 << branch_depth) - 1
    b = np.arange(nbr)
    pb = np.where(b == 0, -1, (b - 1) // 2)
    cells = np.repeat(np.arange(ncells), nbr)
    pbg = np.tile(pb, ncells) + np.where(np.tile(pb, ncells) >= 0, cells * nbr, 0)
    lengths = np.full(ncells * nbr, comp_per_branch, dtype=np.int64)
    return _layout(cells, pbg, lengths, ncells)


def _segment_rank(sorted_keys: np.ndarray, flags: np.ndarray) -> np.ndarray:
    """For keys sorted ascending, the running count of ``flags`` inside each run
    of equal keys (inclusive)."""
    cs = np.cumsum(flags.astype(np.int64))
    if len(sorted_keys) == 0:
        return cs
    starts = np.r_[True, sorted_keys[1:] != sorted_keys[:-1]]
    seg = np.cumsum(starts) - 1
    base = (cs - flags.astype(np.int64))[starts]
    return cs - base[seg]


def grow_random_forest(rng: np.random.Generator, ncells: int, *, max_branches=None,
                       target_size=None, mean_len: float = 12.0, max_len: int = 64) -> Forest:
    """Random binary dendritic trees.

    Growth happens in rounds.  In each round every current tip of a growing cell
    splits into two child branches with probability 1/2, visiting tips left to
    right.  Branch lengths are min(Geometric(1/mean_len), max_len) compartments.

    * ``max_branches`` (int array): a split is taken only while the cell keeps
      at most that many branches; the cell stops when no split fits.
    * ``target_size`` (int array): cells grow until their total length reaches
      the target; afterwards the branches, in creation order, are cut so that
      the total is exactly the target (the crossing branch is shortened, later
      ones are dropped).
    """
    assert (max_branches is None) != (target_size is None)
    p = 1.0 / mean_len

    def draw_len(k):
        return np.minimum(rng.geometric(p, size=k), max_len).astype(np.int64)

    bcell = [np.arange(ncells, dtype=np.int64)]
    bpar = [np.full(ncells, -1, dtype=np.int64)]
    blen = [draw_len(ncells)]
    bround = [np.zeros(ncells, dtype=np.int64)]
    nextid = ncells
    cnt = np.ones(ncells, dtype=np.int64)
    size = blen[0].copy()
    tip_cell = np.arange(ncells, dtype=np.int64)
    tip_id = np.arange(ncells, dtype=np.int64)
    rnd = 0
    while True:
        if max_branches is not None:
            active = cnt + 2 <= max_branches
        else:
            active = size < target_size
        if not active.any():
            break
        rnd += 1
        keep = active[tip_cell]
        tip_cell = tip_cell[keep]
        tip_id = tip_id[keep]
        coin = rng.random(len(tip_cell)) < 0.5
        if max_branches is not None:
            rank = _segment_rank(tip_cell, coin)
            accept = coin & (cnt[tip_cell] + 2 * rank <= max_branches[tip_cell])
        else:
            accept = coin
        k = int(accept.sum())
        if k == 0:
            continue
        par_ids = tip_id[accept]
        par_cells = tip_cell[accept]
        child_ids = nextid + np.arange(2 * k, dtype=np.int64)
        nextid += 2 * k
        clen = draw_len(2 * k)
        bcell.append(np.repeat(par_cells, 2))
        bpar.append(np.repeat(par_ids, 2))
        blen.append(clen)
        bround.append(np.full(2 * k, rnd, dtype=np.int64))
        cnt += 2 * np.bincount(par_cells, minlength=ncells)
        size += np.bincount(np.repeat(par_cells, 2), weights=clen, minlength=ncells).astype(np.int64)
        reps = np.where(accept, 2, 1)
        new_cell = np.repeat(tip_cell, reps)
        new_id = np.repeat(tip_id, reps)
        pos = np.cumsum(reps) - reps  # first output slot of each old tip
        acc_pos = pos[accept]
        new_id[acc_pos] = child_ids[0::2]
        new_id[acc_pos + 1] = child_ids[1::2]
        tip_cell, tip_id = new_cell, new_id

    cell = np.concatenate(bcell)
    par = np.concatenate(bpar)
    length = np.concatenate(blen)
    rounds = np.concatenate(bround)
    nb = len(cell)
    alive = np.ones(nb, dtype=bool)

    if target_size is not None:
        order = np.argsort(cell, kind="stable")  # per cell, creation order
        lo = length[order]
        cs = np.cumsum(lo)
        c_sorted = cell[order]
        starts = np.r_[True, c_sorted[1:] != c_sorted[:-1]]
        seg = np.cumsum(starts) - 1
        base = (cs - lo)[starts]
        within = cs - base[seg]          # inclusive running size inside the cell
        before = within - lo
        tgt = target_size[c_sorted]
        drop = before >= tgt
        cut = (within > tgt) & ~drop
        newlen = lo.copy()
        newlen[cut] = tgt[cut] - before[cut]
        length[order] = newlen
        alive[order[drop]] = False

    # levels: parents are created in earlier rounds, so one pass per round suffices
    level = np.zeros(nb, dtype=np.int64)
    for r in range(1, rnd + 1):
        m = rounds == r
        level[m] = level[par[m]] + 1

    ids = np.flatnonzero(alive)
    # breadth-first order: cell-major, then level, then parent position, then creation
    pos = np.full(nb, -1, dtype=np.int64)
    lvl_alive = level[ids]
    maxlev = int(lvl_alive.max()) if len(ids) else -1
    for ell in range(0, maxlev + 1):
        m = ids[lvl_alive == ell]
        if ell == 0:
            key = np.lexsort((m, cell[m]))
        else:
            key = np.lexsort((m, pos[par[m]]))
        pos[m[key]] = np.arange(len(m))
    final = ids[np.lexsort((pos[ids], level[ids], cell[ids]))]
    rank = np.full(nb, -1, dtype=np.int64)
    rank[final] = np.arange(len(final))
    pb = np.where(par[final] >= 0, rank[np.maximum(par[final], 0)], -1)
    forest = _layout(cell[final], pb, length[final], ncells)
    return forest


def grow_level_forest(rng: np.random.Generator, ncells: int, *, levels: int, p_split: float,
                      len0: int = 40, decay: float = 0.8) -> Forest:
    """Trees shaped like the paper's benchmark networks (§7): every cell has
    ``levels`` levels of branches; on each level every branch splits into two
    child branches with probability ``p_split`` and otherwise continues as a
    single branch on the next level; branches of level l have
    ``max(1, round(len0 * decay**l))`` compartments, so they get shorter away
    from the soma.  A full binary tree for ``p_split = 1``, one chain for 0."""
    lens = np.array([max(1, int(round(len0 * decay ** l))) for l in range(levels)], dtype=np.int64)
    cell = [np.arange(ncells, dtype=np.int64)]
    par = [np.full(ncells, -1, dtype=np.int64)]
    lev = [np.zeros(ncells, dtype=np.int64)]
    tip_id = np.arange(ncells, dtype=np.int64)
    tip_cell = np.arange(ncells, dtype=np.int64)
    nextid = ncells
    for l in range(1, levels):
        reps = np.where(rng.random(len(tip_id)) < p_split, 2, 1)
        new_par = np.repeat(tip_id, reps)
        new_cell = np.repeat(tip_cell, reps)
        ids = nextid + np.arange(len(new_par), dtype=np.int64)
        nextid += len(new_par)
        cell.append(new_cell)
        par.append(new_par)
        lev.append(np.full(len(new_par), l, dtype=np.int64))
        tip_id, tip_cell = ids, new_cell
    cell = np.concatenate(cell)
    par = np.concatenate(par)
    lev = np.concatenate(lev)
    nb = len(cell)
    # creation order inside a level is already breadth first per cell
    order = np.lexsort((np.arange(nb), lev, cell))
    rank = np.empty(nb, dtype=np.int64)
    rank[order] = np.arange(nb)
    pb = np.where(par[order] >= 0, rank[np.maximum(par[order], 0)], -1)
    return _layout(cell[order], pb, lens[lev[order]], ncells)


def cable_values(forest: Forest, rng: np.random.Generator, *, a_kind: str, dt: float = 0.025,
                 sigma_cm=None, rhs: bool = True) -> CableSystem:
    """Coefficients of the implicit-Euler cable system on ``forest``.

    ``a_kind``:
      * ``"uniform"``: a ~ U(0.5, 2.0), c ~ U(0.1, 1.0) (dt is ignored).
      * ``"cable"``: a = 10**U(-2, 2) * r_b**2 with the radius r_b of the
        child's branch, and c = sigma_c_m / dt with sigma_c_m ~ U(0.1, 1.0)
        unless ``sigma_cm`` is given.
    """
    par = forest.parent
    n = forest.n
    nonroot = par >= 0
    if a_kind == "uniform":
        a = rng.uniform(0.5, 2.0, size=n)
        c = rng.uniform(0.1, 1.0, size=n)
        scm = None
    elif a_kind == "cable":
        rad = forest.branch_radius
        nb = forest.nbranches
        if rad is None:
            rad = rng.uniform(0.2, 2.0, size=nb)
            forest.branch_radius = rad
        blen = np.diff(forest.branch_offsets)
        r_of = np.repeat(rad, blen)
        a = (10.0 ** rng.uniform(-2.0, 2.0, size=n)) * r_of * r_of
        scm = rng.uniform(0.1, 1.0, size=n) if sigma_cm is None else np.asarray(sigma_cm)
        c = scm / dt
    else:
        raise ValueError(a_kind)
    a = np.where(nonroot, a, 0.0)
    diag = c + a + np.bincount(par[nonroot], weights=a[nonroot], minlength=n)
    upper = -a
    b = rng.standard_normal(n) if rhs else np.zeros(n)
    return CableSystem(forest, a, c, diag, upper, b, {"a_kind": a_kind, "dt": dt, "sigma_cm": scm})


def assemble(forest: Forest, a: np.ndarray, c: np.ndarray):
    """diag and upper from edge conductances and capacitive terms (paper §1)."""
    par = forest.parent
    nonroot = par >= 0
    a = np.where(nonroot, a, 0.0)
    diag = c + a + np.bincount(par[nonroot], weights=a[nonroot], minlength=forest.n)
    return diag, -a

"""Setup tables of the fine-grained Hines solver, in plain Python.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is an independent
re-derivation of every table the GPU library's host-side setup builds, written
as plain loops over dictionaries and lists, used for bit-exact comparison.

Rules, in the order they run (paper sections in brackets):

S1 validate.  cell_offsets starts at 0, increases strictly, ends at n; a cell's
   first compartment is its root (parent -1); every other compartment i has
   cell_lo <= parent[i] < i  [§2: breadth-first numbering, parent before child].
   A user branch layout must start every cell with a branch, increase strictly,
   end at n, and have parent[i] == i-1 inside a branch.
S2 branches  [§1 Fig 1.1, §2, §5].  A compartment i continues the branch of
   q = parent(i) iff q has exactly one child, |i - q| == 1, the step i - q
   equals the direction of q's branch (when q is not the branch's first
   compartment), and no user branch starts at i.  So a branch is a run of
   consecutive user indices (direction +1, or -1 after re-rooting), and child
   branches always hang off the last compartment of their parent branch.
S3 re-root (option)  [§6 "balance the dependency tree"].  Per cell, the new
   root is the tree centre (minimum eccentricity; the smaller user index when
   there are two), found on a diameter path; edges are re-oriented away from
   it and any user branch layout is ignored.
S4 numbering  [§2, §6].  Branches breadth first from the root branch, the
   children of a branch by ascending user index of their first compartment;
   compartments by branch, then distance to the root.  The plan index of a
   compartment is the cell's first user index + the lengths of earlier
   branches + its position.
S5 split (option)  [§6 "split long branches", §5].  For level l = 0, 1, ...
   over all cells together: S = total length and m = count of level-l
   branches; each branch with len*m > S keeps its first floor(S/m)
   compartments, the rest becomes its only child one level down and adopts
   its children.  The numbering of S4 is then recomputed.
S5' per-group averages (split option 2)  [§8, the outlook: an intermediate
   packing gives local heuristics such as per-block averages].  The cells are
   first packed by S7 on the unsplit trees; then S5 runs inside each of these
   groups, with S and m taken over that group's level-l branches only; the
   final packing (S7) runs on the split trees.
S6 levels: root branch 0, child = parent + 1.
S7 packing  [§4].  Cells in input order (or by size, descending, stable); a
   cell joins the open group iff every level's branch count stays <= the
   group width T and, when a cap is set, the group's compartment count stays
   <= the cap; otherwise a new group opens.
S7' level balancing (option)  [§8, the outlook: let subtrees move one level
   down when that evens out the level widths of a block].  A cell that meets
   the cap but overflows some level of the open group is given a trial: while
   some level l overflows (the smallest such l), one of the cell's branches
   on level l (l > 0) moves down one level together with its whole subtree:
   the branch with the fewest branches in its subtree, then the smallest
   breadth-first rank.  If no level overflows after at most 4 x (branches of
   the cell) moves, the cell joins with the moved levels; otherwise it opens a
   new group with its own levels.  A branch's level then is its step in the
   level-synchronous sweeps (always deeper than its parent's), and S8 and the
   exported tables use it.
S8 lane order  [§4, Fig 4.1].  Inside (group, level): branches by descending
   length, ties by (cell, breadth-first rank in the cell).

Exported tables (the same names as the library's table ids):
  node_plan[n]        plan index of each user compartment
  branches[nb, 8]     per plan branch (cell-major, breadth first):
                      cell, level, first user index, dir, len, parent branch,
                      group, rank in cell
  u_src[n]            per plan index: the user index whose ``upper`` holds the
                      coupling to its plan parent (-1 for roots)
  group_offsets, group_cells   cells of each group, packing order
  group_seg_offsets, seg_offsets, lanes   per (group, level) segment the plan
                      branch ids in lane order
"""
from __future__ import annotations

from collections import deque

import numpy as np


class SetupError(Exception):
    def __init__(self, code: str, msg: str = ""):
        super().__init__(f"{code}: {msg}")
        self.code = code


def _validate(parent, cell_offsets, branch_offsets):
    n = len(parent)
    ncells = len(cell_offsets) - 1
    if ncells < 0:
        raise SetupError("BAD_OFFSETS", "no offsets")
    if cell_offsets[0] != 0 or cell_offsets[ncells] != n:
        raise SetupError("BAD_OFFSETS", "must start at 0 and end at n")
    for c in range(ncells):
        if cell_offsets[c + 1] <= cell_offsets[c]:
            raise SetupError("BAD_OFFSETS", "cells must be non-empty and increasing")
    for c in range(ncells):
        lo, hi = cell_offsets[c], cell_offsets[c + 1]
        if parent[lo] != -1:
            raise SetupError("BAD_PARENT", f"root {lo} must have parent -1")
        for i in range(lo + 1, hi):
            if not (lo <= parent[i] < i):
                raise SetupError("BAD_PARENT", f"parent[{i}]={parent[i]}")
    if branch_offsets is not None:
        nb = len(branch_offsets) - 1
        if nb < 1 and n > 0:
            raise SetupError("BAD_BRANCHES", "empty layout")
        if branch_offsets[0] != 0 or branch_offsets[nb] != n:
            raise SetupError("BAD_BRANCHES", "must start at 0 and end at n")
        starts = set()
        for k in range(nb):
            if branch_offsets[k + 1] <= branch_offsets[k]:
                raise SetupError("BAD_BRANCHES", "branches must be non-empty and increasing")
            starts.add(branch_offsets[k])
            for i in range(branch_offsets[k] + 1, branch_offsets[k + 1]):
                if parent[i] != i - 1:
                    raise SetupError("BAD_BRANCHES", f"parent[{i}] != {i - 1} inside a branch")
        for c in range(ncells):
            if cell_offsets[c] not in starts:
                raise SetupError("BAD_BRANCHES", f"cell {c} does not start a branch")
        return starts
    return None


def _centre(lo, hi, adj):
    def bfs(start):
        dist = {start: 0}
        prev = {start: -1}
        q = deque([start])
        while q:
            v = q.popleft()
            for w in adj[v]:
                if w not in dist:
                    dist[w] = dist[v] + 1
                    prev[w] = v
                    q.append(w)
        far = max(dist.values())
        node = min(v for v, dv in dist.items() if dv == far)
        return node, prev, far

    a, _, _ = bfs(lo)
    b, prev, D = bfs(a)
    path = [b]
    while path[-1] != a:
        path.append(prev[path[-1]])
    path.reverse()  # a ... b
    return min(path[D // 2], path[(D + 1) // 2])


class _Branch:
    __slots__ = ("cell", "first", "dir", "len", "parent", "children", "level", "rank", "gid")

    def __init__(self, cell, first, d, ln, parent):
        self.cell = cell
        self.first = first
        self.dir = d
        self.len = ln
        self.parent = parent
        self.children = []
        self.level = 0
        self.rank = -1
        self.gid = -1

    def node(self, j):
        return self.first + self.dir * j

    def last(self):
        return self.node(self.len - 1)


def _greedy_groups(cells, sizes, counts_of, T, cap):
    """S7 greedy packing by level counts (no level balancing)."""
    groups, cur, cur_cnt, cur_u = [], [], {}, 0
    for c in cells:
        fits = True
        if cur:
            for lvl, k in counts_of(c).items():
                if cur_cnt.get(lvl, 0) + k > T:
                    fits = False
            if cap and cur_u + sizes[c] > cap:
                fits = False
        if not fits:
            groups.append(cur)
            cur, cur_cnt, cur_u = [], {}, 0
        cur.append(c)
        for lvl, k in counts_of(c).items():
            cur_cnt[lvl] = cur_cnt.get(lvl, 0) + k
        cur_u += sizes[c]
    if cur:
        groups.append(cur)
    return groups


def _split_levels(level_list):
    """S5 on the branches reachable from level_list (the top level)."""
    while level_list:
        S = sum(b.len for b in level_list)
        m = len(level_list)
        nxt = []
        for b in level_list:
            if b.len * m > S:
                k = S // m
                t = _Branch(b.cell, b.node(k), b.dir, b.len - k, b)
                t.children = b.children
                for ch in t.children:
                    ch.parent = t
                b.children = [t]
                b.len = k
            nxt.extend(b.children)
        level_list = nxt


def build(parent, cell_offsets, branch_offsets=None, *, rebalance_root=0, split_branches=0,
          group_width=64, cell_order=0, max_group_unknowns=0, level_balance=0):
    parent = [int(v) for v in np.asarray(parent)]
    cell_offsets = [int(v) for v in np.asarray(cell_offsets)]
    bo = None if branch_offsets is None else [int(v) for v in np.asarray(branch_offsets)]
    if group_width < 1 or group_width > 1024 or group_width % 64:
        raise SetupError("OPTION", "group_width must be a multiple of 64 in [64, 1024]")
    if cell_order not in (0, 1) or max_group_unknowns < 0 or split_branches not in (0, 1, 2) \
            or level_balance not in (0, 1):
        raise SetupError("OPTION", "bad option")
    user_starts = _validate(parent, cell_offsets, bo)
    if rebalance_root:
        user_starts = None
    n = len(parent)
    ncells = len(cell_offsets) - 1

    # ---- S2/S3: orientation and branches per cell ----
    newpar = list(parent)
    roots = []
    for c in range(ncells):
        lo, hi = cell_offsets[c], cell_offsets[c + 1]
        root = lo
        if rebalance_root:
            adj = {i: [] for i in range(lo, hi)}
            for i in range(lo + 1, hi):
                adj[i].append(parent[i])
                adj[parent[i]].append(i)
            root = _centre(lo, hi, adj)
            newpar[root] = -1
            seen = {root}
            q = deque([root])
            while q:
                v = q.popleft()
                for w in sorted(adj[v]):
                    if w not in seen:
                        seen.add(w)
                        newpar[w] = v
                        q.append(w)
        roots.append(root)

    children = [[] for _ in range(n)]
    for i in range(n):
        if newpar[i] >= 0:
            children[newpar[i]].append(i)
    for lst in children:
        lst.sort()

    root_branches = []
    for c in range(ncells):
        r = roots[c]
        rb = _Branch(c, r, 1, 1, None)
        root_branches.append(rb)
        # walk: (node, its branch, its position)
        stack = [(r, rb, 0)]
        while stack:
            q, bq, pos = stack.pop()
            kids = children[q]
            for i in kids:
                cont = (len(kids) == 1 and abs(i - q) == 1
                        and (pos == 0 or i - q == bq.dir)
                        and not (user_starts is not None and i in user_starts))
                if cont:
                    if pos == 0:
                        bq.dir = i - q
                    bq.len += 1
                    stack.append((i, bq, pos + 1))
                else:
                    nb_ = _Branch(c, i, 1, 1, bq)
                    bq.children.append(nb_)
                    stack.append((i, nb_, 0))
    for rb in root_branches:
        _sort_children(rb)

    sizes = [cell_offsets[c + 1] - cell_offsets[c] for c in range(ncells)]
    if cell_order == 1:
        cells = sorted(range(ncells), key=lambda c: (-sizes[c], c))
    else:
        cells = list(range(ncells))

    # ---- S5: split, level by level over all cells ----
    if split_branches == 1:
        _split_levels(list(root_branches))
    # ---- S5': split inside the groups of an intermediate packing ----
    if split_branches == 2:
        def natural_counts(c):
            cnt, lvl = {}, [root_branches[c]]
            depth = 0
            while lvl:
                cnt[depth] = len(lvl)
                lvl = [ch for b in lvl for ch in b.children]
                depth += 1
            return cnt
        for grp in _greedy_groups(cells, sizes, natural_counts, group_width, max_group_unknowns):
            _split_levels([root_branches[c] for c in grp])

    # ---- S4/S6: breadth-first numbering and levels ----
    all_branches = []
    node_plan = [0] * n
    u_src = [-1] * n
    for c in range(ncells):
        order = []
        q = deque([root_branches[c]])
        root_branches[c].level = 0
        while q:
            b = q.popleft()
            order.append(b)
            for ch in b.children:
                ch.level = b.level + 1
                q.append(ch)
        off = cell_offsets[c]
        for rank, b in enumerate(order):
            b.rank = rank
            b.gid = len(all_branches)
            all_branches.append(b)
            for j in range(b.len):
                node_plan[b.node(j)] = off + j
            off += b.len
    for b in all_branches:
        for j in range(b.len):
            i = b.node(j)
            if j > 0:
                q = b.node(j - 1)
            elif b.parent is not None:
                q = b.parent.last()
            else:
                continue
            if parent[i] == q:
                u_src[node_plan[i]] = i
            elif parent[q] == i:
                u_src[node_plan[i]] = q
            else:
                raise AssertionError("branch step is not a tree edge")

    # ---- S7: packing (S7': with level balancing) ----
    T = group_width
    cap = max_group_unknowns
    by_cell = {}
    for b in all_branches:
        by_cell.setdefault(b.cell, []).append(b)

    def counts(c, lv=None):
        cnt = {}
        for b in by_cell[c]:
            l_ = b.level if lv is None else lv[b.gid]
            cnt[l_] = cnt.get(l_, 0) + 1
        return cnt

    def subtree(b):
        out, stack = [], [b]
        while stack:
            x = stack.pop()
            out.append(x)
            stack.extend(x.children)
        return out

    subtree_size = {}

    def balance(c, cur_cnt):
        """S7' trial for cell c against the open group's level counts; the
        moved levels (gid -> level) or None."""
        lv = {b.gid: b.level for b in by_cell[c]}
        for b in by_cell[c]:
            if b.gid not in subtree_size:
                subtree_size[b.gid] = len(subtree(b))
        moves, limit = 0, 4 * len(by_cell[c])
        cnt = counts(c, lv)
        while True:
            over = [l_ for l_ in sorted(cnt) if cnt[l_] > 0 and cur_cnt.get(l_, 0) + cnt[l_] > T]
            if not over:
                return lv
            l_ = over[0]
            if l_ == 0 or moves >= limit:
                return None
            cand = [b for b in by_cell[c] if lv[b.gid] == l_]
            b = min(cand, key=lambda x: (subtree_size[x.gid], x.rank))
            for x in subtree(b):
                cnt[lv[x.gid]] -= 1
                lv[x.gid] += 1
                cnt[lv[x.gid]] = cnt.get(lv[x.gid], 0) + 1
            moves += 1

    groups = []
    cur = []
    cur_cnt = {}
    cur_u = 0
    for c in cells:
        fits = True
        if cur:
            for lvl, k in counts(c).items():
                if cur_cnt.get(lvl, 0) + k > T:
                    fits = False
            if cap and cur_u + sizes[c] > cap:
                fits = False
                cap_fail = True
            else:
                cap_fail = False
            if not fits and level_balance and not cap_fail:
                lv = balance(c, cur_cnt)
                if lv is not None:
                    for b in by_cell[c]:
                        b.level = lv[b.gid]
                    fits = True
        if not fits:
            groups.append(cur)
            cur, cur_cnt, cur_u = [], {}, 0
        cur.append(c)
        for lvl, k in counts(c).items():
            cur_cnt[lvl] = cur_cnt.get(lvl, 0) + k
        cur_u += sizes[c]
    if cur:
        groups.append(cur)
    group_of_cell = [0] * ncells
    for g, cs in enumerate(groups):
        for c in cs:
            group_of_cell[c] = g

    # ---- S8: lane order ----
    group_seg_offsets = [0]
    seg_offsets = [0]
    lanes = []
    for g, cs in enumerate(groups):
        nlev = 1 + max(b.level for c in cs for b in by_cell[c])
        for lvl in range(nlev):
            seg = [b for c in cs for b in by_cell[c] if b.level == lvl]
            seg.sort(key=lambda b: (-b.len, b.cell, b.rank))
            lanes.extend(b.gid for b in seg)
            seg_offsets.append(len(lanes))
        group_seg_offsets.append(len(seg_offsets) - 1)

    br = np.zeros((len(all_branches), 8), dtype=np.int64)
    for b in all_branches:
        br[b.gid] = (b.cell, b.level, b.first, b.dir, b.len,
                     -1 if b.parent is None else b.parent.gid, group_of_cell[b.cell], b.rank)
    gofs = [0]
    gcells = []
    for cs in groups:
        gcells.extend(cs)
        gofs.append(len(gcells))
    return {
        "node_plan": np.array(node_plan, dtype=np.int64),
        "branches": br,
        "u_src": np.array(u_src, dtype=np.int64),
        "group_offsets": np.array(gofs, dtype=np.int64),
        "group_cells": np.array(gcells, dtype=np.int64),
        "group_seg_offsets": np.array(group_seg_offsets, dtype=np.int64),
        "seg_offsets": np.array(seg_offsets, dtype=np.int64),
        "lanes": np.array(lanes, dtype=np.int64),
    }


def _sort_children(rb):
    stack = [rb]
    while stack:
        b = stack.pop()
        b.children.sort(key=lambda ch: ch.first)
        stack.extend(b.children)


def permuted_system(tables, parent, diag, upper, rhs):
    """The re-numbered Hines system in plan numbering: plan parent array and
    the values moved along node_plan / u_src (paper §6: a new Hines matrix
    with the same solution up to the permutation)."""
    node_plan = tables["node_plan"]
    n = len(node_plan)
    user_of = np.empty(n, dtype=np.int64)
    user_of[node_plan] = np.arange(n)
    br = tables["branches"]
    ppar = np.full(n, -1, dtype=np.int64)
    for gid in range(br.shape[0]):
        cell, lvl, first, d, ln, pb, g, rank = (int(v) for v in br[gid])
        for j in range(ln):
            k = node_plan[first + d * j]
            if j > 0:
                ppar[k] = k - 1
            elif pb >= 0:
                pfirst, pd, plen = int(br[pb, 2]), int(br[pb, 3]), int(br[pb, 4])
                ppar[k] = node_plan[pfirst + pd * (plen - 1)]
    d2 = np.asarray(diag)[user_of]
    b2 = np.asarray(rhs)[user_of]
    us = tables["u_src"]
    u2 = np.where(us >= 0, np.asarray(upper)[np.maximum(us, 0)], 0.0)
    return ppar.astype(np.int32), d2, u2, b2

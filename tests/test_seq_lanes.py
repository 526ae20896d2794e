"""CPU replay of the index-order cell-lane tables (plan option cell_lanes 2).

The host builder hands k_solve_seq, per wave of 64 lanes, chunks of K = 8
steps: for the gather mapping (lane j, slot r) -> (cell lane 8 r + j // 8,
element j % 8) the position of each element relative to its cell's first
compartment, and per (cell lane, element) a 16-bit step code: the slot the
step's contribution goes into (written by the first child, added by the
others), the slot the step reads, no-carry, padding, and the mailbox flags
of a cut cell.  This test replays the kernel's semantics on those tables in
numpy, lane-parallel like the kernel, and checks

* every compartment eliminated once and substituted once, every slot read by
  the compartment whose children filled it;
* the solution against the FP64 oracle (relative error <= 1e-12 per cell) on
  the workload families, on trees with many children per compartment, on
  trees too wide for the slots in index order (walked depth-first), and on
  cut cells;
* hand-derived codes of a small tree, and tables that do not depend on the
  number of setup threads.
"""
import numpy as np
import pytest

import oracle
from tests.test_cell_lanes import bushy_system, cell_err
from workloads import configs
from workloads.configs import random_system
from workloads.trees import Forest

K = 8
G = 64 // K
SLOT, RD_SHIFT, TIP, PAD, MBOUT, MBIN, FIRST, ROOT = 31, 5, 1024, 2048, 4096, 8192, 16384, 32768
NSLOTS = 26


def seq_replay(plan, f, diag, upper, rhs):
    waves = plan.table("seq_waves").reshape(-1, 3)
    lane_cell = plan.table("seq_lanes").reshape(-1, 64)
    pos = plan.table("seq_pos").reshape(-1, 64, K)    # [chunk][j][r]
    code = plan.table("seq_code").reshape(-1, 64, K)  # [chunk][c][e]
    mbsrc = plan.table("seq_mbsrc").reshape(-1, 64).astype(np.uint64)
    co = f.cell_offsets
    x = np.full(f.n, np.nan)
    seen_b = np.zeros(f.n, dtype=np.int64)
    seen_f = np.zeros(f.n, dtype=np.int64)
    jj = np.arange(64)
    lanes = np.arange(64)
    for w in range(waves.shape[0]):
        off, nk, ncell = (int(v) for v in waves[w])
        cells = lane_cell[w]
        assert 1 <= ncell <= 64 and np.any(cells >= 0)
        base = np.where(cells >= 0, co[np.maximum(cells, 0)], 0)
        mb = np.zeros((64, 2))
        msb = (mbsrc[w] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        msf = (mbsrc[w] >> np.uint64(32)).astype(np.int64)
        scr = np.zeros((nk, K, 64, 2))
        slot = np.zeros((NSLOTS, 64, 2))
        owner = np.full((NSLOTS, 64), -1, dtype=np.int64)  # user index whose children fill the slot
        cd = np.zeros(64)
        cb = np.zeros(64)
        for k in range(nk):
            g = off + k
            D = np.empty((K, 64))
            U = np.empty((K, 64))
            B = np.empty((K, 64))
            I = np.empty((K, 64), dtype=np.int64)
            for r in range(K):  # gather: slot r of every lane j
                c = G * r + jj // K
                e = jj % K
                p = pos[g, jj, r]
                idx = base[c] + np.where(p == 0xFFFF, 0, p)
                D[e, c] = diag[idx]
                U[e, c] = upper[idx]
                B[e, c] = rhs[idx]
                I[e, c] = np.where(p == 0xFFFF, -1, idx)
                real = p != 0xFFFF
                seen_b[idx[real]] += 1
            for e in range(K):
                q = code[g, :, e]
                pad = (q & PAD) != 0
                assert np.array_equal(pad, I[e] < 0)
                root = (q & ROOT) != 0
                assert np.array_equal(root, ~pad & (I[e] == base))
                dd, bb = D[e], B[e]
                uu = np.where(pad | root, 0.0, U[e])
                kc = np.where((q & TIP) != 0, 0.0, 1.0)
                dd = dd - kc * cd
                bb = bb - kc * cb
                mbin = (q & MBIN) != 0
                src = msb & 63
                assert np.all(cells[src[mbin]] == cells[mbin])
                dd = np.where(mbin, dd - mb[src, 0], dd)
                bb = np.where(mbin, bb - mb[src, 1], bb)
                msb = np.where(mbin, msb >> 6, msb)
                rs = (q >> RD_SHIFT) & SLOT
                rl = np.flatnonzero(rs)
                assert np.all(rs <= NSLOTS)
                if len(rl):
                    assert np.array_equal(owner[rs[rl] - 1, rl], I[e, rl]), "slot read by another compartment"
                    dd[rl] = dd[rl] - slot[rs[rl] - 1, rl, 0]
                    bb[rl] = bb[rl] - slot[rs[rl] - 1, rl, 1]
                    owner[rs[rl] - 1, rl] = -1
                rr = 1.0 / dd
                fv = uu * rr
                yv = bb * rr
                cd = uu * fv
                cb = fv * bb
                ds = q & SLOT
                dl = np.flatnonzero(ds)
                assert np.all(ds <= NSLOTS)
                if len(dl):
                    par = f.parent[I[e, dl]]
                    first = (q[dl] & FIRST) != 0
                    assert np.all(owner[ds[dl] - 1, dl][first] == -1), "first contribution into a taken slot"
                    assert np.array_equal(owner[ds[dl] - 1, dl][~first], par[~first]), "added into another slot"
                    owner[ds[dl] - 1, dl] = par
                    old = np.where(first[:, None], 0.0, slot[ds[dl] - 1, dl])
                    slot[ds[dl] - 1, dl] = old + np.stack([cd[dl], cb[dl]], axis=1)
                mbout = (q & MBOUT) != 0
                mb[mbout, 0] = cd[mbout]
                mb[mbout, 1] = cb[mbout]
                scr[k, e, :, 0] = fv
                scr[k, e, :, 1] = yv
        assert np.all(owner == -1), "slot left full at the end of the backward sweep"
        xc = np.zeros(64)
        for k in range(nk - 1, -1, -1):
            g = off + k
            X = np.empty((K, 64))
            for e in range(K - 1, -1, -1):
                q = code[g, :, e]
                xp = xc.copy()
                ds = q & SLOT
                dl = np.flatnonzero(ds)
                xp[dl] = slot[ds[dl] - 1, dl, 0]
                xp = np.where((q & MBOUT) != 0, mb[lanes, 0], xp)
                xv = np.where((q & PAD) != 0, 0.0, scr[k, e, :, 1] - scr[k, e, :, 0] * xp)
                rs = (q >> RD_SHIFT) & SLOT
                rl = np.flatnonzero(rs)
                slot[rs[rl] - 1, rl, 0] = xv[rl]
                mbin = (q & MBIN) != 0
                mb[(msf & 63)[mbin], 0] = xv[mbin]
                msf = np.where(mbin, msf >> 6, msf)
                xc = xv
                X[e] = xv
            for r in range(K):  # scatter through the gather mapping
                c = G * r + jj // K
                e = jj % K
                p = pos[g, jj, r]
                real = p != 0xFFFF
                idx = base[c] + p
                x[idx[real]] = X[e[real], c[real]]
                seen_f[idx[real]] += 1
    assert np.all(seen_b == 1) and np.all(seen_f == 1), "each compartment once per sweep"
    return x


def _plan(f, **kw):
    from paper_1810_12742_amd import Plan
    return Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, cell_lanes=2, **kw)


def _check(f, diag, upper, seed=3, **kw):
    rhs = np.random.default_rng(seed).standard_normal(f.n)
    p = _plan(f, **kw)
    assert p.info["kernel"] == 5
    x = seq_replay(p, f, diag, upper, rhs)
    xo = oracle.solve(f, diag, upper, rhs)
    assert cell_err(f, x, xo) <= 1e-12
    return p


CASES = {
    "random_small": lambda: random_system(300, 5),
    "c2_cells": lambda: configs.c2(70),
    "c1_cells": lambda: configs.c1(64),
    "c3_cells": lambda: configs.c3(60),
}


@pytest.mark.parametrize("name", list(CASES))
def test_seq_replay_matches_oracle(name):
    s = CASES[name]()
    _check(s.forest, s.diag, s.upper)


@pytest.mark.parametrize("seed", [0, 1])
def test_seq_replay_bushy_trees(seed):
    f, diag, upper = bushy_system(90, seed)
    _check(f, diag, upper, seed)


def wide_system(ncells, width, seed=0):
    """Cells of a root with `width` children, each with one child of its own,
    numbered level by level: in decreasing index every grandchild waits for a
    different parent, so the index walk would need `width` slots."""
    m = 1 + 2 * width
    off = np.arange(ncells + 1, dtype=np.int64) * m
    rel = np.empty(m, dtype=np.int64)
    rel[0] = -1
    rel[1:1 + width] = 0
    rel[1 + width:] = np.arange(1, 1 + width)
    par = np.concatenate([np.where(rel < 0, -1, rel + o) for o in off[:-1]]).astype(np.int32)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 2.0, off[-1])
    a[off[:-1]] = 0.0
    diag = rng.uniform(0.1, 1.0, off[-1]) + a
    np.add.at(diag, par[par >= 0], a[par >= 0])
    return Forest(par, off, None), diag, -a


def test_seq_wide_cells_walk_depth_first():
    """40 pending parents in the index walk: more than the 26 slots, so the
    lanes walk depth-first; the replay still matches the oracle and no code
    names a slot above 26 (a depth-first walk of this tree needs one)."""
    f, diag, upper = wide_system(100, 40)
    p = _check(f, diag, upper)
    code = p.table("seq_code")
    assert int((code & SLOT).max()) <= 2 and int(((code >> RD_SHIFT) & SLOT).max()) <= 2


def test_seq_index_walk_uses_many_slots():
    """20 pending parents fit the slots: the index walk is kept and its codes
    name slots up to 20."""
    f, diag, upper = wide_system(100, 20)
    p = _check(f, diag, upper)
    assert int((p.table("seq_code") & SLOT).max()) == 20


def test_seq_codes_of_a_small_tree():
    """Tree 0 <- 1 <- {2, 3}, 2 <- 4, 3 <- 5 (numbered level by level).  The
    backward walk runs 5, 4, 3, 2, 1, 0 after 10 padding steps (user index 5
    sits at step 10: 10 + 5 = 15 mod 16).  5 adds into a new slot 1 for 3; 4
    into a new slot 2 for 2; 3 reads slot 1 and, its parent 1 not being next,
    takes the freed slot 1 for 1; 2 reads slot 2 and carries into 1; 1 reads
    slot 1 and carries into 0."""
    par = np.array([-1, 0, 1, 1, 2, 3], dtype=np.int32)
    f = Forest(par, np.array([0, 6], dtype=np.int64), None)
    p = _plan(f)
    waves = p.table("seq_waves").reshape(-1, 3)
    assert waves.tolist() == [[0, 2, 1]]
    code = p.table("seq_code").reshape(-1, 64, K)[:, 0, :].reshape(-1)
    pos = p.table("seq_pos").reshape(-1, 64, K)
    lane0 = np.concatenate([pos[k, (0 % G) * K + np.arange(K), 0 // G] for k in range(2)])
    assert lane0.tolist() == [0xFFFF] * 10 + [5, 4, 3, 2, 1, 0]
    want = [PAD | TIP] * 10 + [TIP | FIRST | 1, TIP | FIRST | 2, TIP | FIRST | 1 | (1 << RD_SHIFT),
                               TIP | (2 << RD_SHIFT), 1 << RD_SHIFT, ROOT]
    assert code.tolist() == want


@pytest.mark.parametrize("max_cuts", [1, 3])
def test_seq_cut_cells_cross_the_mailbox(max_cuts):
    """Few cells: every cell longer than 64 compartments is cut, the longest
    piece again while it stays that long (up to max_cuts subtrees).  The
    pieces of a cell sit on adjacent lanes of one wave, the first holding the
    cell root; every other piece posts its root's contribution once (mailbox
    flag) and a lane of the same cell takes it at a strictly later step, in
    the order of the taking lane's source list; the replay matches the oracle."""
    s = configs.c2(40)
    p = _check(s.forest, s.diag, s.upper, cell_max_cuts=max_cuts)
    cells = p.table("seq_lanes").reshape(-1, 64)
    src = p.table("seq_mbsrc").reshape(-1, 64).astype(np.uint64)
    code = p.table("seq_code").reshape(-1, 64, K)
    waves = p.table("seq_waves").reshape(-1, 3)
    pieces = []
    for w in range(cells.shape[0]):
        off, nk, _ = waves[w]
        lanes_of = {}
        for c in range(64):
            if cells[w, c] >= 0:
                lanes_of.setdefault(int(cells[w, c]), []).append(c)
        for cell, ls in lanes_of.items():
            assert ls == list(range(ls[0], ls[0] + len(ls)))
            pieces.append(len(ls))
            q = {c: code[off:off + nk, c, :].reshape(-1) for c in ls}
            out_step = {c: np.flatnonzero(q[c] & MBOUT) for c in ls}
            assert len(out_step[ls[0]]) == 0
            assert all(len(out_step[c]) == 1 for c in ls[1:])
            takes = 0
            for c in ls:
                bw = int(src[w, c]) & 0xFFFFFFFF
                for t in np.flatnonzero(q[c] & MBIN):
                    frm = bw & 63
                    bw >>= 6
                    assert frm in ls[1:] and frm != c and out_step[frm][0] < t
                    takes += 1
                assert bw == 0
            assert takes == len(ls) - 1
    assert len(pieces) == 40 and max(pieces) <= max_cuts + 1 and min(pieces) >= 2
    if max_cuts == 3:
        assert max(pieces) > 2


def test_seq_edge_cells():
    """One-compartment cells, a long unbranched cable (one run, no slot) and
    a cell of 20,000 compartments in one plan."""
    rng = np.random.default_rng(4)
    sizes = [1, 1, 5000, 1, 20000, 3]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    par = np.full(off[-1], -1, dtype=np.int32)
    for c, m in enumerate(sizes):
        lo = off[c]
        for i in range(1, m):
            par[lo + i] = lo + (i - 1 if c == 2 else int(rng.integers(max(0, i - 40), i)))
    a = rng.uniform(0.5, 2.0, off[-1])
    a[off[:-1]] = 0.0
    diag = rng.uniform(0.1, 1.0, off[-1]) + a
    np.add.at(diag, par[par >= 0], a[par >= 0])
    _check(Forest(par, off, None), diag, -a)


def test_seq_tables_do_not_depend_on_the_setup_threads(monkeypatch):
    s = configs.c2(600)
    f = s.forest
    got = []
    for th in ("1", "7"):
        monkeypatch.setenv("HINES_SETUP_THREADS", th)
        p = _plan(f)
        got.append({k: p.table(k) for k in ("seq_waves", "seq_lanes", "seq_pos", "seq_code", "seq_mbsrc")})
    for k in got[0]:
        assert np.array_equal(got[0][k], got[1][k]), k


def test_seq_option_errors():
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.hines import HinesError
    s = configs.c2(8)
    f = s.forest
    with pytest.raises(HinesError):
        Plan(f.parent, f.cell_offsets, host_only=1, cell_lanes=3)
    with pytest.raises(HinesError):
        Plan(f.parent, f.cell_offsets, host_only=1, cell_lanes=2, bitwise=True)


@pytest.mark.parametrize("cut,max_cuts", [(1, 1), (1, 3), (100, 2), (1000, 3)])
def test_seq_cut_settings(cut, max_cuts):
    """Cut thresholds of 1%, 100% and 1000% of the mean cell on bushy trees
    and C2 cells: the replay matches the oracle and no cell has more than
    max_cuts + 1 lanes.  These networks are small, so every cell longer than
    a wave slot's share is cut whatever the threshold (as for the depth-first
    lanes)."""
    for f, diag, upper in (bushy_system(60, 7, max_children=4, size=(1, 700)),
                           (lambda s: (s.forest, s.diag, s.upper))(configs.c2(50, seed=3))):
        p = _check(f, diag, upper, cell_cut_percent=cut, cell_max_cuts=max_cuts)
        cells = p.table("seq_lanes")
        cells = cells[cells >= 0]
        assert np.bincount(cells).max() <= max_cuts + 1


def test_seq_many_small_cells_take_the_threshold():
    """40,000 cells (more than half the device's lanes): the cut threshold,
    not a wave slot's share, decides, and cut cells (up to four pieces)
    replay to the oracle."""
    s = random_system(40000, 3)
    p = _check(s.forest, s.diag, s.upper, cell_cut_percent=100, cell_max_cuts=3)
    cells = p.table("seq_lanes")
    per = np.bincount(cells[cells >= 0])
    assert per.max() == 4 and (per == 1).sum() > 0

"""CPU replay of the cell-lane kernel's tables.

The host builder hands the cell-lane kernel, per wave of 64 cells, chunks of
K steps: for the gather mapping (lane j, slot r) -> (cell lane (64 // K) r + j // K,
element j % K) the position of each element relative to its cell's first
compartment, and per (cell lane, element) the flags that steer the register
carry and the per-lane contribution stack.  This test replays the kernel's
semantics on those tables in numpy, lane-parallel like the kernel, and checks

* that every compartment of every cell is eliminated once and substituted
  once, and the stack never underflows or leaves its slots;
* the solution against the FP64 oracle (relative error <= 1e-12 per cell),
  on the workload families and on trees with many children per compartment,
  which exercise the merge of middle children.
"""
import numpy as np
import pytest

import oracle
from workloads import configs
from workloads.configs import random_system
from workloads.trees import Forest

TIP, POP, PUSH, MERGE, PAD, ROOT, MBOUT, MBIN = 1, 2, 4, 8, 16, 32, 64, 128
STACK = 12


def chunk_steps(plan):
    """Steps per chunk, from the table sizes (64 * K entries per chunk)."""
    waves = plan.table("cell_waves").reshape(-1, 3)
    n = plan.table("cell_pos").size
    return n // (64 * int(waves[:, 1].sum()))


def lane_view(plan, table, c):
    """Per chunk, the K entries of cell lane c in step order."""
    K = chunk_steps(plan)
    G = 64 // K
    t = plan.table(table).reshape(-1, 64, K)
    if table == "cell_flags":
        return t[:, c, :]
    return t[:, (c % G) * K + np.arange(K), c // G]


def replay(plan, f, diag, upper, rhs):
    waves = plan.table("cell_waves").reshape(-1, 3)
    lane_cell = plan.table("cell_lanes").reshape(-1, 64)
    K = chunk_steps(plan)
    G = 64 // K                                         # cells per gather slot
    pos = plan.table("cell_pos").reshape(-1, 64, K)     # [chunk][j][r]
    flags = plan.table("cell_flags").reshape(-1, 64, K)  # [chunk][c][e]
    mbsrc = plan.table("cell_mbsrc").reshape(-1, 64).astype(np.uint64)
    rng_ = plan.table("cell_range").reshape(-1, 64).astype(np.uint64)
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
        # each lane's real steps are one run [q0, q1); the rest is padding
        q0 = (rng_[w] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        q1 = (rng_[w] >> np.uint64(32)).astype(np.int64)
        steps = np.arange(nk * K)
        lane_pad = (flags[off:off + nk].transpose(1, 0, 2).reshape(64, -1) & PAD) != 0
        assert np.array_equal(lane_pad, (steps[None, :] < q0[:, None]) | (steps[None, :] >= q1[:, None]))
        mb = np.zeros((64, 2))
        msb = (mbsrc[w] & np.uint64(0xFFFFFFFF)).astype(np.int64)  # next take in the low 6 bits
        msf = (mbsrc[w] >> np.uint64(32)).astype(np.int64)
        scr = np.zeros((nk, K, 64, 2))  # (f, y) per chunk, step and lane
        cd = np.zeros(64)
        cb = np.zeros(64)
        td = np.zeros(64)
        tb = np.zeros(64)
        m = np.zeros(64, dtype=np.int64)
        stk = np.zeros((STACK, 64, 2))
        for k in range(nk):
            g = off + k
            D = np.empty((K, 64))
            U = np.empty((K, 64))
            B = np.empty((K, 64))
            for r in range(K):  # gather: slot r of every lane j
                c = G * r + jj // K
                e = jj % K
                p = pos[g, jj, r]
                idx = base[c] + np.where(p == 0xFFFF, 0, p)
                D[e, c] = diag[idx]
                U[e, c] = upper[idx]
                B[e, c] = rhs[idx]
                real = p != 0xFFFF
                seen_b[idx[real]] += 1
            for e in range(K):
                fe = flags[g, :, e]
                pad = (fe & PAD) != 0
                dd = np.where(pad, 1.0, D[e])
                uu = np.where((fe & (PAD | ROOT)) != 0, 0.0, U[e])
                bb = np.where(pad, 0.0, B[e])
                tip = (fe & TIP) != 0
                cd[tip] = 0.0
                cb[tip] = 0.0
                dd = dd - cd
                bb = bb - cb
                mbin = (fe & MBIN) != 0
                src = msb & 63
                assert np.all(cells[src[mbin]] == cells[mbin])
                dd = np.where(mbin, dd - mb[src, 0], dd)
                bb = np.where(mbin, bb - mb[src, 1], bb)
                msb = np.where(mbin, msb >> 6, msb)
                pop = (fe & POP) != 0
                dd = np.where(pop, dd - td, dd)
                bb = np.where(pop, bb - tb, bb)
                m[pop] -= 1
                assert np.all(m >= 0), "stack underflow"
                top = np.clip(m, 0, STACK - 1)  # lanes that do not pop read nothing in the kernel
                td = np.where(pop, stk[top, lanes, 0], td)
                tb = np.where(pop, stk[top, lanes, 1], tb)
                rr = 1.0 / dd
                fv = uu * rr
                yv = bb * rr
                cd = uu * fv
                cb = uu * yv
                push = (fe & PUSH) != 0
                assert np.all(m[push] < STACK), "stack overflow"
                stk[m[push], lanes[push], 0] = td[push]
                stk[m[push], lanes[push], 1] = tb[push]
                m[push] += 1
                td = np.where(push, cd, td)
                tb = np.where(push, cb, tb)
                merge = (fe & MERGE) != 0
                assert np.all(m[merge] >= 1), "merge into an empty stack"
                td = np.where(merge, td + cd, td)
                tb = np.where(merge, tb + cb, tb)
                mbout = (fe & MBOUT) != 0
                mb[mbout, 0] = cd[mbout]
                mb[mbout, 1] = cb[mbout]
                scr[k, e, :, 0] = fv
                scr[k, e, :, 1] = yv
        assert np.all(m == 0), "backward stack not empty at the end"
        xc = np.zeros(64)
        xt = np.zeros(64)
        stx = np.zeros((STACK, 64))
        for k in range(nk - 1, -1, -1):
            g = off + k
            X = np.empty((K, 64))
            for e in range(K - 1, -1, -1):
                fe = flags[g, :, e]
                use = (fe & (PUSH | MERGE)) != 0
                xp = np.where(use, xt, xc)
                xp = np.where((fe & MBOUT) != 0, mb[lanes, 0], xp)
                push = (fe & PUSH) != 0
                m[push] -= 1
                assert np.all(m >= 0), "forward stack underflow"
                xt = np.where(push, stx[np.clip(m, 0, STACK - 1), lanes], xt)
                xv = scr[k, e, :, 1] - scr[k, e, :, 0] * xp
                pop = (fe & POP) != 0
                assert np.all(m[pop] < STACK), "forward stack overflow"
                stx[m[pop], lanes[pop]] = xt[pop]
                m[pop] += 1
                xt = np.where(pop, xv, xt)
                mbin = (fe & MBIN) != 0
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
        assert np.all(m == 0), "forward stack not empty at the end"
    assert np.all(seen_b == 1) and np.all(seen_f == 1), "each compartment once per sweep"
    return x


def cell_err(f, x, xo):
    e = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    s = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(e / s))


def bushy_system(ncells, seed, max_children=6, size=(1, 400)):
    """Random trees where a compartment may have up to max_children children
    (parent drawn among the last few compartments), so that merges of middle
    children and deep stacks occur."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(size[0], size[1], ncells)
    off = np.zeros(ncells + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    par = np.full(off[-1], -1, dtype=np.int32)
    for c in range(ncells):
        lo, m = off[c], sizes[c]
        nch = np.zeros(m, dtype=np.int64)
        for i in range(1, m):
            for _ in range(8):
                p = int(rng.integers(max(0, i - 12), i))
                if nch[p] < max_children:
                    break
            nch[p] += 1
            par[lo + i] = lo + p
    a = rng.uniform(0.5, 2.0, off[-1])
    cc = rng.uniform(0.1, 1.0, off[-1])
    roots = off[:-1]
    a[roots] = 0.0
    diag = cc + a
    np.add.at(diag, par[par >= 0], a[par >= 0])
    upper = -a
    return Forest(par, off, None), diag, upper


CASES = {
    "random_small": lambda: random_system(300, 5),
    "c2_cells": lambda: configs.c2(70),
    "c1_cells": lambda: configs.c1(64),
    "c3_cells": lambda: configs.c3(60),
}


def _check(f, diag, upper, seed=3):
    from paper_1810_12742_amd import Plan
    rhs = np.random.default_rng(seed).standard_normal(f.n)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, cell_lanes=1)
    assert p.info["kernel"] == 3
    x = replay(p, f, diag, upper, rhs)
    xo = oracle.solve(f, diag, upper, rhs)
    assert cell_err(f, x, xo) <= 1e-12
    return p


@pytest.mark.parametrize("name", list(CASES))
def test_cell_replay_matches_oracle(name):
    s = CASES[name]()
    _check(s.forest, s.diag, s.upper)


@pytest.mark.parametrize("seed", [0, 1])
def test_cell_replay_bushy_trees(seed):
    f, diag, upper = bushy_system(90, seed)
    _check(f, diag, upper, seed)


def test_cell_flags_of_a_small_tree():
    """Hand-checked flags of one tree: root 0 with children 1 (a leaf) and 2;
    2 has children 3, 4, 5; 6 hangs off 5.  Stack needs: 6, 5, 4, 3 need 0;
    node 2 has three children of need 0 -> 1; the root has children of need 0
    and 1 -> max(1, 0 + 1) = 1.  The child with the largest need goes last,
    the highest index among equal needs (5 under 2; 2 under 0), the others in
    ascending order, so the preorder is 0, 1, 2, 3, 4, 5, 6 and the backward
    sweep runs 6 (tip, carries into 5), 5 (last child of 2: push), 4 (tip,
    middle child of 2: merge), 3 (tip, first child of 2: carries), 2 (pop; the
    root's last child: push), 1 (tip, first child of 0: carries), 0 (root,
    pop)."""
    from paper_1810_12742_amd import Plan
    par = np.array([-1, 0, 0, 2, 2, 2, 5], dtype=np.int32)
    off = np.array([0, 7], dtype=np.int64)
    p = Plan(par, off, None, host_only=1, cell_lanes=1)
    waves = p.table("cell_waves").reshape(-1, 3)
    assert waves.tolist() == [[0, 1, 1]] or waves[:, 1].tolist() == [1]
    K = chunk_steps(p)
    order = [int(v) for v in lane_view(p, "cell_pos", 0).reshape(-1)]
    fl = [int(v) for v in lane_view(p, "cell_flags", 0).reshape(-1)]
    npad = len(order) - 7
    assert npad == (-7) % K and order[:npad] == [0xFFFF] * npad and fl[:npad] == [PAD | TIP] * npad
    assert order[npad:] == [6, 5, 4, 3, 2, 1, 0]
    assert fl[npad:] == [TIP, PUSH, TIP | MERGE, TIP, POP | PUSH, TIP, POP | ROOT]
    # every other lane is empty
    flags = p.table("cell_flags").reshape(-1, 64, K)
    pos = p.table("cell_pos").reshape(-1, 64, K)
    assert np.all(flags[0, 1:] == PAD | TIP) and int((pos != 0xFFFF).sum()) == 7


def test_cell_lane_setup_errors():
    from paper_1810_12742_amd import HinesError, Plan
    par = np.r_[-1, np.arange(70000 - 1)].astype(np.int32)
    with pytest.raises(HinesError) as ei:
        Plan(par, np.array([0, 70000], dtype=np.int64), None, host_only=1, cell_lanes=1)
    assert ei.value.code == "TOO_BIG"
    s = random_system(5, 1)
    f = s.forest
    with pytest.raises(HinesError) as ei:
        Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, cell_lanes=1, bitwise=1)
    assert ei.value.code == "OPTION"


def test_stack_need_of_a_full_binary_tree():
    """A full binary tree of compartments of height h needs h stack entries
    at the root (a node whose two children need a entries each needs a + 1:
    one child's entry waits while the other subtree runs).  Heights 12 and 13
    fit once cut into pieces; at height 14 every cut leaves a piece of height
    13 or a remainder whose walk needs more than 12 entries, so setup refuses
    the cell."""
    from paper_1810_12742_amd import HinesError, Plan

    def full(h):
        n = 2 ** (h + 1) - 1
        par = np.r_[-1, (np.arange(1, n) - 1) // 2].astype(np.int32)
        return par, np.array([0, n], dtype=np.int64)

    for h in (12, 13):
        assert Plan(*full(h), None, host_only=1, cell_lanes=1).info["kernel"] == 3
    with pytest.raises(HinesError) as ei:
        Plan(*full(14), None, host_only=1, cell_lanes=1)
    assert ei.value.code == "TOO_BIG"


def test_long_cells_are_cut_into_pieces_on_lanes_of_one_wave():
    """Cells much longer than the mean are cut into two or more pieces walked
    by lanes of one wave: every mailbox post is taken once by a lane of the
    same cell, the lane's source list names the posting lanes, and the
    solution still matches the oracle.  The longest lane is shorter than the
    longest cell."""
    rng = np.random.default_rng(8)
    from workloads import grow_random_forest, cable_values
    sizes = np.r_[np.full(100, 300), np.full(28, 3000)]
    f = grow_random_forest(rng, len(sizes), target_size=sizes)
    s = cable_values(f, np.random.default_rng(9), a_kind="uniform", rhs=False)
    p = _check(f, s.diag, s.upper)
    K = chunk_steps(p)
    fl = p.table("cell_flags").reshape(-1, 64, K)
    waves = p.table("cell_waves").reshape(-1, 3)
    lane_cell = p.table("cell_lanes").reshape(-1, 64)
    mbsrc = p.table("cell_mbsrc").reshape(-1, 64)
    outs = np.nonzero(fl & MBOUT)
    ins = np.nonzero(fl & MBIN)
    assert outs[0].size == ins[0].size >= 28
    posted = set()
    for w in range(waves.shape[0]):
        for c in range(64):
            nin = int(np.count_nonzero(lane_view_flags(p, w, c) & MBIN))
            lst = int(mbsrc[w, c]) & 0xFFFFFFFF
            srcs = [(lst >> (6 * i)) & 63 for i in range(nin)]
            assert lst >> (6 * nin) == 0
            for s_ in srcs:
                assert lane_cell[w, s_] == lane_cell[w, c] and s_ != c
                assert np.count_nonzero(lane_view_flags(p, w, s_) & MBOUT) == 1
                posted.add((w, s_))
    assert len(posted) == outs[0].size
    assert waves[:, 1].max() * K < 3000
    assert p.info["max_makespan"] == waves[:, 1].max()


def lane_view_flags(plan, w, c):
    K = chunk_steps(plan)
    waves = plan.table("cell_waves").reshape(-1, 3)
    off, nk = int(waves[w, 0]), int(waves[w, 1])
    return plan.table("cell_flags").reshape(-1, 64, K)[off:off + nk, c, :].reshape(-1)


def comb_cell(spine, at, tooth_len):
    """A spine of `spine` compartments with unbranched side chains of
    `tooth_len` compartments hanging at the spine compartments `at`."""
    par = list(np.r_[-1, np.arange(spine - 1)])
    for a in at:
        first = len(par)
        par.append(int(a))
        par.extend(range(first, first + tooth_len - 1))
    return np.array(par, dtype=np.int32)


def test_heavy_path_cut_into_four_lanes():
    """A 400-compartment trunk with 2000-compartment side chains at 50, 150
    and 250 has no subtree near one half (one cut leaves 4151 steps): it is
    cut along its heavy path into four lanes, one of which takes three
    mailboxes in turn.  Replay equals the oracle, and the longest lane is
    about 2250 steps."""
    from workloads import Forest, cable_values
    cells = [comb_cell(400, [50, 150, 250], 2000)] + [np.r_[-1, np.arange(199)].astype(np.int32)] * 60
    par, off = [], [0]
    for c in cells:
        par.append(np.where(c >= 0, c + off[-1], -1))
        off.append(off[-1] + c.size)
    f = Forest(np.concatenate(par).astype(np.int32), np.array(off, dtype=np.int64), None)
    s = cable_values(f, np.random.default_rng(3), a_kind="uniform", rhs=False)
    p = _check(f, s.diag, s.upper)
    mbsrc = p.table("cell_mbsrc").reshape(-1, 64)
    lane_cell = p.table("cell_lanes").reshape(-1, 64)
    assert np.count_nonzero(lane_cell == 0) == 4
    lists = [int(v) & 0xFFFFFFFF for v in mbsrc[lane_cell == 0] if v]
    assert len(lists) == 1 and lists[0] >> 12 != 0 and lists[0] >> 18 == 0  # three takes
    K = chunk_steps(p)
    assert 2250 <= p.info["max_makespan"] * K < 2250 + K


def test_largest_cell_and_single_compartment_cells():
    """A cell of kCellMaxSize = 65,535 compartments among small ones is cut
    over several lanes and replays to the oracle; so do 100 one-compartment
    cells (every lane a lone tip that is also its cell's root); one more
    compartment is refused."""
    from paper_1810_12742_amd import HinesError, Plan
    from workloads import Forest, cable_values, grow_random_forest
    rng = np.random.default_rng(30)
    sizes = np.r_[65535, np.full(40, 300)]
    f = grow_random_forest(rng, len(sizes), target_size=sizes)
    s = cable_values(f, np.random.default_rng(31), a_kind="cable", rhs=False)
    p = _check(f, s.diag, s.upper)
    assert np.count_nonzero(p.table("cell_lanes") == 0) >= 2
    one = Forest(np.full(100, -1, dtype=np.int32), np.arange(101, dtype=np.int64), None)
    s1 = cable_values(one, np.random.default_rng(2), a_kind="uniform", rhs=False)
    p1 = _check(one, s1.diag, s1.upper)
    fl = p1.table("cell_flags")
    real = fl[(fl & PAD) == 0]
    assert real.size == 100 and np.all(real == (TIP | ROOT))
    with pytest.raises(HinesError):
        Plan(np.r_[-1, np.arange(65535)].astype(np.int32), np.array([0, 65536]), None, host_only=1, cell_lanes=1)


def test_small_networks_are_cut_to_fill_the_lanes():
    """With too few cells to give the device's 64 x 1,024 wave-slot lanes
    work, every cell longer than a slot's share is cut along its heavy path
    (cells of one size included, which no cut relative to the mean would
    touch): more lanes than cells, a shorter longest lane, same solution."""
    from workloads import cable_values, grow_random_forest
    rng = np.random.default_rng(40)
    f = grow_random_forest(rng, 100, target_size=np.full(100, 1000))
    s = cable_values(f, np.random.default_rng(41), a_kind="cable", rhs=False)
    p = _check(f, s.diag, s.upper)
    lanes = p.table("cell_lanes")
    assert np.count_nonzero(lanes >= 0) >= 2 * f.ncells
    assert p.info["max_makespan"] * chunk_steps(p) < 1000


def test_tables_do_not_depend_on_the_setup_threads():
    """The cell-lane tables are built over blocks of cells by host threads;
    one thread and several give the same tables bit for bit."""
    import os
    import subprocess
    import sys
    code = (
        "import hashlib, sys\n"
        "from workloads import configs\n"
        "from paper_1810_12742_amd import Plan\n"
        "s = configs.c3(600, seed=4)\n"
        "f = s.forest\n"
        "p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, cell_lanes=1)\n"
        "h = hashlib.sha256()\n"
        "for k in ('cell_waves', 'cell_lanes', 'cell_pos', 'cell_flags', 'cell_mbsrc', 'cell_range'):\n"
        "    h.update(p.table(k).tobytes())\n"
        "print(h.hexdigest())\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = []
    for nth in ("1", "5"):
        env = dict(os.environ, HINES_SETUP_THREADS=nth, PYTHONPATH=root)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=root)
        assert r.returncode == 0, r.stderr
        out.append(r.stdout.strip())
    assert out[0] == out[1]


def test_host_out_of_memory_is_a_status():
    """Setup that runs out of host memory (forced with a data-size limit in a
    child process) returns HINES_ERR_OOM through the C ABI instead of
    aborting, for the group tables and the threaded cell-lane tables; with
    the limit lifted the same process builds the plan."""
    import os
    import subprocess
    import sys
    code = (
        "import resource\n"
        "from workloads import configs\n"
        "import paper_1810_12742_amd.hines as H\n"
        "from paper_1810_12742_amd import Plan, HinesError\n"
        "f = configs.c2(8192).forest\n"
        "H.load()\n"
        "cur = [int(l.split()[1]) * 1024 for l in open('/proc/self/status') if l.startswith('VmData:')][0]\n"
        "soft, hard = resource.getrlimit(resource.RLIMIT_DATA)\n"
        "for opts in ({}, {'cell_lanes': 1}):\n"
        "    resource.setrlimit(resource.RLIMIT_DATA, (cur + (64 << 20), hard))\n"
        "    try:\n"
        "        Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, **opts)\n"
        "        print('built')\n"
        "    except HinesError as e:\n"
        "        print(e.code)\n"
        "    resource.setrlimit(resource.RLIMIT_DATA, (soft, hard))\n"
        "print(Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, cell_lanes=1).info['kernel'])\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root,
                       env=dict(os.environ, PYTHONPATH=root), timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["OOM", "OOM", "3"]

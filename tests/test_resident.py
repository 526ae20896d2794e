"""Tables of the LDS-resident solve, checked on the CPU.

The replay below executes the kernel's per-lane program on the exported
tables, step by step in lockstep over the wave's 64 lanes, with the kernel's
timing of every LDS read and write:
  * a path's bottom operands are read when its record becomes the lane's next
    one; every other compartment's operands are read at the end of the step
    before it, after the contributions added in that step;
  * a step's contribution additions happen after all eliminations of the step;
  * the forward sweep reads x of a path top's parent at the top's step.
Its result is compared with the FP64 oracle (paper §2, Listing 2).  A
schedule that eliminated a compartment before one of its children had added
its contribution would read a stale entry and fail the comparison.
"""
import numpy as np
import pytest

import oracle
from workloads import Forest, cable_values, configs, full_binary_forest

TOL = 1e-12
LANES = 64
LANE_TAB_WORDS = 72  # 144 bytes


def cell_rel_err(f, x, xo):
    err = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    scale = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(err / np.maximum(scale, 1e-300)))


def plan_tables(f, **opts):
    from paper_1810_12742_amd import Plan
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=True, resident=True, **opts)
    t = {k: p.table(k) for k in ("res_groups", "res_par", "res_blob")}
    info = p.info
    p.close()
    return t, info


def rcp_fast(d):
    return 1.0 / d


def replay(t, n, diag, upper, rhs):
    groups, par, blob = t["res_groups"], t["res_par"], t["res_blob"]
    x = np.full(n, np.nan)
    parx = np.concatenate([par, np.zeros(2, dtype=np.int64)])
    for g in groups:
        lo, bu0, nslot, ndma, first, count, F, bun, nroot, npath = (int(v) for v in g)
        S = nslot + 2
        zero = nslot
        D = np.zeros(S)
        U = np.zeros(S)
        B = np.zeros(S)
        D[:ndma] = diag[lo:lo + ndma]
        U[:ndma] = upper[lo:lo + ndma]
        B[:ndma] = rhs[lo:lo + ndma]
        PAR = parx[lo:lo + nslot].copy()
        D[zero:] = 1.0
        U[zero:] = 0.0
        B[zero:] = 0.0
        words = blob[8 * bu0:8 * (bu0 + bun)]
        ltab = words[:LANES + 1]
        roots = words[LANE_TAB_WORDS:LANE_TAB_WORDS + nroot]
        U[roots] = 0.0
        rb = LANE_TAB_WORDS + 8 * ((2 * nroot + 15) // 16)
        recs = words[rb:rb + 4 * npath].reshape(-1, 4).copy()  # slot, t0, len, aux
        LINK = np.full(S, zero)

        def rec(k, kb, ke):
            if kb <= k < ke:
                s_, t0, ln, aux = (int(v) for v in recs[k])
                return [s_, t0, t0 + ln, aux]
            return [zero, F + 1, F + 1, zero]

        # ---- backward ----
        st = []
        for l in range(LANES):
            kb, ke = int(ltab[l]), int(ltab[l + 1])
            c, nx = rec(kb, kb, ke), rec(kb + 1, kb, ke)
            st.append(dict(kb=kb, ke=ke, ri=kb, c=c, nx=nx, j=c[0], prev=zero,
                           op1=(D[c[0]], U[c[0]], B[c[0]], PAR[c[0]] if c[0] < nslot else 0),
                           op2=(D[nx[0]], U[nx[0]], B[nx[0]], PAR[nx[0]] if nx[0] < nslot else 0),
                           cd=0.0, cb=0.0))
        for tt in range(F):
            pushes = []
            acts = []
            for l, s in enumerate(st):
                c = s["c"]
                act = c[1] <= tt < c[2]
                if not act:
                    continue
                d1, u1, b1, p1 = s["op1"]
                dd, bb = d1 - s["cd"], b1 - s["cb"]
                r = rcp_fast(dd)
                f_ = u1 * r
                j = s["j"]
                D[j] = f_
                B[j] = bb * r
                LINK[j] = s["prev"]
                s["cd"], s["cb"] = u1 * f_, f_ * bb
                top = tt == c[2] - 1
                if top and c[3]:
                    pushes.append((p1, s["cd"], s["cb"]))
                acts.append((l, top))
            for p1, cd, cb in pushes:
                D[p1] -= cd
                B[p1] -= cb
            for l, top in acts:
                s = st[l]
                if top:
                    j, c = s["j"], s["c"]
                    recs[s["ri"]] = (j, c[1], c[2] - c[1], s["op1"][3])
                    s["cd"] = s["cb"] = 0.0
                    s["prev"] = zero
                    s["ri"] += 1
                    s["c"] = s["nx"]
                    s["j"] = s["c"][0]
                    s["op1"] = s["op2"]
                    s["nx"] = rec(s["ri"] + 1, s["kb"], s["ke"])
                    q = s["nx"][0]
                    s["op2"] = (D[q], U[q], B[q], PAR[q] if q < nslot else 0)
                else:
                    s["prev"] = s["j"]
                    j = s["op1"][3]
                    s["j"] = j
                    s["op1"] = (D[j], U[j], B[j], PAR[j] if j < nslot else 0)
        # ---- forward ----
        st = []
        for l in range(LANES):
            kb, ke = int(ltab[l]), int(ltab[l + 1])
            c, nx = rec(ke - 1, kb, ke), rec(ke - 2, kb, ke)
            st.append(dict(kb=kb, ke=ke, ri=ke - 1, c=c, nx=nx, j=c[0], xp=0.0,
                           op1=(D[c[0]], B[c[0]], LINK[c[0]]), op2=(D[nx[0]], B[nx[0]], LINK[nx[0]])))
        for tt in range(F - 1, -1, -1):
            acts = []
            for l, s in enumerate(st):
                c = s["c"]
                if not (c[1] <= tt < c[2]):
                    continue
                if tt == c[2] - 1:
                    s["xp"] = B[c[3]]
                f1, y1, _ = s["op1"]
                xv = y1 - f1 * s["xp"]
                B[s["j"]] = xv
                s["xp"] = xv
                acts.append(l)
            for l in acts:
                s = st[l]
                if tt == s["c"][1]:
                    s["ri"] -= 1
                    s["c"] = s["nx"]
                    s["j"] = s["c"][0]
                    s["op1"] = s["op2"]
                    s["nx"] = rec(s["ri"] - 1, s["kb"], s["ke"])
                    q = s["nx"][0]
                    s["op2"] = (D[q], B[q], LINK[q])
                else:
                    j = s["op1"][2]
                    s["j"] = j
                    s["op1"] = (D[j], B[j], LINK[j])
        x[lo + first:lo + first + count] = B[first:first + count]
    return x


def _check(f, s, **opts):
    t, info = plan_tables(f, **opts)
    assert info["kernel"] == 4
    x = replay(t, f.n, s.diag, s.upper, s.rhs)
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    assert not np.isnan(x).any()
    assert cell_rel_err(f, x, xo) <= TOL
    return t


def test_replay_c2_slice():
    s = configs.c2(24)
    t = _check(s.forest, s)
    g = t["res_groups"]
    # every compartment once: the groups tile the cells in order
    assert g[:, 5].sum() == s.forest.n
    assert np.all(g[:, 0] % 2 == 0)


def test_replay_small_cells_packed_and_odd_offsets():
    s = configs.random_system(60, seed=21)
    t = _check(s.forest, s)
    g = t["res_groups"]
    assert (g[:, 8] > 1).any()           # several cells share a group
    assert (g[:, 4] == 1).any()          # a group starts on an odd user index


def test_replay_full_binary_and_single_compartments():
    f = full_binary_forest(5, 4, 5)
    # append three one-compartment cells and a bare cable
    par = np.concatenate([f.parent, [-1, -1, -1, -1], np.arange(f.n + 3, f.n + 3 + 9)]).astype(np.int32)
    off = np.concatenate([f.cell_offsets, f.n + np.array([1, 2, 3, 13])]).astype(np.int64)
    ff = Forest(par, off, np.concatenate([f.branch_offsets[:-1], f.n + np.array([0, 1, 2, 3, 13])]))
    s = cable_values(ff, np.random.default_rng(3), a_kind="cable", dt=0.025)
    _check(ff, s)


def test_critical_path_makespan_on_c2_cells():
    """With 64 lanes and cells of about ten-fold parallelism the schedule of a
    single-cell group needs no more steps than its longest root-to-leaf path."""
    s = configs.c2(16)
    f = s.forest
    t, _ = plan_tables(f)
    depth = np.zeros(f.n, dtype=np.int64)
    for i in range(f.n):
        depth[i] = 1 if f.parent[i] < 0 else depth[f.parent[i]] + 1
    for g in t["res_groups"]:
        lo, first, count, F, nroot = int(g[0]), int(g[4]), int(g[5]), int(g[6]), int(g[8])
        if nroot == 1:
            assert F == depth[lo + first:lo + first + count].max()


def test_large_cell_refused():
    from paper_1810_12742_amd import HinesError, Plan
    n = 17000
    par = np.arange(-1, n - 1, dtype=np.int32)
    with pytest.raises(HinesError) as ei:
        Plan(par, np.array([0, n]), None, host_only=True, resident=True)
    assert ei.value.code == "TOO_BIG"
    with pytest.raises(HinesError) as ei:
        Plan(par[:10], np.array([0, 10]), None, host_only=True, resident=True, cell_lanes=True)
    assert ei.value.code == "OPTION"


def test_pack_option_sets_group_sizes():
    s = configs.random_system(80, seed=2)
    f = s.forest
    t1, _ = plan_tables(f, res_pack=1)
    assert (t1["res_groups"][:, 8] == 1).all()          # one cell per group
    t2, _ = plan_tables(f, res_pack=600)
    g = t2["res_groups"]
    multi = g[:, 8] > 1
    assert multi.any() and (g[multi, 5] <= 600).all()
    x = replay(t2, f.n, s.diag, s.upper, s.rhs)
    assert cell_rel_err(f, x, oracle.solve(f, s.diag, s.upper, s.rhs)) <= TOL


def _lanes_per_cell(f, **o):
    from paper_1810_12742_amd import Plan
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=True, cell_lanes=True, **o)
    lc = p.table("cell_lanes")
    p.close()
    return np.bincount(lc[lc >= 0], minlength=f.ncells)


def test_cell_cut_options():
    """cell_max_cuts bounds the lanes of a cut cell.  On a network with more
    cells than half the device's lanes (40,000: 39,990 cables of 10 and ten of
    2,000 compartments) only the threshold decides: the long cables are cut by
    default and stay whole when the threshold is far above them."""
    f = configs.c2(3000).forest
    assert _lanes_per_cell(f).max() >= 3
    assert _lanes_per_cell(f, cell_max_cuts=1).max() <= 2
    sizes = np.array([10] * 39990 + [2000] * 10)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    par = np.arange(-1, off[-1] - 1, dtype=np.int64)
    par[off[:-1]] = -1
    g = Forest(par.astype(np.int32), off, off.copy())
    assert _lanes_per_cell(g)[-10:].min() >= 2
    assert _lanes_per_cell(g, cell_cut_percent=100000).max() == 1

"""Tables of the LDS-resident solve, checked on the CPU.

The replay below executes the kernel's per-lane program on the exported
tables, chunk by chunk in lockstep over the wave's 64 lanes, with the kernel's
timing of every LDS read and write:
  * backward sweep: at the start of chunk c a lane active in chunk c + 1 reads
    that chunk's operands (d, u, b at its four list entries); then every lane
    active in chunk c eliminates its four steps from the operands it read a
    chunk earlier, storing f over u and y over b; then lanes whose path tops
    in chunk c add their contribution into the parent's entry;
  * forward sweep: at the start of chunk c a lane active in chunk c - 1 reads
    (f, y) of that chunk and, if its path tops there, x of the top's parent;
    then every lane active in chunk c substitutes its four steps downward.
Its result is compared with the FP64 oracle (paper §2, Listing 2).  A
schedule that eliminated a compartment before one of its children had added
its contribution, or read a parent's x before it was written, would read a
stale entry and fail the comparison.
"""
import numpy as np
import pytest

import oracle
from workloads import Forest, cable_values, configs, full_binary_forest

TOL = 1e-12
LANES = 64
LANE_TAB_WORDS = 136   # 272 bytes: 65 record offsets, 65 list offsets
NO_PARENT = 0xFFFF
# LDS classes: bytes per group (160 KiB / groups per CU) and plane stride in slots
CLASS_BYTES = (163840, 81920, 54528, 40960, 32768, 27136, 23296, 20480, 16384, 10240)
STRIDES = (6144, 3008, 1984, 1472, 1152, 960, 832, 704, 576, 320)
GROUP_FIELDS = ("lo", "blob", "nslot", "ndma", "first", "count", "nchunk", "blob_units", "nroot", "npath",
                "nlist", "rec_off", "list_off", "cls", "k", "nflip")


def cell_rel_err(f, x, xo):
    err = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    scale = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(err / np.maximum(scale, 1e-300)))


def plan_tables(f, **opts):
    from paper_1810_12742_amd import Plan
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=True, resident=True, **opts)
    t = {k: p.table(k) for k in ("res_groups", "res_blob")}
    t["res_groups"] = t["res_groups"].reshape(-1, len(GROUP_FIELDS))
    info = p.info
    p.close()
    return t, info


def group_view(t, g):
    G = dict(zip(GROUP_FIELDS, (int(v) for v in g)))
    words = t["res_blob"][8 * G["blob"]:8 * (G["blob"] + G["blob_units"])]
    G["rec_first"] = words[:LANES + 1]
    G["list_first"] = words[LANES + 1:2 * LANES + 2]
    G["roots"] = words[LANE_TAB_WORDS:LANE_TAB_WORDS + G["nroot"]]
    f0 = LANE_TAB_WORDS + 8 * ((2 * G["nroot"] + 15) // 16)
    G["flips"] = words[f0:f0 + 2 * G["nflip"]].reshape(-1, 2)  # slot, slot whose u it takes
    r0 = G["rec_off"] // 2
    nrec = G["npath"] + LANES + 1
    G["recs"] = words[r0:r0 + 4 * nrec].reshape(-1, 4)      # c0, nch, parent byte offset, spare
    l0 = G["list_off"] // 2
    K = G["k"]
    G["lists"] = words[l0:l0 + K * G["nlist"]].reshape(-1, K)  # byte offsets of a chunk's steps
    return G


def replay(t, n, diag, upper, rhs):
    x = np.full(n, np.nan)
    for g in t["res_groups"]:
        G = group_view(t, g)
        lo, nslot, ndma, first, count, NC, K = (G[k] for k in ("lo", "nslot", "ndma", "first", "count", "nchunk", "k"))
        zero = nslot
        D = np.zeros(nslot + 1)
        U = np.zeros(nslot + 1)
        B = np.zeros(nslot + 1)
        D[:ndma] = diag[lo:lo + ndma]
        U[:ndma] = upper[lo:lo + ndma]
        B[:ndma] = rhs[lo:lo + ndma]
        D[zero], U[zero], B[zero] = 1.0, 0.0, 0.0
        for dst, src in G["flips"]:   # re-rooted cells: couplings move along the old root's path
            U[dst] = U[src]
        U[G["roots"]] = 0.0
        recs, lists = G["recs"], G["lists"]
        lanes = []
        for l in range(LANES):
            kb, ke = int(G["rec_first"][l]), int(G["rec_first"][l + 1]) - 1
            lb, le = int(G["list_first"][l]), int(G["list_first"][l + 1])
            assert tuple(recs[kb - 1][:3]) == (0xFFFF, 0, NO_PARENT) and tuple(recs[ke][:3]) == (0xFFFF, 0, NO_PARENT)
            paths = [(int(r[0]), int(r[0]) + int(r[1]), int(r[2])) for r in recs[kb:ke]]
            ents = lists[lb:le] // 8
            assert len(ents) == sum(p[1] - p[0] for p in paths)
            chunk_ent = {}
            e = 0
            for c0, c1, _ in paths:
                for c in range(c0, c1):
                    chunk_ent[c] = ents[e]
                    e += 1
            lanes.append((paths, chunk_ent))

        def path_at(paths, c):
            for p in paths:
                if p[0] <= c < p[1]:
                    return p
            return None

        # ---- backward ----
        ops = [dict() for _ in range(LANES)]
        for l, (paths, ce) in enumerate(lanes):
            if 0 in ce:
                a = ce[0]
                ops[l][0] = (D[a].copy(), U[a].copy(), B[a].copy())
        carry = [(0.0, 0.0)] * LANES
        for c in range(NC):
            for l, (paths, ce) in enumerate(lanes):     # reads of chunk c + 1
                if c + 1 < NC and (c + 1) in ce:
                    a = ce[c + 1]
                    ops[l][c + 1] = (D[a].copy(), U[a].copy(), B[a].copy())
            pushes = []
            for l, (paths, ce) in enumerate(lanes):     # eliminations of chunk c
                p = path_at(paths, c)
                if p is None:
                    continue
                a = ce[c]
                d4, u4, b4 = ops[l].pop(c)
                ncd, ncb = carry[l]
                for k in range(K):
                    dd = d4[k] + ncd
                    bb = b4[k] + ncb
                    f_ = u4[k] / dd
                    y_ = bb / dd
                    ncd, ncb = -(u4[k] * f_), -(u4[k] * y_)
                    U[a[k]] = f_
                    B[a[k]] = y_
                carry[l] = (ncd, ncb)
                if c == p[1] - 1:
                    if p[2] != NO_PARENT:
                        pushes.append((p[2] // 8, ncd, ncb))
                    carry[l] = (0.0, 0.0)
            for q, ncd, ncb in pushes:                  # contributions of chunk c
                D[q] += ncd
                B[q] += ncb
        # ---- forward ----
        fops = [dict() for _ in range(LANES)]

        def fread(l, c):
            paths, ce = lanes[l]
            p = path_at(paths, c)
            a = ce[c]
            q = p[2] // 8 if (c == p[1] - 1 and p[2] != NO_PARENT) else zero
            fops[l][c] = (U[a].copy(), B[a].copy(), B[q])

        for l, (paths, ce) in enumerate(lanes):
            if NC - 1 in ce:
                fread(l, NC - 1)
        xp = [0.0] * LANES
        for c in range(NC - 1, -1, -1):
            for l, (paths, ce) in enumerate(lanes):     # reads of chunk c - 1
                if c >= 1 and (c - 1) in ce:
                    fread(l, c - 1)
            for l, (paths, ce) in enumerate(lanes):
                p = path_at(paths, c)
                if p is None:
                    continue
                a = ce[c]
                f4, y4, xq = fops[l].pop(c)
                if c == p[1] - 1:
                    xp[l] = xq
                for k in range(K - 1, -1, -1):
                    xp[l] = y4[k] - f4[k] * xp[l]
                    B[a[k]] = xp[l]
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
    assert np.all(g[:, 2] + 1 <= np.array(STRIDES)[g[:, 13]])


def _eccentricities(par):
    """Hop eccentricity of every node of one tree (parents par, par[0] = -1), by
    a breadth-first search from each node."""
    m = len(par)
    adj = [[] for _ in range(m)]
    for i in range(1, m):
        adj[i].append(par[i])
        adj[par[i]].append(i)
    ecc = np.zeros(m, dtype=np.int64)
    for s0 in range(m):
        dist = np.full(m, -1)
        dist[s0] = 0
        q = [s0]
        for v in q:
            for w in adj[v]:
                if dist[w] < 0:
                    dist[w] = dist[v] + 1
                    q.append(w)
        ecc[s0] = dist.max()
    return ecc


def test_replay_rerooted_cells():
    """Cells re-rooted at their centre (paper §6): the replay with the moved
    couplings solves to the oracle's tolerance, each new root is the
    compartment of least eccentricity (the smaller index on ties, found here by
    brute force), and the schedules get shorter than with the soma as root."""
    for s, opts in ((configs.c2(24), {}), (configs.random_system(60, seed=23), dict(res_pack=600))):
        f = s.forest
        t = _check(f, s, rebalance_root=True, **opts)
        t0, _ = plan_tables(f, **opts)
        assert t["res_groups"][:, 6].sum() < t0["res_groups"][:, 6].sum()
        assert t["res_groups"][:, 15].sum() > 0
        roots = []
        for g in t["res_groups"]:
            G = group_view(t, g)
            roots.extend(int(G["lo"]) + int(r) for r in G["roots"])
        for c in range(min(f.ncells, 12)):
            lo, hi = int(f.cell_offsets[c]), int(f.cell_offsets[c + 1])
            par = f.parent[lo:hi].astype(np.int64) - lo
            par[0] = -1
            ecc = _eccentricities(par)
            want = lo + int(np.flatnonzero(ecc == ecc.min())[0]) if hi - lo > 2 else lo
            assert roots[c] == want


def test_groups_that_do_not_fit_are_split_or_kept_at_their_root():
    """A packed group whose tables overflow LDS (many small re-rooted cells)
    is built again with fewer cells; a near-limit cable that would not fit
    re-rooted keeps its own root.  Both still replay to the oracle."""
    s = configs.random_system(500, seed=31)
    t = _check(s.forest, s, rebalance_root=True, res_pack=3000)
    assert t["res_groups"][:, 5].sum() == s.forest.n
    n = 5500
    par = np.concatenate([np.arange(-1, n - 1), [-1, -1, -1]]).astype(np.int32)
    off = np.array([0, n, n + 1, n + 2, n + 3], dtype=np.int64)
    f = Forest(par, off, off.copy())
    sc = cable_values(f, np.random.default_rng(6), a_kind="cable", dt=0.025)
    t = _check(f, sc, rebalance_root=True)
    g = t["res_groups"]
    assert g[0, 5] == n and g[0, 15] == 0   # the cable alone, from its soma


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
    single-cell group is as long as its longest root-to-leaf path in whole
    chunks, plus at most a few chunks of the two-chunk margins that light
    paths keep before their parents."""
    s = configs.c2(48)
    f = s.forest
    t, _ = plan_tables(f)
    depth = np.zeros(f.n, dtype=np.int64)
    for i in range(f.n):
        depth[i] = 1 if f.parent[i] < 0 else depth[f.parent[i]] + 1
    excess = []
    for g in t["res_groups"]:
        lo, first, count, NC, nroot, K = int(g[0]), int(g[4]), int(g[5]), int(g[6]), int(g[8]), int(g[14])
        if nroot == 1:
            lb = -(-int(depth[lo + first:lo + first + count].max()) // K)
            assert lb <= NC <= lb + 6
            excess.append(NC - lb)
    assert np.mean(excess) < 1.5


def test_lds_class_is_the_smallest_that_fits():
    s = configs.c2(64)
    t, _ = plan_tables(s.forest)
    for g in t["res_groups"]:
        nslot, bu, cls = int(g[2]), int(g[7]), int(g[13])

        def fits(k):
            return nslot + 1 <= STRIDES[k] and 24 * STRIDES[k] + 16 * bu <= CLASS_BYTES[k]
        assert fits(cls)
        assert not any(fits(k) for k in range(cls + 1, len(STRIDES)))


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

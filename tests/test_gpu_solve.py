"""GPU parity of hines_solve (through the C-ABI) against the FP64 oracle.

Bars: the default (reciprocal + fused multiply-add) form within 1e-12
relative error per cell (max norm); the bitwise form equal to the oracle bit
for bit, on the user numbering when the plan keeps it and on the plan
numbering otherwise (the same operations in the same order)."""
import numpy as np
import pytest

import oracle
from oracle import tables as otab
from workloads import Forest, configs, full_binary_forest

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda")


def cell_rel_err(f, x, xo):
    err = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    scale = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(err / np.maximum(scale, 1e-300)))


def gpu_solve(torch_dev, s, rhs=None, alias=False, **opts):
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    f = s.forest
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    d = torch.from_numpy(np.ascontiguousarray(s.diag)).to(dev)
    u = torch.from_numpy(np.ascontiguousarray(s.upper)).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(s.rhs if rhs is None else rhs)).to(dev)
    x = b if alias else torch.empty_like(b)
    p.solve(d, u, b, out=x)
    torch.cuda.synchronize()
    out = x.cpu().numpy()
    p.close()
    return out


def test_c1_bitwise_and_fast(torch_dev):
    s = configs.c1()
    xo = oracle.solve(s.forest, s.diag, s.upper, s.rhs)
    assert np.array_equal(gpu_solve(torch_dev, s, bitwise=True), xo)
    assert cell_rel_err(s.forest, gpu_solve(torch_dev, s), xo) <= TOL


OPTS = [
    dict(),
    dict(split_branches=1),
    dict(rebalance_root=1),
    dict(rebalance_root=1, split_branches=1),
    dict(cell_order=1, max_group_unknowns=1024),
    dict(split_branches=1, max_group_unknowns=512),
    dict(group_width=128, max_group_unknowns=4096),
    dict(group_width=256, max_group_unknowns=5000, split_branches=1),
    dict(level_sync=1),
    dict(level_sync=1, split_branches=1, max_group_unknowns=3000),
    # the outlook (§8): per-group split averages, subtrees moved down a level
    dict(level_sync=1, split_branches=2, max_group_unknowns=4096),
    dict(level_sync=1, level_balance=1, max_group_unknowns=4096),
    dict(split_branches=2, level_balance=1, max_group_unknowns=4096),
]


@pytest.mark.parametrize("opts", OPTS, ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()) or "default")
def test_c2_slice_all_options(torch_dev, opts):
    from paper_1810_12742_amd import Plan
    s = configs.c2(1536)
    f0 = s.forest
    info = Plan(f0.parent, f0.cell_offsets, f0.branch_offsets, **opts).info
    want = 0 if (opts.get("level_sync") or opts.get("rebalance_root")) else 1
    assert info["kernel"] == want
    f = s.forest
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    x = gpu_solve(torch_dev, s, **opts)
    assert cell_rel_err(f, x, xo) <= TOL
    xb = gpu_solve(torch_dev, s, bitwise=True, **opts)
    if not opts.get("rebalance_root"):
        assert np.array_equal(xb, xo)
    else:
        mg = opts.get("max_group_unknowns", 2048)
        o = {k: v for k, v in opts.items() if k != "max_group_unknowns"}
        t = otab.build(f.parent, f.cell_offsets, f.branch_offsets, max_group_unknowns=mg, **o)
        pp, d2, u2, b2 = otab.permuted_system(t, f.parent, s.diag, s.upper, s.rhs)
        x2 = oracle.solve(Forest(pp, f.cell_offsets, np.arange(f.n + 1)), d2, u2, b2)
        assert np.array_equal(xb, x2[t["node_plan"]])
        assert cell_rel_err(f, xb, xo) <= TOL


def test_c2_full_bench_configuration(torch_dev):
    """The full 65,536-cell workload in the launch configuration the bench
    times: the autotuner's shipped pick for this device, or, when this device
    has not been tuned, every candidate the bench would time."""
    from paper_1810_12742_amd.autotune import CELL_CANDIDATES, SHIPPED_CACHE, cached_pick
    s = configs.c2()
    f = s.forest
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    pick = cached_pick(f.parent, f.cell_offsets, f.branch_offsets, candidates=CELL_CANDIDATES,
                       cache_path=SHIPPED_CACHE)
    for opts in ([pick] if pick else CELL_CANDIDATES):
        print(f"c2 full: {opts}", flush=True)
        x = gpu_solve(torch_dev, s, **opts)
        assert cell_rel_err(f, x, xo) <= TOL
    # the layout-resident solve the bench line reports beside it, on the same
    # plan: the same elimination, bit for bit
    from paper_1810_12742_amd import Plan
    torch, dev = torch_dev
    opts = pick or CELL_CANDIDATES[0]
    if opts.get("cell_lanes") != 1:  # the solver layout is a form of the depth-first cell-lane plan
        opts = CELL_CANDIDATES[0]
    if opts.get("cell_lanes") == 1:
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
        d, u, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.rhs))
        xs = p.solve(d, u, b).cpu().numpy()
        dl, ul, bl = p.to_layout(d), p.to_layout(u), p.to_layout(b)
        xl = p.from_layout(p.solve_layout(dl, ul, bl)).cpu().numpy()
        print(f"c2 full, layout-resident: {p.layout_size} slots", flush=True)
        assert np.array_equal(xl, xs)
        assert cell_rel_err(f, xl, xo) <= TOL
        p.close()


def test_rhs_alias_and_determinism(torch_dev):
    s = configs.c2(512)
    xo = oracle.solve(s.forest, s.diag, s.upper, s.rhs)
    x1 = gpu_solve(torch_dev, s, alias=True, split_branches=1)
    x2 = gpu_solve(torch_dev, s, split_branches=1)
    assert np.array_equal(x1, x2)
    assert cell_rel_err(s.forest, x1, xo) <= TOL


def test_unbranched_long_cable(torch_dev):
    """p[i] = i-1: the Thomas special case, one 5000-compartment branch."""
    n = 5000
    par = np.arange(-1, n - 1, dtype=np.int32)
    f = Forest(par, np.array([0, n], dtype=np.int64), np.array([0, n], dtype=np.int64))
    rng = np.random.default_rng(2)
    a = rng.uniform(0.5, 2.0, n)
    a[0] = 0
    c = rng.uniform(0.1, 1.0, n)
    from workloads import assemble
    d, u = assemble(f, a, c)
    from workloads.trees import CableSystem
    s = CableSystem(f, a, c, d, u, rng.standard_normal(n))
    xo = oracle.solve(f, d, u, s.rhs)
    assert cell_rel_err(f, gpu_solve(torch_dev, s), xo) <= TOL
    assert np.array_equal(gpu_solve(torch_dev, s, bitwise=True), xo)


def test_wide_level_multipass_lanes(torch_dev):
    """A soma with 150 child branches: the level is wider than the 64 lanes of
    a group, so lanes take several branches of that level."""
    kids = 150
    parents = [-1]
    for k in range(kids):
        start = len(parents)
        parents.append(0)
        parents.extend(range(start, start + 2))
    one = np.array(parents)
    cells = [one] * 3
    off = np.zeros(4, dtype=np.int64)
    off[1:] = np.cumsum([len(c) for c in cells])
    par = np.concatenate([np.where(c >= 0, c + o, -1) for c, o in zip(cells, off[:-1])]).astype(np.int32)
    f = Forest(par, off, np.arange(off[-1] + 1))
    rng = np.random.default_rng(5)
    from workloads import cable_values
    s = cable_values(f, rng, a_kind="uniform")
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    from paper_1810_12742_amd import Plan
    for gw in (64, 128):
        torch, dev = torch_dev
        p = Plan(f.parent, f.cell_offsets, None, group_width=gw)
        d = torch.from_numpy(s.diag).to(dev)
        u = torch.from_numpy(s.upper).to(dev)
        b = torch.from_numpy(s.rhs).to(dev)
        x = p.solve(d, u, b)
        assert cell_rel_err(f, x.cpu().numpy(), xo) <= TOL


def test_many_small_cells_and_single_compartments(torch_dev):
    s = configs.c3(400)  # sizes 50..20000 mixed; keep the LDS-sized ones
    f = s.forest
    sizes = np.diff(f.cell_offsets)
    keep = np.flatnonzero(sizes <= 5000)
    sub = f.subset(keep)
    from workloads import cable_values
    rng = np.random.default_rng(0)
    ss = cable_values(sub, rng, a_kind="cable")
    # append 7 isolated single-compartment cells
    n0 = sub.n
    par = np.concatenate([sub.parent, np.full(7, -1, dtype=np.int32)])
    off = np.concatenate([sub.cell_offsets, n0 + np.arange(1, 8)])
    bo = np.concatenate([sub.branch_offsets[:-1], n0 + np.arange(0, 8)])
    f2 = Forest(par, off, bo)
    d = np.concatenate([ss.diag, rng.uniform(1, 2, 7)])
    u = np.concatenate([ss.upper, np.zeros(7)])
    b = np.concatenate([ss.rhs, rng.standard_normal(7)])
    from workloads.trees import CableSystem
    s2 = CableSystem(f2, None, None, d, u, b)
    xo = oracle.solve(f2, d, u, b)
    for opts in (dict(), dict(max_group_unknowns=4000, split_branches=1), dict(cell_order=1)):
        assert cell_rel_err(f2, gpu_solve(torch_dev, s2, **opts), xo) <= TOL


def test_error_paths(torch_dev):
    torch, dev = torch_dev
    from paper_1810_12742_amd import HinesError, Plan
    f = full_binary_forest(2, 2, 3)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    d = torch.ones(f.n, dtype=torch.float64, device=dev) * 4
    u = torch.zeros(f.n, dtype=torch.float64, device=dev)
    b = torch.ones(f.n, dtype=torch.float64, device=dev)
    import ctypes
    from paper_1810_12742_amd.hines import load
    lib = load()
    P = ctypes.c_void_p
    st = lib.hines_solve(p._h, P(d.data_ptr()), P(u.data_ptr()), P(b.data_ptr()), P(b.data_ptr()), 3, None)
    assert st == 6  # NCELLS
    st = lib.hines_solve(p._h, P(d.data_ptr()), P(u.data_ptr()), P(b.data_ptr()), P(d.data_ptr()), 2, None)
    assert st == 12  # x aliases diag
    st = lib.hines_solve(p._h, None, P(u.data_ptr()), P(b.data_ptr()), P(b.data_ptr()), 2, None)
    assert st == 1
    # a cell whose compartments exceed LDS runs from the global workspace
    n = 8000
    par = np.arange(-1, n - 1, dtype=np.int32)
    big = Plan(par, np.array([0, n]), None)
    assert big.info["workspace_groups"] == 1
    rng = np.random.default_rng(8)
    dd = 2.0 + rng.random(n)
    uu = -rng.random(n) * 0.9
    bb = rng.standard_normal(n)
    f1 = Forest(par, np.array([0, n]), np.array([0, n]))
    xg = big.solve(torch.from_numpy(dd).to(dev), torch.from_numpy(uu).to(dev), torch.from_numpy(bb).to(dev))
    assert cell_rel_err(f1, xg.cpu().numpy(), oracle.solve(f1, dd, uu, bb)) <= TOL
    # a group whose branch tables alone exceed LDS is refused: a star of 6000 branches
    par = np.concatenate([[-1], np.zeros(6000, dtype=np.int32)]).astype(np.int32)
    with pytest.raises(HinesError) as ei:
        Plan(par, np.array([0, 6001]), None)
    assert ei.value.code == "TOO_BIG"
    # empty forest: nothing to do
    pe = Plan(np.zeros(0, dtype=np.int32), np.zeros(1, dtype=np.int64), None)
    e = torch.zeros(0, dtype=torch.float64, device=dev)
    pe.solve(e, e, e, out=e)
    torch.cuda.synchronize()


def test_check_matrix_through_the_c_abi(torch_dev):
    """hines_check_matrix (paper §1: SDD with a positive diagonal): the
    generated cable matrices pass; a row made non-dominant, a negative
    diagonal and a NaN are reported at their index, the smallest first."""
    import ctypes
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.hines import load
    s = configs.c2(64)
    f = s.forest
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    lib = load()
    P = ctypes.c_void_p
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    bad = ctypes.c_int64(7)
    assert lib.hines_check_matrix(p._h, P(d.data_ptr()), P(u.data_ptr()), ctypes.byref(bad), None) == 0
    assert bad.value == -1
    # the row sum of |off-diagonals| of row i, computed on the host
    par = f.parent
    rowsum = np.abs(np.where(par >= 0, s.upper, 0.0))
    np.add.at(rowsum, par[par >= 0], np.abs(s.upper[par >= 0]))
    i_dom, i_neg, i_nan = 5000, 777, 20000
    d2 = s.diag.copy()
    d2[i_dom] = 0.999 * rowsum[i_dom]  # positive, but below the off-diagonal sum
    d2[i_nan] = np.nan
    dd = torch.from_numpy(d2).to(dev)
    assert lib.hines_check_matrix(p._h, P(dd.data_ptr()), P(u.data_ptr()), ctypes.byref(bad), None) == 11
    assert bad.value == i_dom
    d2[i_neg] = -1.0
    dd = torch.from_numpy(d2).to(dev)
    assert p.check_matrix(dd, u) == i_neg
    # a root's upper entry is ignored, whatever it holds
    u2 = s.upper.copy()
    u2[f.cell_offsets[:-1]] = 1e300
    assert p.check_matrix(d, torch.from_numpy(u2).to(dev)) == -1
    p.close()


def test_resident_kernel_parity(torch_dev):
    """The LDS-resident kernel (plan option resident) on C2 slices, packed
    small cells with odd group offsets, one-compartment cells, an unbranched
    cable and a near-LDS-limit cell; x aliasing rhs; run-to-run equality."""
    from paper_1810_12742_amd import Plan
    cases = [configs.c2(2048), configs.random_system(500, seed=31), configs.c1(1000)]
    # one cell of 5,500 compartments (the image fills most of LDS) plus singletons
    n = 5500
    par = np.concatenate([np.arange(-1, n - 1), [-1, -1, -1]]).astype(np.int32)
    f = Forest(par, np.array([0, n, n + 1, n + 2, n + 3], dtype=np.int64),
               np.array([0, n, n + 1, n + 2, n + 3], dtype=np.int64))
    from workloads import cable_values
    cases.append(cable_values(f, np.random.default_rng(6), a_kind="cable", dt=0.025))
    for s in cases:
        f = s.forest
        xo = oracle.solve(f, s.diag, s.upper, s.rhs)
        assert Plan(f.parent, f.cell_offsets, f.branch_offsets, resident=True).info["kernel"] == 4
        # re-rooted at the tree centres (paper §6), and packed into larger groups
        for opts in (dict(), dict(rebalance_root=1), dict(rebalance_root=1, res_pack=3000)):
            print(f"resident {opts}: {f.ncells} cells, {f.n} unknowns", flush=True)
            x1 = gpu_solve(torch_dev, s, resident=True, **opts)
            assert cell_rel_err(f, x1, xo) <= TOL
            x2 = gpu_solve(torch_dev, s, alias=True, resident=True, **opts)
            assert np.array_equal(x1, x2)


def test_resident_full_c2(torch_dev):
    """The full 65,536-cell C2 workload on the resident kernel, with the soma
    as root and re-rooted at the tree centres."""
    s = configs.c2()
    xo = oracle.solve(s.forest, s.diag, s.upper, s.rhs)
    for opts in (dict(), dict(rebalance_root=1, res_pack=3000)):
        print(f"resident full c2 {opts}", flush=True)
        x = gpu_solve(torch_dev, s, resident=True, **opts)
        assert cell_rel_err(s.forest, x, xo) <= TOL

"""GPU parity of the time loop (in-kernel right-hand side, hipGraph capture,
workspace path for cells too large for LDS) and of the adjoint, against the
FP64 oracle."""
import numpy as np
import pytest

import oracle
from workloads import configs, grow_random_forest, cable_values

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


def mixed_system():
    """Cells of 50, 500, 5000 and 8000 compartments (the last exceed LDS)."""
    rng = np.random.default_rng(12)
    sizes = np.array([50, 500, 5000, 8000, 50, 500, 50, 8000, 5000, 50] * 3)
    f = grow_random_forest(rng, len(sizes), target_size=sizes)
    return cable_values(f, np.random.default_rng(13), a_kind="cable", dt=0.025, rhs=False)


def test_plain_solve_with_workspace_groups(torch_dev):
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = mixed_system()
    f = s.forest
    b = np.random.default_rng(1).standard_normal(f.n)
    xo = oracle.solve(f, s.diag, s.upper, b)
    for opts in (dict(), dict(level_sync=1), dict(bitwise=1), dict(rebalance_root=1, split_branches=1)):
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
        assert p.info["workspace_groups"] >= 6
        d = torch.from_numpy(s.diag).to(dev)
        u = torch.from_numpy(s.upper).to(dev)
        x = p.solve(d, u, torch.from_numpy(b).to(dev))
        xg = x.cpu().numpy()
        assert cell_rel_err(f, xg, xo) <= TOL, opts
        if opts.get("bitwise"):
            assert np.array_equal(xg, xo)


@pytest.mark.parametrize("opts", [dict(), dict(level_sync=1), dict(split_branches=1)])
def test_timestep_noise_vs_oracle(torch_dev, opts):
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = mixed_system()
    f = s.forest
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    c = torch.from_numpy(s.c).to(dev)
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    steps = 4
    for k in range(steps):
        p.timestep(d, u, c, V, V, noise_sigma=0.1, noise_seed=3, step=k)
    Vo = oracle.timeloop(f, s.diag, s.upper, s.c, steps, noise_seed=3, noise_sigma=0.1)
    assert cell_rel_err(f, V.cpu().numpy(), Vo) <= TOL


def test_timestep_constant_current_and_graph(torch_dev):
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = mixed_system()
    f = s.forest
    I = 0.1 * np.random.default_rng(4).standard_normal(f.n)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    c = torch.from_numpy(s.c).to(dev)
    It = torch.from_numpy(I).to(dev)
    steps = 6
    # eager, out of place
    Va = torch.zeros(f.n, dtype=torch.float64, device=dev)
    for k in range(steps):
        Va = p.timestep(d, u, c, Va, i_inj=It, step=k)
    Vo = oracle.timeloop(f, s.diag, s.upper, s.c, steps, I_const=I)
    assert cell_rel_err(f, Va.cpu().numpy(), Vo) <= TOL
    # captured graph, in place; replayed twice with eager work in between
    Vg = torch.zeros(f.n, dtype=torch.float64, device=dev)
    loop = p.timeloop(d, u, c, Vg, steps, i_inj=It)
    loop.launch()
    torch.cuda.synchronize()
    first = Vg.cpu().numpy().copy()
    assert np.array_equal(first, Va.cpu().numpy())
    _ = (d * 2).sum().item()
    loop.launch()
    torch.cuda.synchronize()
    Vo2 = oracle.timeloop(f, s.diag, s.upper, s.c, steps, V0=Vo, I_const=I)
    assert cell_rel_err(f, Vg.cpu().numpy(), Vo2) <= TOL
    loop.close()


def test_noise_graph_and_charge_conservation(torch_dev):
    """Column sums of A equal c, so per cell sum c V^{k+1} = sum c V^k + sum I^k."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = configs.c3(600)
    f = s.forest
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    c = torch.from_numpy(s.c).to(dev)
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    steps = 5
    loop = p.timeloop(d, u, c, V, steps, noise_sigma=0.1, noise_seed=3, first_step=0)
    loop.launch()
    torch.cuda.synchronize()
    Vg = V.cpu().numpy()
    cid = np.repeat(np.arange(f.ncells), np.diff(f.cell_offsets))
    total_I = np.zeros(f.ncells)
    idx = np.arange(f.n, dtype=np.int64)
    for k in range(steps):
        total_I += np.bincount(cid, weights=oracle.noise(3, k, idx, 0.1), minlength=f.ncells)
    lhs = np.bincount(cid, weights=s.c * Vg, minlength=f.ncells)
    scale = np.bincount(cid, weights=np.abs(s.c * Vg), minlength=f.ncells) + 1.0
    assert np.max(np.abs(lhs - total_I) / scale) < 1e-11
    # and a sample of cells against the oracle
    sample = np.arange(0, f.ncells, 37)
    sub = f.subset(sample)
    lo = f.cell_offsets[sample]
    hi = f.cell_offsets[sample + 1]
    gidx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    Vs = np.zeros(sub.n)
    for k in range(steps):
        Is = oracle.noise(3, k, gidx, 0.1)
        Vs = oracle.solve(sub, s.diag[gidx], s.upper[gidx], s.c[gidx] * Vs + Is)
    assert cell_rel_err(sub, Vg[gidx], Vs) <= TOL
    loop.close()


@pytest.mark.parametrize("opts", [dict(), dict(cell_lanes=2)], ids=["groups", "index_order_lanes"])
def test_adjoint_vs_oracle(torch_dev, opts):
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.adjoint import soma_traces
    s = configs.c5(48, size=300)
    f = s.forest
    steps, every = 23, 5
    target = s.meta["target"]
    I = s.meta["I"]
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    a_t = torch.from_numpy(s.a).to(dev).requires_grad_(True)
    c_t = torch.from_numpy(s.c).to(dev).requires_grad_(True)
    I_t = torch.from_numpy(I).to(dev).requires_grad_(True)
    tr = soma_traces(p, a_t, c_t, I_t, steps, every)
    loss = ((tr - torch.from_numpy(target).to(dev)) ** 2).sum()
    loss.backward()
    lo, ga, gc, gI, _ = oracle.adjoint(f, s.a, s.c, I, target, steps)
    assert abs(loss.item() - lo) <= 1e-12 * abs(lo)
    nr = f.parent >= 0

    def rel(x, y):
        return np.max(np.abs(x - y)) / np.max(np.abs(y))
    assert rel(a_t.grad.cpu().numpy()[nr], ga[nr]) <= 1e-10
    assert rel(c_t.grad.cpu().numpy(), gc) <= 1e-10
    assert rel(I_t.grad.cpu().numpy(), gI) <= 1e-10
    assert np.all(a_t.grad.cpu().numpy()[~nr] == 0)


def test_adjoint_central_differences_on_device(torch_dev):
    """Central differences (h = 1e-6) of one cell's loss term against the
    adjoint gradient, for a few parameters."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.adjoint import soma_traces
    s = configs.c5(6, size=120)
    f = s.forest
    steps = 12
    target = torch.from_numpy(s.meta["target"]).to(dev)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    base = {k: torch.from_numpy(v).to(dev) for k, v in (("a", s.a), ("c", s.c), ("I", s.meta["I"]))}

    def loss(params):
        tr = soma_traces(p, params["a"], params["c"], params["I"], steps, 4)
        return ((tr - target) ** 2).sum()

    params = {k: v.clone().requires_grad_(True) for k, v in base.items()}
    loss(params).backward()
    rng = np.random.default_rng(9)
    h = 1e-6
    for kind in ("a", "c", "I"):
        for _ in range(3):
            i = int(rng.integers(1, f.n))
            if kind == "a" and f.parent[i] < 0:
                continue
            vals = []
            for sgn in (1, -1):
                pp = {k: v.clone() for k, v in base.items()}
                pp[kind][i] += sgn * h
                vals.append(loss(pp).item())
            fd = (vals[0] - vals[1]) / (2 * h)
            g = params[kind].grad[i].item()
            assert abs(fd - g) <= 2e-5 * max(abs(g), 1e-2), (kind, i, fd, g)


@pytest.mark.parametrize("dt", [0.001, 0.025, 1.0])
def test_mixed_precision_refinement(torch_dev, dt):
    """FP32 storage + FP64 refinement converges to the FP64 solution of the
    FP32-rounded matrix (the matrix the refinement can reach)."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = configs.c4(dts=(dt,), ncells=768)[dt]
    f = s.forest
    d32 = s.diag.astype(np.float32)
    u32 = s.upper.astype(np.float32)
    xs = oracle.solve(f, d32.astype(np.float64), u32.astype(np.float64), s.rhs)
    oracle_its = oracle.refine(f, d32, u32, s.rhs, sweeps=3)
    # sweep 0 is an FP32 elimination of fl32(rhs): the oracle's FP32 solve of
    # the same system (plain order, IEEE division) is the reference.  Two FP32
    # eliminations of one system differ by rounding only, which is of the size
    # of either one's distance from the FP64 solution; a dropped or misplaced
    # term is orders of magnitude larger.
    e_o32 = cell_rel_err(f, oracle_its[0], xs)
    errs = []
    for opts in (dict(), dict(level_sync=1), dict(split_branches=1, max_group_unknowns=1024)):
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
        D = torch.from_numpy(d32).to(dev)
        U = torch.from_numpy(u32).to(dev)
        B = torch.from_numpy(s.rhs).to(dev)
        errs = []
        for sweeps in range(4):
            x = p.solve_mixed(D, U, B, sweeps=sweeps).cpu().numpy()
            errs.append(cell_rel_err(f, x, xs))
            if sweeps == 0:
                e32 = cell_rel_err(f, x, oracle_its[0])
                assert e32 <= 4.0 * e_o32 + 1e-7, (opts, e32, e_o32)
        assert errs[0] > 1e-10  # FP32 alone is far from FP64
        assert 0.25 * e_o32 <= errs[0] <= 4.0 * e_o32, (opts, errs[0], e_o32)
        assert errs[-1] <= 1e-11, (opts, errs)
        assert errs[1] < errs[0]
        # the oracle's own refinement converges the same way
        oerr = [cell_rel_err(f, xi, xs) for xi in oracle_its]
        assert oerr[-1] <= 1e-11
        # in-place form (x aliases rhs)
        B2 = B.clone()
        p.solve_mixed(D, U, B2, out=B2, sweeps=3)
        assert cell_rel_err(f, B2.cpu().numpy(), xs) <= 1e-11


def test_autotune_picks_a_measured_candidate(torch_dev, tmp_path):
    torch, dev = torch_dev
    from paper_1810_12742_amd.autotune import autotune
    s = configs.c3(400)
    f = s.forest
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    b = torch.from_numpy(np.random.default_rng(2).standard_normal(f.n)).to(dev)
    x = torch.empty_like(b)
    cands = [dict(max_group_unknowns=1024), dict(max_group_unknowns=2048, level_sync=1),
             dict(split_branches=1, cell_order=1)]
    cache = str(tmp_path / "tune.json")
    best, res = autotune(f.parent, f.cell_offsets, f.branch_offsets, lambda p: p.solve(d, u, b, out=x),
                         candidates=cands, reps=2, cache_path=cache)
    assert len(res) == 3 and best in cands
    assert min(res, key=lambda r: r[1])[0] == best
    best2, _ = autotune(f.parent, f.cell_offsets, f.branch_offsets, lambda p: 1 / 0, candidates=cands,
                        cache_path=cache)
    assert best2 == best  # served from the cache, nothing re-timed


def test_autotune_over_whole_cell_kernel_knobs(torch_dev, tmp_path):
    """The candidates the C2 bench tunes over (cut threshold and lanes per cell
    of the one-lane-per-cell kernel, packing of the LDS-resident kernel): each
    builds, solves to the oracle's tolerance, and the pick is the fastest."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.autotune import CELL_CANDIDATES, autotune, cached_pick
    s = configs.c2(1024)
    f = s.forest
    d, u, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.rhs))
    x = torch.empty_like(b)
    cache = str(tmp_path / "tune.json")
    best, res = autotune(f.parent, f.cell_offsets, f.branch_offsets, lambda p: p.solve(d, u, b, out=x),
                         candidates=CELL_CANDIDATES, reps=2, cache_path=cache)
    assert len(res) == len(CELL_CANDIDATES)
    assert min(res, key=lambda r: r[1])[0] == best
    assert cached_pick(f.parent, f.cell_offsets, f.branch_offsets, candidates=CELL_CANDIDATES,
                       cache_path=cache) == best
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    for opts in CELL_CANDIDATES:
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
        p.solve(d, u, b, out=x)
        torch.cuda.synchronize()
        assert cell_rel_err(f, x.cpu().numpy(), xo) <= 1e-12, opts
        p.close()


def test_device_byte_cap_forces_the_out_of_memory_paths(tmp_path):
    """HINES_DEVICE_BYTE_CAP makes the library's device allocations fail past
    a cap, as on a full device: a plan that does not fit returns
    HINES_ERR_OOM, and a time loop whose kept factors do not fit falls back
    to captured plain steps, which give the factored loop's result bit for
    bit (and the oracle's within 1e-12).  Each cap runs in a child process
    (the library reads it once)."""
    import os
    import subprocess
    import sys
    import torch
    from paper_1810_12742_amd import Plan
    s = configs.c3(300, seed=5)
    f = s.forest
    dev = torch.device("cuda")
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
    table_bytes = p.info["device_table_bytes"]
    d, u, c = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.c))
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    loop = p.timeloop(d, u, c, V, 4, noise_sigma=0.1, noise_seed=3)
    loop.launch()
    torch.cuda.synchronize()
    want = V.cpu().numpy()
    loop.close()
    p.close()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys, numpy as np, torch\n"
        "from workloads import configs\n"
        "from paper_1810_12742_amd import Plan, HinesError\n"
        "s = configs.c3(300, seed=5)\n"
        "f = s.forest\n"
        "dev = torch.device('cuda')\n"
        "try:\n"
        "    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)\n"
        "except HinesError as e:\n"
        "    print(e.code)\n"
        "    sys.exit(0)\n"
        "d, u, c = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.c))\n"
        "V = torch.zeros(f.n, dtype=torch.float64, device=dev)\n"
        "loop = p.timeloop(d, u, c, V, 4, noise_sigma=0.1, noise_seed=3)\n"
        "loop.launch()\n"
        "torch.cuda.synchronize()\n"
        "np.save(sys.argv[1], V.cpu().numpy())\n"
        "print('looped')\n")
    out = str(tmp_path / "v.npy")
    for cap, expect in ((1 << 20, "OOM"), (table_bytes + (1 << 20), "looped")):
        env = dict(os.environ, HINES_DEVICE_BYTE_CAP=str(cap), PYTHONPATH=root)
        print(f"cap {cap}: expect {expect}", flush=True)
        r = subprocess.run([sys.executable, "-c", code, out], capture_output=True, text=True, env=env, cwd=root,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        assert r.stdout.split()[-1] == expect
    got = np.load(out)
    assert np.array_equal(got, want)
    Vo = oracle.timeloop(f, s.diag, s.upper, s.c, 4, noise_seed=3, noise_sigma=0.1)
    err = np.max(np.abs(got - Vo)) / np.max(np.abs(Vo))
    assert err <= 1e-12

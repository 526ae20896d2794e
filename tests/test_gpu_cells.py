"""GPU parity of the cell-lane kernel (hines_solve / hines_timestep with
cell_lanes = 1, through the C-ABI) against the FP64 oracle: relative error
<= 1e-12 per cell (max norm), results independent of the run and of aliasing
x with the right-hand side."""
import numpy as np
import pytest

import oracle
from workloads import Forest, cable_values, configs, grow_random_forest

from test_cell_lanes import bushy_system

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


def solve_cells(torch_dev, f, diag, upper, rhs, alias=False):
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
    assert p.info["kernel"] == 3
    d = torch.from_numpy(np.ascontiguousarray(diag)).to(dev)
    u = torch.from_numpy(np.ascontiguousarray(upper)).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(rhs)).to(dev)
    x = b if alias else torch.empty_like(b)
    p.solve(d, u, b, out=x)
    torch.cuda.synchronize()
    out = x.cpu().numpy()
    p.close()
    return out


def test_c2_slice(torch_dev):
    s = configs.c2(1536)
    f = s.forest
    print("cells: c2 slice 1536", flush=True)
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    x1 = solve_cells(torch_dev, f, s.diag, s.upper, s.rhs)
    assert cell_rel_err(f, x1, xo) <= TOL
    x2 = solve_cells(torch_dev, f, s.diag, s.upper, s.rhs, alias=True)
    assert np.array_equal(x1, x2)


def test_fp32_storage_fp64_elimination(torch_dev):
    """hines_solve_stored32: the FP32 matrix widened on load and eliminated in
    FP64 equals the oracle's FP64 solve of the widened matrix to 1e-12, in
    place too; a plan without cell lanes is refused."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.hines import HinesError
    s = configs.c2(1536)
    f = s.forest
    print("cells: fp32 storage", flush=True)
    d32 = s.diag.astype(np.float32)
    u32 = s.upper.astype(np.float32)
    xo = oracle.solve(f, d32.astype(np.float64), u32.astype(np.float64), s.rhs)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
    D = torch.from_numpy(d32).to(dev)
    U = torch.from_numpy(u32).to(dev)
    b = torch.from_numpy(s.rhs).to(dev)
    x = p.solve_stored32(D, U, b)
    torch.cuda.synchronize()
    x1 = x.cpu().numpy()
    assert cell_rel_err(f, x1, xo) <= TOL
    p.solve_stored32(D, U, b, out=b)
    torch.cuda.synchronize()
    assert np.array_equal(b.cpu().numpy(), x1)
    p.close()
    g = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    with pytest.raises(HinesError):
        g.solve_stored32(D, U, torch.from_numpy(s.rhs).to(dev))
    g.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_bushy_trees_and_ragged_waves(torch_dev, seed):
    """Up to 6 children per compartment (middle-child merges, deeper stacks);
    90 cells, so the second wave is partly empty."""
    f, diag, upper = bushy_system(90, seed)
    print(f"cells: bushy seed {seed}", flush=True)
    rhs = np.random.default_rng(seed + 7).standard_normal(f.n)
    xo = oracle.solve(f, diag, upper, rhs)
    assert cell_rel_err(f, solve_cells(torch_dev, f, diag, upper, rhs), xo) <= TOL


def test_mixed_sizes_long_cable_and_single_compartments(torch_dev):
    """Cells of 1 to 20,000 compartments in one plan, an unbranched
    5,000-compartment cable among them."""
    rng = np.random.default_rng(21)
    sizes = np.array([1, 50, 500, 5000, 20000, 1, 2, 3, 500, 50] * 4)
    g = grow_random_forest(rng, len(sizes), target_size=sizes)
    n0 = g.n
    cab = 5000
    par = np.concatenate([g.parent, np.r_[-1, np.arange(n0, n0 + cab - 1)].astype(np.int32)])
    off = np.r_[g.cell_offsets, n0 + cab]
    f = Forest(par.astype(np.int32), off.astype(np.int64), None)
    s = cable_values(f, np.random.default_rng(22), a_kind="uniform", rhs=True)
    print("cells: mixed sizes", flush=True)
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    assert cell_rel_err(f, solve_cells(torch_dev, f, s.diag, s.upper, s.rhs), xo) <= TOL


def test_timestep_forms_and_graph(torch_dev):
    """c V + I, c V + sigma Z and plain c V right-hand sides formed in the
    kernel; a captured multi-step graph equals the eager steps."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = configs.c3(300)
    f = s.forest
    print("cells: timestep forms", flush=True)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    c = torch.from_numpy(s.c).to(dev)
    steps = 3
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    for k in range(steps):
        p.timestep(d, u, c, V, V, noise_sigma=0.1, noise_seed=5, step=k)
    Vo = oracle.timeloop(f, s.diag, s.upper, s.c, steps, noise_seed=5, noise_sigma=0.1)
    assert cell_rel_err(f, V.cpu().numpy(), Vo) <= TOL
    I = 0.1 * np.random.default_rng(4).standard_normal(f.n)
    It = torch.from_numpy(I).to(dev)
    Va = torch.zeros(f.n, dtype=torch.float64, device=dev)
    for k in range(steps):
        Va = p.timestep(d, u, c, Va, i_inj=It, step=k)
    Vo = oracle.timeloop(f, s.diag, s.upper, s.c, steps, I_const=I)
    assert cell_rel_err(f, Va.cpu().numpy(), Vo) <= TOL
    V0 = np.random.default_rng(6).standard_normal(f.n)
    Vc = p.timestep(d, u, c, torch.from_numpy(V0).to(dev), step=0)
    Voc = oracle.timeloop(f, s.diag, s.upper, s.c, 1, V0=V0, I_const=np.zeros(f.n))
    assert cell_rel_err(f, Vc.cpu().numpy(), Voc) <= TOL
    Vg = torch.zeros(f.n, dtype=torch.float64, device=dev)
    loop = p.timeloop(d, u, c, Vg, steps, i_inj=It)
    for rep in range(2):
        Vg.zero_()
        loop.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Vg.cpu().numpy(), Va.cpu().numpy()), rep
        _ = (d * 2).sum().item()
    loop.close()
    p.close()


def test_factored_time_loop_with_noise(torch_dev):
    """A captured loop on a cell-lane plan factors A once per launch and keeps
    V in the walk layout: it equals the eager steps bit for bit and the
    oracle's time loop to 1e-12, over two launches."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = configs.c3(300, seed=5)
    f = s.forest
    print("cells: factored noise loop", flush=True)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    c = torch.from_numpy(s.c).to(dev)
    steps = 4
    Ve = torch.zeros(f.n, dtype=torch.float64, device=dev)
    for k in range(2 * steps):
        p.timestep(d, u, c, Ve, Ve, noise_sigma=0.1, noise_seed=9, step=k)
    Vg = torch.zeros(f.n, dtype=torch.float64, device=dev)
    loop = p.timeloop(d, u, c, Vg, steps, noise_sigma=0.1, noise_seed=9)
    loop.launch()
    torch.cuda.synchronize()
    first = Vg.cpu().numpy().copy()
    Vo = oracle.timeloop(f, s.diag, s.upper, s.c, steps, noise_seed=9, noise_sigma=0.1)
    assert cell_rel_err(f, first, Vo) <= TOL
    loop2 = p.timeloop(d, u, c, Vg, steps, first_step=steps, noise_sigma=0.1, noise_seed=9)
    loop2.launch()
    torch.cuda.synchronize()
    assert np.array_equal(Vg.cpu().numpy(), Ve.cpu().numpy())
    loop.close()
    loop2.close()
    p.close()


def test_edge_cases_empty_single_compartments_and_largest_cell(torch_dev):
    """An empty forest (solve, time step, time loop, FP32 storage: nothing to
    do); 100 one-compartment cells; a cell of 65,535 compartments (the
    largest a cell lane takes, cut over several lanes) among 40 small ones.
    Solves and a kept-factor loop of 3 steps against the oracle."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from workloads import Forest, cable_values, grow_random_forest
    print("cells: empty forest", flush=True)
    pe = Plan(np.zeros(0, dtype=np.int32), np.zeros(1, dtype=np.int64), None, cell_lanes=1)
    e = torch.zeros(0, dtype=torch.float64, device=dev)
    e32 = torch.zeros(0, dtype=torch.float32, device=dev)
    pe.solve(e, e, e, out=e)
    pe.timestep(e, e, e, e, e, noise_sigma=0.1, noise_seed=1)
    pe.solve_stored32(e32, e32, e, out=e)
    le = pe.timeloop(e, e, e, e, 3, noise_sigma=0.1, noise_seed=1)
    le.launch()
    torch.cuda.synchronize()
    le.close()
    pe.close()
    singles = Forest(np.full(100, -1, dtype=np.int32), np.arange(101, dtype=np.int64), np.arange(101, dtype=np.int64))
    rng = np.random.default_rng(30)
    sizes = np.r_[65535, np.full(40, 300)]
    big = grow_random_forest(rng, len(sizes), target_size=sizes)
    for name, f in (("singles", singles), ("largest cell", big)):
        print(f"cells: {name}", flush=True)
        s = cable_values(f, np.random.default_rng(31), a_kind="cable", rhs=True)
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
        d, u, c, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.c, s.rhs))
        x = p.solve(d, u, b)
        torch.cuda.synchronize()
        assert cell_rel_err(f, x.cpu().numpy(), oracle.solve(f, s.diag, s.upper, s.rhs)) <= TOL
        V = torch.zeros(f.n, dtype=torch.float64, device=dev)
        loop = p.timeloop(d, u, c, V, 3, noise_sigma=0.1, noise_seed=4)
        loop.launch()
        torch.cuda.synchronize()
        Vo = oracle.timeloop(f, s.diag, s.upper, s.c, 3, noise_seed=4, noise_sigma=0.1)
        assert cell_rel_err(f, V.cpu().numpy(), Vo) <= TOL
        loop.close()
        if name == "largest cell":  # its groups exceed the 16-bit branch records: only the FP32+refinement solve refuses
            from paper_1810_12742_amd.hines import HinesError
            with pytest.raises(HinesError):
                p.solve_mixed(d.float(), u.float(), b)
        p.close()


@pytest.mark.parametrize("which", ["c3", "bushy"])
def test_assembled_step(torch_dev, which):
    """hines_timestep_assembled: the diagonal c + g + incident edge
    conductances formed inside the cell-lane solve equals the oracle's
    assembled step to 1e-12 (cells cut over several lanes included), in place
    too; a plan without cell lanes is refused."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.hines import HinesError
    if which == "c3":
        s = configs.c3(300, seed=7)
        f, upper = s.forest, s.upper
    else:
        f, _, upper = bushy_system(90, 3)
    print(f"cells: assembled step {which}", flush=True)
    rng = np.random.default_rng(17)
    n = f.n
    c = rng.uniform(0.1, 1.0, n)
    g = rng.uniform(0.0, 3.0, n)
    ge = rng.standard_normal(n)
    v = rng.standard_normal(n)
    want = oracle.timestep_assembled(f, upper, c, g, ge, v)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=1)
    G, U, C, GE, V = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (g, upper, c, ge, v))
    out = p.timestep_assembled(G, U, C, GE, V)
    torch.cuda.synchronize()
    x1 = out.cpu().numpy()
    assert cell_rel_err(f, x1, want) <= TOL
    p.timestep_assembled(G, U, C, GE, V, V)
    torch.cuda.synchronize()
    assert np.array_equal(V.cpu().numpy(), x1)
    p.close()
    q = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    with pytest.raises(HinesError):
        q.timestep_assembled(G, U, C, GE, V, V)
    q.close()


def test_layout_resident_solve_through_the_c_abi():
    """hines_to_layout / hines_solve_layout / hines_from_layout on cell-lane
    plans (whole cells, cells cut over two to four lanes, padding): the same
    elimination as hines_solve on the same plan, bit for bit, and within 1e-12
    of the oracle; x may alias rhs in the layout."""
    import ctypes
    import torch
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.hines import load
    dev = torch.device("cuda")
    lib = load()
    P = ctypes.c_void_p
    for s in (configs.c2(3000), configs.c3(300), configs.random_system(200, seed=5)):
        f = s.forest
        print(f"layout solve: {f.ncells} cells, {f.n} unknowns", flush=True)
        rhs = s.rhs if np.any(s.rhs) else np.random.default_rng(1).standard_normal(f.n)
        xo = oracle.solve(f, s.diag, s.upper, rhs)
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=True)
        d, u, b = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (s.diag, s.upper, rhs))
        m = ctypes.c_int64()
        assert lib.hines_layout_size(p._h, ctypes.byref(m)) == 0 and m.value == p.layout_size >= f.n
        dl, ul, bl = p.to_layout(d), p.to_layout(u), p.to_layout(b)
        xl = torch.empty_like(bl)
        st = lib.hines_solve_layout(p._h, P(dl.data_ptr()), P(ul.data_ptr()), P(bl.data_ptr()), P(xl.data_ptr()),
                                    f.ncells, None)
        assert st == 0
        x = p.from_layout(xl).cpu().numpy()
        assert cell_rel_err(f, x, xo) <= 1e-12
        xs = p.solve(d, u, b).cpu().numpy()
        assert np.array_equal(x, xs)
        p.solve_layout(dl, ul, bl, out=bl)  # in place
        assert np.array_equal(p.from_layout(bl).cpu().numpy(), x)
        assert lib.hines_solve_layout(p._h, P(dl.data_ptr()), P(ul.data_ptr()), P(bl.data_ptr()),
                                      P(dl.data_ptr()), f.ncells, None) == 12
        p.close()
    q = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    assert lib.hines_layout_size(q._h, ctypes.byref(m)) == 12  # not a cell-lane plan

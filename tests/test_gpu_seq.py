"""GPU parity of the index-order cell lanes (plan option cell_lanes 2, kernel
k_solve_seq) through the C-ABI against the FP64 oracle, within 1e-12
relative error per cell (max norm): C2 slices with cut cells, trees with many
children per compartment, trees too wide for the slots (walked depth-first),
unbranched and single-compartment cells, the full 65,536-cell workload, the
right-hand side aliasing x, the time-step forms and their captured loop,
and the forms such a plan refuses."""
import numpy as np
import pytest

import oracle
from tests.test_cell_lanes import bushy_system
from tests.test_gpu_solve import TOL, cell_rel_err, gpu_solve, torch_dev  # noqa: F401
from tests.test_seq_lanes import wide_system
from workloads import configs
from workloads.configs import CableSystem

pytestmark = pytest.mark.gpu


def _system(f, diag, upper, seed=3):
    rhs = np.random.default_rng(seed).standard_normal(f.n)
    return CableSystem(f, -upper, np.zeros(f.n), diag, upper, rhs)


@pytest.mark.parametrize("ncells", [40, 700])
def test_seq_c2_slices(torch_dev, ncells):
    s = configs.c2(ncells)
    xo = oracle.solve(s.forest, s.diag, s.upper, s.rhs)
    for cut in (60, 80):
        print(f"seq c2 {ncells} cells, cut {cut}", flush=True)
        x = gpu_solve(torch_dev, s, cell_lanes=2, cell_cut_percent=cut)
        assert cell_rel_err(s.forest, x, xo) <= TOL


def test_seq_bushy_wide_and_edge_cells(torch_dev):
    rng = np.random.default_rng(4)
    cases = [bushy_system(90, 0), wide_system(100, 40), wide_system(100, 20)]
    sizes = [1, 1, 5000, 1, 20000, 3]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    par = np.full(off[-1], -1, dtype=np.int32)
    for c, m in enumerate(sizes):
        for i in range(1, m):
            par[off[c] + i] = off[c] + (i - 1 if c == 2 else int(rng.integers(max(0, i - 40), i)))
    a = rng.uniform(0.5, 2.0, off[-1])
    a[off[:-1]] = 0.0
    diag = rng.uniform(0.1, 1.0, off[-1]) + a
    np.add.at(diag, par[par >= 0], a[par >= 0])
    from workloads.trees import Forest
    cases.append((Forest(par, off, None), diag, -a))
    for i, (f, d, u) in enumerate(cases):
        print(f"seq case {i}: {f.ncells} cells, {f.n} compartments", flush=True)
        s = _system(f, d, u, seed=i)
        xo = oracle.solve(f, d, u, s.rhs)
        x = gpu_solve(torch_dev, s, cell_lanes=2)
        assert cell_rel_err(f, x, xo) <= TOL


def test_seq_rhs_alias_and_determinism(torch_dev):
    s = configs.c2(512)
    xo = oracle.solve(s.forest, s.diag, s.upper, s.rhs)
    x1 = gpu_solve(torch_dev, s, alias=True, cell_lanes=2)
    x2 = gpu_solve(torch_dev, s, cell_lanes=2)
    assert np.array_equal(x1, x2)
    assert cell_rel_err(s.forest, x1, xo) <= TOL


def test_seq_full_c2(torch_dev):
    """The full 65,536-cell workload, against the oracle and, bit for bit
    aside, against the depth-first cell-lane kernel within the same bar."""
    s = configs.c2()
    f = s.forest
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    for cut in (60, 80):
        print(f"seq full c2, cut {cut}", flush=True)
        x = gpu_solve(torch_dev, s, cell_lanes=2, cell_cut_percent=cut)
        assert cell_rel_err(f, x, xo) <= TOL


def test_seq_timestep_forms_and_graph(torch_dev):
    """c V + I, c V + sigma Z and plain c V right-hand sides formed in the
    index-order kernel, against the oracle's time loop; a captured graph of
    the steps equals the eager steps on every replay."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    s = configs.c3(300)
    f = s.forest
    print("seq: timestep forms", flush=True)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=2)
    assert p.info["kernel"] == 5
    d, u, c = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.c))
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
    for rep in range(3):
        Vg.zero_()
        loop.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Vg.cpu().numpy(), Va.cpu().numpy()), rep
        _ = (d * 2).sum().item()
    loop.close()
    p.close()


def test_seq_plan_refuses_the_depth_first_forms(torch_dev):
    """The solver layout, the FP32-stored matrix and the assembled step are
    forms of the depth-first cell-lane plan: an index-order plan refuses them
    with a status, and its solve still runs."""
    torch, dev = torch_dev
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.hines import HinesError
    s = configs.c2(64)
    f = s.forest
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=2)
    assert p.info["kernel"] == 5
    d, u, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.rhs))
    with pytest.raises(HinesError):
        p.layout_size
    with pytest.raises(HinesError):
        p.solve_stored32(d.float(), u.float(), b)
    with pytest.raises(HinesError):
        p.timestep_assembled(d, u, d, d, b)
    x = p.solve(d, u, b)
    torch.cuda.synchronize()
    assert cell_rel_err(f, x.cpu().numpy(), oracle.solve(f, s.diag, s.upper, s.rhs)) <= TOL
    p.close()

"""GPU parity at the sizes of the measured configurations.

* Config 3 (batching + time loop): 1,000 implicit-Euler steps captured in one
  graph, on a subset of 64 cells from each size class (50, 500, 5,000 and
  20,000 compartments), against the oracle's time loop over the same 1,000
  steps (paper §1: one solve of the discrete system per step).  The oracle
  takes about a second per 100 steps at this size, so the subset is 64 cells
  per class, not the full 200,000.  The full 200,000 cells run once more in
  the bench's plan over 3 steps, and 128 of them are checked against the
  oracle.
* Config 4 (precision): the full C2 cells at dt = 1.0 on the bench's plan,
  FP32 sweep 0 and 3 refinement sweeps against the oracle.
* Config 5 (differentiation): the full 16,384 cells x 1,000 compartments over
  100 steps with checkpoints every 10; central differences (h = 1e-6) on 32
  parameters drawn with seed 5 from the edge conductances, capacitive terms
  and injected currents, against the adjoint gradient.  Each difference is
  taken on the owning cell's loss term, which is the only one the parameter
  changes (cells are independent).
"""
import time

import numpy as np
import pytest

import oracle
from workloads import configs

pytestmark = pytest.mark.gpu


def cell_rel_err(f, x, xo):
    err = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    scale = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(err / np.maximum(scale, 1e-300)))


def c3_class_subset(per_class: int):
    """The first `per_class` cells of every size class of the config-3 recipe."""
    ncells = 1
    while True:
        ncells *= 2
        sizes = configs.c3_sizes(ncells)
        if min(int(np.sum(sizes == s)) for s in configs.C3_SIZES) >= per_class:
            break
    s = configs.c3(ncells)
    sizes = np.diff(s.forest.cell_offsets)
    pick = np.sort(np.concatenate([np.flatnonzero(sizes == z)[:per_class] for z in configs.C3_SIZES]))
    f = s.forest.subset(pick)
    idx = np.concatenate([np.arange(s.forest.cell_offsets[c], s.forest.cell_offsets[c + 1]) for c in pick])
    return f, s.diag[idx], s.upper[idx], s.c[idx]


def test_c3_thousand_captured_steps_per_size_class():
    import torch
    from paper_1810_12742_amd import Plan
    dev = torch.device("cuda")
    f, diag, upper, c = c3_class_subset(64)
    steps = 1000
    print(f"c3 subset: {f.ncells} cells, {f.n} unknowns, {steps} steps", flush=True)
    t0 = time.perf_counter()
    Vo = oracle.timeloop(f, diag, upper, c, steps, noise_seed=3, noise_sigma=0.1)
    print(f"oracle {time.perf_counter() - t0:.1f} s", flush=True)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, cell_lanes=True)
    d = torch.from_numpy(diag).to(dev)
    u = torch.from_numpy(upper).to(dev)
    cc = torch.from_numpy(c).to(dev)
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    loop = p.timeloop(d, u, cc, V, steps, noise_sigma=0.1, noise_seed=3, first_step=0)
    loop.launch()
    torch.cuda.synchronize()
    err = cell_rel_err(f, V.cpu().numpy(), Vo)
    print(f"1000-step error {err:.2e}", flush=True)
    assert err <= 1e-12
    loop.close()
    p.close()


def test_c3_full_configuration_sampled_cells():
    """The full config-3 network (200,000 cells, 6.3e8 compartments) in the
    launch configuration the bench times: the autotuner's shipped pick for it
    and the kept-factor loop captured in one graph, here over 3 noise steps.
    32 cells of every size class, spread over the network, are compared with
    the oracle's time loop on those cells alone (cells are independent), the
    draws keyed by the cells' user indices in the full network.  One step with
    the matrix assembled inside the solve follows, on the same plan, checked
    the same way."""
    import torch
    import bench
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.autotune import SHIPPED_CACHE, cached_pick
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    s = configs.c3(configs.C3_CELLS)
    f = s.forest
    print(f"c3 full: {f.ncells} cells, {f.n} unknowns, generated in {time.perf_counter() - t0:.0f} s", flush=True)
    opts = cached_pick(f.parent, f.cell_offsets, f.branch_offsets, candidates=bench.C3_CANDIDATES,
                       cache_path=SHIPPED_CACHE)
    print(f"plan options {opts}", flush=True)
    assert opts is not None and opts.get("cell_lanes")
    plan = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    d, u, c = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.c))
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    steps = 3
    loop = plan.timeloop(d, u, c, V, steps, first_step=0, noise_sigma=0.1, noise_seed=3)
    loop.launch()
    torch.cuda.synchronize()
    sizes = np.diff(f.cell_offsets)
    pick = []
    for z in configs.C3_SIZES:
        cls = np.flatnonzero(sizes == z)
        pick.append(cls[np.linspace(0, cls.size - 1, 32).astype(np.int64)])
    pick = np.unique(np.concatenate(pick))
    idx = np.concatenate([np.arange(f.cell_offsets[q], f.cell_offsets[q + 1]) for q in pick])
    tidx = torch.from_numpy(idx).to(dev)
    got = V[tidx].cpu().numpy()
    loop.close()
    # one step with the matrix assembled inside the solve (diagonal c + g +
    # incident edge conductances), which the bench times beside the loop,
    # from the loop's state
    rng = np.random.default_rng(5)
    g = rng.uniform(0.0, 1.0, f.n)
    ge = -65.0 * rng.uniform(0.0, 1.0, f.n)
    G, GE = torch.from_numpy(g).to(dev), torch.from_numpy(ge).to(dev)
    plan.timestep_assembled(G, u, c, GE, V, V)
    torch.cuda.synchronize()
    got_a = V[tidx].cpu().numpy()
    plan.close()
    del G, GE, V, d, u, c
    sub = f.subset(pick)
    Vo = oracle.timeloop(sub, s.diag[idx], s.upper[idx], s.c[idx], steps, noise_seed=3, noise_sigma=0.1, index=idx)
    err = cell_rel_err(sub, got, Vo)
    print(f"{pick.size} sampled cells, {idx.size} unknowns: error {err:.2e}", flush=True)
    assert err <= 1e-12
    Va = oracle.timestep_assembled(sub, s.upper[idx], s.c[idx], g[idx], ge[idx], got)
    err_a = cell_rel_err(sub, got_a, Va)
    print(f"assembled step on the sampled cells: error {err_a:.2e}", flush=True)
    assert err_a <= 1e-12


def test_c4_full_configuration_refinement():
    """Config 4 at full size (the 65,536 C2 cells, dt = 1.0, the least
    dominant case) on the plan the bench times: FP32 storage and elimination,
    FP64 residual and accumulation, 3 sweeps.  Sweep 0 against the oracle's
    FP32 solve of the same system (rounding only: within 4x the oracle's own
    distance from the FP64 solution), 3 sweeps within 1e-11 of the oracle's
    FP64 solve of the FP32-stored matrix."""
    import torch
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.autotune import CELL_CANDIDATES, SHIPPED_CACHE, cached_pick
    dev = torch.device("cuda")
    s = configs.c4(dts=(1.0,))[1.0]
    f = s.forest
    d32 = s.diag.astype(np.float32)
    u32 = s.upper.astype(np.float32)
    xs = oracle.solve(f, d32.astype(np.float64), u32.astype(np.float64), s.rhs)
    its = oracle.refine(f, d32, u32, s.rhs, sweeps=0)
    e_o32 = cell_rel_err(f, its[0], xs)
    opts = cached_pick(f.parent, f.cell_offsets, f.branch_offsets, candidates=CELL_CANDIDATES,
                       cache_path=SHIPPED_CACHE) or {}
    print(f"c4 full: {f.ncells} cells, {f.n} unknowns, plan {opts}", flush=True)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    D, U, B = (torch.from_numpy(a).to(dev) for a in (d32, u32, s.rhs))
    x0 = p.solve_mixed(D, U, B, sweeps=0).cpu().numpy()
    x3 = p.solve_mixed(D, U, B, sweeps=3).cpu().numpy()
    p.close()
    e0 = cell_rel_err(f, x0, its[0])
    e3 = cell_rel_err(f, x3, xs)
    print(f"sweep 0 against the oracle's FP32 solve {e0:.2e} (oracle FP32 vs FP64 {e_o32:.2e}); "
          f"3 sweeps {e3:.2e}", flush=True)
    assert e0 <= 4.0 * e_o32 + 1e-7
    assert e3 <= 1e-11


def test_c5_central_differences_full_configuration():
    import torch
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.adjoint import soma_traces
    dev = torch.device("cuda")
    s = configs.c5()
    f = s.forest
    steps, every = s.meta["steps"], s.meta["checkpoint_every"]
    print(f"c5: {f.ncells} cells, {f.n} unknowns, {steps} steps", flush=True)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets)
    target = torch.from_numpy(s.meta["target"]).to(dev)
    base = {"a": torch.from_numpy(s.a).to(dev), "c": torch.from_numpy(s.c).to(dev),
            "I": torch.from_numpy(s.meta["I"]).to(dev)}
    params = {k: v.clone().requires_grad_(True) for k, v in base.items()}
    tr = soma_traces(p, params["a"], params["c"], params["I"], steps, every)
    ((tr - target) ** 2).sum().backward()
    grads = {k: v.grad.cpu().numpy() for k, v in params.items()}
    # 32 parameters drawn uniformly from {a_e (non-root)} U {c_i} U {I_i}
    nonroot = np.flatnonzero(f.parent >= 0)
    pool = len(nonroot) + 2 * f.n
    rng = np.random.default_rng(5)
    draws = rng.choice(pool, size=32, replace=False)
    cell_of = np.searchsorted(f.cell_offsets, np.arange(f.n), side="right") - 1
    h = 1e-6
    worst = 0.0
    with torch.no_grad():
        for q in draws:
            if q < len(nonroot):
                kind, i = "a", int(nonroot[q])
            elif q < len(nonroot) + f.n:
                kind, i = "c", int(q - len(nonroot))
            else:
                kind, i = "I", int(q - len(nonroot) - f.n)
            cell = int(cell_of[i])
            vals = []
            for sgn in (1.0, -1.0):
                pp = {k: v.clone() for k, v in base.items()}
                pp[kind][i] += sgn * h
                t = soma_traces(p, pp["a"], pp["c"], pp["I"], steps, every)
                vals.append(float(((t[:, cell] - target[cell]) ** 2).sum().item()))
            fd = (vals[0] - vals[1]) / (2 * h)
            g = float(grads[kind][i])
            # round-off of a cell's loss term (about 1e2) over 2h bounds the
            # difference quotient's absolute error near 1e-7
            tol = 1e-5 * abs(g) + 5e-7
            worst = max(worst, abs(fd - g) / max(tol, 1e-300))
            assert abs(fd - g) <= tol, (kind, i, fd, g)
    print(f"32 central differences: worst |fd - g| / tol = {worst:.3f}", flush=True)
    p.close()

"""Benchmark of the batched Hines solve on one MI355X.

Default workload (the headline): 65,536 synthetic neuron-shaped cells (random
binary dendritic trees, 16-256 branches, geometric branch lengths of mean 12
capped at 64, about 1.06e8 compartments), cable-equation coefficients at
dt = 0.025, one right-hand side; seed 1.  Inputs are resident in HBM before
the timed region.  A step is one hines_solve over all cells: every matrix
entry is read from HBM once and the solution written once (32 algorithmic
bytes per compartment).  The same line carries the FP32-storage + FP64
refinement form on the same cells at dt in {0.001, 0.025, 1.0}, the
layout-resident solve, the small single-solve case (4,096 cells of 75
compartments), the oracle timed on the host's cores, and (key ``c3``, unless
``--no-c3``) the batched time loop below with the autotuner's cached pick, 1,000
steps per captured graph.

Other workloads (``--workload``): ``c3`` the batched implicit-Euler time loop
(200,000 cells of 50/500/5,000/20,000 compartments, noise current, K steps per
captured graph), ``c5`` the adjoint (16,384 cells x 1,000 compartments, 100
steps, checkpoints every 10), ``scaling`` the paper's comparison of the
one-thread-per-cell solver with the fine-grained one (Figure 7.1's axes): solve
time of both kernels on the first 64 ... 65,536 cells of the headline workload,
``branching`` the same comparison against the branching probability of
paper-style trees (Figure 7.2's axes).

Prints one JSON line.  ``--gpus`` above 1 is refused: the solve is per cell
and needs no communication, and the bench measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Hines unknowns solved/s and % HBM roofline, plain FP64 vs batched/FP32+refine"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UNKNOWN = 32  # read diag, upper, rhs; write x (FP64)
# The fine-grained (flow kernel) plan used for comparisons.
C2_FLOW_OPTIONS = dict(max_group_unknowns=1536, split_branches=0, cell_order=0, group_width=64)
CALIB_BYTES = 512 << 20  # bytes read (and written) by one calibration copy
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hines_solve_c2.json")
TRAFFIC_FILE_C3 = os.path.join(ROOT, "profiles", "traffic_k_cells_step_c3.json")
KERNEL_SRC_DIR = os.path.join(ROOT, "paper_1810_12742_amd", "csrc")
C4_DTS = (0.001, 0.025, 1.0)
# the time loop's plans: the group plan and the cell-lane cut knobs
C3_CANDIDATES = [dict(max_group_unknowns=3000)] + [dict(cell_lanes=1, cell_cut_percent=cp, cell_max_cuts=mc)
                                                   for cp in (60, 80, 110) for mc in (1, 3)]


def _kernel_sha() -> str:
    """SHA-256 over the kernel and plan-builder sources (both decide the bytes
    a launch moves)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_SRC_DIR)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(KERNEL_SRC_DIR, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _traffic(n_launches_per_solve: int, path: str = TRAFFIC_FILE):
    """HBM bytes per launch from the committed PMC measurement, if it was taken
    on the current kernel source; else None."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != _kernel_sha():
        return None
    return t.get("bytes_per_launch")


def copy_calibration(torch, dev):
    """A plain device copy of CALIB_BYTES (read and write), three times: the
    reference kernel whose counter readings scale the HBM byte counters."""
    src = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cell_rel_err(f, x, xo):
    e = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    s = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(e / np.maximum(s, 1e-300)))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(system, threads: int, budget_s: float):
    import oracle
    f = system.forest
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.solve(f, system.diag, system.upper, system.rhs, nthreads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return f.n * reps / el, reps, el


def cpu_baseline(system, budget_s: float = 10.0):
    """The FP64 oracle on the host: repeated full solves of the same workload
    until about ``budget_s`` seconds of wall time have passed, with every host
    thread (OpenMP over cells) and with one thread."""
    import oracle
    oracle.build(force=False)
    f = system.forest
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v, reps, el = _oracle_rate(system, threads, budget_s)
    v1, reps1, el1 = _oracle_rate(system, 1, budget_s)
    return {"value": v, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
            "sample": f"full workload ({f.n} unknowns), {reps} solves, {el:.1f} s, OpenMP over cells",
            "cpu_model": _cpu_model(),
            "single_thread": {"value": v1, "unit": "unknowns/s", "cores": 1,
                              "sample": f"full workload, {reps1} solves, {el1:.1f} s"}}


def run_c1(torch, dev, reps: int = 20):
    """Config 1: 4,096 full binary trees of 75 compartments, one solve, in
    the small-workload regime (the whole system fits the on-chip caches).
    Each solve is timed alone after a 1 GiB device write that evicts the
    caches; reported per plan kind, median over reps."""
    from workloads import configs
    from paper_1810_12742_amd import Plan
    import oracle
    s = configs.c1()
    f = s.forest
    d, u, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.rhs))
    x = torch.empty_like(b)
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    xo = oracle.solve(f, s.diag, s.upper, s.rhs)
    out = {"workload": "c1: 4,096 full binary trees, 15 branches x 5 compartments, seed 0, one solve",
           "unknowns": f.n, "cache_flush_bytes": flush.numel() * 8}
    for name, opts in (("resident", dict(resident=1)), ("flow", dict(C2_FLOW_OPTIONS)),
                       ("cell_lanes", dict(cell_lanes=1))):
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
        times = []
        for k in range(reps + 2):
            flush.fill_(float(k))
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record(stream)
            p.solve(d, u, b, out=x, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if k >= 2:
                times.append(e0.elapsed_time(e1) * 1e3)
        us = float(np.median(times))
        out[name] = {"us_per_solve": us, "unknowns_per_s": f.n / (us * 1e-6),
                     "max_rel_err_vs_oracle": cell_rel_err(f, x.cpu().numpy(), xo)}
        p.close()
    del flush
    return out


def fp32_refine(torch, dev, plan, s, fp64_ms, reps, check):
    """FP32 storage + FP64 refinement on the same cells at each dt: errors
    after 0..3 sweeps against the FP64 solution of the FP32-rounded matrix, and
    throughput with 3 sweeps against the FP64 solve.  On a cell-lane plan also
    the FP32-stored matrix eliminated in FP64 (one sweep, no refinement)."""
    import oracle
    f = s.forest
    out = {}
    b = torch.from_numpy(s.rhs).to(dev)
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()
    nonroot = f.parent >= 0
    child_a = np.bincount(f.parent[nonroot], weights=s.a[nonroot], minlength=f.n)
    for dt in C4_DTS:
        c = s.meta["sigma_cm"] / dt
        diag = c + np.where(nonroot, s.a, 0.0) + child_a
        d32 = diag.astype(np.float32)
        u32 = s.upper.astype(np.float32)
        D = torch.from_numpy(d32).to(dev)
        U = torch.from_numpy(u32).to(dev)
        rec = {"dominance_ratio_median": float(np.median(diag / np.maximum(diag - c, 1e-300)))}
        if check:
            xs = oracle.solve(f, d32.astype(np.float64), u32.astype(np.float64), s.rhs)
            errs = []
            for sw in range(4):
                plan.solve_mixed(D, U, b, out=x, sweeps=sw)
                errs.append(cell_rel_err(f, x.cpu().numpy(), xs))
            rec["err_after_sweeps"] = errs
        ms = _time(torch, lambda: plan.solve_mixed(D, U, b, out=x, sweeps=3), reps, 2, stream)
        rec["ms_3_sweeps"] = ms
        rec["unknowns_per_s"] = f.n / (ms * 1e-3)
        rec["speed_vs_fp64"] = fp64_ms / ms
        if plan.info["kernel"] == 3:
            st = {}
            if check:
                plan.solve_stored32(D, U, b, out=x)
                st["max_rel_err"] = cell_rel_err(f, x.cpu().numpy(), xs)
            ms32 = _time(torch, lambda: plan.solve_stored32(D, U, b, out=x, stream=stream), reps, 2, stream)
            st.update(ms=ms32, unknowns_per_s=f.n / (ms32 * 1e-3), speed_vs_fp64=fp64_ms / ms32)
            rec["fp32_storage_fp64_elimination"] = st
        out[str(dt)] = rec
        del D, U
    return out


def layout_resident(args, torch, plan, s, d, u, b, x, stream):
    """The same solve with d, u, b and x already in the cell-lane solver's
    layout (hines_solve_layout): the permutation into and out of the layout is
    timed apart, as the paper times its permutation kernels apart from its
    solver kernel (section 7)."""
    f = s.forest
    dl, ul, bl = (plan.to_layout(a, stream=stream) for a in (d, u, b))
    xl = torch.empty_like(bl)
    m = plan.layout_size
    ms = _time(torch, lambda: plan.solve_layout(dl, ul, bl, out=xl, stream=stream), args.steps, args.warmup, stream)
    ms_in = _time(torch, lambda: plan.to_layout(b, dst=bl, stream=stream), args.steps, args.warmup, stream)
    ms_out = _time(torch, lambda: plan.from_layout(xl, dst=x, stream=stream), args.steps, args.warmup, stream)
    rec = {"ms_per_solve": ms, "unknowns_per_s": f.n / (ms * 1e-3), "layout_slots": m,
           "padding_share": 1.0 - f.n / m,
           "roofline_frac": BYTES_PER_UNKNOWN * f.n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "to_layout_ms_per_array": ms_in, "from_layout_ms": ms_out,
           "with_permutations_ms": ms + 3 * ms_in + ms_out}
    if not args.no_check:
        import oracle
        plan.solve_layout(dl, ul, bl, out=xl, stream=stream)
        plan.from_layout(xl, dst=x, stream=stream)
        rec["max_rel_err_vs_oracle"] = cell_rel_err(f, x.cpu().numpy(), oracle.solve(f, s.diag, s.upper, s.rhs))
    del dl, ul, bl, xl
    return rec


def run_c2(args, torch, dev):
    from workloads import configs
    from paper_1810_12742_amd import Plan

    s = configs.c2()
    f = s.forest
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    b = torch.from_numpy(s.rhs).to(dev)
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()
    tried = []
    if args.options:
        opts = json.loads(args.options)
    else:
        # the autotuner's pick among the whole-cell kernels and their knobs,
        # from the shipped cache when this device and workload have been tuned
        from paper_1810_12742_amd.autotune import CELL_CANDIDATES, autotune
        opts, tried = autotune(f.parent, f.cell_offsets, f.branch_offsets,
                               lambda p: p.solve(d, u, b, out=x, stream=stream), candidates=CELL_CANDIDATES,
                               reps=5, cache_path=args.tune_cache)
    t0 = time.perf_counter()
    plan = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    setup_s = time.perf_counter() - t0
    info = plan.info
    ms = _time(torch, lambda: plan.solve(d, u, b, out=x, stream=stream), args.steps, args.warmup, stream)

    if args.copy_calibration:
        copy_calibration(torch, dev)

    err = None
    if not args.no_check:
        import oracle
        err = cell_rel_err(f, x.cpu().numpy(), oracle.solve(f, s.diag, s.upper, s.rhs))

    n = f.n
    launches = max(1, int(info["nclasses"]))
    bytes_per_solve = BYTES_PER_UNKNOWN * n
    achieved = bytes_per_solve / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": n / (ms * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "c2: 65,536 random dendritic cells, 16-256 branches, geometric(12) branch "
                        "lengths, dt=0.025, one FP64 solve per step",
            "ncells": f.ncells, "unknowns": n, "groups": info["ngroups"], "launches_per_step": launches,
            "kernel": {5: "index-order cell lanes", 4: "LDS-resident", 3: "cell lanes", 1: "flow",
                       2: "bitwise"}.get(info["kernel"], "level-synchronous"),
            "options": opts, "setup_s": round(setup_s, 3),
            "autotune_ms": [[o, round(t, 4)] for o, t in tried],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": _traffic(launches),
            "kernel": {5: "k_solve_seq", 4: "k_solve_res", 3: "k_solve_cells",
                       1: "k_solve_flow"}.get(info["kernel"], "k_solve_level"),
            "bytes_per_launch": bytes_per_solve / launches,
            "avg_launch_us": ms * 1e3 / launches,
        },
        "max_rel_err_vs_oracle": err,
    }
    if not args.no_forms:
        # the solver layout and the FP32-stored matrix are forms of the
        # depth-first cell-lane plan: when the pick is another kernel, they
        # run on the fastest depth-first cell-lane candidate the tuner timed
        fplan = plan
        if info["kernel"] != 3:
            dfs = [(o, t) for o, t in tried if o.get("cell_lanes") == 1]
            fopts = min(dfs, key=lambda r: r[1])[0] if dfs else dict(cell_lanes=1)
            fplan = Plan(f.parent, f.cell_offsets, f.branch_offsets, **fopts)
            out["forms_options"] = fopts
        out["layout_resident"] = layout_resident(args, torch, fplan, s, d, u, b, x, stream)
        del d, u
        out["fp32_refine"] = fp32_refine(torch, dev, fplan, s, ms, max(3, args.steps // 2), not args.no_check)
        if fplan is not plan:
            fplan.close()
    plan.close()
    if not args.no_forms:
        out["c1"] = run_c1(torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s)
    return out


def run_c3(args, torch, dev):
    """Batched time loop: V^{k+1} = A^-1 (c V^k + 0.1 Z_k), V^0 = 0, K steps in
    one captured graph, the plan (groups or one lane per cell) picked by the
    autotuner on the workload itself."""
    from workloads import configs
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.autotune import autotune

    ncells = args.cells or configs.C3_CELLS
    s = configs.c3(ncells)
    f = s.forest
    print(f"c3: {f.ncells} cells, {f.n} unknowns generated", file=sys.stderr, flush=True)
    d, u, c = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.c))
    if args.options:
        best, tried = json.loads(args.options), []
    else:
        # autotune on the workload itself: the one-lane-per-cell plan is bound by
        # the serial walk of its longest lanes on a small draw and by throughput
        # on the full one, while the group plans scale with the cell count
        vs = torch.zeros(f.n, dtype=torch.float64, device=dev)
        cands = C3_CANDIDATES
        best, tried = autotune(f.parent, f.cell_offsets, f.branch_offsets,
                               lambda p: p.timestep(d, u, c, vs, vs, noise_sigma=0.1, noise_seed=3),
                               candidates=cands, reps=2, cache_path=args.tune_cache, verbose=True)
        del vs
    t0 = time.perf_counter()
    plan = Plan(f.parent, f.cell_offsets, f.branch_offsets, **best)
    setup_s = time.perf_counter() - t0
    V = torch.zeros(f.n, dtype=torch.float64, device=dev)
    K = args.graph_steps
    # step 0 alone: charge conservation over every cell (column sums of A are c)
    plan.timestep(d, u, c, V, V, noise_sigma=0.1, noise_seed=3, step=0)
    torch.cuda.synchronize()
    check = None
    if not args.no_check:
        import oracle
        cid = np.repeat(np.arange(f.ncells), np.diff(f.cell_offsets))
        Vh = V.cpu().numpy()
        inj = np.bincount(cid, weights=oracle.noise(3, 0, np.arange(f.n, dtype=np.int64), 0.1), minlength=f.ncells)
        q = np.bincount(cid, weights=s.c * Vh, minlength=f.ncells)
        scale = np.bincount(cid, weights=np.abs(s.c * Vh), minlength=f.ncells) + 1.0
        check = float(np.max(np.abs(q - inj) / scale))
    loop = plan.timeloop(d, u, c, V, K, first_step=1, noise_sigma=0.1, noise_seed=3)
    stream = torch.cuda.current_stream()
    ms = _time(torch, loop.launch, args.steps, args.warmup, stream)
    if args.copy_calibration:
        copy_calibration(torch, dev)
    assembled = None
    if plan.info["kernel"] == 3:
        # a step whose diagonal changes (linearised current g (V - E)): the
        # matrix assembled inside the solve against hines_assemble + a step
        rng = np.random.default_rng(5)
        g = torch.from_numpy(rng.uniform(0.0, 1.0, f.n)).to(dev)
        ge = torch.from_numpy(-65.0 * rng.uniform(0.0, 1.0, f.n)).to(dev)
        a = -u
        cg = c + g
        d2, u2 = torch.empty_like(c), torch.empty_like(c)
        Vs = torch.zeros_like(c)
        fused = _time(torch, lambda: plan.timestep_assembled(g, u, c, ge, Vs, Vs, stream=stream), max(3, args.steps),
                      1, stream)

        def two_kernels():
            plan.assemble(a, cg, d2, u2, stream=stream)
            plan.timestep(d2, u2, c, Vs, Vs, i_inj=ge, stream=stream)

        unfused = _time(torch, two_kernels, max(3, args.steps), 1, stream)
        assembled = {"fused_ms": fused, "assemble_then_step_ms": unfused, "speedup": unfused / fused,
                     "bytes_per_unknown": {"fused": 48, "assemble_then_step": 80}}
        del g, ge, a, cg, d2, u2, Vs
    n = f.n
    # read d, u, c, V; write V (a cell-lane plan factors A once per graph launch
    # and then reads the pair (f, 1/d') in place of (d, u): the same 40 bytes)
    bytes_per_step = 40 * n
    achieved = bytes_per_step * K / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": n * K / (ms * 1e-3), "unit": "unknown-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"c3: {f.ncells} cells of 50/500/5000/20000 compartments, implicit Euler with "
                               f"noise current, {K} steps per captured graph (one graph launch per step here)",
                   "ncells": f.ncells, "unknowns": n, "graph_steps": K, "options": best,
                   "autotune_ms": [[o, round(t, 4)] for o, t in tried], "setup_s": round(setup_s, 2),
                   "groups": plan.info["ngroups"], "workspace_groups": plan.info["workspace_groups"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _traffic(1, TRAFFIC_FILE_C3) if plan.info["kernel"] == 3 and ncells == configs.C3_CELLS
                     else None,
                     "kernel": {3: "k_cells_step", 1: "k_solve_flow"}.get(plan.info["kernel"], "k_solve_level"),
                     "bytes_per_step": bytes_per_step},
        "charge_conservation_max_rel_err_step0": check,
        "assembled_step": assembled,
    }
    loop.close()
    plan.close()
    return out


def run_c5(args, torch, dev):
    """Adjoint of the soma-trace loss through 100 implicit-Euler steps."""
    from workloads import configs
    from paper_1810_12742_amd import Plan
    from paper_1810_12742_amd.adjoint import soma_traces

    s = configs.c5(args.cells or configs.C5_CELLS)
    f = s.forest
    steps = s.meta["steps"]
    every = s.meta["checkpoint_every"]
    opts = json.loads(args.options) if args.options else {}
    plan = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
    a = torch.from_numpy(s.a).to(dev).requires_grad_(True)
    c = torch.from_numpy(s.c).to(dev).requires_grad_(True)
    I = torch.from_numpy(s.meta["I"]).to(dev).requires_grad_(True)
    target = torch.from_numpy(s.meta["target"]).to(dev)

    def fwd():
        return ((soma_traces(plan, a, c, I, steps, every) - target) ** 2).sum()

    for _ in range(args.warmup):
        fwd().backward()
    torch.cuda.synchronize()
    tf = tb = 0.0
    for _ in range(args.steps):
        a.grad = c.grad = I.grad = None
        e0, e1 = _events(torch)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        loss = fwd()
        e1.record()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        tf += e0.elapsed_time(e1)
        tb += e1.elapsed_time(e2)
    tf /= args.steps
    tb /= args.steps
    err = None
    if not args.no_check:
        import oracle
        lo, ga, gc, gI, _ = oracle.adjoint(f, s.a, s.c, s.meta["I"], s.meta["target"], steps)
        nr = f.parent >= 0

        def rel(x, y):
            return float(np.max(np.abs(x - y)) / np.max(np.abs(y)))
        err = {"loss": abs(loss.item() - lo) / abs(lo), "d_a": rel(a.grad.cpu().numpy()[nr], ga[nr]),
               "d_c": rel(c.grad.cpu().numpy(), gc), "d_I": rel(I.grad.cpu().numpy(), gI)}
    n = f.n
    ms = tf + tb
    return {
        "metric": METRIC, "value": n * steps / (ms * 1e-3), "unit": "unknown-steps/s (forward + adjoint)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"c5: {f.ncells} cells x ~1000 compartments, {steps} implicit-Euler steps, "
                               f"loss sum (V_soma - target)^2, checkpoints every {every}",
                   "ncells": f.ncells, "unknowns": n, "forward_ms": tf, "backward_ms": tb, "options": opts},
        "max_rel_err_vs_oracle_adjoint": err,
    }


SCALING_CELLS = (64, 256, 1024, 4096, 16384, 65536)


def run_scaling(args, torch, dev):
    """Solve time against the number of cells for the cell-lane kernel (one
    lane per cell, the paper's "old" solver, with depth-first walks and with
    walks in index order) and the flow kernel (branch-level parallelism, the
    "fine" solver): the first n cells of the headline workload, each plan
    timed with HIP events.  The speed-up compares the fine solver with the
    depth-first old one."""
    from workloads import configs
    from paper_1810_12742_amd import Plan

    s = configs.c2()
    f = s.forest
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    b = torch.from_numpy(s.rhs).to(dev)
    stream = torch.cuda.current_stream()
    kernels = {"cell_lanes": dict(cell_lanes=1), "cell_lanes_index_order": dict(cell_lanes=2),
               "flow": dict(C2_FLOW_OPTIONS)}
    rows = []
    for nc in SCALING_CELLS:
        sub = f.subset(np.arange(nc)) if nc < f.ncells else f
        n = sub.n
        row = {"ncells": nc, "unknowns": n}
        x = torch.empty(n, dtype=torch.float64, device=dev)
        for name, opts in kernels.items():
            p = Plan(sub.parent, sub.cell_offsets, sub.branch_offsets, **opts)
            ms = _time(torch, lambda: p.solve(d[:n], u[:n], b[:n], out=x, stream=stream), args.steps, args.warmup,
                       stream)
            row[name + "_ms"] = ms
            p.close()
        row["fine_speedup_over_old"] = row["cell_lanes_ms"] / row["flow_ms"]
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    last = rows[-1]
    best = min(last[k + "_ms"] for k in kernels)
    return {
        "metric": METRIC, "value": last["unknowns"] / (best * 1e-3), "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "scaling: first n cells of c2, n = " + ", ".join(map(str, SCALING_CELLS)) +
                               "; value is the faster kernel at the largest n",
                   "kernels": {k: v for k, v in kernels.items()}},
        "rows": rows,
    }


BRANCHING_P = (0.25, 0.5, 0.75, 1.0)
BRANCHING_CELLS = (4096, 65536)


def run_branching(args, torch, dev):
    """Speed-up of the fine solver (flow kernel, without and with branch
    splitting) over the old one-lane-per-cell solver (depth-first walks; the
    index-order walks are timed beside it) against the branching
    probability of the trees: paper-style trees of 8 levels in which a branch
    splits in two with probability p on every level and otherwise continues,
    branches 40 * 0.8^level compartments long."""
    from workloads import cable_values, grow_level_forest
    from paper_1810_12742_amd import Plan

    stream = torch.cuda.current_stream()
    kernels = {"old_cell_lanes": dict(cell_lanes=1), "old_cell_lanes_index_order": dict(cell_lanes=2),
               "fine_flow": dict(C2_FLOW_OPTIONS), "fine_flow_split": dict(C2_FLOW_OPTIONS, split_branches=1)}
    rows = []
    for pr in BRANCHING_P:
        for nc in BRANCHING_CELLS:
            f = grow_level_forest(np.random.default_rng(11), nc, levels=8, p_split=pr)
            s = cable_values(f, np.random.default_rng(12), a_kind="cable", rhs=True)
            d, u, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.rhs))
            x = torch.empty_like(b)
            row = {"p_split": pr, "ncells": nc, "unknowns": f.n}
            for name, opts in kernels.items():
                p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
                row[name + "_ms"] = _time(torch, lambda: p.solve(d, u, b, out=x, stream=stream), args.steps,
                                          args.warmup, stream)
                p.close()
            fine = min(row["fine_flow_ms"], row["fine_flow_split_ms"])
            row["fine_speedup_over_old"] = row["old_cell_lanes_ms"] / fine
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
            del d, u, b, x
    last = rows[-1]
    best = min(last[k + "_ms"] for k in kernels)
    return {
        "metric": METRIC, "value": last["unknowns"] / (best * 1e-3), "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "branching: 8-level trees, split probability p = " +
                               ", ".join(map(str, BRANCHING_P)) + ", cells = " + ", ".join(map(str, BRANCHING_CELLS)) +
                               "; value is the fastest kernel on the last row",
                   "kernels": kernels},
        "rows": rows,
    }


OUTLOOK_OPTIONS = (
    ("split_global", dict(split_branches=1)),
    ("split_per_group", dict(split_branches=2)),
    ("no_split_level_balance", dict(level_balance=1)),
    ("split_per_group_level_balance", dict(split_branches=2, level_balance=1)),
    ("no_split", dict()),
)


def run_outlook(args, torch, dev):
    """The outlook of the paper (section 8) on the level-synchronous kernel it
    concerns: branch splitting with the average over all cells against the
    average over each group of an intermediate packing, and packing with and
    without moving subtrees one level down.  Groups of up to 4,096
    compartments and 64 lanes, so that level widths, not the compartment cap,
    limit the packing.  Default: the first 16,384 cells of the headline
    workload (``--cells``)."""
    from workloads import configs
    from paper_1810_12742_amd import Plan
    import oracle

    nc = args.cells or 16384
    s = configs.c2()
    f = s.forest.subset(np.arange(nc)) if nc < s.forest.ncells else s.forest
    n = f.n
    d, u, b = (torch.from_numpy(np.ascontiguousarray(a[:n])).to(dev) for a in (s.diag, s.upper, s.rhs))
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()
    xo = None if args.no_check else oracle.solve(f, s.diag[:n], s.upper[:n], s.rhs[:n])
    rows = []
    for name, extra in OUTLOOK_OPTIONS:
        opts = dict(level_sync=1, max_group_unknowns=4096, group_width=64, **extra)
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **opts)
        info = p.info
        ms = _time(torch, lambda: p.solve(d, u, b, out=x, stream=stream), args.steps, args.warmup, stream)
        row = {"variant": name, "options": opts, "ms": ms, "groups": info["ngroups"],
               "levels": info["max_level"] + 1, "branches": info["nbranches"], "launches": info["nclasses"]}
        if xo is not None:
            row["max_rel_err_vs_oracle"] = cell_rel_err(f, x.cpu().numpy(), xo)
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        p.close()
    best = min(rows, key=lambda r: r["ms"])
    return {
        "metric": METRIC, "value": n / (best["ms"] * 1e-3), "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"outlook: first {nc} cells of c2 on the level-synchronous kernel, groups of up to "
                               "4,096 compartments and 64 lanes; value is the fastest variant",
                   "unknowns": n},
        "rows": rows,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("c2", "c3", "c5", "scaling", "branching", "outlook"), default="c2")
    ap.add_argument("--cells", type=int, default=0, help="c3/c5/outlook: number of cells (default: the full workload)")
    ap.add_argument("--graph-steps", type=int, default=100, help="c3: time steps per captured graph")
    ap.add_argument("--options", default="", help="plan options as JSON (c2, c3: instead of the autotuner's pick)")
    ap.add_argument("--tune-cache", default=None,
                    help="c2, c3: autotuner cache file (default: the picks shipped with the package)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="c2: skip the FP32+refinement measurement")
    ap.add_argument("--no-c3", action="store_true", help="c2: skip the time-loop (C3) summary on the same line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="c2, c3: after the timed region, run a plain device copy of 512 MiB (read and write) "
                         "three times, the reference kernel for scaling HBM byte counters")
    args = ap.parse_args(argv)
    if args.tune_cache is None:
        from paper_1810_12742_amd.autotune import SHIPPED_CACHE
        args.tune_cache = SHIPPED_CACHE
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the per-cell solve has no cross-GPU step and the path is "
              f"built for a single MI355X (asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    run = {"c2": run_c2, "c3": run_c3, "c5": run_c5, "scaling": run_scaling,
           "branching": run_branching, "outlook": run_outlook}[args.workload]
    out = run(args, torch, dev)
    if args.workload == "c2" and not args.no_c3:
        out["c3"] = c3_summary(args, torch, dev)
    print(json.dumps(out), flush=True)
    return 0


def c3_summary(args, torch, dev):
    """The batched time loop as the configuration states it (200,000 cells,
    1,000 implicit-Euler steps captured in one graph) beside the C2 line: the
    autotuner's cached pick, one untimed and 2 timed graph launches."""
    a = argparse.Namespace(**vars(args))
    a.steps, a.warmup, a.graph_steps, a.options, a.cells = 2, 1, 1000, "", 0
    try:
        r = run_c3(a, torch, dev)
    except Exception as e:  # the C2 line stands on its own
        return {"error": f"{type(e).__name__}: {e}"}
    K = r["config"]["graph_steps"]
    return {"metric": r["metric"], "value": r["value"], "unit": r["unit"], "graph_steps": K,
            "ms_per_graph_launch": r["ms_per_step"], "ms_per_time_step": r["ms_per_step"] / K,
            "launches": r["steps"], "roofline": r["roofline"], "options": r["config"]["options"],
            "workload": r["config"]["workload"], "setup_s": r["config"]["setup_s"],
            "charge_conservation_max_rel_err_step0": r["charge_conservation_max_rel_err_step0"]}


if __name__ == "__main__":
    sys.exit(main())

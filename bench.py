"""Benchmark of the batched FP64 Hines solve on one MI355X.

Workload: 65,536 synthetic neuron-shaped cells (random binary dendritic
trees, 16-256 branches, geometric branch lengths of mean 12 capped at 64,
about 1.06e8 compartments), cable-equation coefficients at dt = 0.025, one
right-hand side; seed 1.  Inputs are resident in HBM before the timed region.
A step is one hines_solve over all cells: every matrix entry is read from HBM
once and the solution written once (32 algorithmic bytes per compartment).

Prints one JSON line.  ``--gpus`` above 1 is refused: the solve is per cell
and needs no communication; this build measures one GPU.
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
# Launch configuration of the timed solve (setup options of the plan).
C2_OPTIONS = dict(max_group_unknowns=1536, split_branches=0, cell_order=0, group_width=64)
CALIB_BYTES = 512 << 20  # bytes read (and written) by one calibration copy
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hines_solve_c2.json")
KERNEL_SRC_DIR = os.path.join(ROOT, "paper_1810_12742_amd", "csrc")


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


def _traffic(n_launches_per_solve: int):
    """HBM bytes per launch from the committed PMC measurement, if it was taken
    on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != _kernel_sha():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(system, budget_s: float = 12.0):
    """The FP64 oracle on the host cores: repeated full solves of the same
    workload until about ``budget_s`` seconds of wall time have passed."""
    import oracle
    oracle.build(force=False)
    f = system.forest
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.solve(f, system.diag, system.upper, system.rhs, nthreads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": f.n * reps / el, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
            "sample": f"full workload ({f.n} unknowns), {reps} solves, {el:.1f} s, OpenMP over cells"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain device copy of 512 MiB (read and write) three "
                         "times, the reference kernel for scaling HBM byte counters")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the per-cell solve has no cross-GPU step and the path is "
              f"built for a single MI355X (asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import torch
    from workloads import configs
    from paper_1810_12742_amd import Plan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = configs.c2()
    f = s.forest
    t0 = time.perf_counter()
    plan = Plan(f.parent, f.cell_offsets, f.branch_offsets, **C2_OPTIONS)
    setup_s = time.perf_counter() - t0
    info = plan.info
    d = torch.from_numpy(s.diag).to(dev)
    u = torch.from_numpy(s.upper).to(dev)
    b = torch.from_numpy(s.rhs).to(dev)
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.solve(d, u, b, out=x, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.solve(d, u, b, out=x, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps

    if args.copy_calibration:
        src = torch.empty(CALIB_BYTES // 8, dtype=torch.float64, device=dev).uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    err = None
    if not args.no_check:
        import oracle
        xo = oracle.solve(f, s.diag, s.upper, s.rhs)
        xg = x.cpu().numpy()
        e = np.maximum.reduceat(np.abs(xg - xo), f.cell_offsets[:-1])
        sc = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
        err = float(np.max(e / sc))

    n = f.n
    launches = max(1, int(info["nclasses"]))
    bytes_per_solve = BYTES_PER_UNKNOWN * n
    achieved = bytes_per_solve / (ms * 1e-3) / 1e9
    traffic = _traffic(launches)
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
            "options": C2_OPTIONS, "setup_s": round(setup_s, 3),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_solve_sched_f64" if info["kernel"] == 1 else "k_solve_lds_f64",
            "bytes_per_launch": bytes_per_solve / launches,
            "avg_launch_us": ms * 1e3 / launches,
        },
        "max_rel_err_vs_oracle": err,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""hines_solve_noalloc through the C-ABI: the cell-lane solve (depth-first or
index-order lanes) with its factors in the library's static device scratch
instead of the plan's allocation.

Its output must equal hines_solve's on the same plan and inputs (same kernel,
same arithmetic; only the scratch address differs), on two calls in a row,
the second on a smaller plan, so stale contents of the shared scratch from the
first call would show.  Both are also checked against the FP64 oracle.  A
plan whose factors exceed the static scratch is refused with
HINES_ERR_TOO_BIG before anything is launched.
"""
import ctypes

import numpy as np
import pytest

import oracle
from workloads import configs

pytestmark = pytest.mark.gpu

TOL = 1e-12
HINES_ERR_TOO_BIG = 10
HINES_ERR_STATE = 12


def cell_rel_err(f, x, xo):
    err = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    scale = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(err / np.maximum(scale, 1e-300)))


def _lib():
    from paper_1810_12742_amd import hines
    lib = hines.load()
    P = ctypes.c_void_p
    lib.hines_solve_noalloc.argtypes = [P, P, P, P, P, ctypes.c_int32, P]
    lib.hines_solve_noalloc.restype = ctypes.c_int32
    lib.hines_solve.argtypes = [P, P, P, P, P, ctypes.c_int32, P]
    lib.hines_solve.restype = ctypes.c_int32
    return lib


def _both(lib, torch, s, **opts):
    """x from hines_solve and from hines_solve_noalloc on one plan."""
    from paper_1810_12742_amd import Plan
    f = s.forest
    dev = torch.device("cuda")
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, **{"cell_lanes": 1, **opts})
    d, u, b = (torch.from_numpy(a).to(dev) for a in (s.diag, s.upper, s.rhs))
    x_ref = torch.full_like(b, np.nan)
    x_new = torch.full_like(b, np.nan)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [ctypes.c_void_p(t.data_ptr()) for t in (d, u, b)]
    assert lib.hines_solve(p._h, *args, ctypes.c_void_p(x_ref.data_ptr()), f.ncells, stream) == 0
    st = lib.hines_solve_noalloc(p._h, *args, ctypes.c_void_p(x_new.data_ptr()), f.ncells, stream)
    assert st == 0, lib.hines_last_error()
    torch.cuda.synchronize()
    p.close()
    return x_ref.cpu().numpy(), x_new.cpu().numpy()


@pytest.mark.parametrize("lanes", [1, 2], ids=["depth_first", "index_order"])
def test_noalloc_equals_solve_on_two_calls(lanes):
    import torch
    lib = _lib()
    for s in (configs.c2(2048), configs.c2(300)):   # the second call is smaller
        f = s.forest
        print(f"noalloc: cell_lanes {lanes}, {f.ncells} cells, {f.n} unknowns", flush=True)
        x_ref, x_new = _both(lib, torch, s, cell_lanes=lanes)
        assert np.array_equal(x_new, x_ref)
        xo = oracle.solve(f, s.diag, s.upper, s.rhs)
        assert cell_rel_err(f, x_new, xo) <= TOL


def test_noalloc_refuses_a_plan_beyond_the_scratch_and_other_kernels():
    import torch
    from paper_1810_12742_amd import Plan
    lib = _lib()
    dev = torch.device("cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # 2,000,000 one-branch cells of 9 compartments: 18e6 walk slots at 16 bytes
    # exceed the 256 MiB scratch
    ncell, m = 2_000_000, 9
    par = np.tile(np.arange(-1, m - 1, dtype=np.int32), ncell)
    par = par + np.repeat(np.arange(ncell, dtype=np.int64) * m, m).astype(np.int32) * (par >= 0)
    off = np.arange(0, ncell * m + 1, m, dtype=np.int64)
    p = Plan(par, off, None, cell_lanes=True)
    n = ncell * m
    buf = torch.zeros(n, dtype=torch.float64, device=dev)
    a = ctypes.c_void_p(buf.data_ptr())
    print("noalloc: oversized plan", flush=True)
    assert lib.hines_solve_noalloc(p._h, a, a, a, ctypes.c_void_p(0), ncell, stream) != 0  # NULL x first
    xb = torch.zeros_like(buf)
    assert lib.hines_solve_noalloc(p._h, a, a, a, ctypes.c_void_p(xb.data_ptr()), ncell, stream) == HINES_ERR_TOO_BIG
    p.close()
    s = configs.c2(64)
    f = s.forest
    q = Plan(f.parent, f.cell_offsets, f.branch_offsets)  # groups, not cell lanes
    d = torch.from_numpy(s.diag).to(dev)
    x = torch.empty_like(d)
    dp = ctypes.c_void_p(d.data_ptr())
    assert lib.hines_solve_noalloc(q._h, dp, dp, dp, ctypes.c_void_p(x.data_ptr()), f.ncells, stream) == \
        HINES_ERR_STATE
    q.close()
    torch.cuda.synchronize()

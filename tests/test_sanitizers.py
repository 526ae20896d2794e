"""The host-side table builders (setup, cell lanes in both walk orders,
resident) compiled with AddressSanitizer and UndefinedBehaviorSanitizer (g++,
CPU only) on forests and option sets of the table-parity suite; the tables
they export must equal the library's (built without sanitizers), so the
sanitized run executes the same code paths.  A heap overflow, use after free
or undefined operation aborts the driver with a report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from workloads import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_12742_amd", "csrc")
TABLES = ["node_plan", "branches", "u_src", "group_offsets", "group_cells", "group_seg_offsets", "seg_offsets",
          "lanes", "flow_groups", "flow_masks", "flow_pos", "flow_aux", "cell_waves", "cell_lanes", "cell_pos",
          "cell_flags", "cell_mbsrc", "res_groups", "cell_range", "res_blob", "seq_waves", "seq_lanes", "seq_pos",
          "seq_code", "seq_mbsrc"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "asan_driver")
    src = [os.path.join(ROOT, "tests", "asan_driver.cpp")] + [os.path.join(CSRC, f) for f in
                                                              ("setup.cpp", "cells.cpp", "resident.cpp")]
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", exe, *src], check=True)
    return exe, d


CASES = [
    ("c2", dict()),
    ("c2", dict(split_branches=1, cell_lanes=1, resident=1)),
    ("c2", dict(split_branches=2, level_balance=1, max_group_unknowns=0)),
    ("c3", dict(rebalance_root=1, split_branches=1, group_width=128, cell_lanes=1)),
    ("c3", dict(level_balance=1, max_group_unknowns=0)),
    ("c2", dict(level_balance=1, max_group_unknowns=0, resident=1)),
    ("small", dict(cell_order=1, max_group_unknowns=900, split_branches=2, cell_lanes=1, resident=1)),
    ("c2", dict(cell_lanes=2)),
    ("small", dict(cell_lanes=2, resident=1)),
]


def _forest(name):
    return {"c2": lambda: configs.c2(64).forest, "c3": lambda: configs.c3(40).forest,
            "small": lambda: configs.random_system(300, seed=11).forest}[name]()


@pytest.mark.parametrize("name,opts", CASES, ids=[f"{n}-{i}" for i, (n, _) in enumerate(CASES)])
def test_builders_under_address_and_ub_sanitizers(driver, name, opts):
    from paper_1810_12742_amd import Plan
    exe, d = driver
    f = _forest(name)
    o = dict(rebalance_root=0, split_branches=0, group_width=64, cell_order=0, max_group_unknowns=2048,
             level_balance=0, cell_lanes=0, resident=0)
    o.update(opts)
    inp, outp = str(d / "in.bin"), str(d / "out.bin")
    with open(inp, "wb") as fh:
        np.array([f.n, f.ncells], dtype=np.int64).tofile(fh)
        f.parent.astype(np.int32).tofile(fh)
        f.cell_offsets.astype(np.int64).tofile(fh)
        np.array([o[k] for k in ("rebalance_root", "split_branches", "group_width", "cell_order",
                                 "max_group_unknowns", "level_balance", "cell_lanes", "resident")],
                 dtype=np.int64).tofile(fh)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, inp, outp], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = np.fromfile(outp, dtype=np.int64)
    got, k = {}, 0
    for name_t in TABLES:
        cnt = int(raw[k])
        k += 1
        if name_t is not None:
            got[name_t] = raw[k:k + max(cnt, 0)]
        k += max(cnt, 0)
    # the library takes one of the two kernels per plan: the resident tables
    # come from a second plan
    base = {k: v for k, v in o.items() if k != "resident"}
    p = Plan(f.parent, f.cell_offsets, None, host_only=True, **base)
    want = p.tables()
    p.close()
    if o["resident"]:
        base.update(cell_lanes=0, resident=1)
        p = Plan(f.parent, f.cell_offsets, None, host_only=True, **base)
        want.update({k: v for k, v in p.tables().items() if k.startswith("res_")})
        p.close()
    for name_t in TABLES:
        if name_t is not None:
            assert np.array_equal(got[name_t], want[name_t].reshape(-1)), name_t

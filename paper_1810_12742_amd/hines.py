"""ctypes binding of libhines.so (include/hines.h): argument marshalling only.

Device arrays are torch tensors (float64, contiguous, on the plan's device);
torch provides the memory and the current stream, the library does the work.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libhines.so")
_lib = None

TABLES = {
    "node_plan": 0, "branches": 1, "u_src": 2, "group_offsets": 3, "group_cells": 4,
    "group_seg_offsets": 5, "seg_offsets": 6, "lanes": 7,
    "flow_groups": 8, "flow_masks": 9, "flow_pos": 10, "flow_aux": 11,
    "cell_waves": 12, "cell_lanes": 13, "cell_pos": 14, "cell_flags": 15, "cell_mbsrc": 16,
    "cell_range": 18, "res_groups": 17, "res_blob": 19,
    "seq_waves": 20, "seq_lanes": 21, "seq_pos": 22, "seq_code": 23, "seq_mbsrc": 24,
}
STATUS = {0: "OK", 1: "NULL", 2: "BAD_OFFSETS", 3: "BAD_PARENT", 4: "BAD_BRANCHES",
          6: "NCELLS", 7: "OPTION", 8: "OOM", 9: "HIP", 10: "TOO_BIG", 11: "NOT_SDD", 12: "STATE"}


class HinesError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"hines error {self.code} ({status}): {message}")


class _Options(ctypes.Structure):
    _fields_ = [("rebalance_root", ctypes.c_int32), ("split_branches", ctypes.c_int32),
                ("group_width", ctypes.c_int32), ("cell_order", ctypes.c_int32),
                ("max_group_unknowns", ctypes.c_int32), ("host_only", ctypes.c_int32),
                ("keep_tables", ctypes.c_int32), ("bitwise", ctypes.c_int32),
                ("level_sync", ctypes.c_int32), ("cell_lanes", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("cell_cut_percent", ctypes.c_int32),
                ("cell_max_cuts", ctypes.c_int32), ("res_pack", ctypes.c_int32),
                ("level_balance", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ncells", ctypes.c_int64), ("nbranches", ctypes.c_int64),
                ("ngroups", ctypes.c_int64), ("nsegments", ctypes.c_int64), ("max_level", ctypes.c_int32),
                ("nclasses", ctypes.c_int32), ("device_table_bytes", ctypes.c_int64),
                ("max_group_lds_bytes", ctypes.c_int64), ("kernel", ctypes.c_int32),
                ("max_makespan", ctypes.c_int32), ("workspace_groups", ctypes.c_int64)]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libhines.so (after torch, so that it binds to torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_1810_12742_amd.build`")
    import torch  # noqa: F401  (HIP runtime of the process)
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.hines_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.hines_default_options.restype = None
    lib.hines_setup.argtypes = [P, I64, P, I64, P, I32, ctypes.POINTER(_Options), ctypes.POINTER(P)]
    lib.hines_solve.argtypes = [P, P, P, P, P, I32, P]
    lib.hines_plan_info_get.argtypes = [P, ctypes.POINTER(_Info)]
    lib.hines_get_table.argtypes = [P, I32, P, I64, ctypes.POINTER(I64)]
    lib.hines_destroy.argtypes = [P]
    lib.hines_status_str.argtypes = [I32]
    lib.hines_status_str.restype = ctypes.c_char_p
    lib.hines_last_error.argtypes = []
    lib.hines_last_error.restype = ctypes.c_char_p
    U32, D = ctypes.c_uint32, ctypes.c_double
    lib.hines_timestep.argtypes = [P, P, P, P, P, P, P, D, U32, U32, I32, P]
    lib.hines_solve_mixed.argtypes = [P, P, P, P, P, I32, I32, P]
    lib.hines_solve_stored32.argtypes = [P, P, P, P, P, I32, P]
    lib.hines_timestep_assembled.argtypes = [P, P, P, P, P, P, P, I32, P]
    lib.hines_timeloop_create.argtypes = [P, P, P, P, P, P, D, U32, U32, I32, I32, ctypes.POINTER(P)]
    lib.hines_timeloop_launch.argtypes = [P, P]
    lib.hines_timeloop_destroy.argtypes = [P]
    lib.hines_assemble.argtypes = [P, P, P, P, P, P]
    lib.hines_gather_roots.argtypes = [P, P, P, P]
    lib.hines_adjoint_rhs.argtypes = [P, P, P, P, P, P]
    lib.hines_adjoint_accumulate.argtypes = [P, P, P, P, P, P, P, P]
    lib.hines_check_matrix.argtypes = [P, P, P, ctypes.POINTER(I64), P]
    lib.hines_layout_size.argtypes = [P, ctypes.POINTER(I64)]
    lib.hines_to_layout.argtypes = [P, P, P, P]
    lib.hines_from_layout.argtypes = [P, P, P, P]
    lib.hines_solve_layout.argtypes = [P, P, P, P, P, I32, P]
    for name in ("hines_setup", "hines_solve", "hines_solve_mixed", "hines_solve_stored32", "hines_timestep_assembled",
                 "hines_plan_info_get",
                 "hines_get_table",
                 "hines_destroy",
                 "hines_timestep", "hines_timeloop_create", "hines_timeloop_launch", "hines_timeloop_destroy",
                 "hines_assemble", "hines_gather_roots", "hines_adjoint_rhs", "hines_adjoint_accumulate",
                 "hines_check_matrix", "hines_layout_size", "hines_to_layout", "hines_from_layout",
                 "hines_solve_layout"):
        getattr(lib, name).restype = I32
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise HinesError(status, load().hines_last_error().decode())


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _dev(t, n, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need contiguous {dtype} with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A setup plan (``hines_setup``) and the solves that use it.

    Options are those of ``hines_options`` in include/hines.h; ``cell_lanes``
    is 0 (groups), 1 (one lane per cell, depth-first walks) or 2 (one lane per
    cell, walks in decreasing user index)."""

    def __init__(self, parent, cell_offsets, branch_offsets=None, *, rebalance_root=False,
                 split_branches=False, group_width=64, cell_order=0, max_group_unknowns=None,
                 host_only=False, keep_tables=True, bitwise=False, level_sync=False, cell_lanes=False,
                 resident=False, cell_cut_percent=0, cell_max_cuts=0, res_pack=0, level_balance=False):
        lib = load()
        opt = _Options()
        lib.hines_default_options(ctypes.byref(opt))
        opt.rebalance_root = int(bool(rebalance_root))
        opt.split_branches = int(split_branches)
        opt.group_width = int(group_width)
        opt.cell_order = int(cell_order)
        if max_group_unknowns is not None:
            opt.max_group_unknowns = int(max_group_unknowns)
        opt.host_only = int(bool(host_only))
        opt.keep_tables = int(bool(keep_tables))
        opt.bitwise = int(bool(bitwise))
        opt.level_sync = int(bool(level_sync))
        opt.cell_lanes = int(cell_lanes)
        opt.resident = int(bool(resident))
        opt.cell_cut_percent = int(cell_cut_percent)
        opt.cell_max_cuts = int(cell_max_cuts)
        opt.res_pack = int(res_pack)
        opt.level_balance = int(bool(level_balance))
        self._par = _host(parent, np.int32)
        self._coff = _host(cell_offsets, np.int64)
        bo = None if branch_offsets is None else _host(branch_offsets, np.int64)
        self.n = int(self._par.shape[0])
        self.ncells = int(self._coff.shape[0] - 1)
        handle = ctypes.c_void_p()
        st = lib.hines_setup(
            ctypes.c_void_p(self._par.ctypes.data), self.n,
            None if bo is None else ctypes.c_void_p(bo.ctypes.data), 0 if bo is None else bo.shape[0] - 1,
            ctypes.c_void_p(self._coff.ctypes.data), self.ncells, ctypes.byref(opt), ctypes.byref(handle))
        _check(st)
        self._h = handle
        self.options = {f: getattr(opt, f) for f, _ in _Options._fields_ if f != "reserved"}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _check(load().hines_destroy(h))
        self._h = None

    @property
    def info(self) -> dict:
        inf = _Info()
        _check(load().hines_plan_info_get(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def table(self, name: str) -> np.ndarray:
        lib = load()
        which = TABLES[name]
        cnt = ctypes.c_int64()
        _check(lib.hines_get_table(self._h, which, None, 0, ctypes.byref(cnt)))
        out = np.empty(cnt.value, dtype=np.int64)
        _check(lib.hines_get_table(self._h, which, ctypes.c_void_p(out.ctypes.data), out.shape[0],
                                   ctypes.byref(cnt)))
        if name == "branches":
            return out.reshape(-1, 8)
        if name == "res_groups":
            return out.reshape(-1, 16)
        return out

    def tables(self) -> dict:
        return {k: self.table(k) for k in TABLES}

    def solve(self, diag, upper, rhs, out=None, stream=None):
        """x = A^-1 rhs on the device (``hines_solve``); returns ``out``."""
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_solve(self._h, _dev(diag, self.n, torch.float64, "diag"),
                                  _dev(upper, self.n, torch.float64, "upper"),
                                  _dev(rhs, self.n, torch.float64, "rhs"),
                                  _dev(out, self.n, torch.float64, "out"), self.ncells,
                                  ctypes.c_void_p(st.cuda_stream)))
        return out

    def solve_mixed(self, diag32, upper32, rhs, out=None, sweeps=3, stream=None):
        """FP32 solve + FP64 refinement (``hines_solve_mixed``); returns ``out``."""
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_solve_mixed(self._h, _dev(diag32, self.n, torch.float32, "diag32"),
                                        _dev(upper32, self.n, torch.float32, "upper32"),
                                        _dev(rhs, self.n, torch.float64, "rhs"),
                                        _dev(out, self.n, torch.float64, "out"), int(sweeps), self.ncells,
                                        ctypes.c_void_p(st.cuda_stream)))
        return out

    def solve_stored32(self, diag32, upper32, rhs, out=None, stream=None):
        """FP32-stored matrix, FP64 elimination on a cell-lane plan
        (``hines_solve_stored32``); returns ``out``."""
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_solve_stored32(self._h, _dev(diag32, self.n, torch.float32, "diag32"),
                                           _dev(upper32, self.n, torch.float32, "upper32"),
                                           _dev(rhs, self.n, torch.float64, "rhs"),
                                           _dev(out, self.n, torch.float64, "out"), self.ncells,
                                           ctypes.c_void_p(st.cuda_stream)))
        return out

    def timestep_assembled(self, g, upper, c, ge, v_in, v_out=None, stream=None):
        """v_out = A^-1 (c v_in + ge) with A assembled from upper = -a, c and g in
        the solve (``hines_timestep_assembled``, cell-lane plans); v_out may be v_in."""
        import torch
        if v_out is None:
            v_out = torch.empty_like(v_in)
        st = stream if stream is not None else torch.cuda.current_stream()
        f64 = torch.float64
        _check(load().hines_timestep_assembled(
            self._h, _dev(g, self.n, f64, "g"), _dev(upper, self.n, f64, "upper"), _dev(c, self.n, f64, "c"),
            _dev(ge, self.n, f64, "ge"), _dev(v_in, self.n, f64, "v_in"), _dev(v_out, self.n, f64, "v_out"),
            self.ncells, ctypes.c_void_p(st.cuda_stream)))
        return v_out

    # ---- time loop (paper §1: one implicit-Euler system per step) ----------
    def timestep(self, diag, upper, c, v_in, v_out=None, i_inj=None, noise_sigma=0.0, noise_seed=0, step=0,
                 stream=None):
        """v_out = A^-1 (c v_in + I) (``hines_timestep``); v_out may be v_in."""
        import torch
        if v_out is None:
            v_out = torch.empty_like(v_in)
        st = stream if stream is not None else torch.cuda.current_stream()
        f64 = torch.float64
        _check(load().hines_timestep(
            self._h, _dev(diag, self.n, f64, "diag"), _dev(upper, self.n, f64, "upper"), _dev(c, self.n, f64, "c"),
            _dev(v_in, self.n, f64, "v_in"), _dev(v_out, self.n, f64, "v_out"),
            None if i_inj is None else _dev(i_inj, self.n, f64, "i_inj"), float(noise_sigma),
            int(noise_seed) & 0xFFFFFFFF, int(step) & 0xFFFFFFFF, self.ncells, ctypes.c_void_p(st.cuda_stream)))
        return v_out

    def timeloop(self, diag, upper, c, v, nsteps, first_step=0, i_inj=None, noise_sigma=0.0, noise_seed=0):
        """A captured graph of ``nsteps`` in-place steps of ``v`` (``hines_timeloop_create``)."""
        import torch
        f64 = torch.float64
        h = ctypes.c_void_p()
        keep = (diag, upper, c, v, i_inj)
        _check(load().hines_timeloop_create(
            self._h, _dev(diag, self.n, f64, "diag"), _dev(upper, self.n, f64, "upper"), _dev(c, self.n, f64, "c"),
            _dev(v, self.n, f64, "v"), None if i_inj is None else _dev(i_inj, self.n, f64, "i_inj"),
            float(noise_sigma), int(noise_seed) & 0xFFFFFFFF, int(first_step) & 0xFFFFFFFF, int(nsteps),
            self.ncells, ctypes.byref(h)))
        return TimeLoop(h, self, keep)

    # ---- solver layout of a cell-lane plan (paper §7: permutation kernels) ----
    @property
    def layout_size(self) -> int:
        n = ctypes.c_int64()
        _check(load().hines_layout_size(self._h, ctypes.byref(n)))
        return int(n.value)

    def to_layout(self, src, dst=None, stream=None):
        import torch
        m = self.layout_size
        dst = torch.empty(m, dtype=torch.float64, device=src.device) if dst is None else dst
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_to_layout(self._h, _dev(src, self.n, torch.float64, "src"),
                                      _dev(dst, m, torch.float64, "dst"), ctypes.c_void_p(st.cuda_stream)))
        return dst

    def from_layout(self, src, dst=None, stream=None):
        import torch
        m = self.layout_size
        dst = torch.empty(self.n, dtype=torch.float64, device=src.device) if dst is None else dst
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_from_layout(self._h, _dev(src, m, torch.float64, "src"),
                                        _dev(dst, self.n, torch.float64, "dst"), ctypes.c_void_p(st.cuda_stream)))
        return dst

    def solve_layout(self, diag_l, upper_l, rhs_l, out=None, stream=None):
        """A x = rhs with every array in the solver layout (``hines_solve_layout``)."""
        import torch
        m = self.layout_size
        out = torch.empty_like(rhs_l) if out is None else out
        st = stream if stream is not None else torch.cuda.current_stream()
        f64 = torch.float64
        _check(load().hines_solve_layout(self._h, _dev(diag_l, m, f64, "diag_l"), _dev(upper_l, m, f64, "upper_l"),
                                         _dev(rhs_l, m, f64, "rhs_l"), _dev(out, m, f64, "out"), self.ncells,
                                         ctypes.c_void_p(st.cuda_stream)))
        return out

    def check_matrix(self, diag, upper, stream=None):
        """Strict diagonal dominance with a positive diagonal (``hines_check_matrix``).
        Returns -1 when every row passes, else the smallest failing user index."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        bad = ctypes.c_int64(-1)
        status = load().hines_check_matrix(self._h, _dev(diag, self.n, torch.float64, "diag"),
                                           _dev(upper, self.n, torch.float64, "upper"), ctypes.byref(bad),
                                           ctypes.c_void_p(st.cuda_stream))
        if status == 11:
            return int(bad.value)
        _check(status)
        return -1

    # ---- element-wise kernels of the adjoint ----------------------------------
    def assemble(self, a, c, diag=None, upper=None, stream=None):
        import torch
        diag = torch.empty_like(c) if diag is None else diag
        upper = torch.empty_like(c) if upper is None else upper
        st = stream if stream is not None else torch.cuda.current_stream()
        f64 = torch.float64
        _check(load().hines_assemble(self._h, _dev(a, self.n, f64, "a"), _dev(c, self.n, f64, "c"),
                                     _dev(diag, self.n, f64, "diag"), _dev(upper, self.n, f64, "upper"),
                                     ctypes.c_void_p(st.cuda_stream)))
        return diag, upper

    def gather_roots(self, v, out=None, stream=None):
        import torch
        out = torch.empty(self.ncells, dtype=torch.float64, device=v.device) if out is None else out
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_gather_roots(self._h, _dev(v, self.n, torch.float64, "v"),
                                         _dev(out, self.ncells, torch.float64, "out"), ctypes.c_void_p(st.cuda_stream)))
        return out

    def adjoint_rhs(self, c, lam_next, g_roots, mu=None, stream=None):
        import torch
        mu = torch.empty_like(c) if mu is None else mu
        st = stream if stream is not None else torch.cuda.current_stream()
        f64 = torch.float64
        _check(load().hines_adjoint_rhs(self._h, _dev(c, self.n, f64, "c"),
                                        None if lam_next is None else _dev(lam_next, self.n, f64, "lam_next"),
                                        _dev(g_roots, self.ncells, f64, "g_roots"), _dev(mu, self.n, f64, "mu"),
                                        ctypes.c_void_p(st.cuda_stream)))
        return mu

    def adjoint_accumulate(self, lam, v, v_prev, grad_a, grad_c, grad_i, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        f64 = torch.float64
        _check(load().hines_adjoint_accumulate(
            self._h, _dev(lam, self.n, f64, "lam"), _dev(v, self.n, f64, "v"), _dev(v_prev, self.n, f64, "v_prev"),
            _dev(grad_a, self.n, f64, "grad_a"), _dev(grad_c, self.n, f64, "grad_c"),
            _dev(grad_i, self.n, f64, "grad_i"), ctypes.c_void_p(st.cuda_stream)))


class TimeLoop:
    """A captured multi-step graph (``hines_timeloop_*``)."""

    def __init__(self, handle, plan, keep):
        self._h = handle
        self._plan = plan   # the plan must outlive the loop
        self._keep = keep   # and so must the bound arrays

    def launch(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(load().hines_timeloop_launch(self._h, ctypes.c_void_p(st.cuda_stream)))

    def close(self):
        if self._h is not None and self._h.value:
            _check(load().hines_timeloop_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""MI355X batched Hines solver (paper: F. Huber, "Efficient Tree Solver for
Hines Matrices on the GPU").

The compute path is the C-ABI library ``libhines.so`` (HIP kernels for gfx950,
built in-tree by ``paper_1810_12742_amd.build``); :mod:`.hines` is a thin
ctypes binding that only marshals arguments.  Nothing here computes on the
CPU: if the library is missing, every call raises.
"""
from .hines import HinesError, Plan, TABLES, TimeLoop, library_path, load

__all__ = ["HinesError", "Plan", "TABLES", "TimeLoop", "library_path", "load"]

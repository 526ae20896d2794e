"""FP64 CPU oracle for the batched Hines solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  It shares no code with
the GPU library ``paper_1810_12742_amd`` and never imports it; both sides take
their inputs from ``workloads``.

Contents (each cites the passage of the paper it follows):

* ``solve`` / ``solve_f32``: the Hines algorithm (paper §2, Listing 2) in the
  user numbering, plain C, one cell after another (cells are independent, §3).
* ``spmv`` / ``residual``: the tree matrix of §1 applied to a vector.
* ``noise``: the injected-current draws of the time loop (Philox4x32-10).
* ``timeloop``: repeated implicit-Euler steps of the discrete system of §1.
* ``refine``: FP32 solve + FP64 residual iterative refinement.
* ``adjoint``: discrete adjoint of the time loop (A is symmetric, §1).
* ``tables`` (submodule): the setup tables of §4-§6 in plain Python.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hines_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_hines.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no FMA contraction, IEEE division)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                        "-fPIC", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_solve_f64.argtypes = [I64, P, P, P, P, P, ctypes.c_int]
        lib.oracle_solve_f64.restype = I64
        lib.oracle_solve_f32.argtypes = [I64, P, P, P, P, P, ctypes.c_int]
        lib.oracle_solve_f32.restype = I64
        lib.oracle_spmv_f64.argtypes = [I64, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_spmv_f64.restype = None
        lib.oracle_philox.argtypes = [P, P, P]
        lib.oracle_philox.restype = None
        lib.oracle_noise.argtypes = [ctypes.c_uint32, ctypes.c_uint32, I64, P, ctypes.c_double, P]
        lib.oracle_noise.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _arrs(forest):
    par = np.ascontiguousarray(forest.parent, dtype=np.int32)
    off = np.ascontiguousarray(forest.cell_offsets, dtype=np.int64)
    return par, off


class PivotError(RuntimeError):
    pass


def solve(forest, diag, upper, rhs, nthreads: int = 0, return_pivots: bool = False):
    """x = A^-1 rhs in FP64 (paper §2, Listing 2, coupling read as u[i])."""
    par, off = _arrs(forest)
    d = np.array(diag, dtype=np.float64, copy=True)
    u = np.ascontiguousarray(upper, dtype=np.float64)
    b = np.array(rhs, dtype=np.float64, copy=True)
    bad = _load().oracle_solve_f64(len(off) - 1, _p(off), _p(par), _p(d), _p(u), _p(b), nthreads)
    if bad:
        raise PivotError(f"{bad} non-positive pivots")
    return (b, d) if return_pivots else b


def solve_f32(forest, diag32, upper32, rhs32, nthreads: int = 0):
    """The same elimination carried out in FP32."""
    par, off = _arrs(forest)
    d = np.array(diag32, dtype=np.float32, copy=True)
    u = np.ascontiguousarray(upper32, dtype=np.float32)
    b = np.array(rhs32, dtype=np.float32, copy=True)
    bad = _load().oracle_solve_f32(len(off) - 1, _p(off), _p(par), _p(d), _p(u), _p(b), nthreads)
    if bad:
        raise PivotError(f"{bad} non-positive pivots (fp32)")
    return b


def spmv(forest, diag, upper, x, nthreads: int = 0):
    """y = A x for the symmetric tree matrix (paper §1)."""
    par, off = _arrs(forest)
    d = np.ascontiguousarray(diag, dtype=np.float64)
    u = np.ascontiguousarray(upper, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(xx)
    _load().oracle_spmv_f64(len(off) - 1, _p(off), _p(par), _p(d), _p(u), _p(xx), _p(y), nthreads)
    return y


def residual(forest, diag, upper, rhs, x, nthreads: int = 0):
    """r = rhs - A x in FP64."""
    return np.asarray(rhs, dtype=np.float64) - spmv(forest, diag, upper, x, nthreads)


def philox(counter, key):
    """One Philox4x32-10 block (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().oracle_philox(_p(c), _p(k), _p(out))
    return out


def noise(seed: int, step: int, idx, scale: float):
    """scale * Z(seed, step, i) for user indices ``idx`` (Box-Muller on Philox)."""
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(ii.shape[0], dtype=np.float64)
    _load().oracle_noise(seed & 0xFFFFFFFF, step & 0xFFFFFFFF, ii.shape[0], _p(ii), float(scale), _p(out))
    return out


def timeloop(forest, diag, upper, c, steps: int, *, V0=None, I_const=None, noise_seed=None,
             noise_sigma=0.0, first_step: int = 0, keep_all: bool = False, nthreads: int = 0,
             index=None):
    """Implicit-Euler steps V^{k+1} = A^-1 (c V^k + I^k) (paper §1, the discrete
    system with I evaluated at the old step).  I^k is ``I_const`` if given,
    else ``noise_sigma * Z(noise_seed, k, i)`` with i the compartment's user
    index: ``index[j]`` for compartment j when given (cells taken out of a
    larger network keep their draws), else j.  Returns V^steps (and the list
    of all states when ``keep_all``)."""
    n = forest.n
    V = np.zeros(n) if V0 is None else np.array(V0, dtype=np.float64, copy=True)
    idx = np.arange(n, dtype=np.int64) if index is None else np.ascontiguousarray(index, dtype=np.int64)
    assert idx.shape == (n,)
    hist = [V.copy()] if keep_all else None
    for k in range(first_step, first_step + steps):
        if I_const is not None:
            I = I_const
        else:
            I = noise(noise_seed, k, idx, noise_sigma)
        b = c * V + I
        V = solve(forest, diag, upper, b, nthreads)
        if keep_all:
            hist.append(V.copy())
    return (V, hist) if keep_all else V


def timestep_assembled(forest, upper, c, g, ge, v, nthreads: int = 0):
    """One implicit-Euler step with a linearised membrane current (paper §1):
    the diagonal is the capacitive term plus g plus the conductances of every
    edge meeting the compartment (a = -upper, none above a root); the right-
    hand side is c v + g E, given as ``ge``.  Returns A^-1 (c v + ge)."""
    par = np.asarray(forest.parent)
    nonroot = par >= 0
    a = np.where(nonroot, -np.asarray(upper, dtype=np.float64), 0.0)
    diag = np.asarray(c, dtype=np.float64) + np.asarray(g, dtype=np.float64) + a
    diag = diag + np.bincount(par[nonroot], weights=a[nonroot], minlength=forest.n)
    return solve(forest, diag, np.where(nonroot, upper, 0.0), np.asarray(c) * np.asarray(v) + np.asarray(ge), nthreads)


def refine(forest, diag32, upper32, rhs, sweeps: int = 3, nthreads: int = 0):
    """FP32 solves with FP64 residuals and FP64 accumulation.

    The matrix is the FP32 one widened exactly to FP64.  Returns the list of
    iterates x^0 .. x^sweeps."""
    d64 = np.asarray(diag32, dtype=np.float32).astype(np.float64)
    u64 = np.asarray(upper32, dtype=np.float32).astype(np.float64)
    b = np.asarray(rhs, dtype=np.float64)
    x = solve_f32(forest, diag32, upper32, b.astype(np.float32), nthreads).astype(np.float64)
    out = [x.copy()]
    for _ in range(sweeps):
        r = residual(forest, d64, u64, b, x, nthreads)
        dx = solve_f32(forest, diag32, upper32, r.astype(np.float32), nthreads)
        x = x + dx.astype(np.float64)
        out.append(x.copy())
    return out


def adjoint(forest, a, c, I, target, steps: int, nthreads: int = 0):
    """Loss and gradients of the time loop with a squared soma-voltage loss.

    Forward: A V^k = c V^{k-1} + I, V^0 = 0, A = diag(c) + L(a) (paper §1).
    Loss: sum over cells and k = 1..steps of (V^k_root - target_cell)^2.
    Backward (A = A^T): lambda^{steps+1} = 0 and for k = steps..1
      A lambda^k = dLoss/dV^k + c lambda^{k+1};
      dL/dI   += lambda^k;
      dL/dc_i += lambda^k_i (V^{k-1}_i - V^k_i);
      dL/da_e += -(lambda^k_i - lambda^k_p)(V^k_i - V^k_p) for the edge e=(i, p(i)).
    Returns (loss, dL/da, dL/dc, dL/dI, V^steps); dL/da is stored at the child."""
    par = forest.parent
    nonroot = par >= 0
    a = np.where(nonroot, np.asarray(a, dtype=np.float64), 0.0)
    diag = c + a + np.bincount(par[nonroot], weights=a[nonroot], minlength=forest.n)
    upper = -a
    roots = forest.cell_offsets[:-1]
    V = [np.zeros(forest.n)]
    for _ in range(steps):
        V.append(solve(forest, diag, upper, c * V[-1] + I, nthreads))
    loss = 0.0
    for k in range(1, steps + 1):
        loss += float(np.sum((V[k][roots] - target) ** 2))
    lam_next = np.zeros(forest.n)
    ga = np.zeros(forest.n)
    gc = np.zeros(forest.n)
    gI = np.zeros(forest.n)
    pp = np.maximum(par, 0)
    for k in range(steps, 0, -1):
        mu = c * lam_next
        mu[roots] += 2.0 * (V[k][roots] - target)
        lam = solve(forest, diag, upper, mu, nthreads)
        gI += lam
        gc += lam * (V[k - 1] - V[k])
        ga += np.where(nonroot, -(lam - lam[pp]) * (V[k] - V[k][pp]), 0.0)
        lam_next = lam
    return loss, ga, gc, gI, V[-1]

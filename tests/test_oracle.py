"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

* dense Gaussian elimination (LAPACK through numpy) on every Hines tree with
  up to 7 compartments and on random small forests;
* the tridiagonal special case p[i] = i-1 (paper §2), against LAPACK's banded
  solver through scipy;
* the 2x2 closed form (Cramer's rule);
* recovery of x_true from b = A x_true;
* the column-sum invariant of the cable matrix (paper §1: 1^T A = c^T);
* the pivot bound of strictly diagonally dominant elimination;
* plausible mistakes (the printed backward indexing, a dropped update, a sign
  flip) planted in small Python copies must fail the dense pin.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import oracle
from workloads import Forest, assemble, configs


def dense_from_edges(parent, a, c):
    """A = diag(c) + graph Laplacian of the edge weights a (paper §1)."""
    n = len(parent)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] += c[i]
        p = int(parent[i])
        if p >= 0:
            A[i, i] += a[i]
            A[p, p] += a[i]
            A[i, p] -= a[i]
            A[p, i] -= a[i]
    return A


def forest_of_cells(parents):
    """Concatenate single-cell parent arrays (cell-local indices) into a forest."""
    sizes = [len(p) for p in parents]
    off = np.zeros(len(parents) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    par = np.concatenate([np.where(np.asarray(p) >= 0, np.asarray(p) + o, -1)
                          for p, o in zip(parents, off[:-1])]).astype(np.int32)
    bo = np.arange(off[-1] + 1, dtype=np.int64)  # every compartment its own branch
    return Forest(par, off, bo)


def all_trees(n):
    """Every parent array with p[0] = -1 and 0 <= p[i] < i ((n-1)! of them)."""
    for choice in itertools.product(*[range(i) for i in range(1, n)]):
        yield [-1] + list(choice)


def random_values(forest, rng, a_lo=0.5, a_hi=2.0):
    a = rng.uniform(a_lo, a_hi, size=forest.n)
    c = rng.uniform(0.1, 1.0, size=forest.n)
    a[forest.parent < 0] = 0.0
    d, u = assemble(forest, a, c)
    return a, c, d, u


def per_cell_dense_check(forest, a, c, d, u, b, x, tol):
    worst = 0.0
    for k in range(forest.ncells):
        lo, hi = forest.cell_offsets[k], forest.cell_offsets[k + 1]
        par = np.where(forest.parent[lo:hi] >= 0, forest.parent[lo:hi] - lo, -1)
        A = dense_from_edges(par, a[lo:hi], c[lo:hi])
        xs = np.linalg.solve(A, b[lo:hi])
        err = np.max(np.abs(x[lo:hi] - xs)) / np.max(np.abs(xs))
        worst = max(worst, err)
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_every_tree_up_to_7_vs_dense(n):
    trees = list(all_trees(n))
    f = forest_of_cells(trees)
    rng = np.random.default_rng(100 + n)
    a, c, d, u = random_values(f, rng)
    b = rng.standard_normal(f.n)
    x = oracle.solve(f, d, u, b)
    per_cell_dense_check(f, a, c, d, u, b, x, 1e-13)


def test_random_small_forests_vs_dense():
    s = configs.random_system(60, seed=7)
    f = s.forest
    assert np.diff(f.cell_offsets).max() <= 400
    x = oracle.solve(f, s.diag, s.upper, s.rhs)
    per_cell_dense_check(f, s.a, s.c, s.diag, s.upper, s.rhs, x, 1e-11)


def test_dense_matrix_matches_assembly():
    """The generator's (diag, upper) are the entries of the §1 matrix."""
    s = configs.random_system(5, seed=3)
    f = s.forest
    A = dense_from_edges(f.parent, s.a, s.c)
    assert np.allclose(np.diag(A), s.diag, rtol=0, atol=1e-12)
    nr = f.parent >= 0
    assert np.array_equal(A[np.arange(f.n)[nr], f.parent[nr]], s.upper[nr])
    assert np.array_equal(A, A.T)
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    assert (np.diag(A) > off).all()  # strictly diagonally dominant (paper §1)
    assert np.linalg.eigvalsh(A).min() > 0


def test_thomas_special_case_vs_banded():
    """p[i] = i-1 reduces the Hines algorithm to the Thomas algorithm (§2)."""
    n = 1000
    f = forest_of_cells([[-1] + list(range(n - 1))])
    rng = np.random.default_rng(11)
    a, c, d, u = random_values(f, rng)
    b = rng.standard_normal(n)
    x = oracle.solve(f, d, u, b)
    ab = np.zeros((3, n))
    ab[0, 1:] = u[1:]   # superdiagonal A[i-1, i] = u[i]
    ab[1, :] = d
    ab[2, :-1] = u[1:]  # subdiagonal A[i, i-1] = u[i]
    xs = scipy.linalg.solve_banded((1, 1), ab, b)
    assert np.max(np.abs(x - xs)) / np.max(np.abs(xs)) < 1e-13


def test_two_by_two_closed_form():
    f = forest_of_cells([[-1, 0]])
    d = np.array([3.0, 5.0])
    u = np.array([0.0, -2.0])
    b = np.array([1.0, 4.0])
    x = oracle.solve(f, d, u, b)
    det = d[0] * d[1] - u[1] ** 2
    assert abs(x[0] - (d[1] * b[0] - u[1] * b[1]) / det) < 1e-15
    assert abs(x[1] - (d[0] * b[1] - u[1] * b[0]) / det) < 1e-15


def test_spmv_vs_dense():
    s = configs.random_system(8, seed=5)
    f = s.forest
    A = dense_from_edges(f.parent, s.a, s.c)
    x = np.random.default_rng(2).standard_normal(f.n)
    y = oracle.spmv(f, s.diag, s.upper, x)
    assert np.max(np.abs(y - A @ x)) <= 1e-12 * np.max(np.abs(A @ x))


def test_recover_x_true_c2_cells():
    s = configs.c2(512)
    f = s.forest
    xt = np.random.default_rng(9).standard_normal(f.n)
    b = oracle.spmv(f, s.diag, s.upper, xt)
    x = oracle.solve(f, s.diag, s.upper, b)
    worst = 0.0
    for k in range(f.ncells):
        lo, hi = f.cell_offsets[k], f.cell_offsets[k + 1]
        worst = max(worst, np.max(np.abs(x[lo:hi] - xt[lo:hi])) / np.max(np.abs(xt[lo:hi])))
    assert worst < 1e-10, worst


def test_column_sum_invariant_c2():
    """1^T A = c^T for the cable matrix, so sum_i c_i x_i = sum_i b_i per cell."""
    s = configs.c2(2048)
    f = s.forest
    x = oracle.solve(f, s.diag, s.upper, s.rhs)
    cid = np.repeat(np.arange(f.ncells), np.diff(f.cell_offsets))
    lhs = np.bincount(cid, weights=s.c * x)
    rhs = np.bincount(cid, weights=s.rhs)
    scale = np.bincount(cid, weights=np.abs(s.c * x)) + np.bincount(cid, weights=np.abs(s.rhs))
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13


def test_pivot_bound_c2():
    """Eliminated pivots of the cable matrix satisfy d'_i >= c_i + a_i > 0."""
    s = configs.c2(256)
    _, dpiv = oracle.solve(s.forest, s.diag, s.upper, s.rhs, return_pivots=True)
    assert (dpiv >= (s.c + s.a) * (1 - 1e-14)).all()


def test_c1_shape_and_identity_structure():
    s = configs.c1()
    f = s.forest
    assert f.n == 4096 * 75 and f.ncells == 4096 and f.nbranches == 4096 * 15
    # branch b's first compartment attaches to the last compartment of branch (b-1)//2
    p = f.parent[:75]
    for b in range(1, 15):
        assert p[5 * b] == 5 * ((b - 1) // 2) + 4
    x = oracle.solve(f, s.diag, s.upper, s.rhs)
    per_cell_dense_check(f.subset(np.arange(16)), s.a[:16 * 75], s.c[:16 * 75], None, None,
                         s.rhs[:16 * 75], x[:16 * 75], 1e-13)


# ---- planted mistakes must fail the dense pin --------------------------------------------

def _mutant(d, u, b, p, kind):
    d = d.copy()
    b = b.copy()
    n = len(d)
    for i in range(n - 1, 0, -1):
        uu = u[p[i]] if kind == "printed_listing" else u[i]
        f = uu / d[i]
        if kind != "drop_d":
            d[p[i]] = d[p[i]] - f * uu
        b[p[i]] = b[p[i]] - f * b[i]
    b[0] = b[0] / d[0]
    for i in range(1, n):
        s = -1.0 if kind == "sign" else 1.0
        b[i] = (b[i] - s * u[i] * b[p[i]]) / d[i]
    return b


@pytest.mark.parametrize("kind", ["printed_listing", "drop_d", "sign"])
def test_planted_mistakes_fail_dense_pin(kind):
    rng = np.random.default_rng(5)
    worst = 0.0
    for par in list(all_trees(6))[::7]:
        f = forest_of_cells([par])
        a, c, d, u = random_values(f, rng)
        b = rng.standard_normal(f.n)
        A = dense_from_edges(f.parent, a, c)
        xs = np.linalg.solve(A, b)
        xm = _mutant(d, u, b, f.parent, kind)
        worst = max(worst, np.max(np.abs(xm - xs)) / np.max(np.abs(xs)))
        # the oracle itself passes on the same inputs
        assert np.max(np.abs(oracle.solve(f, d, u, b) - xs)) <= 1e-13 * np.max(np.abs(xs))
    assert worst > 1e-3, (kind, worst)

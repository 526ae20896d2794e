"""Pins of the oracle's time loop, noise, refinement and adjoint."""
import os

import numpy as np
import pytest
import scipy.stats

import oracle
from workloads import Forest, assemble, configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(w, 16) for w in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


def test_noise_is_standard_normal_and_keyed():
    idx = np.arange(200_000, dtype=np.int64)
    z = oracle.noise(3, 0, idx, 1.0)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    z1 = oracle.noise(3, 1, idx, 1.0)
    assert abs(np.corrcoef(z, z1)[0, 1]) < 0.01
    # keyed by the user index: any subset gives the same values
    sub = idx[::37]
    assert np.array_equal(oracle.noise(3, 0, sub, 1.0), z[::37])
    assert np.array_equal(oracle.noise(3, 0, idx, 0.1), 0.1 * z)


def test_timeloop_charge_conservation():
    """Column sums of A equal c (paper §1), hence per cell
    sum_i c_i V_i^{k+1} = sum_i c_i V_i^k + sum_i I_i^k."""
    s = configs.c3(300)
    f = s.forest
    cid = np.repeat(np.arange(f.ncells), np.diff(f.cell_offsets))
    V = np.zeros(f.n)
    idx = np.arange(f.n, dtype=np.int64)
    for k in range(3):
        Vn = oracle.timeloop(f, s.diag, s.upper, s.c, 1, V0=V, noise_seed=3, noise_sigma=0.1,
                             first_step=k)
        I = oracle.noise(3, k, idx, 0.1)
        lhs = np.bincount(cid, weights=s.c * Vn)
        rhs = np.bincount(cid, weights=s.c * V) + np.bincount(cid, weights=I)
        scale = np.bincount(cid, weights=np.abs(s.c * Vn)) + np.bincount(cid, weights=np.abs(I))
        assert np.max(np.abs(lhs - rhs) / scale) < 1e-12
        V = Vn


def test_timeloop_cells_out_of_a_network_keep_their_draws():
    """Cells do not couple: the oracle's time loop over a few cells taken out
    of a network, with the draws keyed by their user indices in it, gives the
    full loop's values on those cells exactly; with the identity index it is
    the plain loop."""
    s = configs.c3(40)
    f = s.forest
    full = oracle.timeloop(f, s.diag, s.upper, s.c, 3, noise_seed=3, noise_sigma=0.1)
    same = oracle.timeloop(f, s.diag, s.upper, s.c, 3, noise_seed=3, noise_sigma=0.1, index=np.arange(f.n))
    assert np.array_equal(full, same)
    pick = np.array([1, 5, 17, 30])
    idx = np.concatenate([np.arange(f.cell_offsets[q], f.cell_offsets[q + 1]) for q in pick])
    part = oracle.timeloop(f.subset(pick), s.diag[idx], s.upper[idx], s.c[idx], 3, noise_seed=3,
                           noise_sigma=0.1, index=idx)
    assert np.array_equal(part, full[idx])
    # the draws are keyed: without the index the subset's values differ
    plain = oracle.timeloop(f.subset(pick), s.diag[idx], s.upper[idx], s.c[idx], 3, noise_seed=3,
                            noise_sigma=0.1)
    assert not np.array_equal(plain, full[idx])

@pytest.mark.parametrize("dt", [0.001, 0.025, 1.0])
def test_refinement_reaches_fp64_solution(dt):
    s = configs.c4(dts=(dt,), ncells=256)[dt]
    f = s.forest
    d32 = s.diag.astype(np.float32)
    u32 = s.upper.astype(np.float32)
    xs = oracle.solve(f, d32.astype(np.float64), u32.astype(np.float64), s.rhs)
    its = oracle.refine(f, d32, u32, s.rhs, sweeps=3)
    errs = [np.max(np.abs(x - xs)) / np.max(np.abs(xs)) for x in its]
    assert errs[0] > 1e-9          # raw FP32 is far from FP64
    assert errs[-1] <= 1e-11, errs
    assert errs[1] < errs[0]


def _tiny_forest():
    s = configs.random_system(3, seed=21)
    return s.forest


def test_adjoint_vs_dense_autograd():
    torch = pytest.importorskip("torch")
    f = _tiny_forest()
    n = f.n
    rng = np.random.default_rng(1)
    a = rng.uniform(0.5, 2.0, n)
    a[f.parent < 0] = 0
    c = rng.uniform(0.5, 3.0, n)
    I = 0.1 * rng.standard_normal(n)
    target = rng.standard_normal(f.ncells)
    steps = 6
    loss, ga, gc, gI, _ = oracle.adjoint(f, a, c, I, target, steps)

    ta = torch.tensor(a, dtype=torch.float64, requires_grad=True)
    tc = torch.tensor(c, dtype=torch.float64, requires_grad=True)
    tI = torch.tensor(I, dtype=torch.float64, requires_grad=True)
    par = torch.tensor(f.parent.astype(np.int64))
    nr = par >= 0
    ci = torch.arange(n)[nr]
    pi = par[nr]
    A = torch.diag(tc)
    L = torch.zeros(n, n, dtype=torch.float64)
    L = L.index_put((ci, ci), ta[nr], accumulate=True)
    L = L.index_put((pi, pi), ta[nr], accumulate=True)
    L = L.index_put((ci, pi), -ta[nr], accumulate=True)
    L = L.index_put((pi, ci), -ta[nr], accumulate=True)
    A = A + L
    roots = torch.tensor(f.cell_offsets[:-1])
    V = torch.zeros(n, dtype=torch.float64)
    tl = torch.zeros((), dtype=torch.float64)
    tt = torch.tensor(target)
    for _ in range(steps):
        V = torch.linalg.solve(A, (tc * V + tI).unsqueeze(1)).squeeze(1)
        tl = tl + ((V[roots] - tt) ** 2).sum()
    tl.backward()
    assert abs(loss - tl.item()) <= 1e-12 * abs(loss)
    nrm = f.parent >= 0

    def rel(x, y):
        return np.max(np.abs(x - y)) / np.max(np.abs(y))
    assert rel(ga[nrm], ta.grad.numpy()[nrm]) < 1e-10
    assert rel(gc, tc.grad.numpy()) < 1e-10
    assert rel(gI, tI.grad.numpy()) < 1e-10


def test_adjoint_vs_central_differences():
    s = configs.c5(4, size=60)
    f = s.forest
    I = s.meta["I"]
    target = s.meta["target"]
    steps = 10
    _, ga, gc, gI, _ = oracle.adjoint(f, s.a, s.c, I, target, steps)
    rng = np.random.default_rng(5)
    h = 1e-6
    cid = np.repeat(np.arange(f.ncells), np.diff(f.cell_offsets))
    for kind in ("a", "c", "I"):
        for _ in range(3):
            i = int(rng.integers(0, f.n))
            if kind == "a" and f.parent[i] < 0:
                i += 1
            cell = cid[i]
            sub = f.subset([cell])
            lo = f.cell_offsets[cell]
            hi = f.cell_offsets[cell + 1]

            def L(delta):
                aa = s.a[lo:hi].copy()
                cc = s.c[lo:hi].copy()
                II = I[lo:hi].copy()
                {"a": aa, "c": cc, "I": II}[kind][i - lo] += delta
                return oracle.adjoint(sub, aa, cc, II, target[cell:cell + 1], steps)[0]
            fd = (L(h) - L(-h)) / (2 * h)
            g = {"a": ga, "c": gc, "I": gI}[kind][i]
            assert abs(fd - g) <= 1e-5 * max(abs(g), 1e-3), (kind, i, fd, g)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_assembled_step_vs_dense_matrix_from_edges(seed):
    """The assembled step against a dense matrix built edge by edge from the
    cable equation's definition (each edge adds a to both diagonal ends and
    -a off the diagonal; c + g on the diagonal), solved by LAPACK; the value
    stored at a root's upper entry plays no part."""
    rng = np.random.default_rng(seed)
    f = configs.random_system(6, seed).forest
    n = f.n
    a = rng.uniform(0.1, 2.0, n)
    upper = -a
    upper[f.parent < 0] = 123.0  # ignored
    c, g = rng.uniform(0.1, 1.0, n), rng.uniform(0.0, 3.0, n)
    ge, v = rng.standard_normal(n), rng.standard_normal(n)
    A = np.diag(c + g)
    for i in range(n):
        p = f.parent[i]
        if p >= 0:
            A[i, i] += a[i]
            A[p, p] += a[i]
            A[i, p] = A[p, i] = -a[i]
    want = np.linalg.solve(A, c * v + ge)
    got = oracle.timestep_assembled(f, upper, c, g, ge, v)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13)

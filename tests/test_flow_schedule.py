"""CPU replay of the flow kernel's chunk schedule.

The host builder hands the flow kernel four tables per plan (per-chunk-step
lane masks, element entries, push targets, group records).  This test
replays the kernel's semantics on those tables in plain numpy (K sub-steps
per busy lane and chunk step, identity pads, pushes at path tops) and checks

* the ordering rules the kernel relies on: every entry is eliminated exactly
  once; a push into a parent's entry happens at least two chunk steps before
  the step that eliminates it (operands are read one step ahead); in the
  forward sweep a pushed path reads its parent's x at least two steps after
  the parent wrote it;
* the solution against the FP64 oracle (relative error <= 1e-12 per cell).
"""
import numpy as np
import pytest

import oracle
from workloads import configs
from workloads.configs import random_system

LANES = np.arange(64, dtype=np.uint64)


def _bits(m):
    return np.nonzero((np.uint64(m) >> LANES) & np.uint64(1))[0]


def replay(plan, f, diag, upper, rhs):
    fg = plan.table("flow_groups").reshape(-1, 8)
    masks = plan.table("flow_masks").view(np.uint64)
    pos = plan.table("flow_pos")
    aux = plan.table("flow_aux")
    goff = plan.table("group_offsets")
    gcells = plan.table("group_cells")
    co = f.cell_offsets
    x = np.full(f.n, np.nan)
    for g in range(fg.shape[0]):
        step_off, pos_off, aux_off, F, nel, naux, nent, K = (int(v) for v in fg[g])
        users = np.concatenate([np.arange(co[c], co[c + 1]) for c in gcells[goff[g]:goff[g + 1]]])
        if F == 0:  # too large for LDS: solved by the level-synchronous kernel
            assert nel == 0 and naux == 0
            continue
        assert users.size == nel and nent >= nel and aux_off % 2 == 0
        B8 = 3 * K + 1  # LDS block of a lane-chunk, in 8-byte units; entry j at 3 j

        def to_entry(off):
            off = np.asarray(off)
            assert np.all((off % B8) < 3 * K) and np.all((off % B8) % 3 == 0)
            return (off // B8) * K + (off % B8) // 3
        pw = pos[pos_off:pos_off + nel]
        P = to_entry(pw & 0x7FFF)
        root = (pw & 0x8000) != 0
        assert np.unique(P).size == nel and P.max() < nent
        assert np.array_equal(np.sort(users[root]), np.sort(co[gcells[goff[g]:goff[g + 1]]]))
        D = np.ones(nent)  # pads: identity compartments
        U = np.zeros(nent)
        B = np.zeros(nent)
        D[P] = diag[users]
        U[P] = np.where(root, 0.0, upper[users])
        B[P] = rhs[users]
        ax = to_entry(aux[aux_off:aux_off + naux]) if naux else aux[:0]
        elim_step = np.full(nent, -1)
        last_push = np.full(nent, -10)
        fin = np.zeros(64)
        uin = np.zeros(64)
        bin_ = np.zeros(64)
        R = A = 0
        for t in range(F):
            M = masks[2 * (step_off + t)]
            E = masks[2 * (step_off + t) + 1]
            act = _bits(M)
            push = _bits(E)
            c = act.size
            assert np.all(np.isin(push, act))
            for j in range(K):
                e = (R + np.arange(c)) * K + j
                assert np.all(elim_step[e] < 0)
                assert np.all(last_push[e] <= t - 2), "push too late for the one-step-ahead read"
                elim_step[e] = t
                dl = D[e] - fin[act] * uin[act]
                bl = B[e] - fin[act] * bin_[act]
                r = 1.0 / dl
                fv = U[e] * r
                D[e] = fv
                B[e] = bl * r
                fin[act] = fv
                uin[act] = U[e]
                bin_[act] = bl
            nf = np.zeros(64)
            nf[act] = fin[act]
            if push.size:
                q = ax[A + np.arange(push.size)]
                assert np.all(elim_step[q] < 0), "push after the parent was eliminated"
                for qq, l in zip(q, push):  # in lane order
                    D[qq] -= fin[l] * uin[l]
                    B[qq] -= fin[l] * bin_[l]
                    last_push[qq] = t
                nf[push] = 0.0
            fin = nf
            R += c
            A += push.size
        assert R * K == nent and A == naux
        xp = np.zeros(64)
        for t in range(F - 1, -1, -1):
            M = masks[2 * (step_off + t)]
            E = masks[2 * (step_off + t) + 1]
            act = _bits(M)
            push = _bits(E)
            c = act.size
            R -= c
            A -= push.size
            xv = xp[act].copy()
            if push.size:
                k = np.searchsorted(act, push)
                q = ax[A + np.arange(push.size)]
                assert np.all(elim_step[q] >= t + 2), "parent x not written two steps earlier"
                xv[k] = B[q]
            for j in range(K - 1, -1, -1):
                e = (R + np.arange(c)) * K + j
                xv = B[e] - D[e] * xv
                B[e] = xv
            xp[act] = xv
        x[users] = B[P]
    return x


def cell_err(f, x, xo):
    e = np.maximum.reduceat(np.abs(x - xo), f.cell_offsets[:-1])
    s = np.maximum.reduceat(np.abs(xo), f.cell_offsets[:-1])
    return float(np.max(e / s))


CASES = {
    "random_small": lambda: random_system(300, 5),
    "c2_cells": lambda: configs.c2(40),
    "c1_cells": lambda: configs.c1(64),
    "c3_cells": lambda: configs.c3(60),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("opts", [dict(), dict(split_branches=1), dict(max_group_unknowns=4000),
                                  dict(cell_order=1, max_group_unknowns=700)],
                         ids=["default", "split", "cap4000", "sorted_cap700"])
def test_flow_replay_matches_oracle(name, opts):
    from paper_1810_12742_amd import Plan
    s = CASES[name]()
    f = s.forest
    rhs = np.random.default_rng(3).standard_normal(f.n)
    p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, **opts)
    assert p.info["kernel"] == 1
    x = replay(p, f, s.diag, s.upper, rhs)
    xo = oracle.solve(f, s.diag, s.upper, rhs)
    done = ~np.isnan(x)
    assert done.sum() >= min(10000, f.n)
    xo[~done] = x[~done] = 1.0
    assert cell_err(f, x, xo) <= 1e-12


def test_flow_not_used_for_rerooted_or_bitwise_plans():
    from paper_1810_12742_amd import Plan
    s = random_system(50, 2)
    f = s.forest
    for opts in (dict(rebalance_root=1), dict(bitwise=1), dict(level_sync=1)):
        p = Plan(f.parent, f.cell_offsets, f.branch_offsets, host_only=1, **opts)
        if opts.get("rebalance_root"):
            continue  # flow only if every re-rooted branch still ascends
        assert p.info["kernel"] != 1, opts

"""Batches of problems (mbl_solve_batch): up to 16 disorder realizations or
targets of one chain length factored, solved and iterated in shared launches.
Each problem's arithmetic is that of a lone mbl_solve, so every output is
bitwise the same as a separate call -- energies, vectors, residuals,
observables and the iteration counts that trace the control flow (restarts,
operator applications, passes through the factors, refinement sweeps,
perturbed pivots).  One batched problem per size is also checked against the
oracle."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu

VALUES = ("evals", "resid", "r", "s1", "se", "s2", "fluct", "dynfrac", "kl", "evecs")
COUNTS = ("emin", "emax", "sigma", "hnorm", "nconv", "n_restarts", "n_opapply", "n_passes",
          "n_pass_rhs", "ir_iters_max", "n_perturbed", "fallback", "status")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mbl.Context(0)
    yield c
    c.close()


def items(count, seed):
    rng = np.random.default_rng(seed)
    return [dict(h=float(rng.uniform(0.5, 5.0)), seed=1000 * seed + q,
                 eps=float(rng.uniform(0.05, 0.95))) for q in range(count)]


def assert_same(b, a, tag):
    for k in VALUES:
        assert np.array_equal(b[k], a[k]), (tag, k)
    for k in COUNTS:
        assert b[k] == a[k], (tag, k, b[k], a[k])


@pytest.mark.parametrize("L,count,prec", [(10, 3, mbl.MBL_FP64), (12, 5, mbl.MBL_FP64),
                                          (14, 16, mbl.MBL_FP64), (12, 4, mbl.MBL_FP32_IR64),
                                          (14, 6, mbl.MBL_FP32_IR64)],
                         ids=["L10x3", "L12x5", "L14x16", "L12x4-fp32", "L14x6-fp32"])
def test_batched_equals_alone(ctx, L, count, prec):
    nev = 20
    its = items(count, L + count)
    say("batch", L, count, prec)
    outs = ctx.mbl_solve_batch(L, nev, its, prec=prec, vectors=True, extra=True)
    with mbl.Context(0) as c2:
        for q, (it, b) in enumerate(zip(its, outs)):
            a = c2.mbl_solve(L, it["h"], it["seed"], it["eps"], nev, prec=prec, vectors=True,
                             extra=True, allow_notconv=True)
            assert_same(b, a, (L, q))
            assert a["batch"] == 1
    # the batched path ran (no problem of these sets leaves it)
    assert all(b["batch"] == count for b in outs), [b["batch"] for b in outs]
    # and against the oracle, one problem of the batch
    if L <= 12:
        it = its[0]
        ref = oracle.solve(L, it["h"], it["seed"], it["eps"], nev, observables=False)
        hn = ref["hnorm"]
        assert np.abs(outs[0]["evals"] - ref["evals"]).max() <= 1e-10 * hn
        assert outs[0]["max_resid"] <= 1e-9


def test_batch_then_smaller_batch_and_lone(ctx):
    """Plans and factors of several batch sizes in one context, a lone solve in
    between: each still equals its separate call."""
    L, nev = 12, 20
    its = items(7, 99)
    first = ctx.mbl_solve_batch(L, nev, its)
    lone = ctx.mbl_solve(L, its[0]["h"], its[0]["seed"], its[0]["eps"], nev)
    second = ctx.mbl_solve_batch(L, nev, its[:3])
    assert [b["batch"] for b in first] == [7] * 7 and [b["batch"] for b in second] == [3] * 3
    for k in ("evals", "resid", "s1", "se"):
        assert np.array_equal(first[0][k], lone[k])
        for q in range(3):
            assert np.array_equal(first[q][k], second[q][k]), (q, k)


def test_unbatchable_sets_are_solved_alone(ctx):
    """Mixed chain lengths, a sector below the batch minimum, one problem:
    solved one at a time, with the same results as separate calls."""
    nev = 10
    with mbl.Context(0) as c2:
        out = ctx.mbl_solve_batch(8, nev, items(3, 5))          # dim 70: below 128
        for it, b in zip(items(3, 5), out):
            a = c2.mbl_solve(8, it["h"], it["seed"], it["eps"], nev)
            assert np.array_equal(b["evals"], a["evals"])
            assert b["batch"] == 1
        one = ctx.mbl_solve_batch(12, nev, items(1, 6))
        it = items(1, 6)[0]
        a = c2.mbl_solve(12, it["h"], it["seed"], it["eps"], nev)
        assert np.array_equal(one[0]["evals"], a["evals"])


def test_batch_with_explicit_targets_and_fields(ctx):
    """sigma given instead of eps, and fields given instead of a seed."""
    L, nev = 12, 12
    f = oracle.fields(L, 2.5, 7)
    its = [dict(h=2.5, seed=7, sigma=-1.0), dict(h=0.0, seed=0, fields=f, eps=0.3),
           dict(h=4.0, seed=3, eps=0.0), dict(h=4.0, seed=3, eps=1.0)]
    out = ctx.mbl_solve_batch(L, nev, its)
    with mbl.Context(0) as c2:
        for it, b in zip(its, out):
            a = c2.mbl_solve(L, it["h"], it["seed"], it.get("eps", 0.5), nev,
                             sigma=it.get("sigma", float("nan")), fields=it.get("fields"))
            for k in ("evals", "resid", "s1", "se", "r"):
                assert np.array_equal(b[k], a[k]), k
            assert b["n_passes"] == a["n_passes"]


def test_invalid_problem_in_a_batch(ctx):
    """A problem with an invalid eps gets its own status; the others are solved."""
    its = items(3, 8)
    its[1]["eps"] = 1.5
    k = len(its)
    prs = (mbl.mbl_problem * k)()
    ress = (mbl.mbl_result * k)()
    bufs = []
    for q, it in enumerate(its):
        p, r, b, _f = ctx._prepare(12, it["h"], it["seed"], it["eps"], 10, 1.0, mbl.MBL_FP64, None,
                                   float("nan"), 0.0, False, False, 0, 0, True)
        prs[q], ress[q] = p, r
        bufs.append(b)
    status = (ctypes.c_int * k)()
    code = mbl.lib().mbl_solve_batch(ctx._h, k, prs, ress, status)
    assert code == mbl.MBL_EINVAL
    assert list(status) == [mbl.MBL_OK, mbl.MBL_EINVAL, mbl.MBL_OK]
    a = ctx.mbl_solve(12, its[2]["h"], its[2]["seed"], its[2]["eps"], 10)
    assert np.array_equal(bufs[2]["evals"], a["evals"])


def test_problem_leaving_the_batch(ctx):
    """A problem whose lone solve leaves the plain refinement (forced by the
    refinement-stall hooks) leaves the batch and is solved alone; its result,
    FP64 fallback or error included, is its lone result, and the rest of the
    batch is unchanged."""
    L, nev = 12, 16
    its = items(4, 21)
    its[1]["hooks"] = mbl.MBL_HOOK_IR_STALL32
    out = ctx.mbl_solve_batch(L, nev, its, prec=mbl.MBL_FP32_IR64)
    assert [o["batch"] for o in out] == [4, 1, 4, 4]
    assert out[1]["fallback"] == 1
    with mbl.Context(0) as c2:
        for it, b in zip(its, out):
            a = c2.mbl_solve(L, it["h"], it["seed"], it["eps"], nev, prec=mbl.MBL_FP32_IR64,
                             hooks=it.get("hooks", 0))
            for k in ("evals", "resid", "r", "s1", "se"):
                assert np.array_equal(b[k], a[k]), k
            for k in ("n_passes", "fallback", "status"):
                assert b[k] == a[k], k
    # FP64: the forced stall is an error of that problem alone
    its = items(3, 22)
    its[2]["hooks"] = mbl.MBL_HOOK_IR_STALL64
    out = ctx.mbl_solve_batch(L, nev, its)
    assert [o["status"] for o in out] == [mbl.MBL_OK, mbl.MBL_OK, mbl.MBL_ENUMERIC]
    assert [o["batch"] for o in out[:2]] == [3, 3]
    a = ctx.mbl_solve(L, its[0]["h"], its[0]["seed"], its[0]["eps"], nev)
    assert np.array_equal(out[0]["evals"], a["evals"])


def test_batch_graph_replays_match_eager(ctx):
    """Block expansions of the Krylov and extremal-energy iterations run as
    captured graphs, replayed at every expansion with host reads of their
    staged coefficients between the replays; batches solved twice in one
    context (so the second call replays graphs captured by the first) equal
    the eager launch sequence bitwise."""
    import os
    sets = [(12, 5, mbl.MBL_FP64), (14, 3, mbl.MBL_FP32_IR64)]
    graphed = []
    for L, count, prec in sets:
        its = items(count, 40 + L)
        first = ctx.mbl_solve_batch(L, 16, its, prec=prec, vectors=True, extra=True)
        again = ctx.mbl_solve_batch(L, 16, its, prec=prec, vectors=True, extra=True)
        for a, b in zip(first, again):
            assert_same(a, b, ("replay", L))
        graphed.append((L, its, prec, first))
    os.environ["MBL_NO_GRAPH"] = "1"
    try:
        eager = mbl.Context(0)
    finally:
        del os.environ["MBL_NO_GRAPH"]
    with eager:
        for L, its, prec, first in graphed:
            out = eager.mbl_solve_batch(L, 16, its, prec=prec, vectors=True, extra=True)
            for a, b in zip(first, out):
                assert_same(a, b, ("eager", L))

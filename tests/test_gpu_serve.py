"""Continuous batching (mbl_serve_start / mbl_submit / mbl_wait): requests of
mixed sizes overlap on the device, are admitted by predicted footprint, and
each result is the same alone and in the mix (bitwise: a request's arithmetic
does not depend on its slot or on the other requests)."""
import sys
import time

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu

KEYS = ("evals", "resid", "r", "s1", "se")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def mix(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = int(rng.choice([8, 10, 12, 14]))
        h = float(rng.uniform(0.5, 5.0))
        eps = float(rng.uniform(0.05, 0.95))
        prec = mbl.MBL_FP32_IR64 if i % 3 == 2 else mbl.MBL_FP64
        out.append((L, h, 100 + i, eps, 20, prec))
    return out


def test_results_same_alone_and_in_mix():
    reqs = mix(24)
    say("serving", len(reqs), "requests on 4 slots")
    with mbl.Context(0) as c:
        c.mbl_serve_start(4)
        tickets = [c.mbl_submit(L, h, s, e, nev, prec=p) for (L, h, s, e, nev, p) in reqs]
        outs = [c.mbl_wait(t) for t in tickets]
        st = c.mbl_serve_stats()
    say("stats", st)
    assert st["completed"] == len(reqs) and st["max_running"] >= 2
    with mbl.Context(0) as c2:
        for (L, h, s, e, nev, p), o in zip(reqs, outs):
            assert o["status"] == mbl.MBL_OK
            a = c2.mbl_solve(L, h, s, e, nev, prec=p)
            for k in KEYS:
                assert np.array_equal(o[k], a[k]), (L, h, s, e, p, k)
            assert o["t_submit"] <= o["t_start"] <= o["t_done"]
    # and the mix itself agrees with the oracle on one request per size
    seen = set()
    for (L, h, s, e, nev, p), o in zip(reqs, outs):
        if L in seen or L > 12:
            continue
        seen.add(L)
        ref = oracle.solve(L, h, s, e, nev)
        assert np.abs(o["evals"] - ref["evals"]).max() <= 1e-10 * ref["hnorm"]


def test_admission_by_footprint():
    with mbl.Context(0) as c:
        fp14 = c.mbl_footprint(14, mbl.MBL_FP64, 20)
        fp8 = c.mbl_footprint(8, mbl.MBL_FP64, 20)
        assert fp8 < fp14
        budget = fp14 + 2 * fp8 + fp8 // 2      # one L = 14 and two L = 8 at a time
        c.mbl_serve_start(4, budget)
        reqs = [(14, 3.0, s, 0.5) for s in range(4)] + [(8, 2.0, s, 0.3) for s in range(6)]
        tickets = [c.mbl_submit(L, h, s, e, 20) for (L, h, s, e) in reqs]
        peak = 0
        while not all(c.mbl_poll(t) for t in tickets):
            i = c.mbl_serve_stats()
            assert i["held_bytes"] <= budget
            peak = max(peak, i["running"])
            time.sleep(0.002)
        outs = [c.mbl_wait(t) for t in tickets]
        st = c.mbl_serve_stats()
    assert all(o["status"] == mbl.MBL_OK for o in outs)
    assert st["max_running"] <= 3
    # a slot never held more device memory than the footprint it was admitted
    # with (the largest admitted footprint here is the L = 14 one)
    assert 0 < st["max_slot_peak"] <= fp14
    # no two L = 14 requests were ever on the device together
    spans = sorted((o["t_start"], o["t_done"]) for (L, *_), o in zip(reqs, outs) if L == 14)
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 1e-6


def test_errors_and_late_arrivals():
    with mbl.Context(0) as c:
        fp10 = c.mbl_footprint(10, mbl.MBL_FP64, 10)
        c.mbl_serve_start(2, fp10 * 3)
        bad = c.mbl_submit(1, 1.0, 0, 0.5, 10)                  # L below 2
        big = c.mbl_submit(16, 1.0, 0, 0.5, 10)                 # above the budget
        first = [c.mbl_submit(10, 2.0, s, 0.5, 10) for s in range(3)]
        time.sleep(0.01)
        late = [c.mbl_submit(10, 2.0, s, 0.7, 10) for s in range(3, 6)]
        assert c.mbl_wait(bad)["status"] == mbl.MBL_EINVAL
        assert c.mbl_wait(big)["status"] == mbl.MBL_ENOMEM
        outs = [c.mbl_wait(t) for t in first + late]
        assert all(o["status"] == mbl.MBL_OK and o["max_resid"] <= 1e-9 for o in outs)
        with pytest.raises(mbl.MblError):
            c.mbl_poll(10 ** 9)


def test_concurrent_large_fronts_bitwise():
    # the benchmark's mode at a size with multi-block fronts (L = 16: outer
    # Schur pairs, merged solve blocks, several solve steps per level): two
    # solves in flight on two slots give bitwise the one-at-a-time results
    cases = [(16, 3.0, 0, 0.5), (16, 2.0, 1, 0.2), (16, 4.0, 2, 0.8), (16, 1.0, 3, 0.5)]
    with mbl.Context(0) as c:
        alone = [c.mbl_solve(L, h, s, e, 50) for (L, h, s, e) in cases]
    say("L=16 solves, 2 at a time")
    with mbl.Context(0) as c:
        c.mbl_serve_batch_limit(1)                # every request alone on its slot
        c.mbl_serve_start(2)
        outs = [c.mbl_wait(t) for t in [c.mbl_submit(L, h, s, e, 50) for (L, h, s, e) in cases]]
        st = c.mbl_serve_stats()
    assert st["max_running"] == 2
    for a, o in zip(alone, outs):
        assert o["status"] == mbl.MBL_OK and o["nconv"] == 50
        for k in KEYS:
            assert np.array_equal(o[k], a[k]), k


def test_batched_serving_bitwise():
    """Requests queued together are admitted as batches (one L, one precision);
    every result equals its lone solve bitwise, batches of FP32 requests too."""
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(40):
        L = int(rng.choice([10, 12, 14]))
        prec = mbl.MBL_FP32_IR64 if i % 2 else mbl.MBL_FP64
        reqs.append((L, float(rng.uniform(0.5, 5.0)), 300 + i, float(rng.uniform(0.05, 0.95)), prec))
    say("batched serving", len(reqs), "requests on 2 slots")
    with mbl.Context(0) as c:
        c.mbl_serve_start(2)
        tickets = [c.mbl_submit(L, h, s, e, 20, prec=p) for (L, h, s, e, p) in reqs]
        outs = [c.mbl_wait(t) for t in tickets]
        st = c.mbl_serve_stats()
    say("stats", st)
    assert st["completed"] == len(reqs) and st["batches"] >= 2
    assert 4 <= sum(o["batch"] > 1 for o in outs) <= st["batched"]
    with mbl.Context(0) as c2:
        for (L, h, s, e, p), o in zip(reqs, outs):
            assert o["status"] == mbl.MBL_OK
            a = c2.mbl_solve(L, h, s, e, 20, prec=p)
            for k in KEYS:
                assert np.array_equal(o[k], a[k]), (L, h, s, e, p, k, o["batch"])
            for k in ("n_restarts", "n_opapply", "n_passes", "ir_iters_max", "fallback"):
                assert o[k] == a[k], (k, o["batch"])

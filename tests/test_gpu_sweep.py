"""Energy sweep of one realization (mbl_sweep) and disorder averages
(mbl_disorder_average): the protocol of the paper's "Numerical method"
section.  Bins are compared with the oracle's (dense spectrum per
realization, every target), each target with a separate mbl_solve call
(identical arithmetic), and the averages over realizations with the oracle's
averages of its own bins."""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu

EPS = [0.1, 0.3, 0.5, 0.7, 0.9]
# bins compared with the oracle: r, S_1, S_2, S_E, S_E^2, F, f, KL, energy density
TOL = {"r": 1e-8, "s1": 1e-8, "s2": 1e-8, "se": 1e-8, "se2": 1e-7, "fluct": 1e-9,
       "dynfrac": 1e-9, "kl": 1e-6, "edens": 1e-10, "nconv": 0.0}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bins_of_solve(g, nev):
    """The binning rule applied to one mbl_solve result (test-side helper)."""
    def fmean(v):
        v = [float(x) for x in v if math.isfinite(float(x))]
        return sum(v) / len(v) if v else math.nan
    b = np.full(mbl.MBL_NBIN, math.nan)
    b[0] = fmean(g["r"][:nev - 2]) if nev >= 3 else math.nan
    b[1], b[2], b[3] = fmean(g["s1"]), fmean(g["s2"]), fmean(g["se"])
    b[4] = sum(float(x) * float(x) for x in g["se"]) / nev
    b[5], b[6] = fmean(g["fluct"]), fmean(g["dynfrac"])
    b[7] = fmean(g["kl"][:nev - 1]) if nev >= 2 else math.nan
    w = g["emax"] - g["emin"]
    b[8] = sum((float(E) - g["emin"]) / w for E in g["evals"]) / nev
    b[9] = g["nconv"]
    return b


@pytest.mark.parametrize("L,h,seed,nev", [(10, 1.0, 3, 16), (12, 0.7, 1, 20)])
def test_sweep_bins_match_oracle(L, h, seed, nev):
    say("sweep", L, h, seed, nev, EPS)
    with mbl.Context(0) as c:
        sw = c.mbl_sweep(L, h, seed, EPS, nev)
    assert sw["code"] == mbl.MBL_OK and (sw["status"] == mbl.MBL_OK).all()
    refs = oracle.solve_targets(L, h, seed, EPS, nev)
    for k, ref in enumerate(refs):
        rb = oracle.realization_bins(ref)
        for q, name in enumerate(mbl.BIN_NAMES):
            got, want = sw["bins"][k, q], rb[q]
            assert abs(got - want) <= TOL[name] * max(1.0, abs(want)), (EPS[k], name, got, want)


def test_sweep_equals_separate_solves():
    L, h, seed, nev = 12, 3.0, 7, 20
    with mbl.Context(0) as c:
        sw = c.mbl_sweep(L, h, seed, EPS, nev)
        for k, e in enumerate(EPS):
            g = c.mbl_solve(L, h, seed, e, nev, extra=True)
            assert np.array_equal(sw["bins"][k], _bins_of_solve(g, nev), equal_nan=True), e


def test_disorder_average_over_realizations():
    L, h, nev, seeds = 10, 2.5, 12, [0, 1, 2, 3]
    eps = [0.5]
    with mbl.Context(0) as c:
        B = np.array([c.mbl_sweep(L, h, s, eps, nev)["bins"][0] for s in seeds])
    R = np.array([oracle.realization_bins(oracle.solve_targets(L, h, s, eps, nev)[0])
                  for s in seeds])
    got, ref = mbl.mbl_disorder_average(B), oracle.disorder_average(R)
    for q, name in enumerate(mbl.BIN_NAMES):
        assert abs(got["mean"][q] - ref["mean"][q]) <= TOL[name] * max(1.0, abs(ref["mean"][q]))
    assert got["sigma_e"] == pytest.approx(ref["sigma_e"], rel=1e-6, abs=1e-8)
    assert got["sem"][3] == pytest.approx(ref["sem"][3], rel=1e-5, abs=1e-9)


def test_sweep_errors():
    with mbl.Context(0) as c:
        with pytest.raises(mbl.MblError):
            c.mbl_sweep(10, 1.0, 0, [], 10)
        with pytest.raises(mbl.MblError):
            c.mbl_sweep(10, 1.0, 0, [0.5, 1.5], 10)
        with pytest.raises(mbl.MblError):
            c.mbl_sweep(23, 1.0, 0, [0.5], 10)

"""GPU parity at the benchmarked sizes.

L = 14 and 16: the whole path (mbl_solve, FP64, nev = 50, five targets per
realization) against stored oracle results (tests/golden, written by
make_oracle_golden.py from the dense oracle).

L = 18 and 20, where the dense oracle does not fit: certificates the oracle
computes one eigenpair at a time, in the launch configuration the benchmark
times (mbl_solve, FP64, nev = 50): residuals ||H psi - E psi|| and Rayleigh
quotients of every pair with H applied by the oracle's own CPU code, S_1 of
every vector and S_E of all (L = 18) or eight (L = 20) vectors recomputed by
the oracle, orthonormality, and window completeness from a second solve at a
shifted target whose window overlaps the first; the FP32 LU + FP64 refinement
path at L = 20 under the same certificates and against the FP64 path.
"""
import glob
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl
from parity import assert_subspaces, kl_tolerance

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EIG_TOL = 1e-10
RES_TOL = 1e-9
OBS_TOL = 1e-8
GAP_MIN = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mbl.Context(0)
    yield c
    c.close()


GOLDEN = sorted(glob.glob(os.path.join(HERE, "golden", "oracle_L*_h*_s*.json")))


def _separated(E, hn):
    gaps = np.diff(E)
    sep = np.ones(E.size, dtype=bool)
    sep[:-1] &= gaps >= GAP_MIN * hn
    sep[1:] &= gaps >= GAP_MIN * hn
    return sep, gaps


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[7:-5] for p in GOLDEN])
def test_golden_parity(ctx, path):
    rec = json.load(open(path))
    L, h, seed, nev = rec["L"], rec["h"], rec["seed"], rec["nev"]
    f = np.array(rec["fields"])
    assert np.array_equal(f, oracle.fields(L, h, seed))       # stored fields = the generator's
    hn = max(abs(rec["emin"]), abs(rec["emax"]))
    for t in rec["targets"]:
        say("golden", os.path.basename(path), "eps", t["eps"])
        g = ctx.mbl_solve(L, h, seed, t["eps"], nev, extra=True, vectors=True)
        assert abs(g["emin"] - rec["emin"]) <= 1e-12 * hn
        assert abs(g["emax"] - rec["emax"]) <= 1e-12 * hn
        assert abs(g["sigma"] - t["sigma"]) <= 1e-12 * hn
        E = np.array(t["evals"])
        assert np.abs(g["evals"] - E).max() <= EIG_TOL * hn, (t["eps"], np.abs(g["evals"] - E).max() / hn)
        assert g["max_resid"] <= RES_TOL
        sep, gaps = _separated(E, hn)
        # a level of a cluster cut by the window edge has its partner outside
        # the window: not separated either (stored clusters, L = 14)
        for cl in t.get("clusters", []):
            sep &= ~((E >= cl["evals"][0] - EIG_TOL * hn) & (E <= cl["evals"][-1] + EIG_TOL * hn))
        for key in ("s1", "se", "s2", "fluct", "dynfrac"):
            d = np.abs(g[key] - np.array(t[key]))[sep]
            assert d.max(initial=0.0) <= OBS_TOL, (t["eps"], key, d.max())
        rmask = np.minimum(gaps[:-1], gaps[1:]) >= GAP_MIN * hn
        d = np.abs(g["r"] - np.array(t["r"]))[rmask]
        assert d.max(initial=0.0) <= OBS_TOL, (t["eps"], "r", d.max())
        # residuals of the GPU vectors with H applied by the oracle's own code
        Z = g["evecs"]
        Eg = g["evals"]
        b = oracle.basis(L)
        ores = np.array([oracle.residual(L, 1.0, f, Z[:, k], Eg[k], b) for k in range(nev)])
        assert ores.max() <= RES_TOL * hn, ores.max() / hn
        # levels closer than GAP_MIN ||H||: eigenvectors compared as subspaces
        # against the oracle's vectors of the whole cluster (stored at L = 14)
        if "clusters" in t:
            for cl in t["clusters"]:
                Ec = np.array(cl["evals"])
                Zo = np.array(cl["vecs"]).T
                inside = np.flatnonzero((Eg >= Ec[0] - EIG_TOL * hn) & (Eg <= Ec[-1] + EIG_TOL * hn))
                assert inside.size >= 1
                assert_subspaces(Eg[inside], Z[:, inside], Ec, Zo, hn)
        # KL(p_n | p_n+1), gated on separated pairs with a tolerance from the
        # oracle's residuals of the GPU vectors (tests/parity.py: kl_tolerance)
        kmask = sep[:-1] & sep[1:]
        ktol = kl_tolerance(Z, Eg, ores, hn)
        d = np.abs(g["kl"] - np.array(t["kl"]))
        assert np.all(d[kmask] <= ktol[kmask]), (t["eps"], "kl", (d - ktol)[kmask].max())


# (L, h, seed, eps, vectors whose S_E the oracle recomputes: all at L = 18,
# eight spread over the window at L = 20, where each takes the oracle seconds)
SPREAD = (0, 7, 14, 21, 28, 35, 42, 49)
LARGE = [(18, 3.0, 0, 0.5, tuple(range(50))), (20, 2.0, 0, 0.2, SPREAD), (20, 3.0, 1, 0.8, SPREAD)]


def certify(ctx, g, L, h, seed, eps, nev, se_idx):
    """Certificates of one L >= 18 window, every one computed by the oracle's
    own code from the GPU's eigenvectors."""
    Z, E = g["evecs"], g["evals"]
    n = math.comb(L, L // 2)
    assert Z.shape == (n, nev)
    hn = g["hnorm"]
    f = oracle.fields(L, h, seed)
    b = oracle.basis(L)
    assert abs(g["sigma"] - (g["emin"] + eps * (g["emax"] - g["emin"]))) <= 1e-13 * hn
    # orthonormality of the returned basis
    G = Z.T @ Z
    assert np.abs(G - np.eye(nev)).max() <= 1e-12
    assert np.all(np.diff(E) >= 0)
    # residuals and Rayleigh quotients of every pair with H applied by the oracle
    for k in range(nev):
        res = oracle.residual(L, 1.0, f, Z[:, k], E[k], b)
        assert res <= RES_TOL * hn, (k, res / hn)
        assert abs(oracle.rayleigh(L, 1.0, f, Z[:, k], b) - E[k]) <= EIG_TOL * hn, k
    # observables of the returned vectors recomputed by the oracle
    sep, gaps = _separated(E, hn)
    for k in range(nev):
        assert abs(oracle.participation_entropy(Z[:, k]) - g["s1"][k]) <= OBS_TOL, k
    for k in se_idx:
        assert abs(oracle.entanglement_entropy(L, Z[:, k], b) - g["se"][k]) <= OBS_TOL, k
    ro, _ = oracle.gap_ratios(E)
    rmask = np.minimum(gaps[:-1], gaps[1:]) >= GAP_MIN * hn
    assert np.abs(ro - g["r"])[rmask].max(initial=0.0) <= 1e-12
    return sep


@pytest.mark.parametrize("L,h,seed,eps,se_idx", LARGE, ids=[f"L{c[0]}-h{c[1]}-s{c[2]}-e{c[3]}" for c in LARGE])
def test_large_certificates(ctx, L, h, seed, eps, se_idx):
    nev = 50
    say("certificates", L, h, seed, eps)
    g = ctx.mbl_solve(L, h, seed, eps, nev, vectors=True)
    certify(ctx, g, L, h, seed, eps, nev, se_idx)
    E, hn = g["evals"], g["hnorm"]
    # window completeness: a second, independent solve centred half a window
    # above; inside the overlap of the two windows both must list the same levels
    half = 0.5 * (E[-1] - g["sigma"])
    g2 = ctx.mbl_solve(L, h, seed, eps, nev, sigma=g["sigma"] + half)
    E2 = g2["evals"]
    lo, hi = max(E[0], E2[0]), min(E[-1], E2[-1])
    pad = 1e-9 * hn
    a = E[(E > lo + pad) & (E < hi - pad)]
    c = E2[(E2 > lo + pad) & (E2 < hi - pad)]
    assert a.size >= nev // 4 and a.size == c.size, (a.size, c.size)
    assert np.abs(a - c).max() <= EIG_TOL * hn


def test_fp32_refined_matches_fp64_L18(ctx):
    L, h, nev = 18, 3.0, 50
    say("fp32 vs fp64 L18")
    g64 = ctx.mbl_solve(L, h, 3, 0.5, nev)
    g32 = ctx.mbl_solve(L, h, 3, 0.5, nev, prec=mbl.MBL_FP32_IR64)
    hn = g64["hnorm"]
    assert g32["max_resid"] <= RES_TOL
    assert np.abs(g32["evals"] - g64["evals"]).max() <= EIG_TOL * hn
    sep, _ = _separated(g64["evals"], hn)
    for key in ("s1", "se"):
        assert np.abs(g32[key] - g64[key])[sep].max() <= OBS_TOL, key


def test_fp32_refined_certificates_L20(ctx):
    """The L = 20 benchmark configuration at its own precision (FP32 LU on the
    matrix cores, every shifted solve refined in FP64): the FP64 certificates
    computed by the oracle, and per-eigenpair agreement with the FP64 path."""
    L, h, seed, eps, nev = 20, 3.0, 0, 0.5, 50
    say("fp32+ir certificates L20")
    g32 = ctx.mbl_solve(L, h, seed, eps, nev, prec=mbl.MBL_FP32_IR64, vectors=True)
    assert g32["max_resid"] <= RES_TOL
    sep = certify(ctx, g32, L, h, seed, eps, nev, (0, 25, 49))
    g64 = ctx.mbl_solve(L, h, seed, eps, nev, vectors=True)
    hn = g64["hnorm"]
    dE = np.abs(g32["evals"] - g64["evals"])
    say(f"  fp32+ir vs fp64: max |dE| / ||H|| = {dE.max() / hn:.2e}, fallback={g32['fallback']}")
    assert dE.max() <= EIG_TOL * hn
    assert_subspaces(g32["evals"], g32["evecs"], g64["evals"], g64["evecs"], hn)
    for key in ("s1", "se"):
        assert np.abs(g32[key] - g64[key])[sep].max() <= OBS_TOL, key

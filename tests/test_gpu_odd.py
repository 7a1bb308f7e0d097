"""Odd chains (the paper's L = 15, 17, 19 sizes) in the S^z = +1/2 sector:
every step of the path against the oracle through the C ABI, as for even L.
The half chain A is sites 1..(L-1)/2, so the entanglement blocks are
rectangular (B has one site more)."""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu

KEYS_TOL = {"s1": 1e-8, "s2": 1e-8, "se": 1e-8, "fluct": 1e-9, "dynfrac": 1e-9}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mbl.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("L", [3, 5, 7, 9, 11, 13, 15, 17, 19, 21])
def test_odd_basis_bit_exact(ctx, L):
    say("odd basis L", L)
    b = ctx.mbl_basis(L)
    assert b.size == mbl.mbl_sector_dim(L) == math.comb(L, (L + 1) // 2)
    assert np.array_equal(b, oracle.basis(L))


@pytest.mark.parametrize("L", [3, 9, 15, 21])
def test_odd_rank_bit_exact(ctx, L):
    say("odd rank L", L)
    b = oracle.basis(L)
    assert np.array_equal(ctx.mbl_rank(L, b), np.arange(b.size))
    # the S^z = -1/2 words and words with bits above L are outside the sector
    bad = np.array([(1 << (L // 2)) - 1, (1 << L) - 1, (1 << ((L + 1) // 2)) - 1 + (1 << L)],
                   dtype=np.uint64).astype(np.uint32)
    assert np.all(ctx.mbl_rank(L, bad) == -1)


@pytest.mark.parametrize("L,J", [(3, 1.0), (5, 1.0), (9, 0.7), (11, 1.0), (11, 0.0)])
def test_odd_hamiltonian_matches_dense_oracle(ctx, L, J):
    say("odd hamiltonian L", L, "J", J)
    f = oracle.fields(L, 3.0, 17)
    rp, col, val = ctx.mbl_hamiltonian(L, J, f)
    n = rp.size - 1
    H = np.zeros((n, n))
    for k in range(n):
        H[k, col[rp[k]:rp[k + 1]]] = val[rp[k]:rp[k + 1]]
    Ho = oracle.dense_H(L, J, f)
    assert np.array_equal(np.diag(H), np.diag(Ho))
    assert np.abs(H - Ho).max() <= 1e-15
    if J != 0.0:
        nup = (L + 1) // 2
        assert col.size == n + 2 * L * math.comb(L - 2, nup - 1)


@pytest.mark.parametrize("L,h,seed,eps,nev", [(5, 1.0, 0, 0.5, 4), (7, 2.0, 1, 0.3, 10),
                                              (9, 3.0, 2, 0.5, 20), (11, 0.8, 3, 0.7, 20),
                                              (13, 4.0, 4, 0.5, 30)])
def test_odd_solve_matches_oracle(ctx, L, h, seed, eps, nev):
    say("odd solve", L, h, seed, eps, nev)
    g = ctx.mbl_solve(L, h, seed, eps, nev, extra=True)
    o = oracle.solve(L, h, seed, eps, nev)
    hn = o["hnorm"]
    assert g["nconv"] == nev and g["max_resid"] <= 1e-9
    assert abs(g["emin"] - o["emin"]) <= 1e-10 * hn and abs(g["emax"] - o["emax"]) <= 1e-10 * hn
    assert np.abs(g["evals"] - o["evals"]).max() <= 1e-10 * hn
    gaps = np.diff(o["evals"])
    sep = np.minimum(np.r_[np.inf, gaps], np.r_[gaps, np.inf]) >= 1e-6 * hn
    for k, tol in KEYS_TOL.items():
        d = np.abs(g[k] - o[k])[sep]
        assert d.max() <= tol, (k, d.max())
    assert np.abs(g["r"] - o["r"]).max() <= 1e-8


def test_odd_solve_through_a_front_without_pivots(ctx):
    """L = 17 (S^z = 1/2, dim 24310): one front of its tree has no pivots (its
    subgraph was split with an empty separator), so the factorization, the
    solves and the extend-add pass its children's updates straight through it.
    Certified by the oracle's residuals and Rayleigh quotients of every pair."""
    L, h, seed, eps, nev = 17, 3.0, 0, 0.5, 20
    say("odd solve through a front without pivots, L", L)
    ft = ctx.mbl_front_tree(L)
    assert (ft["npiv"] == 0).any()
    g = ctx.mbl_solve(L, h, seed, eps, nev, vectors=True)
    Z, E, hn = g["evecs"], g["evals"], g["hnorm"]
    assert g["nconv"] == nev and g["max_resid"] <= 1e-9
    f = oracle.fields(L, h, seed)
    b = oracle.basis(L)
    for k in range(nev):
        assert oracle.residual(L, 1.0, f, Z[:, k], E[k], b) <= 1e-9 * hn, k
        assert abs(oracle.rayleigh(L, 1.0, f, Z[:, k], b) - E[k]) <= 1e-10 * hn, k
    assert np.abs(Z.T @ Z - np.eye(nev)).max() <= 1e-12


def test_odd_tiny_sector_full_space(ctx):
    # L = 3: dim 3, every eigenpair; r of the three levels
    g = ctx.mbl_solve(3, 1.5, 5, 0.5, 3, extra=True)
    o = oracle.solve(3, 1.5, 5, 0.5, 3)
    assert np.abs(g["evals"] - o["evals"]).max() <= 1e-12 * o["hnorm"]
    assert np.abs(g["se"] - o["se"]).max() <= 1e-10


def test_odd_sweep_bins(ctx):
    eps = [0.2, 0.5, 0.8]
    sw = ctx.mbl_sweep(11, 1.0, 6, eps, 16)
    assert sw["code"] == mbl.MBL_OK
    for k, ref in enumerate(oracle.solve_targets(11, 1.0, 6, eps, 16)):
        rb = oracle.realization_bins(ref)
        for q in (0, 1, 2, 3, 4, 5, 6, 8):
            assert abs(sw["bins"][k, q] - rb[q]) <= 1e-7 * max(1.0, abs(rb[q]))

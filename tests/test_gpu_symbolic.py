"""The symbolic analysis behind the LU (ordering, assembly tree of dense
fronts, predicted fill and flops) checked against an exact symbolic
factorization of the permuted pattern of H computed here, on the host, from the
CSR pattern the device assembled."""
import sys

import numpy as np
import pytest

import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mbl.Context(0)
    yield c
    c.close()


def exact_lower_structure(n, rowptr, col, perm):
    """Row indices below the diagonal of every column of the Cholesky factor of
    P A P^T (A symmetric pattern, P from perm[k] = old index eliminated k-th):
    struct(L_j) = {i > j : A'_ij != 0} united with struct(L_c) - {j} over the
    columns c whose first subdiagonal entry is j (the elimination tree)."""
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    kids = [[] for _ in range(n)]
    struct = [None] * n
    for j in range(n):
        old = perm[j]
        s = set(int(iperm[c]) for c in col[rowptr[old]:rowptr[old + 1]])
        s = {i for i in s if i > j}
        for c in kids[j]:
            s |= struct[c]
        s.discard(j)
        struct[j] = s
        if s:
            kids[min(s)].append(j)
    return struct


@pytest.mark.parametrize("L", [6, 8, 10, 12, 9, 11])
def test_front_tree_contains_the_exact_fill(ctx, L):
    say("symbolic", L)
    info = ctx.mbl_symbolic(L)
    n = mbl.mbl_sector_dim(L)
    perm = ctx.mbl_ordering(L)
    # the ordering is a permutation of the basis indices
    assert perm.shape == (n,) and np.array_equal(np.sort(perm), np.arange(n))
    rp, col, _ = ctx.mbl_hamiltonian(L, 1.0, np.zeros(L))
    ft = ctx.mbl_front_tree(L)
    first, npiv, nc, parent, cptr = ft["first"], ft["npiv"], ft["ncontrib"], ft["parent"], ft["cptr"]
    nf = first.size
    assert info["n_fronts"] == nf
    # the pivot blocks tile 0..n-1 in post-order, parents after their children
    order = np.argsort(first, kind="stable")
    assert np.array_equal(order, np.arange(nf))
    assert first[0] == 0 and np.array_equal(first[1:], (first + npiv)[:-1])
    assert first[-1] + npiv[-1] == n and np.all(npiv >= 1)
    for f in range(nf):
        rows = ft["contrib"][cptr[f]:cptr[f] + nc[f]]
        assert np.all(np.diff(rows) > 0)
        if nc[f]:
            assert rows[0] >= first[f] + npiv[f]
        if parent[f] < 0:
            assert nc[f] == 0
            continue
        P = parent[f]
        assert P > f
        # the parent front holds every contribution row (as pivot or contribution)
        prow = set(range(first[P], first[P] + npiv[P])) | set(
            ft["contrib"][cptr[P]:cptr[P] + nc[P]].tolist())
        assert set(rows.tolist()) <= prow
    # every entry of the exact factor lies in its front
    struct = exact_lower_structure(n, rp, col, perm)
    owner = np.repeat(np.arange(nf), npiv)
    exact_nnz = n
    for j in range(n):
        f = owner[j]
        allowed = set(range(j + 1, first[f] + npiv[f])) | set(
            ft["contrib"][cptr[f]:cptr[f] + nc[f]].tolist())
        assert struct[j] <= allowed, (j, sorted(struct[j] - allowed)[:5])
        exact_nnz += 2 * len(struct[j])
    # predicted fill and flops are the counts of these fronts
    p = npiv.astype(np.float64)
    c = nc.astype(np.float64)
    assert info["nnz_factor"] == int(np.sum(npiv.astype(np.int64) ** 2 + 2 * npiv.astype(np.int64) * nc))
    assert info["front_entries"] == int(np.sum((npiv.astype(np.int64) + nc) ** 2))
    flops = np.sum(2.0 / 3.0 * p ** 3 + 2 * p ** 2 * c + 2 * p * c ** 2)
    assert abs(info["flops_factor"] - flops) <= 1e-12 * flops
    assert info["max_front"] == int((npiv + nc).max()) and info["max_pivots"] == int(npiv.max())
    # fronts are dense: the prediction bounds the exact fill from above
    assert info["nnz_factor"] >= exact_nnz
    say(f"  L={L} fronts={nf} predicted nnz(L+U)={info['nnz_factor']} exact={exact_nnz}")

"""The Rayleigh-Ritz eigensolver of the Krylov iteration (mbl_ritz_eig): the
device Jacobi kernels against the oracle's Householder + QL eigenvalues, the
eigenpair residual and orthogonality of the returned vectors, and the two
kernels (orders up to 128 in LDS, the general one) against each other bit
for bit.  Matrices: dense random, degenerate (repeated eigenvalues in a random
basis), and the shape of a restarted Krylov-Schur projection (diagonal of kept
Ritz values, a coupling row block, then block-tridiagonal expansion blocks)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = mbl.Context(0)
    yield c
    c.close()


def random_sym(m, rng):
    A = rng.standard_normal((m, m))
    return (A + A.T) / 2


def degenerate(m, rng):
    """Eigenvalues with multiplicities up to 4, in a random orthonormal basis."""
    vals = np.repeat(rng.standard_normal((m + 3) // 4), 4)[:m]
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    B = (Q * vals) @ Q.T
    return (B + B.T) / 2


def krylov_shaped(m, rng, b=4):
    """Restarted block Krylov-Schur projection: kept Ritz values on the
    diagonal, their coupling to the residual block, then expansion blocks
    (symmetric diagonal blocks, upper-triangular subdiagonal R blocks)."""
    nkeep = (m // 2) // b * b
    A = np.zeros((m, m))
    A[np.arange(nkeep), np.arange(nkeep)] = np.sort(rng.standard_normal(nkeep))[::-1] * 10
    c0 = nkeep
    while c0 < m:
        w = min(b, m - c0)
        D = rng.standard_normal((w, w))
        A[c0:c0 + w, c0:c0 + w] = (D + D.T) / 2
        if c0 == nkeep:
            A[c0:c0 + w, :nkeep] = rng.standard_normal((w, nkeep)) * 1e-3
        elif c0 >= b:
            A[c0:c0 + w, c0 - b:c0] = np.triu(rng.standard_normal((w, b)))[:w]
        c0 += w
    return np.tril(A) + np.tril(A, -1).T


KINDS = {"random": random_sym, "degenerate": degenerate, "krylov": krylov_shaped}


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("m", [1, 2, 3, 17, 56, 64, 89, 90, 91, 128, 150])
def test_eigenpairs(ctx, kind, m):
    rng = np.random.default_rng(1000 * m + len(kind))
    A = KINDS[kind](m, rng)
    say("ritz_eig", kind, m)
    w, Z = ctx.mbl_ritz_eig(A)
    nrm = max(np.abs(np.linalg.eigvalsh(A)).max(), 1e-300)
    tol = 1e-13 * nrm
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - oracle.eigh_full(A)[0]).max() <= tol
    assert np.abs(A @ Z - Z * w).max() <= tol
    assert np.abs(Z.T @ Z - np.eye(m)).max() <= 1e-13


@pytest.mark.parametrize("m", [2, 5, 33, 60, 64, 68, 90, 91, 101, 127, 128])
def test_lds_kernel_equals_general_kernel(ctx, m):
    """Orders up to 128 run in the LDS kernel (rotations in LDS up to 90, in
    global memory above); the general kernel applies the same rotations with
    the same arithmetic, so the bits agree."""
    rng = np.random.default_rng(m)
    As = np.stack([KINDS[k](m, rng) for k in sorted(KINDS)])
    w1, Z1 = ctx.mbl_ritz_eig(As)
    w2, Z2 = ctx.mbl_ritz_eig(As, general=True)
    assert np.array_equal(w1, w2) and np.array_equal(Z1, Z2)


def test_batch_equals_single_calls(ctx):
    """One workgroup per matrix: a batch of 16 gives each matrix's own result."""
    rng = np.random.default_rng(7)
    m = 60
    As = np.stack([KINDS[sorted(KINDS)[k % 3]](m, rng) for k in range(16)])
    w, Z = ctx.mbl_ritz_eig(As)
    for k in (0, 5, 15):
        wk, Zk = ctx.mbl_ritz_eig(As[k])
        assert np.array_equal(w[k], wk) and np.array_equal(Z[k], Zk)


def test_diagonal_and_zero_matrices(ctx):
    """No rotation moves: eigenvalues are the sorted diagonal, vectors the
    permuted identity (zero sweeps of rotations)."""
    d = np.array([3.0, -1.0, 2.0, -1.0, 0.0])
    w, Z = ctx.mbl_ritz_eig(np.diag(d))
    assert np.array_equal(w, np.sort(d))
    assert np.array_equal(np.abs(Z).sum(axis=0), np.ones(5))
    assert np.array_equal(Z.T @ np.diag(d) @ Z, np.diag(w))
    w0, Z0 = ctx.mbl_ritz_eig(np.zeros((4, 4)))
    assert np.array_equal(w0, np.zeros(4)) and np.array_equal(Z0, np.eye(4))


def test_rejections(ctx):
    lib = mbl.lib()
    A = np.eye(3)
    w = np.zeros(3)
    Z = np.zeros(9)
    p = mbl._pd_of
    assert lib.mbl_ritz_eig(ctx._h, 1, 0, p(A), p(w), p(Z), 0) == mbl.MBL_EINVAL
    assert lib.mbl_ritz_eig(ctx._h, 1, 1025, p(A), p(w), p(Z), 0) == mbl.MBL_EINVAL
    assert lib.mbl_ritz_eig(ctx._h, 1, 3, p(A), p(w), p(Z), 2) == mbl.MBL_EINVAL
    assert lib.mbl_ritz_eig(ctx._h, -1, 3, p(A), p(w), p(Z), 0) == mbl.MBL_EINVAL
    assert lib.mbl_ritz_eig(ctx._h, 0, 3, None, None, None, 0) == mbl.MBL_OK

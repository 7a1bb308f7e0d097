"""mbl_observables_noalloc, the allocation-free variant of mbl_observables, on
device buffers owned by the caller (torch tensors here), against the existing
entry point on the same vectors: two calls in a row, the second smaller, a
size whose entanglement work is done in chunks of vectors, a leading
dimension above the sector dimension, and the documented rejections."""
import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vectors(L, nev, seed):
    b = oracle.basis(L)
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((b.size, nev))
    Z[:, 0] = 1.0                                   # uniform sector state
    if nev > 1:
        Z[:, 1] = 0.0
        Z[2, 1] = 1.0                               # a basis state
    if nev > 2:
        Z[:, 2] *= np.exp(-np.arange(b.size) / 40.0)
    Z /= np.linalg.norm(Z, axis=0)
    E = np.sort(rng.standard_normal(nev))
    return Z, E


def _noalloc(L, Z, E, ld=None):
    dim, nev = Z.shape
    ld = dim if ld is None else ld
    Zp = np.zeros((nev, max(ld, dim)))
    Zp[:, :dim] = Z.T                               # column j at j * ld
    dev = torch.device("cuda:0")
    Zd = torch.from_numpy(Zp).to(dev)
    Ed = torch.from_numpy(E.copy()).to(dev)
    rd = torch.full((max(nev - 2, 1),), np.nan, dtype=torch.float64, device=dev)
    s1d = torch.full((nev,), np.nan, dtype=torch.float64, device=dev)
    sed = torch.full((nev,), np.nan, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = mbl.mbl_observables_noalloc(L, nev, Ed.data_ptr(), Zd.data_ptr(), ld, rd.data_ptr(),
                                     s1d.data_ptr(), sed.data_ptr(), stream)
    torch.cuda.synchronize(dev)
    return rc, rd.cpu().numpy()[:max(nev - 2, 0)], s1d.cpu().numpy(), sed.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    c = mbl.Context(0)
    yield c
    c.close()


def _check(ctx, L, nev, seed, ld=None):
    Z, E = _vectors(L, nev, seed)
    rc, r, s1, se = _noalloc(L, Z, E, ld)
    assert rc == mbl.MBL_OK
    r0, s10, se0 = ctx.mbl_observables(L, E, Z)
    # same kernels, same per-vector arithmetic: bitwise the existing entry point
    assert np.array_equal(r, r0)
    assert np.array_equal(s1, s10)
    assert np.array_equal(se, se0)
    return Z, se


def test_two_calls_second_smaller(ctx):
    _check(ctx, 16, 24, 1)
    Z, se = _check(ctx, 10, 5, 2)
    b = oracle.basis(10)
    for k in range(5):
        assert abs(oracle.entanglement_entropy(10, Z[:, k], b) - se[k]) <= 1e-8


def test_chunked_entanglement_and_padded_leading_dimension(ctx):
    # L = 20: the work array holds the entanglement work of a few vectors at a
    # time, so twelve vectors take several chunks
    _check(ctx, 20, 12, 3)
    _check(ctx, 12, 9, 4, ld=mbl.mbl_sector_dim(12) + 7)


def test_rejections():
    Z, E = _vectors(8, 4, 5)
    rc, *_ = _noalloc(8, Z, E, ld=Z.shape[0] - 1)
    assert rc == mbl.MBL_EINVAL
    Z, E = _vectors(8, 300, 6)
    rc, *_ = _noalloc(8, Z, E)
    assert rc == mbl.MBL_EINVAL
    # and the array is still usable afterwards
    Z, E = _vectors(8, 4, 7)
    rc, r, s1, se = _noalloc(8, Z, E)
    assert rc == mbl.MBL_OK and np.all(np.isfinite(se))

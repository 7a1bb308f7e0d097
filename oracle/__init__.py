"""CPU FP64 oracle for the shift-invert eigenproblem of the random-field
Heisenberg chain (Eq. (1) of Luitz, Laflorencie, Alet 2014).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it.  The arithmetic lives in ``oracle.c`` (plain C, no LAPACK); this
module only builds it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_l = ctypes.c_long
_i = ctypes.c_int
_u64 = ctypes.c_uint64
_pd = ctypes.POINTER(ctypes.c_double)
_pu32 = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, strict IEEE FP64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_splitmix64_next.restype = _u64
        L.orc_splitmix64_next.argtypes = [ctypes.POINTER(_u64)]
        L.orc_fields.argtypes = [_i, _d, _u64, _pd]
        L.orc_sector_basis.restype = _l
        L.orc_sector_basis.argtypes = [_i, _i, _pu32]
        L.orc_rank.restype = _l
        L.orc_rank.argtypes = [_pu32, _l, ctypes.c_uint32]
        L.orc_dense_H.argtypes = [_i, _d, _pd, _pu32, _l, _pd]
        L.orc_apply_H.argtypes = [_i, _d, _pd, _pu32, _l, _pd, _pd]
        L.orc_tridiagonalize.restype = _l
        L.orc_tridiagonalize.argtypes = [_l, _pd, _pd, _pd, _pd, _l]
        L.orc_tridiag_ql.restype = _i
        L.orc_tridiag_ql.argtypes = [_l, _pd, _pd, _pd, _l]
        L.orc_tridiag_invit.argtypes = [_l, _pd, _pd, _l, _pd, _pd]
        L.orc_backtransform.argtypes = [_l, _pd, _pd, _l, _pd]
        L.orc_eigvalsh.restype = _i
        L.orc_eigvalsh.argtypes = [_l, _pd, _pd]
        L.orc_eigh_full.restype = _i
        L.orc_eigh_full.argtypes = [_l, _pd, _pd, _pd]
        L.orc_nearest_eigenpairs.restype = _i
        L.orc_nearest_eigenpairs.argtypes = [_l, _pd, _d, _d, _l, _pd, _pd, _pd, _pd]
        L.orc_nearest_eigenpairs_multi.restype = _i
        L.orc_nearest_eigenpairs_multi.argtypes = [_l, _pd, _l, _pd, _pd, _l, _pd, _pd, _pd, _pd]
        L.orc_gap_ratios.restype = _d
        L.orc_gap_ratios.argtypes = [_l, _pd, _pd]
        L.orc_participation_entropy.restype = _d
        L.orc_participation_entropy.argtypes = [_l, _pd, _d]
        L.orc_entanglement_entropy.restype = _d
        L.orc_entanglement_entropy.argtypes = [_i, _pu32, _l, _pd]
        L.orc_bipartite_fluct.restype = _d
        L.orc_bipartite_fluct.argtypes = [_i, _pu32, _l, _pd]
        L.orc_kl_divergence.restype = _d
        L.orc_kl_divergence.argtypes = [_l, _pd, _pd]
        L.orc_dynamical_fraction.restype = _d
        L.orc_dynamical_fraction.argtypes = [_i, _pu32, _l, _pd]
        L.orc_residual.restype = _d
        L.orc_residual.argtypes = [_i, _d, _pd, _pu32, _l, _pd, _d]
        L.orc_rayleigh.restype = _d
        L.orc_rayleigh.argtypes = [_i, _d, _pd, _pu32, _l, _pd]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_pd)


def _pu(a):
    return a.ctypes.data_as(_pu32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- primitives
def splitmix64(seed: int, count: int) -> list[int]:
    st = _u64(seed)
    return [int(lib().orc_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def fields(L: int, h: float, seed: int) -> np.ndarray:
    out = np.zeros(L)
    lib().orc_fields(L, h, seed, _p(out))
    return out


def sector_nup(L: int) -> int:
    """Up spins of the sector: L/2 (S^z = 0) for even L, (L+1)/2 (S^z = +1/2,
    the smallest |S^z| of an odd chain) for odd L."""
    return (L + 1) // 2


def sector_dim(L: int, nup: int | None = None) -> int:
    return math.comb(L, sector_nup(L) if nup is None else nup)


def basis(L: int, nup: int | None = None) -> np.ndarray:
    nup = sector_nup(L) if nup is None else nup
    out = np.zeros(sector_dim(L, nup), dtype=np.uint32)
    n = lib().orc_sector_basis(L, nup, _pu(out))
    assert n == out.size
    return out


def rank(b: np.ndarray, s: int) -> int:
    return int(lib().orc_rank(_pu(b), b.size, s))


def dense_H(L: int, J: float, f: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    b = basis(L) if b is None else b
    n = b.size
    H = np.zeros((n, n))  # filled column-major == H^T row-major; H symmetric
    lib().orc_dense_H(L, J, _p(_f64(f)), _pu(b), n, _p(H))
    return H.T.copy()


def apply_H(L: int, J: float, f: np.ndarray, x: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    b = basis(L) if b is None else b
    x = _f64(x)
    y = np.zeros_like(x)
    lib().orc_apply_H(L, J, _p(_f64(f)), _pu(b), b.size, _p(x), _p(y))
    return y


def eigvalsh(A: np.ndarray) -> np.ndarray:
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    w = np.zeros(n)
    rc = lib().orc_eigvalsh(n, A.ctypes.data_as(_pd), _p(w))
    assert rc == 0
    return w


def eigh_full(A: np.ndarray):
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    w = np.zeros(n)
    Z = np.zeros((n, n), order="F")
    rc = lib().orc_eigh_full(n, A.ctypes.data_as(_pd), _p(w), Z.ctypes.data_as(_pd))
    assert rc == 0
    return w, Z


def tridiag_eigvals(d: np.ndarray, e: np.ndarray) -> np.ndarray:
    d = _f64(d).copy()
    e = np.concatenate([_f64(e), [0.0]])
    rc = lib().orc_tridiag_ql(d.size, _p(d), _p(e), None, 0)
    assert rc == 0
    return np.sort(d)


def nearest_eigenpairs(H: np.ndarray, eps: float, nev: int, sigma: float = math.nan,
                       vectors: bool = True, full_spectrum: bool = False):
    """The nev eigenpairs of dense symmetric H closest to the target; see oracle.c."""
    n = H.shape[0]
    A = np.array(H, dtype=np.float64, order="F", copy=True)
    ev = np.zeros(nev)
    Z = np.zeros((n, nev), order="F") if vectors else None
    allw = np.zeros(n) if full_spectrum else None
    o3 = np.zeros(3)
    rc = lib().orc_nearest_eigenpairs(
        n, A.ctypes.data_as(_pd), eps, sigma, nev, _p(ev),
        Z.ctypes.data_as(_pd) if vectors else None,
        _p(allw) if full_spectrum else None, _p(o3))
    assert rc == 0
    out = dict(evals=ev, emin=o3[0], emax=o3[1], sigma=o3[2])
    if vectors:
        out["evecs"] = np.ascontiguousarray(Z)
    if full_spectrum:
        out["spectrum"] = allw
    return out


def gap_ratios(E: np.ndarray):
    E = _f64(E)
    r = np.zeros(max(E.size - 2, 0))
    mean = lib().orc_gap_ratios(E.size, _p(E), _p(r) if r.size else None)
    return r, mean


def participation_entropy(psi: np.ndarray, q: float = 1.0) -> float:
    psi = _f64(psi)
    return float(lib().orc_participation_entropy(psi.size, _p(psi), q))


def entanglement_entropy(L: int, psi: np.ndarray, b: np.ndarray | None = None) -> float:
    b = basis(L) if b is None else b
    psi = _f64(psi)
    return float(lib().orc_entanglement_entropy(L, _pu(b), b.size, _p(psi)))


def bipartite_fluct(L: int, psi: np.ndarray, b: np.ndarray | None = None) -> float:
    b = basis(L) if b is None else b
    psi = _f64(psi)
    return float(lib().orc_bipartite_fluct(L, _pu(b), b.size, _p(psi)))


def kl_divergence(psi: np.ndarray, phi: np.ndarray) -> float:
    psi, phi = _f64(psi), _f64(phi)
    return float(lib().orc_kl_divergence(psi.size, _p(psi), _p(phi)))


def dynamical_fraction(L: int, psi: np.ndarray, b: np.ndarray | None = None) -> float:
    b = basis(L) if b is None else b
    psi = _f64(psi)
    return float(lib().orc_dynamical_fraction(L, _pu(b), b.size, _p(psi)))


def residual(L: int, J: float, f: np.ndarray, psi: np.ndarray, E: float,
             b: np.ndarray | None = None) -> float:
    b = basis(L) if b is None else b
    psi = _f64(psi)
    return float(lib().orc_residual(L, J, _p(_f64(f)), _pu(b), b.size, _p(psi), E))


def rayleigh(L: int, J: float, f: np.ndarray, psi: np.ndarray, b: np.ndarray | None = None) -> float:
    b = basis(L) if b is None else b
    psi = _f64(psi)
    return float(lib().orc_rayleigh(L, J, _p(_f64(f)), _pu(b), b.size, _p(psi)))


# ---------------------------------------------------------- whole problem
def solve(L: int, h: float, seed: int, eps: float, nev: int, J: float = 1.0,
          fields_in: np.ndarray | None = None, sigma: float = math.nan,
          vectors: bool = True, observables: bool = True, full_spectrum: bool = False):
    """One realization and target: fields -> dense H -> nearest eigenpairs ->
    observables (r, S_1, S_E and, for completeness, S_2, F, f, KL)."""
    f = fields(L, h, seed) if fields_in is None else _f64(fields_in)
    b = basis(L)
    H = dense_H(L, J, f, b)
    nev = min(nev, b.size)
    out = nearest_eigenpairs(H, eps, nev, sigma, vectors=vectors or observables,
                             full_spectrum=full_spectrum)
    out["fields"] = f
    out["hnorm"] = max(abs(out["emin"]), abs(out["emax"]))
    r, rmean = gap_ratios(out["evals"])
    out["r"], out["r_mean"] = r, rmean
    if observables:
        Z = out["evecs"]
        out["s1"] = np.array([participation_entropy(Z[:, j], 1.0) for j in range(nev)])
        out["s2"] = np.array([participation_entropy(Z[:, j], 2.0) for j in range(nev)])
        out["se"] = np.array([entanglement_entropy(L, Z[:, j], b) for j in range(nev)])
        out["fluct"] = np.array([bipartite_fluct(L, Z[:, j], b) for j in range(nev)])
        out["dynfrac"] = np.array([dynamical_fraction(L, Z[:, j], b) for j in range(nev)])
        out["kl"] = np.array([kl_divergence(Z[:, j], Z[:, j + 1]) for j in range(nev - 1)])
    if not vectors:
        out.pop("evecs", None)
    return out


def solve_targets(L: int, h: float, seed: int, eps_list, nev: int, J: float = 1.0,
                  fields_in: np.ndarray | None = None, observables: bool = True,
                  vectors: bool = False):
    """One realization, several targets from a single dense spectrum (the
    paper's eps grid per disorder sample).  Returns one dict per target."""
    f = fields(L, h, seed) if fields_in is None else _f64(fields_in)
    b = basis(L)
    n = b.size
    nev = min(nev, n)
    A = np.array(dense_H(L, J, f, b), order="F")
    eps = _f64(eps_list)
    nt = eps.size
    sig = np.full(nt, math.nan)
    ev = np.zeros(nt * nev)
    Z = np.zeros(nt * nev * n)
    o3 = np.zeros(3 * nt)
    rc = lib().orc_nearest_eigenpairs_multi(n, A.ctypes.data_as(_pd), nt, _p(eps), _p(sig), nev,
                                            _p(ev), _p(Z), None, _p(o3))
    assert rc == 0
    del A
    outs = []
    for t in range(nt):
        out = dict(L=L, h=h, seed=seed, eps=float(eps[t]), nev=nev, fields=f,
                   evals=ev[t * nev:(t + 1) * nev].copy(),
                   emin=o3[3 * t], emax=o3[3 * t + 1], sigma=o3[3 * t + 2])
        out["hnorm"] = max(abs(out["emin"]), abs(out["emax"]))
        Zt = Z[t * nev * n:(t + 1) * nev * n].reshape(nev, n).T
        out["r"], out["r_mean"] = gap_ratios(out["evals"])
        if observables:
            out["s1"] = np.array([participation_entropy(Zt[:, j], 1.0) for j in range(nev)])
            out["s2"] = np.array([participation_entropy(Zt[:, j], 2.0) for j in range(nev)])
            out["se"] = np.array([entanglement_entropy(L, Zt[:, j], b) for j in range(nev)])
            out["fluct"] = np.array([bipartite_fluct(L, Zt[:, j], b) for j in range(nev)])
            out["dynfrac"] = np.array([dynamical_fraction(L, Zt[:, j], b) for j in range(nev)])
            out["kl"] = np.array([kl_divergence(Zt[:, j], Zt[:, j + 1]) for j in range(nev - 1)])
        if vectors:
            out["evecs"] = np.ascontiguousarray(Zt)
        outs.append(out)
    return outs


# ---- the sweep protocol ("Numerical method" section): per-realization bins,
# then averages over realizations with the standard error over the bins

BIN_NAMES = ("r", "s1", "s2", "se", "se2", "fluct", "dynfrac", "kl", "edens", "nconv")


def _finite_mean(values) -> float:
    vals = [float(v) for v in values if math.isfinite(float(v))]
    return sum(vals) / len(vals) if vals else math.nan


def realization_bins(out: dict, nconv: int | None = None) -> np.ndarray:
    """One realization's bin for one target: each observable averaged over the
    nev eigenstates of that realization (the paper bins over the eigenstates
    of a sample because they are correlated).  r and KL average their finite
    values; edens is the mean of (E - E_min) / (E_max - E_min)."""
    nev = len(out["evals"])
    w = out["emax"] - out["emin"]
    b = np.full(len(BIN_NAMES), math.nan)
    b[0] = _finite_mean(out["r"]) if nev >= 3 else math.nan
    b[1] = _finite_mean(out["s1"])
    b[2] = _finite_mean(out["s2"])
    b[3] = _finite_mean(out["se"])
    b[4] = sum(float(x) * float(x) for x in out["se"]) / nev
    b[5] = _finite_mean(out["fluct"])
    b[6] = _finite_mean(out["dynfrac"])
    b[7] = _finite_mean(out["kl"]) if nev >= 2 else math.nan
    b[8] = sum(((float(E) - out["emin"]) / w if w > 0 else 0.0) for E in out["evals"]) / nev
    b[9] = float(nev if nconv is None else nconv)
    return b


def disorder_average(bins) -> dict:
    """Mean over realizations of each bin (finite bins only), the standard
    error over those bins, sqrt(sum (b - mean)^2 / (k (k - 1))), and sigma_E,
    the standard deviation of S_E over all eigenstates of all realizations:
    sqrt(<S_E^2> - <S_E>^2) with each realization weighted equally."""
    B = np.asarray(bins, dtype=np.float64).reshape(-1, len(BIN_NAMES))
    mean = np.full(B.shape[1], math.nan)
    sem = np.full(B.shape[1], math.nan)
    for q in range(B.shape[1]):
        col = [float(x) for x in B[:, q] if math.isfinite(float(x))]
        k = len(col)
        if k == 0:
            continue
        m = sum(col) / k
        mean[q] = m
        if k >= 2:
            sem[q] = math.sqrt(sum((x - m) ** 2 for x in col) / (k * (k - 1)))
    sig = math.sqrt(max(0.0, mean[4] - mean[3] * mean[3]))
    return {"mean": mean, "sem": sem, "sigma_e": sig}

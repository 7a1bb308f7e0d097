"""Python binding of libmbl, the MI355X shift-invert eigensolver for the
random-field Heisenberg chain (Eq. (1) of Luitz, Laflorencie, Alet 2014).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libmbl.so`` behind the C ABI declared in ``include/mbl.h``.  The functions
keep the C names (``mbl_solve``, ``mbl_basis``, ...); :class:`Context` wraps
a context handle for convenience.  There is no fallback: if the library is
missing or no GPU is visible the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbl.so")

MBL_OK, MBL_EINVAL, MBL_ENOMEM, MBL_ENOTCONV = 0, -1, -2, -3
MBL_ENUMERIC, MBL_EDEVICE, MBL_EBUSY, MBL_ENOTFOUND = -4, -5, -6, -7
MBL_FP64, MBL_FP32_IR64 = 0, 1
MBL_WANT_VECTORS, MBL_WANT_OBS, MBL_WANT_OBS_EXTRA = 1, 2, 4
MBL_HOOK_IR_STALL32, MBL_HOOK_IR_STALL64, MBL_HOOK_NO_CONV = 0x100, 0x200, 0x400
MBL_EIG_GENERAL = 1
MBL_NBIN = 10
BIN_NAMES = ("r", "s1", "s2", "se", "se2", "fluct", "dynfrac", "kl", "edens", "nconv")
MBL_L_MAX = 22

# every symbol include/mbl.h declares
EXPORTS = ("mbl_create", "mbl_destroy", "mbl_strerror", "mbl_last_error", "mbl_problem_init",
           "mbl_sector_dim", "mbl_fields", "mbl_basis", "mbl_rank", "mbl_hamiltonian",
           "mbl_spmv", "mbl_extremal", "mbl_ritz_eig", "mbl_symbolic", "mbl_ordering",
           "mbl_front_tree", "mbl_shift_solve",
           "mbl_observables", "mbl_observables_extra", "mbl_observables_noalloc", "mbl_solve",
           "mbl_solve_batch", "mbl_footprint",
           "mbl_serve_start", "mbl_serve_batch_limit", "mbl_submit", "mbl_poll", "mbl_wait", "mbl_serve_stats",
           "mbl_profile_enable", "mbl_profile_read", "mbl_sweep", "mbl_disorder_average")

_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


class mbl_problem(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("J", _d), ("h", _d), ("seed", ctypes.c_uint64),
                ("fields", _pd), ("eps", _d), ("sigma", _d), ("nev", ctypes.c_int),
                ("prec", ctypes.c_int), ("tol", _d), ("flags", ctypes.c_uint32),
                ("block", ctypes.c_int), ("ncv", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("fail_alloc_bytes", ctypes.c_size_t)]


class mbl_result(ctypes.Structure):
    _fields_ = [("evals", _pd), ("evecs", _pd), ("resid", _pd), ("r", _pd), ("s1", _pd),
                ("se", _pd), ("s2", _pd), ("fluct", _pd), ("dynfrac", _pd), ("kl", _pd),
                ("emin", _d), ("emax", _d), ("sigma", _d), ("hnorm", _d), ("r_mean", _d),
                ("max_resid", _d), ("nconv", ctypes.c_int), ("n_restarts", ctypes.c_int),
                ("n_opapply", ctypes.c_int), ("n_passes", ctypes.c_int),
                ("n_pass_rhs", ctypes.c_int), ("ir_iters_max", ctypes.c_int),
                ("n_perturbed", ctypes.c_int), ("fallback", ctypes.c_int),
                ("t_phase", _d * 8),
                ("t_submit", _d), ("t_start", _d), ("t_done", _d), ("batch", ctypes.c_int)]


class mbl_symbolic_info(ctypes.Structure):
    _fields_ = [("dim", _i64), ("nnz_h", _i64), ("n_fronts", _i64), ("n_levels", _i64),
                ("max_front", _i64), ("max_pivots", _i64), ("nnz_factor", _i64),
                ("front_entries", _i64), ("flops_factor", _d), ("seconds", _d)]


class mbl_kernel_profile(ctypes.Structure):
    _fields_ = [("launches", _i64), ("seconds", _d), ("bytes", _d), ("flops", _d)]


class mbl_serve_info(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("budget_bytes", ctypes.c_size_t),
                ("held_bytes", ctypes.c_size_t), ("submitted", _i64), ("admitted", _i64),
                ("completed", _i64), ("running", _i64), ("queued", _i64), ("max_running", _i64),
                ("bypasses", _i64), ("trims", _i64), ("retries", _i64),
                ("max_slot_peak", ctypes.c_size_t), ("batches", _i64), ("batched", _i64)]


class mbl_solve_info(ctypes.Structure):
    _fields_ = [("ir_iters", ctypes.c_int), ("n_perturbed", ctypes.c_int),
                ("backward_error", _d), ("t_factor", _d), ("t_solve", _d)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmbl.so (built in-tree by ``paper_1411_0660_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1411_0660_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.mbl_create.argtypes = [ctypes.c_int, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.mbl_destroy.argtypes = [vp]
    L.mbl_strerror.restype = ctypes.c_char_p
    L.mbl_strerror.argtypes = [ctypes.c_int]
    L.mbl_last_error.restype = ctypes.c_char_p
    L.mbl_problem_init.argtypes = [ctypes.POINTER(mbl_problem)]
    L.mbl_problem_init.restype = None
    L.mbl_sector_dim.restype = _i64
    L.mbl_sector_dim.argtypes = [ctypes.c_int]
    L.mbl_fields.argtypes = [ctypes.c_int, _d, ctypes.c_uint64, _pd]
    L.mbl_basis.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]
    L.mbl_rank.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32), _i64,
                           ctypes.POINTER(_i64)]
    L.mbl_hamiltonian.argtypes = [vp, ctypes.c_int, _d, _pd, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), _pd, ctypes.POINTER(_i64)]
    L.mbl_spmv.argtypes = [vp, ctypes.c_int, _d, _pd, ctypes.c_int, _pd, _pd]
    L.mbl_extremal.argtypes = [vp, ctypes.c_int, _d, _pd, _pd, _pd]
    L.mbl_ritz_eig.argtypes = [vp, ctypes.c_int, ctypes.c_int, _pd, _pd, _pd, ctypes.c_int]
    L.mbl_symbolic.argtypes = [vp, ctypes.c_int, ctypes.POINTER(mbl_symbolic_info)]
    L.mbl_ordering.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
    _pi32 = ctypes.POINTER(ctypes.c_int32)
    L.mbl_front_tree.argtypes = [vp, ctypes.c_int, _pi32, _pi32, _pi32, _pi32,
                                 ctypes.POINTER(_i64), _pi32, ctypes.POINTER(_i64),
                                 ctypes.POINTER(_i64)]
    L.mbl_shift_solve.argtypes = [vp, ctypes.c_int, _d, _pd, _d, ctypes.c_int, ctypes.c_int, _pd,
                                  _pd, ctypes.POINTER(mbl_solve_info)]
    L.mbl_observables.argtypes = [vp, ctypes.c_int, ctypes.c_int, _pd, _pd, _pd, _pd, _pd]
    L.mbl_observables_extra.argtypes = [vp, ctypes.c_int, ctypes.c_int, _pd, _pd, _pd, _pd, _pd]
    L.mbl_observables_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, _i64, vp, vp, vp, vp]
    L.mbl_solve.argtypes = [vp, ctypes.POINTER(mbl_problem), ctypes.POINTER(mbl_result)]
    L.mbl_solve_batch.argtypes = [vp, ctypes.c_int, ctypes.POINTER(mbl_problem),
                                  ctypes.POINTER(mbl_result), ctypes.POINTER(ctypes.c_int)]
    L.mbl_footprint.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_size_t)]
    L.mbl_serve_start.argtypes = [vp, ctypes.c_int, ctypes.c_size_t]
    L.mbl_serve_batch_limit.argtypes = [vp, ctypes.c_int]
    L.mbl_serve_stats.argtypes = [vp, ctypes.POINTER(mbl_serve_info)]
    L.mbl_submit.argtypes = [vp, ctypes.POINTER(mbl_problem), ctypes.POINTER(mbl_result),
                             ctypes.POINTER(ctypes.c_uint64)]
    L.mbl_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    L.mbl_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    L.mbl_profile_enable.argtypes = [vp, ctypes.c_char_p]
    L.mbl_profile_read.argtypes = [vp, ctypes.POINTER(mbl_kernel_profile)]
    L.mbl_sweep.argtypes = [vp, ctypes.POINTER(mbl_problem), _pd, ctypes.c_int, _pd,
                            ctypes.POINTER(ctypes.c_int)]
    L.mbl_disorder_average.argtypes = [_pd, ctypes.c_int, _pd, _pd, _pd]
    _lib = L
    return L


class MblError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().mbl_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib().mbl_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code: int, where: str, allow=()):
    if code != MBL_OK and code not in allow:
        raise MblError(code, where)
    return code


def _pd_of(a):
    return None if a is None else a.ctypes.data_as(_pd)


# ------------------------------------------------------------------ functions
def mbl_sector_dim(L: int) -> int:
    return int(lib().mbl_sector_dim(L))


def mbl_disorder_average(bins) -> dict:
    """Mean and standard error over realizations of one target's bins
    (n_real x MBL_NBIN), and sigma_E; host arithmetic in the library."""
    b = np.ascontiguousarray(bins, dtype=np.float64).reshape(-1, MBL_NBIN)
    mean, sem, sig = np.zeros(MBL_NBIN), np.zeros(MBL_NBIN), ctypes.c_double(0.0)
    _check(lib().mbl_disorder_average(_pd_of(b), b.shape[0], _pd_of(mean), _pd_of(sem),
                                      ctypes.byref(sig)), "mbl_disorder_average")
    return {"mean": mean, "sem": sem, "sigma_e": sig.value}


def mbl_observables_noalloc(L: int, nev: int, evals_dev: int, evecs_dev: int, ld: int,
                            r_dev: int, s1_dev: int, se_dev: int, stream: int = 0) -> int:
    """Allocation-free observables on device buffers (addresses as ints, 0 for
    NULL) of the current device; enqueues on `stream` and returns its status."""
    return lib().mbl_observables_noalloc(L, nev, evals_dev or None, evecs_dev or None, ld,
                                         r_dev or None, s1_dev or None, se_dev or None,
                                         stream or None)


def mbl_fields(L: int, h: float, seed: int) -> np.ndarray:
    out = np.zeros(L)
    _check(lib().mbl_fields(L, h, seed, _pd_of(out)), "mbl_fields")
    return out


class Context:
    """A libmbl context on one HIP device (``mbl_create`` / ``mbl_destroy``)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, stream=None):
        self._pending = {}          # ticket -> buffers the library writes into
        self._h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream) if stream else None
        _check(lib().mbl_create(device, hbm_budget, s, ctypes.byref(self._h)), "mbl_create")

    def close(self):
        if self._h:
            lib().mbl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- single steps
    def mbl_basis(self, L: int) -> np.ndarray:
        out = np.zeros(mbl_sector_dim(L), dtype=np.uint32)
        _check(lib().mbl_basis(self._h, L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))),
               "mbl_basis")
        return out

    def mbl_rank(self, L: int, words) -> np.ndarray:
        w = np.ascontiguousarray(words, dtype=np.uint32)
        r = np.zeros(w.size, dtype=np.int64)
        _check(lib().mbl_rank(self._h, L, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), w.size,
                              r.ctypes.data_as(ctypes.POINTER(_i64))), "mbl_rank")
        return r

    def mbl_hamiltonian(self, L: int, J: float, fields):
        f = np.ascontiguousarray(fields, dtype=np.float64)
        n = mbl_sector_dim(L)
        nnz = _i64()
        _check(lib().mbl_hamiltonian(self._h, L, J, _pd_of(f), None, None, None, ctypes.byref(nnz)),
               "mbl_hamiltonian")
        rp = np.zeros(n + 1, dtype=np.int32)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        _check(lib().mbl_hamiltonian(self._h, L, J, _pd_of(f),
                                     rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     _pd_of(val), ctypes.byref(nnz)), "mbl_hamiltonian")
        return rp, col, val

    def mbl_spmv(self, L: int, J: float, fields, x) -> np.ndarray:
        f = np.ascontiguousarray(fields, dtype=np.float64)
        x = np.asfortranarray(x, dtype=np.float64)
        nvec = 1 if x.ndim == 1 else x.shape[1]
        y = np.zeros_like(x)
        _check(lib().mbl_spmv(self._h, L, J, _pd_of(f), nvec, _pd_of(x), _pd_of(y)), "mbl_spmv")
        return y

    def mbl_extremal(self, L: int, J: float, fields):
        f = np.ascontiguousarray(fields, dtype=np.float64)
        a, b = _d(), _d()
        _check(lib().mbl_extremal(self._h, L, J, _pd_of(f), ctypes.byref(a), ctypes.byref(b)),
               "mbl_extremal")
        return a.value, b.value

    def mbl_ritz_eig(self, A, general: bool = False):
        """Eigenpairs of a batch of small symmetric matrices (count x m x m, or
        one m x m): eigenvalues ascending (count x m) and unit eigenvectors
        (count x m x m, column j for eigenvalue j)."""
        A = np.asarray(A, dtype=np.float64)
        one = A.ndim == 2
        if one:
            A = A[None]
        count, m = A.shape[0], A.shape[1]
        Af = np.ascontiguousarray(np.transpose(A, (0, 2, 1)))        # column-major blocks
        w = np.zeros((count, m))
        Z = np.zeros((count, m, m))
        _check(lib().mbl_ritz_eig(self._h, count, m, _pd_of(Af), _pd_of(w), _pd_of(Z),
                                  MBL_EIG_GENERAL if general else 0), "mbl_ritz_eig")
        Z = np.transpose(Z, (0, 2, 1))
        return (w[0], Z[0]) if one else (w, Z)

    def mbl_symbolic(self, L: int) -> dict:
        info = mbl_symbolic_info()
        _check(lib().mbl_symbolic(self._h, L, ctypes.byref(info)), "mbl_symbolic")
        return {k: getattr(info, k) for k, _ in info._fields_}

    def mbl_ordering(self, L: int) -> np.ndarray:
        out = np.zeros(mbl_sector_dim(L), dtype=np.int32)
        _check(lib().mbl_ordering(self._h, L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "mbl_ordering")
        return out

    def mbl_front_tree(self, L: int) -> dict:
        """Fronts of the symbolic analysis: first, npiv, ncontrib, parent, cptr
        (per front, post-order) and the concatenated contribution rows."""
        nf, nc = _i64(), _i64()
        _check(lib().mbl_front_tree(self._h, L, None, None, None, None, None, None,
                                    ctypes.byref(nf), ctypes.byref(nc)), "mbl_front_tree")
        out = {k: np.zeros(nf.value, dtype=np.int32) for k in ("first", "npiv", "ncontrib", "parent")}
        out["cptr"] = np.zeros(nf.value, dtype=np.int64)
        out["contrib"] = np.zeros(max(nc.value, 1), dtype=np.int32)
        p32 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        _check(lib().mbl_front_tree(self._h, L, p32(out["first"]), p32(out["npiv"]),
                                    p32(out["ncontrib"]), p32(out["parent"]),
                                    out["cptr"].ctypes.data_as(ctypes.POINTER(_i64)),
                                    p32(out["contrib"]), None, None), "mbl_front_tree")
        out["contrib"] = out["contrib"][:nc.value]
        return out

    def mbl_shift_solve(self, L: int, J: float, fields, sigma: float, b, prec: int = MBL_FP64):
        f = np.ascontiguousarray(fields, dtype=np.float64)
        b = np.asfortranarray(b, dtype=np.float64)
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        x = np.zeros_like(b)
        info = mbl_solve_info()
        _check(lib().mbl_shift_solve(self._h, L, J, _pd_of(f), sigma, prec, nrhs, _pd_of(b),
                                     _pd_of(x), ctypes.byref(info)), "mbl_shift_solve")
        return x, {k: getattr(info, k) for k, _ in info._fields_}

    def mbl_observables(self, L: int, evals, evecs):
        Z = np.asfortranarray(evecs, dtype=np.float64)
        nev = Z.shape[1]
        E = np.ascontiguousarray(evals, dtype=np.float64)
        r = np.zeros(max(nev - 2, 1))
        s1 = np.zeros(nev)
        se = np.zeros(nev)
        _check(lib().mbl_observables(self._h, L, nev, _pd_of(E), _pd_of(Z), _pd_of(r), _pd_of(s1),
                                     _pd_of(se)), "mbl_observables")
        return r[:max(nev - 2, 0)], s1, se

    def mbl_observables_extra(self, L: int, evecs):
        Z = np.asfortranarray(evecs, dtype=np.float64)
        nev = Z.shape[1]
        s2, fl, df, kl = np.zeros(nev), np.zeros(nev), np.zeros(nev), np.zeros(max(nev - 1, 1))
        _check(lib().mbl_observables_extra(self._h, L, nev, _pd_of(Z), _pd_of(s2), _pd_of(fl),
                                           _pd_of(df), _pd_of(kl)), "mbl_observables_extra")
        return s2, fl, df, kl[:max(nev - 1, 0)]

    # -- whole path
    def _prepare(self, L, h, seed, eps, nev, J, prec, fields, sigma, tol, vectors, extra, block,
                 ncv, entanglement, hooks=0, max_restarts=0, fail_alloc=0):
        pr = mbl_problem()
        lib().mbl_problem_init(ctypes.byref(pr))
        pr.L, pr.J, pr.h, pr.seed, pr.eps, pr.sigma, pr.nev = L, J, h, seed, eps, sigma, nev
        pr.prec, pr.tol, pr.block, pr.ncv = prec, tol, block, ncv
        pr.max_restarts, pr.fail_alloc_bytes = max_restarts, fail_alloc
        f = None
        if fields is not None:
            f = np.ascontiguousarray(fields, dtype=np.float64)
            pr.fields = _pd_of(f)
        pr.flags = MBL_WANT_OBS | (MBL_WANT_VECTORS if vectors else 0) | \
            (MBL_WANT_OBS_EXTRA if extra else 0) | hooks
        n = mbl_sector_dim(L) if 2 <= L <= MBL_L_MAX else 1
        nb = max(nev, 1)
        bufs = dict(evals=np.zeros(nb), resid=np.zeros(nb), r=np.zeros(max(nev - 2, 1)),
                    s1=np.zeros(nb))
        if entanglement:
            bufs["se"] = np.zeros(nb)
        if vectors:
            bufs["evecs"] = np.zeros((nb, n))
        if extra:
            bufs.update(s2=np.zeros(nb), fluct=np.zeros(nb), dynfrac=np.zeros(nb),
                        kl=np.zeros(max(nev - 1, 1)))
        res = mbl_result()
        for k, v in bufs.items():
            setattr(res, k, _pd_of(v))
        return pr, res, bufs, f

    @staticmethod
    def _collect(res, bufs, nev, vectors):
        out = {k: v for k, v in bufs.items()}
        out["r"] = out["r"][:max(nev - 2, 0)]
        if "kl" in out:
            out["kl"] = out["kl"][:max(nev - 1, 0)]
        if vectors:
            out["evecs"] = out["evecs"].T.copy()      # dim x nev
        for k in ("emin", "emax", "sigma", "hnorm", "r_mean", "max_resid", "nconv", "n_restarts",
                  "n_opapply", "n_passes", "n_pass_rhs", "ir_iters_max", "n_perturbed", "fallback",
                  "t_submit", "t_start", "t_done", "batch"):
            out[k] = getattr(res, k)
        out["t_phase"] = list(res.t_phase)
        return out

    def mbl_solve(self, L: int, h: float, seed: int, eps: float, nev: int, *, J: float = 1.0,
                  prec: int = MBL_FP64, fields=None, sigma: float = math.nan, tol: float = 0.0,
                  vectors: bool = False, extra: bool = False, block: int = 0, ncv: int = 0,
                  entanglement: bool = True, allow_notconv: bool = False, hooks: int = 0,
                  max_restarts: int = 0, fail_alloc: int = 0) -> dict:
        pr, res, bufs, _f = self._prepare(L, h, seed, eps, nev, J, prec, fields, sigma, tol,
                                          vectors, extra, block, ncv, entanglement, hooks,
                                          max_restarts, fail_alloc)
        code = lib().mbl_solve(self._h, ctypes.byref(pr), ctypes.byref(res))
        _check(code, "mbl_solve", allow=(MBL_ENOTCONV,) if allow_notconv else ())
        out = self._collect(res, bufs, nev, vectors)
        out["status"] = code
        return out

    def mbl_solve_batch(self, L: int, nev: int, items, *, J: float = 1.0, prec: int = MBL_FP64,
                        tol: float = 0.0, vectors: bool = False, extra: bool = False,
                        block: int = 0, ncv: int = 0, entanglement: bool = True,
                        max_restarts: int = 0) -> list:
        """Solve the problems ``items`` (dicts with h, seed, eps and optionally
        sigma, fields or hooks) together; one result dict (as mbl_solve, plus
        ``status``) per item."""
        items = list(items)
        k = len(items)
        prs = (mbl_problem * k)()
        ress = (mbl_result * k)()
        keep = []
        for q, it in enumerate(items):
            pr, res, bufs, f = self._prepare(L, it["h"], it["seed"], it.get("eps", 0.5), nev, J,
                                             prec, it.get("fields"), it.get("sigma", math.nan),
                                             tol, vectors, extra, block, ncv, entanglement,
                                             it.get("hooks", 0), max_restarts, 0)
            prs[q] = pr
            ress[q] = res
            keep.append((bufs, f))
        status = (ctypes.c_int * max(k, 1))(*([MBL_EBUSY] * max(k, 1)))
        code = lib().mbl_solve_batch(self._h, k, prs, ress, status)
        if code == MBL_EDEVICE or all(status[q] == MBL_EBUSY for q in range(k)):
            _check(code, "mbl_solve_batch")     # a device error, or nothing attempted
        out = []
        for q in range(k):
            d = self._collect(ress[q], keep[q][0], nev, vectors)
            d["status"] = status[q]
            out.append(d)
        return out

    def mbl_sweep(self, L: int, h: float, seed: int, eps, nev: int, *, J: float = 1.0,
                  prec: int = MBL_FP64, fields=None, tol: float = 0.0, block: int = 0,
                  ncv: int = 0) -> dict:
        """One realization at every target of `eps`: bins (n_eps x MBL_NBIN,
        columns BIN_NAMES) and per-target status."""
        e = np.ascontiguousarray(eps, dtype=np.float64).ravel()
        pr, _res, _bufs, f = self._prepare(L, h, seed, float(e[0]) if e.size else 0.5, nev, J, prec,
                                           fields, math.nan, tol, False, True, block, ncv, True)
        bins = np.zeros((max(e.size, 1), MBL_NBIN))
        status = (ctypes.c_int * max(e.size, 1))()
        code = lib().mbl_sweep(self._h, ctypes.byref(pr), _pd_of(e), int(e.size), _pd_of(bins),
                               status)
        _check(code, "mbl_sweep", allow=(MBL_ENOTCONV, MBL_ENUMERIC))
        return {"bins": bins[:e.size], "status": np.array(status[:e.size], dtype=np.int32),
                "code": code, "fields": f}

    # -- serving (continuous batching)
    def mbl_serve_start(self, slots: int = 0, budget_bytes: int = 0):
        _check(lib().mbl_serve_start(self._h, slots, budget_bytes), "mbl_serve_start")

    def mbl_serve_batch_limit(self, max_batch: int):
        _check(lib().mbl_serve_batch_limit(self._h, max_batch), "mbl_serve_batch_limit")

    def mbl_submit(self, L: int, h: float, seed: int, eps: float, nev: int, *, J: float = 1.0,
                   prec: int = MBL_FP64, fields=None, sigma: float = math.nan, tol: float = 0.0,
                   vectors: bool = False, extra: bool = False, block: int = 0, ncv: int = 0,
                   entanglement: bool = True) -> int:
        pr, res, bufs, f = self._prepare(L, h, seed, eps, nev, J, prec, fields, sigma, tol,
                                         vectors, extra, block, ncv, entanglement)
        t = ctypes.c_uint64()
        _check(lib().mbl_submit(self._h, ctypes.byref(pr), ctypes.byref(res), ctypes.byref(t)),
               "mbl_submit")
        self._pending[t.value] = (pr, res, bufs, f, nev, vectors)
        return t.value

    def mbl_poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        _check(lib().mbl_poll(self._h, ticket, ctypes.byref(done)), "mbl_poll")
        return bool(done.value)

    def mbl_wait(self, ticket: int) -> dict:
        """Result dict of the request (as mbl_solve) plus ``status``."""
        st = ctypes.c_int()
        _check(lib().mbl_wait(self._h, ticket, ctypes.byref(st)), "mbl_wait")
        pr, res, bufs, f, nev, vectors = self._pending.pop(ticket)
        out = self._collect(res, bufs, nev, vectors)
        out["status"] = st.value
        return out

    def mbl_serve_stats(self) -> dict:
        i = mbl_serve_info()
        _check(lib().mbl_serve_stats(self._h, ctypes.byref(i)), "mbl_serve_stats")
        return {k: getattr(i, k) for k, _ in i._fields_}

    def mbl_profile_enable(self, kernel_class: str | None):
        _check(lib().mbl_profile_enable(self._h, kernel_class.encode() if kernel_class else None),
               "mbl_profile_enable")

    def mbl_profile_read(self) -> dict:
        p = mbl_kernel_profile()
        _check(lib().mbl_profile_read(self._h, ctypes.byref(p)), "mbl_profile_read")
        return {k: getattr(p, k) for k, _ in p._fields_}

    def mbl_footprint(self, L: int, prec: int, nev: int, block: int = 0) -> int:
        b = ctypes.c_size_t()
        _check(lib().mbl_footprint(self._h, L, prec, nev, block, ctypes.byref(b)), "mbl_footprint")
        return b.value

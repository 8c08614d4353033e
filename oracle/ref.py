"""Python face of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle_dd.so`` (built from ``oracle_dd.c`` by
``oracle/build.py``).  Everything here is the paper's Algorithm 1 carried out
with a double-double (dd, unit roundoff ~2^-104) higher precision:

* :func:`gram_dd`       Alg. 1 steps 1-2, eq. (ATA)
* :func:`jacobi2_dd`    Alg. 1 step 3 with two-sided cyclic Jacobi (Sec. 2.1)
* :func:`sigma_sort`    Alg. 1 steps 3-5, eq. (sqrt); sigma_1 >= ... >= sigma_n
* :func:`u_rows_dd`     Alg. 1 step 6, eq. (AV-0)
* :func:`chol_dd`       Alg. 2 step 1
* :func:`equilibrate_dd` / :func:`kappa_b`   A = B D (Sec. 1, Thm. 1)
* :func:`orth`, :func:`resid`   the quantities bounded in Thm. 1

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg use this
module.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_dd.so")

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # noqa: WPS433 -- build on first use
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, ci, cd = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.oracle_gram_dd.argtypes = [i64, i64, vp, i64, ci, _dp, _dp]
    lib.oracle_gram_dd.restype = None
    lib.oracle_jacobi2_dd.argtypes = [i64, _dp, _dp, cd, ci, _dp, _dp]
    lib.oracle_jacobi2_dd.restype = ci
    lib.oracle_sigma_sort.argtypes = [i64, _dp, _dp, _dp, _dp]
    lib.oracle_sigma_sort.restype = ci
    lib.oracle_u_rows_dd.argtypes = [i64, vp, i64, ci, _dp, _dp, _dp, _dp, i64, _i64p, _dp, _dp]
    lib.oracle_u_rows_dd.restype = None
    lib.oracle_chol_dd.argtypes = [i64, _dp, _dp, _dp, _dp]
    lib.oracle_chol_dd.restype = ci
    lib.oracle_equilibrate_dd.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_equilibrate_dd.restype = None
    lib.oracle_orth_dd.argtypes = [i64, i64, vp, i64, ci]
    lib.oracle_orth_dd.restype = cd
    lib.oracle_resid_rows.argtypes = [i64, vp, i64, vp, i64, vp, vp, i64, ci, i64, _i64p, _dp]
    lib.oracle_resid_rows.restype = None
    lib.oracle_eft.argtypes = [cd, cd, _dp]
    lib.oracle_eft.restype = None
    lib.oracle_dd_ops.argtypes = [_dp, _dp, _dp]
    lib.oracle_dd_ops.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ci
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _colmajor(A: np.ndarray) -> tuple[np.ndarray, int]:
    """Return (F-ordered array, is_f32).  The stored values are used exactly."""
    if A.dtype not in (np.float64, np.float32):
        raise TypeError("oracle expects float64 or float32 input")
    A = np.asfortranarray(A)
    return A, int(A.dtype == np.float32)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def gram_dd(A: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """M = A^T A in double-double; returns (Mhi, Mlo), full symmetric, C-order."""
    lib = _load()
    A, f32 = _colmajor(A)
    m, n = A.shape
    Mhi = np.zeros((n, n), dtype=np.float64, order="F")
    Mlo = np.zeros((n, n), dtype=np.float64, order="F")
    lib.oracle_gram_dd(m, n, A.ctypes.data, max(m, 1), f32, _p(Mhi), _p(Mlo))
    return np.ascontiguousarray(Mhi), np.ascontiguousarray(Mlo)


def jacobi2_dd(Mhi, Mlo, tol: float = 1e-30, max_sweeps: int = 60):
    """Two-sided cyclic Jacobi in dd.  Returns (lam_hi, lam_lo, Vhi, Vlo, sweeps)."""
    lib = _load()
    n = Mhi.shape[0]
    Mh = np.array(Mhi, dtype=np.float64, order="F", copy=True)
    Ml = np.array(Mlo, dtype=np.float64, order="F", copy=True)
    Vh = np.zeros((n, n), order="F")
    Vl = np.zeros((n, n), order="F")
    sweeps = lib.oracle_jacobi2_dd(n, _p(Mh), _p(Ml), tol, max_sweeps, _p(Vh), _p(Vl))
    return (np.diag(Mh).copy(), np.diag(Ml).copy(), np.ascontiguousarray(Vh),
            np.ascontiguousarray(Vl), int(sweeps))


def sigma_sort(lam_hi, lam_lo, Vhi, Vlo):
    """sigma = sqrt(lambda) in dd, sorted descending, V permuted and sign-fixed."""
    lib = _load()
    n = len(lam_hi)
    sh = np.array(lam_hi, dtype=np.float64, copy=True)
    sl = np.array(lam_lo, dtype=np.float64, copy=True)
    Vh = np.array(Vhi, dtype=np.float64, order="F", copy=True)
    Vl = np.array(Vlo, dtype=np.float64, order="F", copy=True)
    bad = lib.oracle_sigma_sort(n, _p(sh), _p(sl), _p(Vh), _p(Vl))
    return sh, sl, np.ascontiguousarray(Vh), np.ascontiguousarray(Vl), int(bad)


def u_rows_dd(A, Vhi, Vlo, shi, slo, rows=None):
    """Rows of U = A V Sigma^{-1} in dd.  Returns (Uhi, Ulo) of shape (len(rows), n)."""
    lib = _load()
    A, f32 = _colmajor(A)
    m, n = A.shape
    rows = np.arange(m, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    rows = np.ascontiguousarray(rows)
    Vh = np.asfortranarray(Vhi, dtype=np.float64)
    Vl = np.asfortranarray(Vlo, dtype=np.float64)
    sh = np.ascontiguousarray(shi, dtype=np.float64)
    sl = np.ascontiguousarray(slo, dtype=np.float64)
    nr = len(rows)
    Uh = np.zeros((nr, n), order="F")
    Ul = np.zeros((nr, n), order="F")
    lib.oracle_u_rows_dd(n, A.ctypes.data, max(m, 1), f32, _p(Vh), _p(Vl), _p(sh), _p(sl),
                         nr, rows.ctypes.data_as(_i64p), _p(Uh), _p(Ul))
    return Uh, Ul


def chol_dd(Mhi, Mlo):
    """Upper Cholesky factor in dd.  Returns (Rhi, Rlo, info)."""
    lib = _load()
    n = Mhi.shape[0]
    Mh = np.asfortranarray(Mhi, dtype=np.float64)
    Ml = np.asfortranarray(Mlo, dtype=np.float64)
    Rh = np.zeros((n, n), order="F")
    Rl = np.zeros((n, n), order="F")
    info = lib.oracle_chol_dd(n, _p(Mh), _p(Ml), _p(Rh), _p(Rl))
    return np.ascontiguousarray(Rh), np.ascontiguousarray(Rl), int(info)


def equilibrate_dd(Mhi, Mlo):
    """(Hhi, Hlo, dhi, dlo) with d_j = sqrt(m_jj) and H = D^-1 M D^-1 in dd."""
    lib = _load()
    n = Mhi.shape[0]
    Mh = np.asfortranarray(Mhi, dtype=np.float64)
    Ml = np.asfortranarray(Mlo, dtype=np.float64)
    Hh = np.zeros((n, n), order="F")
    Hl = np.zeros((n, n), order="F")
    dh = np.zeros(n)
    dl = np.zeros(n)
    lib.oracle_equilibrate_dd(n, _p(Mh), _p(Ml), _p(Hh), _p(Hl), _p(dh), _p(dl))
    return np.ascontiguousarray(Hh), np.ascontiguousarray(Hl), dh, dl


def kappa_b(Mhi, Mlo) -> float:
    """kappa(B) for A = B D, from the eigenvalues of H = B^T B (dd Jacobi)."""
    Hh, Hl, _, _ = equilibrate_dd(Mhi, Mlo)
    lh, ll, _, _, _ = jacobi2_dd(Hh, Hl)
    lam = lh + ll
    if lam.min() <= 0:
        return float("inf")
    return float(np.sqrt(lam.max() / lam.min()))


def orth(U: np.ndarray) -> float:
    """||U^T U - I||_F with the Gram of U in dd (Thm. 1, eq. (orthU1))."""
    lib = _load()
    U, f32 = _colmajor(U)
    m, n = U.shape
    return float(lib.oracle_orth_dd(m, n, U.ctypes.data, max(m, 1), f32))


def resid(A, U, S, V, rows=None) -> float:
    """||A - U diag(S) V^T||_F / ||A||_F over the given rows, in dd (Thm. 1)."""
    lib = _load()
    A, f32 = _colmajor(A)
    U = np.asfortranarray(U, dtype=A.dtype)
    S = np.ascontiguousarray(S, dtype=A.dtype)
    V = np.asfortranarray(V, dtype=A.dtype)
    m, n = A.shape
    rows = np.arange(m, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    rows = np.ascontiguousarray(rows)
    out = np.zeros(2)
    lib.oracle_resid_rows(n, A.ctypes.data, max(m, 1), U.ctypes.data, max(m, 1), S.ctypes.data,
                          V.ctypes.data, max(n, 1), f32, len(rows),
                          rows.ctypes.data_as(_i64p), _p(out))
    return float(np.sqrt(out[0] / out[1])) if out[1] > 0 else 0.0


def eft(a: float, b: float):
    """(TwoSum(a, b), TwoProduct(a, b)) as ((s, e), (p, f))."""
    out = np.zeros(4)
    _load().oracle_eft(a, b, _p(out))
    return (out[0], out[1]), (out[2], out[3])


def dd_ops(x, y):
    """dd add, mul, div of x, y and sqrt of x; each returned as (hi, lo)."""
    xa = np.ascontiguousarray(x, dtype=np.float64)
    ya = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(8)
    _load().oracle_dd_ops(_p(xa), _p(ya), _p(out))
    return (out[0], out[1]), (out[2], out[3]), (out[4], out[5]), (out[6], out[7])


@dataclass
class OracleSVD:
    sigma_hi: np.ndarray
    sigma_lo: np.ndarray
    V_hi: np.ndarray
    V_lo: np.ndarray
    M_hi: np.ndarray
    M_lo: np.ndarray
    kappa_b: float
    sweeps: int
    not_spd: bool

    @property
    def sigma(self) -> np.ndarray:
        return self.sigma_hi + self.sigma_lo


def svd(A: np.ndarray, tol: float = 1e-30, max_sweeps: int = 60,
        want_kappa: bool = True, gram=None) -> OracleSVD:
    """Alg. 1 end to end with a dd higher precision (U is left to u_rows_dd).

    ``gram`` may pass a precomputed (Mhi, Mlo) of the same A to save time.
    """
    Mhi, Mlo = gram_dd(A) if gram is None else gram
    lh, ll, Vh, Vl, sweeps = jacobi2_dd(Mhi, Mlo, tol, max_sweeps)
    sh, sl, Vh, Vl, bad = sigma_sort(lh, ll, Vh, Vl)
    kb = kappa_b(Mhi, Mlo) if want_kappa else float("nan")
    return OracleSVD(sh, sl, Vh, Vl, Mhi, Mlo, kb, sweeps, bool(bad))


def sigma_rel_err(sigma_hat: np.ndarray, ref: OracleSVD) -> np.ndarray:
    """|sigma_hat_i - sigma_i| / sigma_i with the reference kept in dd."""
    s = np.asarray(sigma_hat, dtype=np.float64)
    return np.abs((s - ref.sigma_hi) - ref.sigma_lo) / ref.sigma_hi

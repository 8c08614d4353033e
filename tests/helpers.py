"""Shared helpers for the GPU tests: column-major device copies, the paper's
tolerances, and oracle-side measurements of a GPU result."""
from __future__ import annotations

import sys

import numpy as np

from oracle import ref

U = {np.float64: 2.0 ** -53, np.float32: 2.0 ** -24}
U_DD = 2.0 ** -104


def say(*a):
    """Name the case before a GPU step (flushed, so it survives a lost box)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def u_of(A) -> float:
    return U[np.float64 if A.dtype == np.float64 else np.float32]


def to_dev(A: np.ndarray):
    """Column-major CUDA copy of a numpy matrix (strides (1, rows))."""
    import torch
    A = np.asarray(A)
    t = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda")
    return t.t()


def to_np(t) -> np.ndarray:
    """numpy copy (Fortran order) of a column-major CUDA matrix or a vector."""
    if t.dim() == 1:
        return t.detach().cpu().numpy().copy()
    return np.asfortranarray(t.t().contiguous().cpu().numpy().T)


def sigma_tol(n: int, u: float, kb: float) -> float:
    """max_i |s_i - sigma_i| / sigma_i <= 50 n u kappa(B)."""
    return 50.0 * n * u * kb


def orth_tol(n: int, u: float) -> float:
    """||U^T U - I||_F <= 50 n u (the kappa(B)-free target)."""
    return 50.0 * n * u


def orth_tol_alg2(n: int, u: float, kb: float) -> float:
    """Orthogonality bound of Algorithm 2 (Remark 2: O(u) kappa(B) + O(u_h) kappa(B)^2; the
    u_h term is negligible here), with the same constant 50 n."""
    return 50.0 * n * u * max(1.0, kb)


def info_ok(info) -> bool:
    """No failure code: the low byte is 0 (bits 256 and 512 are warnings)."""
    return (int(info) & 0xFF) == 0


def check_thin(A, S, V, Uo, o: ref.OracleSVD, rows=None, label="", alg2=False):
    """The paper's three measures for a GPU result (S, V, U as numpy arrays).

    ||U^T U - I||_F is held to the kappa(B)-free 50 n u -- the bound of the two-sided
    Jacobi on M_h at u_h (Remark 1), the library default -- and reported against
    50 n u kappa(B) beside it.  ``alg2``: the result came from Algorithm 2 alone, whose
    bound (the remark after Lemma 1) carries kappa(B)."""
    n = A.shape[1]
    u = u_of(A)
    err = ref.sigma_rel_err(S.astype(np.float64), o)
    report = {"sigma_rel_err": float(err.max()), "sigma_tol": sigma_tol(n, u, o.kappa_b),
              "kappa_b": o.kappa_b}
    assert err.max() <= report["sigma_tol"], (label, report)
    VtV = V.astype(np.float64).T @ V.astype(np.float64) - np.eye(n)
    report["v_orth"] = float(np.linalg.norm(VtV))
    assert report["v_orth"] <= orth_tol(n, u), (label, report)
    if Uo is not None:
        report["u_orth"] = ref.orth(Uo)
        report["u_orth_meets_50nu"] = report["u_orth"] <= orth_tol(n, u)
        report["u_orth_tol_50nu_kappab"] = orth_tol_alg2(n, u, o.kappa_b)
        bound = orth_tol_alg2(n, u, o.kappa_b) if alg2 else orth_tol(n, u)
        assert report["u_orth"] <= bound, (label, report)
        report["resid"] = ref.resid(A, Uo, S, V, rows=rows)
        assert report["resid"] <= orth_tol(n, u), (label, report)
    return report

"""Brute-force tier of the oracle -- TEST INFRASTRUCTURE ONLY.

Independent of ``oracle_dd.c``: the Gram matrix of the stored binary matrix
is formed exactly with Python integers (every binary float is an integer
times a power of two), and the spectrum is taken with mpmath at 60 digits.
Used to pin the dd oracle on small inputs.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np


def _int_scaled(A: np.ndarray) -> tuple[list[list[int]], int]:
    """Columns of A as Python ints C[j][k] with A[k, j] == C[j][k] * 2**e0 exactly."""
    A64 = np.asarray(A, dtype=np.float64)  # FP32 values are exact in FP64
    m, n = A64.shape
    mant, ex = np.frexp(A64)  # A = mant * 2**ex, 0.5 <= |mant| < 1
    imant = (mant * 2.0 ** 53).astype(np.int64)  # exact: 53-bit integer significands
    ex = ex.astype(np.int64) - 53
    nz = imant != 0
    e0 = int(ex[nz].min()) if nz.any() else 0
    cols = []
    for j in range(n):
        col = []
        for k in range(m):
            v = int(imant[k, j])
            col.append(v << int(ex[k, j] - e0) if v else 0)
        cols.append(col)
    return cols, e0


def exact_gram(A: np.ndarray) -> list[list[Fraction]]:
    """A^T A exactly, as a list of rows of Fractions."""
    cols, e0 = _int_scaled(A)
    n = len(cols)
    scale = Fraction(2) ** (2 * e0)
    G = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        ci = cols[i]
        for j in range(i, n):
            cj = cols[j]
            s = sum(x * y for x, y in zip(ci, cj))
            G[i][j] = G[j][i] = s * scale
    return G


def fraction_to_dd(x: Fraction) -> tuple[float, float]:
    """Round an exact rational to the nearest (hi, lo) double pair."""
    hi = float(x)
    lo = float(x - Fraction(hi))
    return hi, lo


def mp_sigma(A: np.ndarray, dps: int = 60, G=None) -> list:
    """Singular values of the stored A (descending), as mpmath mpf at `dps` digits.

    sigma_i = sqrt(lambda_i(A^T A)) with the exact Gram and mpmath's symmetric
    eigensolver; at 60 digits the eigensolver's absolute error is far below the
    smallest eigenvalue for every matrix the tests use.
    """
    G = exact_gram(A) if G is None else G
    n = len(G)
    with mpmath.workdps(dps):
        M = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                M[i, j] = mpmath.mpf(G[i][j].numerator) / G[i][j].denominator
        if n == 1:
            ev = [M[0, 0]]
        else:
            E, _ = mpmath.eigsy(M)
            ev = [E[i] for i in range(n)]
        sig = sorted((mpmath.sqrt(e) for e in ev), reverse=True)
    return sig


def mp_sigma_2x2(a: Fraction, b: Fraction, c: Fraction, dps: int = 60) -> list:
    """Closed form for M = [[a, b], [b, c]]: lambda = (a+c)/2 +- sqrt(((a-c)/2)^2 + b^2)."""
    with mpmath.workdps(dps):
        a_, b_, c_ = (mpmath.mpf(x.numerator) / x.denominator for x in (a, b, c))
        mid = (a_ + c_) / 2
        rad = mpmath.sqrt(((a_ - c_) / 2) ** 2 + b_ ** 2)
        l1 = mid + rad
        l2 = (a_ * c_ - b_ ** 2) / l1  # product of roots, no cancellation
        return [mpmath.sqrt(l1), mpmath.sqrt(l2)]


def rel_err_mp(hi: float, lo: float, ref, dps: int = 60) -> float:
    """|(hi + lo) - ref| / ref evaluated in mpmath."""
    with mpmath.workdps(dps):
        v = mpmath.mpf(hi) + mpmath.mpf(lo)
        return float(abs(v - ref) / ref)


def mp_eigvecs(A: np.ndarray, dps: int = 60, G=None):
    """(sigma, V) of the stored A from the exact Gram and mpmath's eigsy at `dps` digits:
    sigma descending (mpf), V as an n x n numpy array of mpf whose columns are the unit
    eigenvectors in that order, each with the sign mpmath returned (no sign rule)."""
    G = exact_gram(A) if G is None else G
    n = len(G)
    with mpmath.workdps(dps):
        M = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                M[i, j] = mpmath.mpf(G[i][j].numerator) / G[i][j].denominator
        E, Q = mpmath.eigsy(M)
        order = sorted(range(n), key=lambda i: -E[i])
        sig = [mpmath.sqrt(E[i]) for i in order]
        V = np.empty((n, n), dtype=object)
        for c, i in enumerate(order):
            for r in range(n):
                V[r, c] = Q[r, i]
    return sig, V

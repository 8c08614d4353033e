"""Seeded synthetic inputs for the Gram-based thin SVD.

Shared by the tests, the benchmark and the oracle's checks; it holds none of
the method's arithmetic (no Gram, no eigensolver, no back-multiplication).

Two families:

* :func:`make_a` -- the paper's random test matrices A = B D (Sec. 4.1,
  Tables 2-3): D and Sigma from the DLATM1 modes of Table 3, B = W1 Sigma W2 W3
  with W1, W2 orthonormal factors of Gaussian matrices and W3 a sequence of
  plane rotations that gives B unit-norm columns (the Bendel-Mickey /
  Davies-Higham construction of a matrix with prescribed singular values and
  unit column norms).
* :func:`hadamard_exact` / :func:`orthogonal_columns` -- matrices whose stored
  binary entries have an exactly known SVD, used to pin the oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

BASE_SEED = 11953


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def latm1(mode: int, kappa: float, n: int, rng: np.random.Generator) -> np.ndarray:
    """Diagonal entries with condition number kappa, per Table 3 of the paper.

    1: d(1) = 1, d(2:n) = 1/kappa        2: d(1:n-1) = 1, d(n) = 1/kappa
    3: d(i) = kappa^(-(i-1)/(n-1))       4: d(i) = 1 - (i-1)/(n-1) (1 - 1/kappa)
    5: log-uniform in (1/kappa, 1) (endpoints not forced)
    """
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    if mode == 1:
        d = np.full(n, 1.0 / kappa)
        d[0] = 1.0
    elif mode == 2:
        d = np.ones(n)
        d[-1] = 1.0 / kappa
    elif mode == 3:
        d = kappa ** (-i / (n - 1))
    elif mode == 4:
        d = 1.0 - i / (n - 1) * (1.0 - 1.0 / kappa)
    elif mode == 5:
        d = np.exp(-np.log(kappa) * rng.random(n))
    else:
        raise ValueError(f"unknown DLATM1 mode {mode}")
    return d


def _orth_factor(G: np.ndarray) -> np.ndarray:
    """Q factor of G (Householder QR, LAPACK via scipy) with diag(R) > 0."""
    Q, R = scipy.linalg.qr(np.asfortranarray(G), mode="economic", overwrite_a=True,
                           check_finite=False)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def unit_columns(X: np.ndarray) -> np.ndarray:
    """Rotate column pairs of X (n x n, sum of squared column norms == n) until
    every column has unit norm; singular values are unchanged.

    Each step picks i with ||x_i|| < 1 and j with ||x_j|| > 1 and applies the
    plane rotation [c s; -s c] (t = s/c) that solves
    (c_jj - 1) t^2 - 2 c_ij t + (c_ii - 1) = 0, so the new column i has norm 1.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    n = X.shape[1]
    nrm2 = np.einsum("ij,ij->j", X, X)
    for _ in range(4 * n):
        dev = nrm2 - 1.0
        if np.max(np.abs(dev)) <= 1e-15:
            break
        lo = np.where(dev < 0)[0]
        hi = np.where(dev > 0)[0]
        if len(lo) == 0 or len(hi) == 0:
            break
        i = lo[np.argmin(dev[lo])]
        j = hi[np.argmax(dev[hi])]
        cii, cjj = nrm2[i], nrm2[j]
        cij = float(X[:, i] @ X[:, j])
        disc = np.sqrt(cij * cij - (cii - 1.0) * (cjj - 1.0))
        sg = 1.0 if cij >= 0 else -1.0
        t = (cii - 1.0) / (cij + sg * disc)
        c = 1.0 / np.sqrt(1.0 + t * t)
        s = c * t
        xi, xj = X[:, i].copy(), X[:, j].copy()
        X[:, i] = c * xi - s * xj
        X[:, j] = s * xi + c * xj
        nrm2[i] = X[:, i] @ X[:, i]
        nrm2[j] = X[:, j] @ X[:, j]
    X /= np.sqrt(np.einsum("ij,ij->j", X, X))
    return X


@dataclass
class MatrixSpec:
    """Recipe for one A = B D test matrix (Sec. 4.1 of the paper)."""

    m: int
    n: int
    kappa_b: float
    kappa_d: float
    mode_b: int = 3
    mode_d: int = 3
    seed: int = BASE_SEED
    dtype: str = "f64"          # stored precision of A: "f64" or "f32"
    shuffle: bool = False       # permute the columns (D no longer monotone)
    w1: str = "qr"              # "qr": orthonormal W1; "gauss": Gaussian / sqrt(m)
    extra: dict = field(default_factory=dict)


def make_a(spec: MatrixSpec) -> np.ndarray:
    """The m x n matrix A = B D of the spec, column-major (Fortran order).

    B = W1 (Sigma W2 W3): Sigma from DLATM1(mode_b, kappa_b) rescaled so that
    sum(sigma^2) = n, W2 the orthonormal factor of an n x n Gaussian, W3 the
    rotations of :func:`unit_columns`, W1 the orthonormal factor of an m x n
    Gaussian (or, for very large m, a Gaussian scaled by 1/sqrt(m), whose
    columns are orthonormal only up to O(sqrt(n/m))).  D = DLATM1(mode_d,
    kappa_d).  FP32 inputs are generated in FP64 and then rounded: the rounded
    array is the input.
    """
    m, n = spec.m, spec.n
    if m < n or n < 1:
        raise ValueError("need m >= n >= 1")
    rng = rng_for(spec.seed)
    sig = latm1(spec.mode_b, spec.kappa_b, n, rng)
    sig = sig * np.sqrt(n / np.sum(sig * sig))
    W2 = _orth_factor(rng.standard_normal((n, n)))
    X = unit_columns(sig[:, None] * W2)
    d = latm1(spec.mode_d, spec.kappa_d, n, rng)
    G = np.asfortranarray(rng.standard_normal((n, m)).T)
    if spec.w1 == "qr":
        W1 = _orth_factor(G)
    elif spec.w1 == "gauss":
        W1 = G
        W1 *= 1.0 / np.sqrt(m)
    else:
        raise ValueError(spec.w1)
    del G
    A = W1 @ (X * d[None, :])
    del W1
    if spec.shuffle:
        A = A[:, rng.permutation(n)]
    A = np.asfortranarray(A)
    if spec.dtype == "f32":
        A = np.asfortranarray(A.astype(np.float32))
    elif spec.dtype != "f64":
        raise ValueError(spec.dtype)
    return A


def small_factor(spec: MatrixSpec) -> tuple[np.ndarray, np.random.Generator]:
    """Y = (Sigma W2 W3) D of the spec, n x n, with the spec's column permutation applied
    (the draws of make_a without W1), and the generator after those draws."""
    n = spec.n
    rng = rng_for(spec.seed)
    sig = latm1(spec.mode_b, spec.kappa_b, n, rng)
    sig = sig * np.sqrt(n / np.sum(sig * sig))
    W2 = _orth_factor(rng.standard_normal((n, n)))
    X = unit_columns(sig[:, None] * W2)
    d = latm1(spec.mode_d, spec.kappa_d, n, rng)
    Y = X * d[None, :]
    if spec.shuffle:
        Y = Y[:, rng.permutation(n)]
    return np.asfortranarray(Y), rng


def make_a_device(spec: MatrixSpec, device):
    """A = W1 Y built on the GPU for workloads too large for the host recipe.

    Y is :func:`small_factor` (numpy, FP64).  W1 is an m x n Gaussian from a torch
    generator seeded with spec.seed, made orthonormal by a QR factorization when
    spec.w1 == "qr" (then sigma(A) equals sigma(Y) up to the rounding of the product),
    else scaled by 1/sqrt(m).  Returns (A, Y): A a column-major (strides (1, m)) torch
    tensor in the spec's dtype, Y the numpy factor.
    """
    import torch
    m, n = spec.m, spec.n
    if m < n or n < 1:
        raise ValueError("need m >= n >= 1")
    Y, _ = small_factor(spec)
    gen = torch.Generator(device=device).manual_seed(int(spec.seed))
    G = torch.randn((n, m), generator=gen, device=device, dtype=torch.float64)  # W1^T
    if spec.w1 == "qr":
        Q, _ = torch.linalg.qr(G.t(), mode="reduced")
        del G
        W1t = Q.t().contiguous()
        del Q
    elif spec.w1 == "gauss":
        W1t = G.mul_(1.0 / np.sqrt(m))
    else:
        raise ValueError(spec.w1)
    Yt = torch.from_numpy(np.ascontiguousarray(Y.T)).to(device)
    At = Yt @ W1t  # (n x m) row-major = A column-major
    del W1t
    if spec.dtype == "f32":
        At = At.to(torch.float32)
    elif spec.dtype != "f64":
        raise ValueError(spec.dtype)
    return At.t(), Y


# --------------------------------------------------------------------------
# matrices with an exactly known SVD
# --------------------------------------------------------------------------

def sylvester(m: int) -> np.ndarray:
    """Sylvester Hadamard matrix of order m (a power of two): H[i,j] = (-1)^popcount(i & j)."""
    if m & (m - 1):
        raise ValueError("order must be a power of two")
    i = np.arange(m, dtype=np.int64)
    x = i[:, None] & i[None, :]
    par = np.zeros_like(x)
    while np.any(x):
        par ^= x & 1
        x >>= 1
    return (1 - 2 * par).astype(np.float64)


@dataclass
class ExactSVD:
    A: np.ndarray         # stored matrix, Fortran order
    sigma: np.ndarray     # exact singular values, descending
    U: np.ndarray         # exact left singular vectors matching sigma (m x n)
    V: np.ndarray         # exact right singular vectors matching sigma (n x n)
    kappa_b: float        # exact kappa(B)


def hadamard_exact(k: int, n: int, block_exps=None, dtype: str = "f64", seed: int = BASE_SEED,
                   col_perm: bool = False) -> ExactSVD:
    """A = Q diag(s) W^T with an exactly known SVD and kappa(B) << kappa(A).

    m = 4^k; Q = H_m[:, :n] / 2^k (orthonormal columns, entries +-2^-k);
    W = blockdiag(H_4 / 2) (orthogonal, entries +-1/2); s_j = c_j 2^-e_b with c_j drawn from
    {1, 7/8, ..., 1/4} (distinct within a block, e_b per block), so every entry of A is a
    sum of four values with 3-bit significands within three binades: exactly
    representable in FP32 and FP64.  The s_j are distinct, so V is unique up to
    column signs.  All columns of a block have the same norm, so D is constant
    per block and kappa(B) = max/min of s_j / d_block(j), while kappa(A) grows
    with the spread between blocks.
    """
    if n % 4:
        raise ValueError("n must be a multiple of 4")
    m = 4 ** k
    if n > m:
        raise ValueError("n must be <= 4^k")
    nb = n // 4
    rng = rng_for(seed)
    if block_exps is None:
        block_exps = [10 * b for b in range(nb)]
    # four distinct values with 3-bit significands inside [1/4, 1]
    palette = np.array([1.0, 0.875, 0.75, 0.625, 0.5, 0.375, 0.25])
    s = np.empty(n)
    for b in range(nb):
        pick = rng.choice(len(palette), size=4, replace=False)
        s[4 * b:4 * b + 4] = np.ldexp(palette[pick], -int(block_exps[b]))
    H = sylvester(m)[:, :n]
    Q = H / 2.0 ** k
    H4 = sylvester(4) / 2.0
    W = np.zeros((n, n))
    for b in range(nb):
        W[4 * b:4 * b + 4, 4 * b:4 * b + 4] = H4
    A = (Q * s[None, :]) @ W.T
    if col_perm:
        p = rng.permutation(n)
        A = A[:, p]
        W = W[p, :]
    order = np.argsort(-s, kind="stable")
    d_block = np.sqrt(np.array([np.sum(s[4 * b:4 * b + 4] ** 2) / 4.0 for b in range(nb)]))
    ratios = s / np.repeat(d_block, 4)
    kb = float(ratios.max() / ratios.min())
    A = np.asfortranarray(A)
    if dtype == "f32":
        A32 = A.astype(np.float32)
        if not np.array_equal(A32.astype(np.float64), A):
            raise ValueError("construction not exact in FP32")
        A = np.asfortranarray(A32)
    return ExactSVD(A=A, sigma=s[order], U=Q[:, order], V=W[:, order], kappa_b=kb)


def orthogonal_columns(k: int, n: int, scales: np.ndarray, dtype: str = "f64") -> ExactSVD:
    """A = (H_m[:, :n] / 2^k) diag(scales): kappa(B) = 1, sigma = sorted |scales|."""
    m = 4 ** k
    Q = sylvester(m)[:, :n] / 2.0 ** k
    A = np.asfortranarray(Q * np.asarray(scales, dtype=np.float64)[None, :])
    if dtype == "f32":
        A = np.asfortranarray(A.astype(np.float32))
    absd = np.abs(np.asarray(A, dtype=np.float64)[0, :]) * 2.0 ** k
    order = np.argsort(-absd, kind="stable")
    V = np.eye(n)[:, order]
    return ExactSVD(A=A, sigma=absd[order], U=(Q * np.sign(scales)[None, :])[:, order], V=V,
                    kappa_b=1.0)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def spec_small_f64(seed: int = BASE_SEED + 1) -> MatrixSpec:
    """FP64, m = 2000, n = 20, kappa(B) = 10 (log-spaced), D log-spaced over 1e8."""
    return MatrixSpec(m=2000, n=20, kappa_b=10.0, kappa_d=1e8, mode_b=3, mode_d=3, seed=seed)


def spec_tall_f64(m: int = 1_000_000, seed: int = BASE_SEED + 2) -> MatrixSpec:
    """FP64, m = 1e6, n = 64, kappa(B) = 100, D log-spaced over 1e10, columns shuffled."""
    return MatrixSpec(m=m, n=64, kappa_b=100.0, kappa_d=1e10, mode_b=3, mode_d=3, seed=seed,
                      shuffle=True)


def spec_tall_f32(m: int = 4_000_000, seed: int = BASE_SEED + 3) -> MatrixSpec:
    """FP32 working, m = 4e6, n = 128, kappa(B) = 1e2, kappa(D) = 1e6."""
    return MatrixSpec(m=m, n=128, kappa_b=100.0, kappa_d=1e6, mode_b=3, mode_d=3, seed=seed,
                      dtype="f32", w1="qr" if m <= 1_000_000 else "gauss")


def spec_large_f64(m: int = 2_000_000, seed: int = BASE_SEED + 5) -> MatrixSpec:
    """FP64, m = 2e6, n = 512, kappa(B) = 1e3, kappa(D) = 1e12."""
    return MatrixSpec(m=m, n=512, kappa_b=1e3, kappa_d=1e12, mode_b=3, mode_d=3, seed=seed,
                      w1="gauss")


def batch_specs(count: int = 512, m_lo: int = 10_000, m_hi: int = 200_000,
                ns=(16, 32, 48, 64, 96), seed: int = BASE_SEED + 4) -> list[MatrixSpec]:
    """The batched workload: m ~ U[m_lo, m_hi], n from ns, kappa(B) log-U[10, 1e3],
    kappa(D) log-U[1e4, 1e12], columns shuffled; matrix i seeded seed + 1000 i."""
    rng = rng_for(seed)
    out = []
    for i in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        n = int(rng.choice(ns))
        kb = float(10 ** rng.uniform(1, 3))
        kd = float(10 ** rng.uniform(4, 12))
        out.append(MatrixSpec(m=m, n=n, kappa_b=kb, kappa_d=kd, mode_b=3, mode_d=3,
                              seed=seed + 1000 * (i + 1), shuffle=True, w1="gauss"))
    return out

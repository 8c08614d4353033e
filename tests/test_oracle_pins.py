"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes one part of the oracle against mathematics the paper relies on:
exact rational arithmetic, an exact integer Gram, a 60-digit eigensolver,
matrices with an exactly known SVD, closed forms, invariances, and LAPACK's
one-sided Jacobi SVD (the paper's own accuracy reference, Sec. 4.1.1).
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from gen import matrices as g
from oracle import brute, ref

U_DD = 2.0 ** -104          # unit roundoff of the dd format used by the oracle
U64 = 2.0 ** -53


def _fr(x: float) -> Fraction:
    return Fraction(x)


# ---------------------------------------------------------------- dd primitives

@pytest.mark.parametrize("seed", range(5))
def test_eft_exact(seed):
    """TwoSum and TwoProduct are error-free: s + e == a + b, p + f == a * b exactly."""
    rng = np.random.default_rng(seed)
    for _ in range(400):
        a = float(rng.standard_normal() * 2.0 ** rng.integers(-60, 60))
        b = float(rng.standard_normal() * 2.0 ** rng.integers(-60, 60))
        (s, e), (p, f) = ref.eft(a, b)
        assert _fr(s) + _fr(e) == _fr(a) + _fr(b)
        assert _fr(p) + _fr(f) == _fr(a) * _fr(b)
        assert s == a + b and p == a * b


def test_dd_ops_accuracy():
    """dd add/mul/div/sqrt agree with exact rationals (mpmath for sqrt) to ~2^-100."""
    rng = np.random.default_rng(7)
    with mpmath.workdps(50):
        for _ in range(300):
            xh, yh = rng.uniform(0.5, 2.0, size=2) * 2.0 ** rng.integers(-20, 20, size=2)
            x = (float(xh), float(xh) * float(rng.uniform(-1, 1)) * 2.0 ** -54)
            y = (float(yh), float(yh) * float(rng.uniform(-1, 1)) * 2.0 ** -54)
            X = _fr(x[0]) + _fr(x[1])
            Y = _fr(y[0]) + _fr(y[1])
            add, mul, div, sq = ref.dd_ops(x, y)
            for got, exact in ((add, X + Y), (mul, X * Y), (div, X / Y)):
                err = abs(_fr(got[0]) + _fr(got[1]) - exact) / abs(exact)
                assert err <= 2.0 ** -100, (got, float(exact))
            s = mpmath.sqrt(mpmath.mpf(X.numerator) / X.denominator)
            err = abs(mpmath.mpf(sq[0]) + mpmath.mpf(sq[1]) - s) / s
            assert err <= 2.0 ** -100


# ---------------------------------------------------------------- Gram (Alg. 1 step 2)

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gram_vs_exact_integer_gram(dtype):
    """dd Gram within eq. (ATA) with eps = 2 m u_dd of the exact Gram of the stored A."""
    spec = g.MatrixSpec(m=600, n=12, kappa_b=30.0, kappa_d=1e8, mode_b=3, mode_d=5,
                        seed=101, dtype=dtype, shuffle=True)
    A = g.make_a(spec)
    Mhi, Mlo = ref.gram_dd(A)
    G = brute.exact_gram(A)
    absA = np.abs(A.astype(np.float64))
    bound = 2 * A.shape[0] * U_DD * (absA.T @ absA)
    n = A.shape[1]
    for i in range(n):
        for j in range(n):
            err = abs(_fr(Mhi[i, j]) + _fr(Mlo[i, j]) - G[i][j])
            assert float(err) <= bound[i, j], (i, j, float(err), bound[i, j])


def test_gram_symmetric_and_blocking_independent():
    """Full symmetric output; row blocks merged in fixed order give the same hi part for any m split."""
    A = g.make_a(g.MatrixSpec(m=3000, n=8, kappa_b=10, kappa_d=1e4, seed=5))
    Mhi, Mlo = ref.gram_dd(A)
    assert np.array_equal(Mhi, Mhi.T) and np.array_equal(Mlo, Mlo.T)
    # the sum of the Grams of two row blocks equals the Gram (dd rounding only)
    M1 = ref.gram_dd(A[:1234])
    M2 = ref.gram_dd(A[1234:])
    for i in range(8):
        for j in range(8):
            tot = (_fr(M1[0][i, j]) + _fr(M1[1][i, j]) + _fr(M2[0][i, j]) + _fr(M2[1][i, j])
                   - _fr(Mhi[i, j]) - _fr(Mlo[i, j]))
            assert abs(float(tot)) <= 1e-28 * np.sqrt(Mhi[i, i] * Mhi[j, j])


# ---------------------------------------------------------------- sigma (Alg. 1 steps 3-5)

def _bound_dd(n, kb):
    # Remark 1 with u and u_h both the dd unit roundoff, constants made explicit
    return 16.0 * n * n * U_DD * kb * kb + 64 * n * U_DD


@pytest.mark.parametrize("spec", [
    g.spec_small_f64(),
    g.MatrixSpec(m=400, n=16, kappa_b=1e3, kappa_d=1e6, mode_b=5, mode_d=1, seed=77),
    g.MatrixSpec(m=300, n=10, kappa_b=50, kappa_d=1e9, mode_b=4, mode_d=2, seed=78, dtype="f32",
                 shuffle=True),
], ids=["m2000n20", "mode5-1", "f32"])
def test_sigma_vs_brute_force(spec):
    """sigma from the dd oracle equals sqrt(eig(exact Gram)) at 60 digits."""
    A = g.make_a(spec)
    o = ref.svd(A)
    assert o.sweeps > 0 and not o.not_spd
    ref_sig = brute.mp_sigma(A)
    errs = [brute.rel_err_mp(o.sigma_hi[i], o.sigma_lo[i], ref_sig[i]) for i in range(A.shape[1])]
    assert max(errs) <= _bound_dd(A.shape[1], o.kappa_b), max(errs)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("perm", [False, True])
def test_hadamard_exact_spectrum(dtype, perm):
    """A = Q diag(s) W^T with exact dyadic sigma: oracle sigma, V and U exact to dd rounding,
    although kappa(A) is ~1e9 (FP64 case) while kappa(B) is tiny (Sec. 1, [DV1992])."""
    exps = [0, 10, 20, 30] if dtype == "f64" else [0, 8, 16, 24]
    E = g.hadamard_exact(5, 16, block_exps=exps, dtype=dtype, col_perm=perm, seed=3)
    o = ref.svd(E.A)
    err = np.abs((o.sigma_hi - E.sigma) + o.sigma_lo) / E.sigma
    assert err.max() <= 8 * U_DD
    assert abs(o.kappa_b - E.kappa_b) <= 1e-14 * E.kappa_b
    sgn = np.sign(np.sum(o.V_hi * E.V, axis=0))
    assert np.all(sgn != 0)
    assert np.abs((o.V_hi * sgn - E.V) + o.V_lo * sgn).max() <= 1e-28
    Uh, Ul = ref.u_rows_dd(E.A, o.V_hi, o.V_lo, o.sigma_hi, o.sigma_lo)
    assert np.abs((Uh * sgn - E.U) + Ul * sgn).max() <= 1e-28


def test_n1_closed_form():
    """n = 1: sigma = ||a||_2, V = [1], U = a / ||a||."""
    rng = np.random.default_rng(11)
    a = np.asfortranarray(rng.standard_normal((777, 1)) * 1e-3)
    o = ref.svd(a)
    ss = sum(_fr(x) ** 2 for x in a[:, 0])
    with mpmath.workdps(60):
        s = mpmath.sqrt(mpmath.mpf(ss.numerator) / ss.denominator)
    assert brute.rel_err_mp(o.sigma_hi[0], o.sigma_lo[0], s) <= 4 * U_DD
    assert o.V_hi[0, 0] == 1.0 and o.V_lo[0, 0] == 0.0
    Uh, Ul = ref.u_rows_dd(a, o.V_hi, o.V_lo, o.sigma_hi, o.sigma_lo, rows=[0, 5, 776])
    with mpmath.workdps(60):
        for r, k in enumerate([0, 5, 776]):
            ex = mpmath.mpf(a[k, 0]) / s
            assert abs(mpmath.mpf(Uh[r, 0]) + mpmath.mpf(Ul[r, 0]) - ex) <= 1e-30 * abs(ex) + 1e-40


def test_n2_closed_form():
    """n = 2: eigenvalues of [[a, b], [b, c]] by the quadratic formula on the exact Gram."""
    rng = np.random.default_rng(12)
    A = np.asfortranarray(rng.standard_normal((500, 2)) * np.array([1.0, 3e-7]))
    A[:, 1] += 1e-7 * A[:, 0]
    o = ref.svd(A)
    G = brute.exact_gram(A)
    s = brute.mp_sigma_2x2(G[0][0], G[0][1], G[1][1])
    for i in range(2):
        assert brute.rel_err_mp(o.sigma_hi[i], o.sigma_lo[i], s[i]) <= 1e-29


def _sign_rule(V):
    """The output sign convention, stated plainly: flip each column so that its entry of
    largest magnitude is positive; among entries of equal magnitude the lowest row index
    counts.  (Written here, independently of the oracle's code.)"""
    V = V.copy()
    for c in range(V.shape[1]):
        mags = [abs(x) for x in V[:, c]]
        best = max(mags)
        r = mags.index(best)  # first (lowest) index of the largest magnitude
        if V[r, c] < 0:
            V[:, c] = -V[:, c]
    return V


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (5, 3), (8, 4)])
def test_sign_rule_against_brute_force(n, seed):
    """V of the oracle, compared entry by entry with NO sign alignment, against the
    60-digit eigenvectors of the exact Gram with the sign convention applied in the test:
    a wrong convention (smallest entry positive, first entry positive, highest index on
    ties) or a column permutation fails."""
    rng = np.random.default_rng(300 + seed)
    A = np.asfortranarray(rng.standard_normal((40, n)) * np.logspace(0, -3, n)[None, :])
    o = ref.svd(A)
    sig, Vb = brute.mp_eigvecs(A)
    with mpmath.workdps(60):  # (mpmath rounds even a negation to the working precision)
        Vb = _sign_rule(Vb)
        for c in range(n):
            mags = sorted((abs(x) for x in Vb[:, c]), reverse=True)
            assert mags[0] - mags[1] > mpmath.mpf(10) ** -6  # no near-tie: the rule decides
            for r in range(n):
                d = mpmath.mpf(o.V_hi[r, c]) + mpmath.mpf(o.V_lo[r, c]) - Vb[r, c]
                assert abs(d) <= mpmath.mpf(10) ** -25, (r, c, float(d))


def test_sign_rule_exact_ties_take_the_lowest_index():
    """A = [[1, 0], [1, 1], [0, 1]]: A^T A = [[2, 1], [1, 2]], eigenvectors (1, 1)/sqrt(2)
    (sigma = sqrt(3)) and (1, -1)/sqrt(2) (sigma = 1).  Both columns tie in magnitude
    exactly, so the lowest row index carries the positive sign: V = [[c, c], [c, -c]]."""
    A = np.asfortranarray(np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]]))
    o = ref.svd(A)
    V = o.V_hi + o.V_lo
    c = 2.0 ** -0.5
    assert np.abs(V - np.array([[c, c], [c, -c]])).max() <= 1e-15
    assert V[0, 0] > 0 and V[0, 1] > 0 and V[1, 1] < 0
    assert abs(o.V_hi[0, 1]) == abs(o.V_hi[1, 1])  # the tie is exact in the oracle


def test_orthogonal_columns():
    """kappa(B) = 1: sigma are the column norms, V a permutation."""
    scales = np.array([3.0, -1e-6, 0.25, 7e5, 1e-12, -2.5, 1.0, 9e-3])
    E = g.orthogonal_columns(4, 8, scales)
    o = ref.svd(E.A)
    err = np.abs((o.sigma_hi - E.sigma) + o.sigma_lo) / E.sigma
    assert err.max() <= 8 * U_DD
    assert np.array_equal(np.abs(np.round(o.V_hi)), E.V)
    assert abs(o.kappa_b - 1.0) < 1e-28 + 1e-15


def test_invariances():
    """Power-of-two scaling is exact; row/column permutations and sign flips leave sigma."""
    A = g.make_a(g.MatrixSpec(m=500, n=12, kappa_b=100, kappa_d=1e7, seed=21, shuffle=True))
    o = ref.svd(A)
    o2 = ref.svd(np.asfortranarray(A * 2.0 ** 37))
    assert np.array_equal(o2.sigma_hi, o.sigma_hi * 2.0 ** 37)
    assert np.array_equal(o2.sigma_lo, o.sigma_lo * 2.0 ** 37)
    rng = np.random.default_rng(1)
    tol = _bound_dd(12, o.kappa_b)
    for B in (A[rng.permutation(500)], A[:, rng.permutation(12)],
              A * np.where(rng.random(12) < 0.5, -1.0, 1.0)):
        ob = ref.svd(np.asfortranarray(B))
        err = np.abs((ob.sigma_hi - o.sigma_hi) + (ob.sigma_lo - o.sigma_lo)) / o.sigma_hi
        assert err.max() <= tol


def test_jacobi_decomposition():
    """V orthogonal to dd precision; V diag(lambda) V^T reproduces M (rounded to FP64 for the check)."""
    A = g.make_a(g.MatrixSpec(m=800, n=24, kappa_b=100, kappa_d=1e3, seed=31))
    Mhi, Mlo = ref.gram_dd(A)
    lh, ll, Vh, Vl, sweeps = ref.jacobi2_dd(Mhi, Mlo)
    assert 2 <= sweeps <= 20
    VtV = Vh.T @ Vh - np.eye(24)
    assert np.abs(VtV).max() < 4e-16
    rec = (Vh * (lh + ll)) @ Vh.T
    assert np.abs(rec - Mhi).max() <= 1e-14 * np.abs(Mhi).max()


def test_jacobi_not_converged_flag():
    """A sweep cap of 1 on a non-diagonal matrix reports non-convergence (-1)."""
    A = g.make_a(g.MatrixSpec(m=200, n=10, kappa_b=100, kappa_d=10, seed=3))
    Mhi, Mlo = ref.gram_dd(A)
    *_, sweeps = ref.jacobi2_dd(Mhi, Mlo, max_sweeps=1)
    assert sweeps == -1


def test_not_spd_detected():
    """A rank-deficient A (duplicated column) gives lambda <= 0 or an SPD failure."""
    A = g.make_a(g.MatrixSpec(m=100, n=6, kappa_b=10, kappa_d=10, seed=4))
    A[:, 3] = A[:, 1]
    o = ref.svd(np.asfortranarray(A), want_kappa=False)
    Rh, Rl, info = ref.chol_dd(o.M_hi, o.M_lo)
    assert o.not_spd or info != 0 or o.sigma[-1] < 1e-25 * o.sigma[0]


def test_chol_dd():
    """R^T R equals M to dd rounding (checked in exact rationals), R upper triangular."""
    A = g.make_a(g.MatrixSpec(m=300, n=8, kappa_b=30, kappa_d=1e6, seed=41))
    Mhi, Mlo = ref.gram_dd(A)
    Rh, Rl, info = ref.chol_dd(Mhi, Mlo)
    assert info == 0
    assert np.all(np.tril(Rh, -1) == 0)
    n = 8
    for i in range(n):
        for j in range(i, n):
            s = sum((_fr(Rh[k, i]) + _fr(Rl[k, i])) * (_fr(Rh[k, j]) + _fr(Rl[k, j]))
                    for k in range(n))
            mij = _fr(Mhi[i, j]) + _fr(Mlo[i, j])
            bound = 8 * n * U_DD * float(np.abs(Rh[:, i]) @ np.abs(Rh[:, j]))
            assert float(abs(s - mij)) <= bound


def test_kappa_b_matches_generator():
    """The generator's B has singular values exactly Sigma (up to W1's rounding): kappa(B) as set."""
    for kb, mode in ((10.0, 3), (1e3, 5), (100.0, 2)):
        A = g.make_a(g.MatrixSpec(m=2000, n=16, kappa_b=kb, kappa_d=1e8, mode_b=mode, seed=9))
        Mhi, Mlo = ref.gram_dd(A)
        sig = g.latm1(mode, kb, 16, g.rng_for(9))  # mode 5 does not force its endpoints
        realised = sig.max() / sig.min()
        assert abs(ref.kappa_b(Mhi, Mlo) - realised) <= 1e-11 * realised


def test_orth_and_resid_closed_forms():
    """||U^T U - I||_F of Q diag(1 + delta) and ||Q diag(ds) W^T||_F / ||A||_F are known in closed form."""
    E = g.hadamard_exact(4, 8, block_exps=[0, 3], seed=8)
    assert ref.orth(E.U) == 0.0
    delta = np.array([1, -2, 3, 0, 0, 5, -1, 2]) * 2.0 ** -40
    U2 = E.U * (1 + delta)
    want = np.sqrt(np.sum((2 * delta + delta ** 2) ** 2))
    assert abs(ref.orth(U2) - want) <= 1e-6 * want
    assert ref.resid(E.A, E.U, E.sigma, E.V) == 0.0
    ds = np.array([0, 1, 0, 0, -2, 0, 0, 1]) * 2.0 ** -30
    got = ref.resid(E.A, E.U, E.sigma + ds, E.V)
    want = np.sqrt(np.sum(ds ** 2)) / np.sqrt(np.sum(E.sigma ** 2))
    assert abs(got - want) <= 1e-10 * want


def test_cross_check_lapack_dgejsv():
    """The paper's own reference (one-sided Jacobi SVD in double, DGEJSV) agrees to ~u_64 kappa(B)."""
    A = g.make_a(g.MatrixSpec(m=1024, n=64, kappa_b=100, kappa_d=1e8, mode_b=3, mode_d=5,
                              seed=13, dtype="f32"))
    o = ref.svd(A)
    sva, u, v, work, iwork, info = lapack.dgejsv(A.astype(np.float64), joba=1, jobu=3, jobv=3)
    assert info == 0
    sig = np.sort(sva * (work[0] / work[1]))[::-1]
    err = ref.sigma_rel_err(sig, o)
    assert err.max() <= 50 * 64 * U64 * o.kappa_b


def test_negative_control_tracks_kappa_b_not_kappa_a():
    """Paper Sec. 1 / Remark 1: with a FP64 Gram, Jacobi's sigma error is flat in kappa(D) while a
    QR-type eigensolver (numpy eigh, LAPACK syevd) degrades as kappa(D) grows (columns shuffled:
    a QR-type solver can keep relative accuracy on a matrix graded along its diagonal)."""
    errs_j, errs_e = [], []
    for kd in (1.0, 1e4, 1e8):
        A = g.make_a(g.MatrixSpec(m=1024, n=32, kappa_b=10, kappa_d=kd, mode_b=3, mode_d=3,
                                  seed=17, dtype="f32", shuffle=True))
        o = ref.svd(A)
        M64 = o.M_hi  # Gram rounded to FP64: u_h = u_64
        lh, ll, Vh, Vl, _ = ref.jacobi2_dd(M64, np.zeros_like(M64))
        sj = np.sort(np.sqrt(lh))[::-1]
        se = np.sort(np.sqrt(np.abs(np.linalg.eigvalsh(M64))))[::-1]
        errs_j.append(ref.sigma_rel_err(sj, o).max())
        errs_e.append(ref.sigma_rel_err(se, o).max())
    assert max(errs_j) < 1e-12
    assert errs_e[-1] > 1e3 * max(errs_j)

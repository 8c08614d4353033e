"""The synthetic inputs follow the paper's test-matrix recipe (Sec. 4.1, Tables 2-3)."""
import numpy as np
import pytest

from gen import matrices as g


def test_latm1_modes_table3():
    n, k = 6, 1e4
    rng = g.rng_for(0)
    assert np.array_equal(g.latm1(1, k, n, rng), np.array([1.0] + [1e-4] * 5))
    assert np.array_equal(g.latm1(2, k, n, rng), np.array([1.0] * 5 + [1e-4]))
    d3 = g.latm1(3, k, n, rng)
    assert np.allclose(d3, k ** (-np.arange(n) / (n - 1)), rtol=1e-15)
    d4 = g.latm1(4, k, n, rng)
    assert np.allclose(d4, 1 - np.arange(n) / (n - 1) * (1 - 1 / k), rtol=1e-15)
    d5 = g.latm1(5, k, 1000, rng)
    assert np.all((d5 > 1 / k) & (d5 < 1))
    # logarithms uniform on (log 1/k, 0): mean near half the range
    assert abs(np.mean(np.log10(d5)) + 2.0) < 0.15


def test_unit_columns_keeps_singular_values():
    rng = g.rng_for(3)
    sig = g.latm1(3, 1e3, 12, rng)
    sig *= np.sqrt(12 / np.sum(sig ** 2))
    W2 = np.linalg.qr(rng.standard_normal((12, 12)))[0]
    X = g.unit_columns(sig[:, None] * W2)
    assert np.allclose(np.linalg.norm(X, axis=0), 1.0, atol=1e-15)
    sv = np.linalg.svd(X, compute_uv=False)
    assert np.allclose(np.sort(sv), np.sort(sig), rtol=1e-12)


def test_seed_reproducible_and_layout():
    spec = g.MatrixSpec(m=300, n=7, kappa_b=10, kappa_d=1e5, seed=42, shuffle=True)
    A1, A2 = g.make_a(spec), g.make_a(spec)
    assert np.array_equal(A1, A2)
    assert A1.flags.f_contiguous and A1.dtype == np.float64
    spec.dtype = "f32"
    A3 = g.make_a(spec)
    assert A3.dtype == np.float32 and A3.flags.f_contiguous
    assert np.array_equal(A3, A1.astype(np.float32))


def test_column_norms_are_d():
    """With W1 orthonormal and B of unit columns, ||a_j|| equals d_j (MODE 3, kappa(D))."""
    spec = g.MatrixSpec(m=500, n=9, kappa_b=50, kappa_d=1e6, seed=5)
    A = g.make_a(spec)
    d = np.linalg.norm(A, axis=0)
    assert np.allclose(d, 1e6 ** (-np.arange(9) / 8), rtol=1e-13)


@pytest.mark.parametrize("k,n", [(3, 8), (5, 16)])
def test_hadamard_exact_is_exact(k, n):
    E = g.hadamard_exact(k, n)
    A = E.A
    # U diag(sigma) V^T reproduces the stored A exactly, U and V orthonormal exactly
    assert np.array_equal((E.U * E.sigma) @ E.V.T, A)
    assert np.array_equal(E.U.T @ E.U, np.eye(n))
    assert np.array_equal(E.V.T @ E.V, np.eye(n))


def test_batch_specs_ranges():
    specs = g.batch_specs(64)
    assert all(10_000 <= s.m <= 200_000 for s in specs)
    assert {s.n for s in specs} <= {16, 32, 48, 64, 96}
    assert all(10 <= s.kappa_b <= 1e3 and 1e4 <= s.kappa_d <= 1e12 for s in specs)

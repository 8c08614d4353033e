"""Parity of the operand-split Gram (integer slices on the int8 matrix cores) with the oracle.

Error model of the split form.  Rows are processed in slabs (the same slab
plan as the library: about m / 1024 rows, rounded up to 64, unless a slab
height is given); within a slab the exponent E_j of column j never exceeds
ilogb(slab max of column j) + 6.  Each entry is cut to S balanced base-256
digits with a tail below (128 / 255) 2^(E - 8 S) + 2^(E - 96), and digit pairs
r + t > S + 1 are dropped (sum below S 2^(E_i + E_j - 8 S - 2)), so a row adds
an error of at most (S + 3) 2^(E_i + E_j - 8 S), plus double-double rounding.
"""
import numpy as np
import pytest

from gen import matrices as g
from oracle import ref
from tests.helpers import U_DD, check_thin, say, sigma_tol, to_dev, to_np, u_of

pytestmark = pytest.mark.gpu


def _slab_rows(m):
    rps = -(-m // 1024)
    return max(64, -(-rps // 64) * 64)


def _split_bound(A, S):
    A = np.abs(A.astype(np.float64))
    m, n = A.shape
    rps = _slab_rows(m)
    pad = (-m) % rps
    Ap = np.vstack([A, np.zeros((pad, n))])
    smax = Ap.reshape(-1, rps, n).max(axis=1)  # slab column maxima
    with np.errstate(divide="ignore"):
        e = np.where(smax > 0, np.floor(np.log2(np.where(smax > 0, smax, 1.0))) + 6, -np.inf)
    p2 = np.where(np.isfinite(e), 2.0 ** e, 0.0)  # 2^E per slab and column
    return (S + 3) * 2.0 ** (-8 * S) * rps * (p2.T @ p2)


def _gram_split(A, S):
    import ctypes

    import torch

    import paper_2603_11953_amd as gs
    w = gs.GSVD_F64 if A.dtype == np.float64 else gs.GSVD_F32
    m, n = A.shape
    o = gs.opts(w, gs.GSVD_GRAM_SPLIT, n_slices=S, slab_rows=_slab_rows(m))
    dA = to_dev(A)
    Mhi = gs.colmajor_empty(n, n, torch.float64, dA.device)
    Mlo = gs.colmajor_empty(n, n, torch.float64, dA.device)
    work = gs.workspace(gs.gsvd_gram_workspace_size(m, n, ctypes.byref(o)), dA.device)
    rc = gs.gsvd_gram(m, n, dA.data_ptr(), m, Mhi.data_ptr(), Mlo.data_ptr(), n, work.data_ptr(),
                      work.numel(), ctypes.byref(o), gs._stream(None))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return to_np(Mhi), to_np(Mlo)


@pytest.mark.parametrize("m,n,dt,S", [
    (1, 1, "f64", 10), (63, 5, "f64", 10), (65, 17, "f64", 10), (5000, 20, "f64", 10),
    (100_003, 64, "f64", 10), (3001, 96, "f64", 10), (2000, 64, "f64", 4), (777, 33, "f64", 12),
    (1, 1, "f32", 6), (5000, 20, "f32", 6), (50_001, 128, "f32", 6), (4097, 100, "f32", 3),
])
def test_split_gram_parity(m, n, dt, S):
    spec = g.MatrixSpec(m=max(m, n), n=n, kappa_b=30, kappa_d=1e6, mode_b=3, mode_d=5,
                        seed=3000 + m + n, dtype=dt, shuffle=True, w1="gauss")
    A = g.make_a(spec)
    say("split gram", m, n, dt, S)
    Mh, Ml = _gram_split(A, S)
    oh, ol = ref.gram_dd(A)
    diff = np.abs((Mh - oh) + (Ml - ol)) if dt == "f64" else np.abs((Mh - oh) - ol)
    absA = np.abs(A.astype(np.float64))
    rnd = (4 * A.shape[0] * (U_DD if dt == "f64" else 2.0 ** -53)) * (absA.T @ absA)
    bound = _split_bound(A, S) + rnd
    assert np.array_equal(Mh, Mh.T)
    assert np.all(diff <= bound + 1e-300), float(np.max(diff / np.maximum(bound, 1e-300)))


def test_split_gram_exact_on_short_integer_entries():
    """Entries that fit in the first few digits are cut without a tail, and when every pair of
    non-zero digits is kept the Gram of such a matrix must be exact."""
    rng = np.random.default_rng(5)
    # 20-bit integers times 2^c: a column's exponent is at most c + 25, so the 96-bit
    # fixed-point value of every entry has its low 71 bits zero and only digits 1..4
    # can be non-zero; S = 7 keeps every pair r + t <= 8, i.e. all 16 pairs of them
    A = rng.integers(-(2 ** 20), 2 ** 20, size=(3000, 24)).astype(np.float64)
    A *= 2.0 ** rng.integers(-30, 30, size=24)[None, :]
    A = np.asfortranarray(A)
    say("split gram exact")
    Mh, Ml = _gram_split(A, 7)
    oh, ol = ref.gram_dd(A)
    assert np.array_equal(Mh, oh) and np.array_equal(Ml, ol)


def test_split_gram_deterministic():
    A = g.make_a(g.MatrixSpec(m=200_001, n=64, kappa_b=100, kappa_d=1e10, seed=6, shuffle=True,
                              w1="gauss"))
    say("split gram determinism")
    r1 = _gram_split(A, 10)
    r2 = _gram_split(A, 10)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


def _thin_split(A, S=0):
    import paper_2603_11953_amd as gs
    import torch
    S_, V, U, info = gs.thin(to_dev(A), gram=gs.GSVD_GRAM_SPLIT, n_slices=S)
    torch.cuda.synchronize()
    return to_np(S_), to_np(V), to_np(U), int(info.item())


@pytest.mark.parametrize("spec", [
    g.MatrixSpec(m=100_000, n=64, kappa_b=100, kappa_d=1e10, mode_b=3, mode_d=3, seed=11955,
                 shuffle=True),
    g.MatrixSpec(m=50_000, n=128, kappa_b=100, kappa_d=1e6, mode_b=3, mode_d=3, seed=11956,
                 dtype="f32"),
    g.spec_small_f64(),
], ids=["m1e5n64-f64", "m5e4n128-f32", "m2000n20-f64"])
def test_thin_split_end_to_end(spec):
    """With the default slice counts the split form meets the same tolerances as the plain one."""
    A = g.make_a(spec)
    o = ref.svd(A)
    say("thin split", spec.m, spec.n, spec.dtype)
    S, V, Uo, info = _thin_split(A)
    assert info == 0
    rep = check_thin(A, S, V, Uo, o, label=str(spec))
    assert rep["u_orth_meets_50nu"], rep


def test_target_rel_err_raises_the_slice_count_and_is_met():
    """The requested sigma accuracy sets the split Gram's slice count: each tighter target
    gives at least as many slices, and every run meets its own target (and the
    tolerance 50 n u kappa(B)) against the oracle."""
    import paper_2603_11953_amd as gs
    A = g.make_a(g.MatrixSpec(m=100_000, n=64, kappa_b=100, kappa_d=1e10, mode_b=3, mode_d=3,
                              seed=12_345, shuffle=True, w1="gauss"))
    o = ref.svd(A)
    prev = 0
    for target in (1e-5, 1e-9, 1e-12):
        S_used = gs.gram_config(A.shape[0], 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT,
                                target_rel_err=target, kappa_b=100)["n_slices"]
        assert S_used >= prev
        prev = S_used
        say("target", target, "S", S_used)
        import torch
        S, V, U, info = gs.thin(to_dev(A), gram=gs.GSVD_GRAM_SPLIT, target_rel_err=target,
                                kappa_b=100)
        torch.cuda.synchronize()
        assert (int(info.item()) & 0xFF) == 0
        err = ref.sigma_rel_err(to_np(S), o).max()
        assert err <= target, (target, S_used, err)
        assert err <= sigma_tol(64, 2.0 ** -53, o.kappa_b)
    assert prev > gs.gram_config(A.shape[0], 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT,
                                 target_rel_err=1e-5, kappa_b=100)["n_slices"]

"""Parity of the wide path (n > 128 for the Gram and U kernels, n > 96 for the
FP64 eigensolver stage) with the CPU oracle, through the C-ABI.

The wide kernels are a different design from the one-workgroup ones: 64-column
panel pairs for the Gram, 256 x 128 tiles with W staged in k-chunks for U, and
Algorithm 2 spread over launches (blocked dd Cholesky, block one-sided Jacobi)
for the eigensolver.  Sizes span several panels with ragged tails.
"""
import numpy as np
import pytest

from gen import matrices as g
from oracle import ref
from tests.helpers import U_DD, check_thin, say, sigma_tol, to_dev, to_np, u_of

pytestmark = pytest.mark.gpu


def _sync():
    import torch
    torch.cuda.synchronize()


def _thin(A, **kw):
    import paper_2603_11953_amd as gs
    S, V, U, info = gs.thin(to_dev(A), **kw)
    _sync()
    return to_np(S), to_np(V), (to_np(U) if U is not None else None), int(info.item())


@pytest.mark.parametrize("m,n,dt", [(3000, 129, "f64"), (1001, 200, "f64"), (20_011, 512, "f64"),
                                    (777, 300, "f64"), (5000, 257, "f32"), (640, 512, "f32")])
def test_wide_gram_parity(m, n, dt):
    """Panel-pair Gram vs the dd oracle within eq. (ATA): |dM| <= eps |A|^T |A|."""
    import paper_2603_11953_amd as gs
    A = g.make_a(g.MatrixSpec(m=m, n=n, kappa_b=30, kappa_d=1e6, mode_b=3, mode_d=5,
                              seed=3000 + m + n, dtype=dt, shuffle=True, w1="gauss"))
    say("wide gram", m, n, dt)
    Mhi_d, Mlo_d = gs.gram(to_dev(A))
    _sync()
    Mh, Ml = to_np(Mhi_d), to_np(Mlo_d)
    oh, ol = ref.gram_dd(A)
    absA = np.abs(A.astype(np.float64))
    scale = absA.T @ absA
    if dt == "f64":
        diff = np.abs((Mh - oh) + (Ml - ol))
        eps = 4 * m * U_DD
    else:
        diff = np.abs((Mh - oh) - ol)
        eps = 2 * m * 2.0 ** -53
    assert np.array_equal(Mh, Mh.T) and np.array_equal(Ml, Ml.T)
    assert np.all(diff <= eps * scale + 1e-300), float(np.max(diff / np.maximum(scale, 1e-300)))


def test_wide_gram_deterministic():
    import paper_2603_11953_amd as gs
    A = g.make_a(g.MatrixSpec(m=50_001, n=200, kappa_b=100, kappa_d=1e10, seed=6, shuffle=True,
                              w1="gauss"))
    say("wide gram determinism")
    M1 = [to_np(t) for t in gs.gram(to_dev(A))]
    M2 = [to_np(t) for t in gs.gram(to_dev(A))]
    _sync()
    assert np.array_equal(M1[0], M2[0]) and np.array_equal(M1[1], M2[1])


@pytest.mark.parametrize("m,n,dt", [(1000, 129, "f64"), (5003, 512, "f64"), (257, 257, "f64"),
                                    (777, 300, "f32"), (4099, 512, "f32")])
def test_wide_u_recover_parity(m, n, dt):
    """U = A W within eq. (AV-0): |dU| <= (n + 2) u |A| |W|, against the dd product."""
    import paper_2603_11953_amd as gs
    rng = np.random.default_rng(m + n)
    npdt = np.float64 if dt == "f64" else np.float32
    A = np.asfortranarray(rng.standard_normal((m, n)).astype(npdt))
    Wm = np.asfortranarray((rng.standard_normal((n, n)) * np.logspace(0, 6, n)).astype(npdt))
    say("wide u_recover", m, n, dt)
    Ud = gs.u_recover(to_dev(A), to_dev(Wm))
    _sync()
    Ug = to_np(Ud).astype(np.float64)
    Uh, Ul = ref.u_rows_dd(A, Wm.astype(np.float64), np.zeros((n, n)), np.ones(n), np.zeros(n))
    bound = (n + 2) * u_of(A) * (np.abs(A.astype(np.float64)) @ np.abs(Wm.astype(np.float64)))
    assert np.all(np.abs((Ug - Uh) - Ul) <= bound)


@pytest.mark.parametrize("n", [97, 128, 160, 257])
def test_wide_eig_parity(n):
    """Multi-launch Algorithm 2 on the oracle's M_h: sigma within 50 n u kappa(B), V orthogonal
    and equal to the oracle's eigenvectors (same sign rule), W == fl(V / S) bitwise."""
    import torch

    import paper_2603_11953_amd as gs
    A = g.make_a(g.MatrixSpec(m=4 * n + 50, n=n, kappa_b=100, kappa_d=1e8, mode_b=3, mode_d=3,
                              seed=200 + n, shuffle=True))
    o = ref.svd(A)
    say("wide eig", n)
    S, V, W, info = gs.eig(to_dev(o.M_hi), to_dev(o.M_lo), gs.GSVD_F64)
    _sync()
    assert int(info.item()) == 0
    S, V, W = to_np(S), to_np(V), to_np(W)
    u = 2.0 ** -53
    err = ref.sigma_rel_err(S, o)
    assert err.max() <= sigma_tol(n, u, o.kappa_b), err.max()
    assert np.all(np.diff(S) <= 0)
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 50 * n * u
    assert np.abs(V - o.V_hi).max() <= 1e3 * n * u * o.kappa_b
    idx = np.argmax(np.abs(V), axis=0)
    assert np.all(V[idx, np.arange(n)] > 0)
    Wref = (torch.from_numpy(np.ascontiguousarray(V)) / torch.from_numpy(S)[None, :]).numpy()
    assert np.array_equal(W, Wref)


@pytest.mark.parametrize("spec", [
    g.MatrixSpec(m=30_000, n=200, kappa_b=100, kappa_d=1e10, mode_b=3, mode_d=3, seed=11,
                 shuffle=True),
    g.MatrixSpec(m=9_001, n=131, kappa_b=1e3, kappa_d=1e12, mode_b=3, mode_d=3, seed=12,
                 shuffle=True, w1="gauss"),
], ids=["m3e4n200-f64", "m9001n131-f64-kb1e3"])
def test_wide_thin_end_to_end(spec):
    """sigma <= 50 n u kappa(B); ||V^T V - I||, ||A - U S V^T|| / ||A|| <= 50 n u;
    ||U^T U - I|| within Remark 2's bound; U on sampled rows against the oracle's."""
    A = g.make_a(spec)
    o = ref.svd(A)
    say("wide thin", spec.m, spec.n)
    S, V, Uo, info = _thin(A)
    assert info == 0
    rep = check_thin(A, S, V, Uo, o, label=str(spec))
    if o.kappa_b <= 100.5:
        assert rep["u_orth_meets_50nu"], rep
    rows = np.unique(np.r_[0, spec.m - 1, np.random.default_rng(1).integers(0, spec.m, 300)])
    Uh, Ul = ref.u_rows_dd(A, o.V_hi, o.V_lo, o.sigma_hi, o.sigma_lo, rows=rows)
    du = np.abs((Uo[rows] - Uh) - Ul)
    assert du.max() <= 1e3 * spec.n * u_of(A) * o.kappa_b, (du.max(), rep)


def test_wide_exact_spectrum_n512():
    """Hadamard construction at n = 512 (m = 1024): exact sigma, kappa(B) < 8 while
    kappa(A) ~ 2^38; the GPU sigma error stays at 50 n u kappa(B).  Blocks share
    exponents, so sigma values repeat and V is not unique: V and U are checked by
    orthogonality and the residual."""
    exps = [int(36 * b / 127) for b in range(128)]
    E = g.hadamard_exact(5, 512, block_exps=exps, dtype="f64", seed=9, col_perm=True)
    say("wide hadamard 512")
    S, V, Uo, info = _thin(E.A)
    assert (info & 0xFF) == 0, info  # repeated sigma: the dd stage may flag the tied pairs
    u = 2.0 ** -53
    err = np.abs(S - E.sigma) / E.sigma
    assert err.max() <= sigma_tol(512, u, E.kappa_b), err.max()
    assert np.linalg.norm(V.T @ V - np.eye(512)) <= 50 * 512 * u
    assert ref.orth(Uo) <= 50 * 512 * u * E.kappa_b
    assert ref.resid(E.A, Uo, S, V) <= 50 * 512 * u


@pytest.mark.parametrize("form", ["plain", "split"])
def test_wide_info_codes(form):
    """Zero column -> 1 (M_h not positive definite), NaN or Inf -> 3 (also through the split
    Gram, which flags them), one sweep -> 2."""
    import paper_2603_11953_amd as gs
    gram = gs.GSVD_GRAM_SPLIT if form == "split" else gs.GSVD_GRAM_PLAIN
    A = g.make_a(g.MatrixSpec(m=2000, n=160, kappa_b=100, kappa_d=1e4, seed=13, shuffle=True))
    Z = A.copy(order="F")
    Z[:, 77] = 0.0
    say("wide info zero column", form)
    assert _thin(Z, gram=gram)[3] == 1
    for bad in (np.nan, np.inf):
        Nn = A.copy(order="F")
        Nn[5, 140] = bad
        say("wide info nonfinite", bad, form)
        assert _thin(Nn, gram=gram)[3] == 3
    say("wide info max_sweeps=1", form)
    assert _thin(A, max_sweeps=1, gram=gram)[3] == 2


# ------------------------------------------------------------------ wide split Gram

def _wide_split_bound(A, S):
    """Error model of the wide split form: exponents per 2048-row slab,
    E_j = ilogb(slab max of column j) + 4; each row adds at most (S + 3) 2^(E_i + E_j - 8 S)."""
    A = np.abs(A.astype(np.float64))
    m, n = A.shape
    rps = 2048
    Ap = np.vstack([A, np.zeros(((-m) % rps, n))])
    smax = Ap.reshape(-1, rps, n).max(axis=1)
    with np.errstate(divide="ignore"):
        e = np.where(smax > 0, np.floor(np.log2(np.where(smax > 0, smax, 1.0))) + 4, -np.inf)
    p2 = np.where(np.isfinite(e), 2.0 ** e, 0.0)
    return (S + 3) * 2.0 ** (-8 * S) * rps * (p2.T @ p2)


def _gram_split_wide(A, S, rows_cap=0):
    import ctypes

    import torch

    import paper_2603_11953_amd as gs
    w = gs.GSVD_F64 if A.dtype == np.float64 else gs.GSVD_F32
    m, n = A.shape
    o = gs.opts(w, gs.GSVD_GRAM_SPLIT, n_slices=S, slab_rows=rows_cap)
    dA = to_dev(A)
    Mhi = gs.colmajor_empty(n, n, torch.float64, dA.device)
    Mlo = gs.colmajor_empty(n, n, torch.float64, dA.device)
    work = gs.workspace(gs.gsvd_gram_workspace_size(m, n, ctypes.byref(o)), dA.device)
    rc = gs.gsvd_gram(m, n, dA.data_ptr(), m, Mhi.data_ptr(), Mlo.data_ptr(), n, work.data_ptr(),
                      work.numel(), ctypes.byref(o), gs._stream(None))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return to_np(Mhi), to_np(Mlo)


@pytest.mark.parametrize("m,n,dt,S,cap", [
    (3000, 129, "f64", 10, 0), (20_011, 512, "f64", 9, 0), (9001, 200, "f64", 4, 0),
    (300, 300, "f64", 12, 0), (3 * 8192 + 123, 150, "f64", 9, 8192),
    (5000, 257, "f32", 6, 0), (777, 300, "f32", 3, 0), (2 * 8192 + 5, 190, "f32", 8, 8192),
])
def test_wide_split_gram_parity(m, n, dt, S, cap):
    """Panel-pair split Gram vs the dd oracle within the digit error model plus dd rounding;
    cap > 0 forces several passes over the digit planes."""
    A = g.make_a(g.MatrixSpec(m=m, n=n, kappa_b=30, kappa_d=1e6, mode_b=3, mode_d=5,
                              seed=4000 + m + n, dtype=dt, shuffle=True, w1="gauss"))
    say("wide split gram", m, n, dt, S, cap)
    Mh, Ml = _gram_split_wide(A, S, cap)
    oh, ol = ref.gram_dd(A)
    diff = np.abs((Mh - oh) + (Ml - ol)) if dt == "f64" else np.abs((Mh - oh) - ol)
    absA = np.abs(A.astype(np.float64))
    rnd = (4 * m * (U_DD if dt == "f64" else 2.0 ** -53)) * (absA.T @ absA)
    bound = _wide_split_bound(A, S) + rnd
    assert np.array_equal(Mh, Mh.T)
    assert np.all(diff <= bound + 1e-300), float(np.max(diff / np.maximum(bound, 1e-300)))


def test_wide_split_gram_exact_on_short_integer_entries():
    """20-bit integers times 2^c: only the first three digits are non-zero, S = 7 keeps all
    their pairs, so the Gram must equal the oracle's bit for bit (checks the plane layout,
    the LDS swizzle and the exact combination)."""
    rng = np.random.default_rng(7)
    A = rng.integers(-(2 ** 20), 2 ** 20, size=(5000, 200)).astype(np.float64)
    A *= 2.0 ** rng.integers(-30, 30, size=200)[None, :]
    A = np.asfortranarray(A)
    say("wide split gram exact")
    Mh, Ml = _gram_split_wide(A, 7, 8192)
    oh, ol = ref.gram_dd(A)
    assert np.array_equal(Mh, oh) and np.array_equal(Ml, ol)


def test_wide_split_gram_deterministic_and_pass_invariant():
    """Same result run to run; with exponents fixed per slab the sums are exact per slab, so the
    pass structure only changes the dd rounding of the slot additions."""
    A = g.make_a(g.MatrixSpec(m=5 * 8192 + 77, n=160, kappa_b=100, kappa_d=1e10, seed=8,
                              shuffle=True, w1="gauss"))
    say("wide split gram determinism")
    r1 = _gram_split_wide(A, 9)
    r2 = _gram_split_wide(A, 9)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
    r3 = _gram_split_wide(A, 9, 8192)
    scale = np.abs(A).T @ np.abs(A)
    assert np.all(np.abs((r3[0] - r1[0]) + (r3[1] - r1[1])) <= 64 * U_DD * scale)


@pytest.mark.parametrize("spec", [
    g.MatrixSpec(m=30_000, n=200, kappa_b=100, kappa_d=1e10, mode_b=3, mode_d=3, seed=11,
                 shuffle=True),
    g.MatrixSpec(m=9_001, n=131, kappa_b=1e3, kappa_d=1e12, mode_b=3, mode_d=3, seed=12,
                 shuffle=True, w1="gauss"),
], ids=["m3e4n200-f64", "m9001n131-f64-kb1e3"])
def test_wide_thin_split_end_to_end(spec):
    """The split form with the default slice count meets the plain form's tolerances."""
    import paper_2603_11953_amd as gs
    A = g.make_a(spec)
    o = ref.svd(A)
    say("wide thin split", spec.m, spec.n)
    S, V, Uo, info = _thin(A, gram=gs.GSVD_GRAM_SPLIT)
    assert info == 0
    rep = check_thin(A, S, V, Uo, o, label=str(spec))
    if o.kappa_b <= 100.5:
        assert rep["u_orth_meets_50nu"], rep


def test_wide_split_exact_spectrum_n512():
    import paper_2603_11953_amd as gs
    exps = [int(36 * b / 127) for b in range(128)]
    E = g.hadamard_exact(5, 512, block_exps=exps, dtype="f64", seed=9, col_perm=True)
    say("wide split hadamard 512")
    S, V, Uo, info = _thin(E.A, gram=gs.GSVD_GRAM_SPLIT)
    assert (info & 0xFF) == 0, info  # repeated sigma: the dd stage may flag the tied pairs
    err = np.abs(S - E.sigma) / E.sigma
    assert err.max() <= sigma_tol(512, 2.0 ** -53, E.kappa_b), err.max()

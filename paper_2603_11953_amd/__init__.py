"""MI355X (gfx950) mixed precision Gram-based thin SVD.

Python face of ``libgsvd.so`` (the C-ABI in ``include/gsvd.h``).  The raw entry
points keep their C names (``gsvd_thin``, ``gsvd_gram``, ``gsvd_eig``,
``gsvd_u_recover`` ...) and take plain integers / device addresses; the
``thin``/``gram``/``eig``/``u_recover`` helpers marshal torch CUDA tensors
(torch supplies device memory and the current stream only -- every step of
the computation runs in the library's HIP kernels).

Importing the package never falls back to anything else: if the library is
missing the import raises, naming the build command.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

__all__ = [
    "GSVD_F32", "GSVD_F64", "GSVD_GRAM_AUTO", "GSVD_GRAM_PLAIN", "GSVD_GRAM_SPLIT",
    "GSVD_EIG_AUTO", "GSVD_EIG_JACOBI2", "GSVD_EIG_CHOL_JACOBI1", "GSVD_WANT_U", "GSVD_U_FP32_MFMA",
    "GSVD_MAX_N",
    "GsvdOpts", "GsvdError", "lib", "lib_path", "opts", "thin", "gram", "eig", "u_recover",
    "gsvd_opts_default", "gsvd_status_string", "gsvd_thin", "gsvd_thin_workspace_size",
    "gsvd_gram", "gsvd_gram_workspace_size", "gsvd_gram_config", "gram_config", "gsvd_eig", "gsvd_eig_workspace_size",
    "gsvd_u_recover", "gsvd_thin_batched", "gsvd_thin_batched_workspace_size", "thin_batched",
    "Batch", "gsvd_cholqr", "gsvd_cholqr_workspace_size", "cholqr", "gsvd_thin_noalloc", "gsvd_noalloc_max_bytes", "GSVD_ERR_SCRATCH", "GSVD_INFO_WARN_ASSUMPTION", "GSVD_INFO_WARN_REFINE",
]

GSVD_F32, GSVD_F64 = 0, 1
GSVD_GRAM_AUTO, GSVD_GRAM_PLAIN, GSVD_GRAM_SPLIT = 0, 1, 2
GSVD_EIG_AUTO, GSVD_EIG_JACOBI2, GSVD_EIG_CHOL_JACOBI1 = 0, 1, 2
GSVD_WANT_U = 1
GSVD_U_FP32_MFMA = 2
GSVD_MAX_N = 512
GSVD_ERR_SCRATCH = -102
GSVD_INFO_WARN_ASSUMPTION, GSVD_INFO_WARN_REFINE = 256, 512

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libgsvd.so")


class GsvdOpts(ctypes.Structure):
    _fields_ = [
        ("working", ctypes.c_int),
        ("gram", ctypes.c_int),
        ("eig", ctypes.c_int),
        ("n_slices", ctypes.c_int),
        ("jacobi_tol", ctypes.c_double),
        ("max_sweeps", ctypes.c_int),
        ("flags", ctypes.c_uint),
        ("slab_rows", ctypes.c_int64),
        ("target_rel_err", ctypes.c_double),
        ("kappa_b", ctypes.c_double),
    ]


class GsvdError(RuntimeError):
    pass


def _load() -> ctypes.CDLL:
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
    # first makes libgsvd.so bind to that same runtime, so device pointers and
    # stream handles from torch are valid in the library.  Loading the library
    # first would pull in a second HIP runtime from /opt/rocm.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover -- the C-ABI itself does not need torch
        pass
    if not os.path.exists(lib_path):
        raise ImportError(
            f"{lib_path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
            " (or python paper_2603_11953_amd/build.py)")
    L = ctypes.CDLL(lib_path)
    i64, vp, sz, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    op = ctypes.POINTER(GsvdOpts)
    L.gsvd_opts_default.argtypes = [op, ci]
    L.gsvd_opts_default.restype = None
    L.gsvd_status_string.argtypes = [ci]
    L.gsvd_status_string.restype = ctypes.c_char_p
    L.gsvd_thin_workspace_size.argtypes = [i64, i64, op]
    L.gsvd_thin_workspace_size.restype = sz
    L.gsvd_thin.argtypes = [i64, i64, vp, i64, vp, vp, i64, vp, i64, vp, sz, vp, op, vp]
    L.gsvd_thin.restype = ci
    L.gsvd_gram_workspace_size.argtypes = [i64, i64, op]
    L.gsvd_gram_workspace_size.restype = sz
    L.gsvd_gram_config.argtypes = [i64, i64, op, vp, vp, vp]
    L.gsvd_gram_config.restype = ci
    L.gsvd_gram.argtypes = [i64, i64, vp, i64, vp, vp, i64, vp, sz, op, vp]
    L.gsvd_gram.restype = ci
    L.gsvd_eig_workspace_size.argtypes = [i64, op]
    L.gsvd_eig_workspace_size.restype = sz
    L.gsvd_eig.argtypes = [i64, vp, vp, i64, vp, vp, i64, vp, i64, vp, vp, sz, op, vp]
    L.gsvd_eig.restype = ci
    L.gsvd_u_recover.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, op, vp]
    L.gsvd_u_recover.restype = ci
    L.gsvd_thin_batched_workspace_size.argtypes = [ci, vp, vp, op]
    L.gsvd_thin_batched_workspace_size.restype = sz
    L.gsvd_thin_batched.argtypes = [ci, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, op, vp]
    L.gsvd_thin_batched.restype = ci
    L.gsvd_cholqr_workspace_size.argtypes = [i64, i64, op]
    L.gsvd_cholqr_workspace_size.restype = sz
    L.gsvd_cholqr.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, vp, sz, vp, op, vp]
    L.gsvd_cholqr.restype = ci
    L.gsvd_noalloc_max_bytes.argtypes = []
    L.gsvd_noalloc_max_bytes.restype = sz
    L.gsvd_thin_noalloc.argtypes = [i64, i64, vp, i64, vp, vp, i64, vp, i64, vp, op, vp]
    L.gsvd_thin_noalloc.restype = ci
    return L


lib = _load()

# raw C entry points, same names as in gsvd.h
gsvd_opts_default = lib.gsvd_opts_default
gsvd_thin = lib.gsvd_thin
gsvd_thin_workspace_size = lib.gsvd_thin_workspace_size
gsvd_gram = lib.gsvd_gram
gsvd_gram_workspace_size = lib.gsvd_gram_workspace_size
gsvd_gram_config = lib.gsvd_gram_config
gsvd_eig = lib.gsvd_eig
gsvd_eig_workspace_size = lib.gsvd_eig_workspace_size
gsvd_u_recover = lib.gsvd_u_recover
gsvd_thin_batched = lib.gsvd_thin_batched
gsvd_thin_batched_workspace_size = lib.gsvd_thin_batched_workspace_size
gsvd_thin_noalloc = lib.gsvd_thin_noalloc
gsvd_cholqr = lib.gsvd_cholqr
gsvd_cholqr_workspace_size = lib.gsvd_cholqr_workspace_size
gsvd_noalloc_max_bytes = lib.gsvd_noalloc_max_bytes


def gsvd_status_string(code: int) -> str:
    return lib.gsvd_status_string(int(code)).decode()


def gram_config(m: int, n: int, working: int = GSVD_F64, gram: int = GSVD_GRAM_AUTO,
                **kw) -> dict:
    """The Gram launch shape the library resolves for (m, n) and these options:
    slab height, slab count and (split form) int8 slice count; n_slices 0 means the
    plain form (also what GSVD_GRAM_AUTO resolved to)."""
    o = opts(working, gram, **kw)
    rows, slabs, sl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
    rc = lib.gsvd_gram_config(m, n, ctypes.byref(o), ctypes.addressof(rows),
                              ctypes.addressof(slabs), ctypes.addressof(sl))
    _check(rc, "gsvd_gram_config")
    return {"slab_rows": rows.value, "n_slabs": slabs.value, "n_slices": sl.value}


def opts(working: int, gram: int = GSVD_GRAM_AUTO, eig: int = GSVD_EIG_AUTO, *,
         want_u: bool = True, jacobi_tol: float = 0.0, max_sweeps: int = 0,
         n_slices: int = 0, slab_rows: int = 0, target_rel_err: float = 0.0,
         kappa_b: float = 0.0, u_fp32_mfma: bool = False) -> GsvdOpts:
    o = GsvdOpts()
    lib.gsvd_opts_default(ctypes.byref(o), int(working))
    o.gram, o.eig, o.n_slices = int(gram), int(eig), int(n_slices)
    o.jacobi_tol, o.max_sweeps = float(jacobi_tol), int(max_sweeps)
    o.flags = (GSVD_WANT_U if want_u else 0) | (GSVD_U_FP32_MFMA if u_fp32_mfma else 0)
    o.slab_rows = int(slab_rows)
    o.target_rel_err, o.kappa_b = float(target_rel_err), float(kappa_b)
    return o


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise GsvdError(f"{what} returned {rc}: {gsvd_status_string(rc)}")


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch  # noqa: WPS433 -- torch is only the memory/stream provider
    return torch


def _working_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return GSVD_F64
    if t.dtype == torch.float32:
        return GSVD_F32
    raise TypeError("A must be float32 or float64")


def colmajor_empty(rows: int, cols: int, dtype, device):
    """A (rows x cols) tensor with column-major strides (1, rows)."""
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("matrices must be column-major: stride (1, ld); use A.t().contiguous().t()")
    return max(int(t.stride(1)), int(t.shape[0]), 1)


def _stream(stream) -> ctypes.c_void_p:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(int(s.cuda_stream))


def _on(stream):
    """Allocate on the stream the library will run on: torch's caching allocator
    then hands the blocks (workspace, outputs, info) to later work only in that
    stream's order, after the library's kernels."""
    torch = _torch()
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def thin(A, *, gram: int = GSVD_GRAM_AUTO, eig: int = GSVD_EIG_AUTO, want_u: bool = True,
         jacobi_tol: float = 0.0, max_sweeps: int = 0, n_slices: int = 0, slab_rows: int = 0,
         target_rel_err: float = 0.0, kappa_b: float = 0.0, u_fp32_mfma: bool = False,
         work=None, stream=None):
    """Thin SVD of a column-major CUDA tensor A (m x n).  Returns (S, V, U, info) tensors;
    info is a one-element int32 device tensor (check it after synchronising)."""
    torch = _torch()
    w = _working_of(A)
    m, n = int(A.shape[0]), int(A.shape[1])
    lda = _ld(A)
    o = opts(w, gram, eig, want_u=want_u, jacobi_tol=jacobi_tol, max_sweeps=max_sweeps,
             n_slices=n_slices, slab_rows=slab_rows, target_rel_err=target_rel_err,
             kappa_b=kappa_b, u_fp32_mfma=u_fp32_mfma)
    with _on(stream):
        S = torch.empty(n, dtype=A.dtype, device=A.device)
        V = colmajor_empty(n, n, A.dtype, A.device)
        U = colmajor_empty(m, n, A.dtype, A.device) if want_u else None
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
        need = lib.gsvd_thin_workspace_size(m, n, ctypes.byref(o))
        if work is None:
            work = workspace(need, A.device)
        rc = lib.gsvd_thin(m, n, A.data_ptr(), lda, S.data_ptr(), V.data_ptr(), n,
                           U.data_ptr() if want_u else None, m, work.data_ptr(), work.numel(),
                           info.data_ptr(), ctypes.byref(o), _stream(stream))
    _check(rc, "gsvd_thin")
    return S, V, U, info


def cholqr(A, *, gram: int = GSVD_GRAM_AUTO, n_slices: int = 0, target_rel_err: float = 0.0,
           kappa_b: float = 0.0, stream=None):
    """Mixed precision Cholesky QR of a column-major CUDA tensor A (m x n): returns
    (Q, R, info) with Q m x n and R n x n upper triangular in A's precision."""
    torch = _torch()
    w = _working_of(A)
    m, n = int(A.shape[0]), int(A.shape[1])
    lda = _ld(A)
    o = opts(w, gram, n_slices=n_slices, target_rel_err=target_rel_err, kappa_b=kappa_b)
    with _on(stream):
        Q = colmajor_empty(m, n, A.dtype, A.device)
        R = colmajor_empty(n, n, A.dtype, A.device)
        info = torch.full((1,), -1, dtype=torch.int32, device=A.device)
        need = lib.gsvd_cholqr_workspace_size(m, n, ctypes.byref(o))
        work = workspace(need, A.device)
        rc = lib.gsvd_cholqr(m, n, A.data_ptr(), lda, Q.data_ptr(), m, R.data_ptr(), n,
                             work.data_ptr(), work.numel(), info.data_ptr(), ctypes.byref(o),
                             _stream(stream))
    _check(rc, "gsvd_cholqr")
    return Q, R, info


def gram(A, *, work=None, stream=None):
    """M_h = A^T A: returns (Mhi, Mlo) float64 n x n column-major tensors."""
    torch = _torch()
    w = _working_of(A)
    m, n = int(A.shape[0]), int(A.shape[1])
    lda = _ld(A)
    o = opts(w, GSVD_GRAM_PLAIN)
    with _on(stream):
        Mhi = colmajor_empty(n, n, torch.float64, A.device)
        Mlo = colmajor_empty(n, n, torch.float64, A.device)
        need = lib.gsvd_gram_workspace_size(m, n, ctypes.byref(o))
        if work is None:
            work = workspace(need, A.device)
        rc = lib.gsvd_gram(m, n, A.data_ptr(), lda, Mhi.data_ptr(), Mlo.data_ptr(), n,
                           work.data_ptr(), work.numel(), ctypes.byref(o), _stream(stream))
    _check(rc, "gsvd_gram")
    return Mhi, Mlo


def eig(Mhi, Mlo, working: int, *, eig: int = GSVD_EIG_AUTO, jacobi_tol: float = 0.0,
        max_sweeps: int = 0, stream=None):
    """Eigensolver stage on a device Gram: returns (S, V, W, info) in the working precision."""
    torch = _torch()
    n = int(Mhi.shape[0])
    dt = torch.float64 if working == GSVD_F64 else torch.float32
    o = opts(working, GSVD_GRAM_PLAIN, eig, jacobi_tol=jacobi_tol, max_sweeps=max_sweeps)
    with _on(stream):
        S = torch.empty(n, dtype=dt, device=Mhi.device)
        V = colmajor_empty(n, n, dt, Mhi.device)
        W = colmajor_empty(n, n, dt, Mhi.device)
        info = torch.full((1,), -1, dtype=torch.int32, device=Mhi.device)
        need = lib.gsvd_eig_workspace_size(n, ctypes.byref(o))
        work = workspace(need, Mhi.device) if need > 0 else None
        rc = lib.gsvd_eig(n, Mhi.data_ptr(), Mlo.data_ptr() if Mlo is not None else None,
                          _ld(Mhi), S.data_ptr(), V.data_ptr(), n, W.data_ptr(), n,
                          info.data_ptr(), work.data_ptr() if work is not None else None,
                          work.numel() if work is not None else 0, ctypes.byref(o),
                          _stream(stream))
    _check(rc, "gsvd_eig")
    return S, V, W, info


def u_recover(A, W, *, u_fp32_mfma: bool = False, stream=None):
    """U = A W in the working precision of A (FP32: the BF16 operand-split form unless
    u_fp32_mfma)."""
    w = _working_of(A)
    m, n = int(A.shape[0]), int(A.shape[1])
    o = opts(w, u_fp32_mfma=u_fp32_mfma)
    with _on(stream):
        U = colmajor_empty(m, n, A.dtype, A.device)
        rc = lib.gsvd_u_recover(m, n, A.data_ptr(), _ld(A), W.data_ptr(), _ld(W), U.data_ptr(),
                                m, ctypes.byref(o), _stream(stream))
    _check(rc, "gsvd_u_recover")
    return U


class Batch:
    """Everything one gsvd_thin_batched call needs, prepared once: outputs, the device
    pointer arrays, the host shape arrays and the workspace.  ``run()`` enqueues the
    call (capturable in a graph: it only launches kernels)."""

    def __init__(self, As, *, gram: int = GSVD_GRAM_AUTO, eig: int = GSVD_EIG_AUTO,
                 want_u: bool = True, jacobi_tol: float = 0.0, max_sweeps: int = 0,
                 n_slices: int = 0, slab_rows: int = 0, target_rel_err: float = 0.0,
                 kappa_b: float = 0.0):
        torch = _torch()
        if len(As) < 1:
            raise ValueError("empty batch")
        dev = As[0].device
        w = _working_of(As[0])
        if any(_working_of(a) != w for a in As):
            raise TypeError("all matrices of a batch share one dtype")
        self.count = len(As)
        self.As = list(As)
        self.o = opts(w, gram, eig, want_u=want_u, jacobi_tol=jacobi_tol,
                      max_sweeps=max_sweeps, n_slices=n_slices, slab_rows=slab_rows,
                      target_rel_err=target_rel_err, kappa_b=kappa_b)
        i64 = ctypes.c_int64 * self.count
        self.hM = i64(*[int(a.shape[0]) for a in As])
        self.hN = i64(*[int(a.shape[1]) for a in As])
        self.hLda = i64(*[_ld(a) for a in As])
        self.S = [torch.empty(int(a.shape[1]), dtype=a.dtype, device=dev) for a in As]
        self.V = [colmajor_empty(int(a.shape[1]), int(a.shape[1]), a.dtype, dev) for a in As]
        self.U = ([colmajor_empty(int(a.shape[0]), int(a.shape[1]), a.dtype, dev) for a in As]
                  if want_u else None)
        self.hLdv = i64(*[int(a.shape[1]) for a in As])
        self.hLdu = i64(*[int(a.shape[0]) for a in As])
        self.info = torch.full((self.count,), -1, dtype=torch.int32, device=dev)

        def ptrs(ts):
            return torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)

        self.dA, self.dS, self.dV = ptrs(self.As), ptrs(self.S), ptrs(self.V)
        self.dU = ptrs(self.U) if want_u else None
        need = lib.gsvd_thin_batched_workspace_size(self.count, self.hM, self.hN,
                                                     ctypes.byref(self.o))
        if need == 0:
            raise GsvdError("gsvd_thin_batched_workspace_size: invalid shapes or options")
        self.work = workspace(need, dev)

    def run(self, stream=None) -> None:
        """Enqueue the call on ``stream`` (default: torch's current stream).  The buffers
        were allocated on the stream current at construction; on another stream they are
        recorded as used there, so the caching allocator keeps them until that work ends."""
        if stream is not None:
            for t in [self.work, self.info, self.dA, self.dS, self.dV, *self.S, *self.V,
                      *(self.U or []), *([self.dU] if self.dU is not None else [])]:
                t.record_stream(stream)
        rc = lib.gsvd_thin_batched(
            self.count, self.hM, self.hN, self.dA.data_ptr(), self.hLda, self.dS.data_ptr(),
            self.dV.data_ptr(), self.hLdv, self.dU.data_ptr() if self.dU is not None else None,
            self.hLdu, self.work.data_ptr(), self.work.numel(), self.info.data_ptr(),
            ctypes.byref(self.o), _stream(stream))
        _check(rc, "gsvd_thin_batched")


def thin_batched(As, *, stream=None, **kw):
    """Thin SVDs of a list of column-major CUDA tensors in one batched call.
    Returns (S list, V list, U list or None, info tensor)."""
    b = Batch(As, **kw)
    b.run(stream)
    return b.S, b.V, b.U, b.info

"""gsvd_thin_noalloc (workspace in the library's fixed per-device array) against gsvd_thin
with a caller's workspace: the same kernels and plan, so the outputs agree bit for bit; two
calls in a row, the second on a smaller input (the array keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

from gen import matrices as g
from tests.helpers import say, to_dev

pytestmark = pytest.mark.gpu


def _both(A, **kw):
    import torch

    import paper_2603_11953_amd as gs
    dA = to_dev(A)
    m, n = A.shape
    o = gs.opts(gs.GSVD_F64 if A.dtype == np.float64 else gs.GSVD_F32, **kw)
    ob = ctypes.byref(o)
    outs = []
    for noalloc in (False, True):
        S = torch.full((n,), -1.0, dtype=dA.dtype, device=dA.device)
        V = gs.colmajor_empty(n, n, dA.dtype, dA.device).fill_(-1.0)
        U = gs.colmajor_empty(m, n, dA.dtype, dA.device).fill_(-1.0)
        info = torch.full((1,), -7, dtype=torch.int32, device=dA.device)
        st = gs._stream(None)
        if noalloc:
            rc = gs.gsvd_thin_noalloc(m, n, dA.data_ptr(), m, S.data_ptr(), V.data_ptr(), n,
                                      U.data_ptr(), m, info.data_ptr(), ob, st)
        else:
            need = gs.gsvd_thin_workspace_size(m, n, ob)
            work = gs.workspace(need, dA.device)
            rc = gs.gsvd_thin(m, n, dA.data_ptr(), m, S.data_ptr(), V.data_ptr(), n, U.data_ptr(),
                              m, work.data_ptr(), work.numel(), info.data_ptr(), ob, st)
        assert rc == 0, (noalloc, rc, gs.gsvd_status_string(rc))
        torch.cuda.synchronize()
        outs.append((S, V, U, info))
    return outs


@pytest.mark.parametrize("kw", [{}, {"gram": 1}], ids=["auto", "plain"])
def test_noalloc_matches_gsvd_thin_twice(kw):
    import torch

    import paper_2603_11953_amd as gs
    big = g.make_a(g.MatrixSpec(m=300_000, n=64, kappa_b=100, kappa_d=1e10, seed=401,
                                shuffle=True, w1="gauss"))
    small = g.make_a(g.MatrixSpec(m=5_000, n=20, kappa_b=1e3, kappa_d=1e8, seed=402, shuffle=True))
    for A, label in ((big, "first, 300000 x 64"), (small, "second, 5000 x 20")):
        m, n = A.shape
        o = gs.opts(gs.GSVD_F64, **kw)
        assert 0 < gs.gsvd_thin_workspace_size(m, n, ctypes.byref(o)) <= gs.gsvd_noalloc_max_bytes()
        say("noalloc", label, kw)
        ref_out, got = _both(A, **kw)
        assert int(got[3].item()) == 0 and int(ref_out[3].item()) == 0
        for x, y in zip(ref_out[:3], got[:3]):
            assert torch.equal(x, y), label


def test_noalloc_fp32_and_wide():
    import torch
    A = g.make_a(g.MatrixSpec(m=60_000, n=100, kappa_b=100, kappa_d=1e6, seed=403,
                              dtype="f32", w1="gauss"))
    W = g.make_a(g.MatrixSpec(m=20_000, n=160, kappa_b=100, kappa_d=1e6, seed=404, w1="gauss"))
    for X, label in ((A, "fp32 60000 x 100"), (W, "fp64 20000 x 160")):
        say("noalloc", label)
        ref_out, got = _both(X)
        for x, y in zip(ref_out, got):
            assert torch.equal(x, y), label

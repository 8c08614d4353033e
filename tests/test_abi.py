"""The C-ABI library loads, exports every function include/gsvd.h declares, and
rejects bad arguments synchronously (no kernel is launched, so no GPU is needed)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2603_11953_amd as gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(gsvd_\w+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol():
    decl = _declared()
    assert {"gsvd_thin", "gsvd_gram", "gsvd_eig", "gsvd_u_recover"} <= decl
    out = subprocess.run(["nm", "-D", "--defined-only", gs.lib_path], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (gsvd_\w+)", out))
    assert decl <= exported, decl - exported
    for name in decl:
        assert hasattr(gs.lib, name)


def test_opts_default_and_status():
    o = gs.opts(gs.GSVD_F64)
    assert o.working == gs.GSVD_F64 and o.flags == gs.GSVD_WANT_U and o.max_sweeps == 0
    assert gs.gsvd_status_string(0) == "success"
    assert "info 1" in gs.gsvd_status_string(1)
    assert "invalid argument" in gs.gsvd_status_string(-4)


def test_workspace_sizes_positive_and_aligned():
    for w in (gs.GSVD_F32, gs.GSVD_F64):
        o = gs.opts(w)
        for m, n in ((1, 1), (2000, 20), (1_000_000, 64), (4_000_000, 128)):
            t = gs.gsvd_thin_workspace_size(m, n, ctypes.byref(o))
            g = gs.gsvd_gram_workspace_size(m, n, ctypes.byref(o))
            assert t > 0 and t % 256 == 0 and g % 256 == 0 and t >= g + 2 * n * n * 8


def test_gram_config_resolves_the_launch_shape():
    for w in (gs.GSVD_F32, gs.GSVD_F64):
        smax = 12 if w == gs.GSVD_F64 else 8
        for m, n in ((64, 1), (2000, 20), (1_000_000, 64), (4_000_000, 128)):
            for gram in (gs.GSVD_GRAM_PLAIN, gs.GSVD_GRAM_SPLIT):
                c = gs.gram_config(m, n, w, gram)
                # the slabs cover the rows once: none is empty
                assert c["slab_rows"] >= 1 and c["n_slabs"] >= 1
                assert c["slab_rows"] * c["n_slabs"] >= m > c["slab_rows"] * (c["n_slabs"] - 1)
                if gram == gs.GSVD_GRAM_PLAIN:
                    assert c["n_slices"] == 0
                else:
                    assert 1 <= c["n_slices"] <= smax
                    assert gs.gram_config(m, n, w, gram, n_slices=3)["n_slices"] == 3
            c = gs.gram_config(1_000_000, 64, w, gs.GSVD_GRAM_SPLIT, slab_rows=4096)
            assert c["slab_rows"] == 4096 and c["n_slabs"] == -(-1_000_000 // 4096)
    o = gs.opts(gs.GSVD_F64)
    out = ctypes.c_int64()
    assert gs.gsvd_gram_config(0, 4, ctypes.byref(o), None, None, None) == -1
    assert gs.gsvd_gram_config(3, 4, ctypes.byref(o), ctypes.addressof(out), None, None) == -2
    assert gs.gsvd_gram_config(10, 4, None, None, None, None) == -3
    o = gs.opts(gs.GSVD_F32, gs.GSVD_GRAM_SPLIT, n_slices=9)
    assert gs.gsvd_gram_config(1000, 4, ctypes.byref(o), None, None, None) == -101


def test_plain_gram_slabs_fill_whole_rounds():
    """Host logic of the single-problem dd Gram plan: without a caller's slab
    height, the slab count at an m off the tuning size is set so that the
    workgroups (two per slab at n = 64) fill whole rounds of the 256 CUs, to within
    one slab (slab heights are whole LDS chunks); a caller's height is kept as given
    (rounded up to whole LDS chunks)."""
    for m in (1_000_000, 1_010_000, 1_500_000, 3_000_000):
        c = gs.gram_config(m, 64, gs.GSVD_F64, gs.GSVD_GRAM_PLAIN)
        wgs = 2 * c["n_slabs"]
        rounds = -(-wgs // 256)
        assert rounds * 256 - 2 < wgs + 2 and wgs <= rounds * 256, (m, c)
        assert c["slab_rows"] * c["n_slabs"] >= m > c["slab_rows"] * (c["n_slabs"] - 1)
    c = gs.gram_config(1_010_000, 64, gs.GSVD_F64, gs.GSVD_GRAM_PLAIN, slab_rows=7813)
    assert 7813 <= c["slab_rows"] < 7813 + 256  # one LDS chunk at most
    assert c["n_slabs"] == -(-1_010_000 // c["slab_rows"])


FAKE = 0x7F0000000000  # never dereferenced: validation fails first


def _gpu_visible() -> bool:
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:  # pragma: no cover
        return False


# Cases that pass a never-valid device address and expect the synchronous
# validation to refuse it: run only where no GPU is visible, so that a
# regression in the validation cannot launch kernels on that address.
fake_pointers = pytest.mark.skipif(_gpu_visible(), reason="fake device pointers: CPU-only check")


@fake_pointers
@pytest.mark.parametrize("args,code", [
    (dict(m=0), -1),
    (dict(n=0), -2),
    (dict(m=10, n=20), -2),
    (dict(n=gs.GSVD_MAX_N + 1, m=10_000), -2),
    (dict(A=None), -3),
    (dict(lda=99), -4),
    (dict(S=None), -5),
    (dict(V=None), -6),
    (dict(ldv=3), -7),
    (dict(U=None), -8),
    (dict(ldu=50), -9),
    (dict(work=FAKE + 8), -10),
    (dict(work_bytes=16), -11),
    (dict(info=None), -12),
])
def test_thin_rejects_bad_arguments(args, code):
    o = gs.opts(gs.GSVD_F64)
    a = dict(m=100, n=8, A=FAKE, lda=100, S=FAKE, V=FAKE, ldv=8, U=FAKE, ldu=100, work=FAKE,
             work_bytes=1 << 40, info=FAKE)
    a.update(args)
    rc = gs.gsvd_thin(a["m"], a["n"], a["A"], a["lda"], a["S"], a["V"], a["ldv"], a["U"], a["ldu"],
                      a["work"], a["work_bytes"], a["info"], ctypes.byref(o), None)
    assert rc == code


@fake_pointers
def test_bad_options_rejected():
    o = gs.opts(gs.GSVD_F64)
    o.working = 7
    rc = gs.gsvd_thin(100, 8, FAKE, 100, FAKE, FAKE, 8, FAKE, 100, FAKE, 1 << 40, FAKE,
                      ctypes.byref(o), None)
    assert rc == -13
    rc = gs.gsvd_thin(100, 8, FAKE, 100, FAKE, FAKE, 8, FAKE, 100, FAKE, 1 << 40, FAKE, None, None)
    assert rc == -13


@fake_pointers
def test_gram_eig_u_reject_bad_arguments():
    o = gs.opts(gs.GSVD_F64)
    assert gs.gsvd_gram(100, 8, FAKE, 100, FAKE, None, 8, FAKE, 1 << 40, ctypes.byref(o), None) == -6
    assert gs.gsvd_gram(100, 8, FAKE, 100, FAKE, FAKE, 7, FAKE, 1 << 40, ctypes.byref(o), None) == -7
    assert gs.gsvd_gram(100, 8, FAKE, 100, FAKE, FAKE, 8, FAKE, 0, ctypes.byref(o), None) == -9
    assert gs.gsvd_eig(8, FAKE, None, 8, FAKE, FAKE, 8, FAKE, 8, FAKE, None, 0,
                       ctypes.byref(o), None) == -3
    assert gs.gsvd_eig(8, FAKE, FAKE, 8, FAKE, FAKE, 8, FAKE, 8, None, None, 0,
                       ctypes.byref(o), None) == -10
    assert gs.gsvd_u_recover(100, 8, FAKE, 100, FAKE, 8, FAKE, 99, ctypes.byref(o), None) == -8


@fake_pointers
def test_unsupported_combinations_report_so():
    for w, s in ((gs.GSVD_F64, 13), (gs.GSVD_F32, 9)):
        o = gs.opts(w, gs.GSVD_GRAM_SPLIT, n_slices=s)
        rc = gs.gsvd_thin(100, 8, FAKE, 100, FAKE, FAKE, 8, FAKE, 100, FAKE, 1 << 40, FAKE,
                          ctypes.byref(o), None)
        assert rc == -101


def test_single_hip_runtime_in_process():
    """torch and libgsvd.so must share one HIP runtime (stream handles and pointers pass between them)."""
    import torch  # noqa: F401
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    assert len(paths) == 1, paths


def test_wide_limits():
    """n in 129..512 runs the wide kernels, for both working precisions (from n = 97 on
    for the default eigensolver); the eigensolver scratch covers the multi-workgroup
    preconditioner and the double-double Jacobi stage (11 n^2 doubles)."""
    for w in (gs.GSVD_F64, gs.GSVD_F32):
        for eig in (gs.GSVD_EIG_AUTO, gs.GSVD_EIG_CHOL_JACOBI1):
            o = gs.opts(w, eig=eig)
            for n in (97, 128, 129, 512):
                t = gs.gsvd_thin_workspace_size(4 * n, n, ctypes.byref(o))
                e = gs.gsvd_eig_workspace_size(n, ctypes.byref(o))
                if w == gs.GSVD_F32 and n <= 128 and eig == gs.GSVD_EIG_CHOL_JACOBI1:
                    assert e == 0  # the one-workgroup Algorithm 2
                    continue
                assert t % 256 == 0 and e > 4 * n * n * 8 and t > e, (w, eig, n)
                if eig == gs.GSVD_EIG_AUTO:
                    assert e >= 11 * n * n * 8
    # FP64, n <= 96: Algorithm 2 alone needs no scratch; the default adds the dd stage
    assert gs.gsvd_eig_workspace_size(96, ctypes.byref(gs.opts(gs.GSVD_F64, eig=gs.GSVD_EIG_CHOL_JACOBI1))) == 0
    assert gs.gsvd_eig_workspace_size(96, ctypes.byref(gs.opts(gs.GSVD_F64))) >= 11 * 96 * 96 * 8
    c = gs.gram_config(2_000_000, 512, gs.GSVD_F64, gs.GSVD_GRAM_PLAIN)
    assert c["n_slices"] == 0 and c["slab_rows"] % 16 == 0
    assert c["slab_rows"] * c["n_slabs"] >= 2_000_000 > c["slab_rows"] * (c["n_slabs"] - 1)


def _batch_call(batch=3, M=(1000, 2000, 500), N=(16, 64, 8), lda=None, ldv=None, ldu=None,
                work_bytes=1 << 40, null=(), o=None, working=gs.GSVD_F64):
    i64 = ctypes.c_int64 * max(len(M), 1)
    hM, hN = i64(*M), i64(*N)
    hLda = i64(*(lda or M))
    hLdv = i64(*(ldv or N))
    hLdu = i64(*(ldu or M))
    o = o or gs.opts(working)
    args = dict(dA=FAKE, dS=FAKE, dV=FAKE, dU=FAKE, work=FAKE, dInfo=FAKE, hM=hM, hN=hN,
                hLda=hLda, hLdv=hLdv, hLdu=hLdu)
    for k in null:
        args[k] = None
    return gs.gsvd_thin_batched(batch, args["hM"], args["hN"], args["dA"], args["hLda"],
                                args["dS"], args["dV"], args["hLdv"], args["dU"], args["hLdu"],
                                args["work"], work_bytes, args["dInfo"], ctypes.byref(o), None)


@fake_pointers
@pytest.mark.parametrize("kw,code", [
    (dict(batch=0), -1),
    (dict(null=("hM",)), -2),
    (dict(null=("hN",)), -3),
    (dict(null=("dA",)), -4),
    (dict(null=("hLda",)), -5),
    (dict(null=("dS",)), -6),
    (dict(null=("dV",)), -7),
    (dict(null=("hLdv",)), -8),
    (dict(null=("dU",)), -9),
    (dict(null=("hLdu",)), -10),
    (dict(null=("work",)), -11),
    (dict(work_bytes=0), -12),
    (dict(null=("dInfo",)), -13),
    (dict(M=(1000, 10, 500)), -2),          # m < n
    (dict(N=(16, 0, 8)), -3),
    (dict(N=(16, 97, 8)), -3),              # FP64 eigensolver limit
    (dict(lda=(1000, 1999, 500)), -5),
    (dict(ldv=(16, 63, 8)), -8),
    (dict(ldu=(999, 2000, 500)), -10),
])
def test_batched_argument_errors(kw, code):
    assert _batch_call(**kw) == code


@fake_pointers
def test_batched_workspace_and_unsupported():
    i64 = ctypes.c_int64 * 3
    hM, hN = i64(1000, 2000, 500), i64(16, 64, 8)
    for w in (gs.GSVD_F32, gs.GSVD_F64):
        for g in (gs.GSVD_GRAM_PLAIN, gs.GSVD_GRAM_SPLIT):
            o = gs.opts(w, g)
            t = gs.gsvd_thin_batched_workspace_size(3, hM, hN, ctypes.byref(o))
            assert t > 0 and t % 256 == 0
    o = gs.opts(gs.GSVD_F64)
    assert gs.gsvd_thin_batched_workspace_size(3, hM, i64(16, 97, 8), ctypes.byref(o)) == 0
    assert gs.gsvd_thin_batched_workspace_size(0, hM, hN, ctypes.byref(o)) == 0
    # FP32 working allows n up to 128 in a batch
    o32 = gs.opts(gs.GSVD_F32)
    assert gs.gsvd_thin_batched_workspace_size(3, i64(1000, 2000, 500), i64(16, 128, 8),
                                               ctypes.byref(o32)) > 0
    assert _batch_call(o=gs.opts(gs.GSVD_F64, gs.GSVD_GRAM_SPLIT, n_slices=13)) == -101


def test_target_rel_err_sets_the_slice_count():
    """The split slice count follows the requested accuracy: a tighter target never
    lowers S, a looser one never raises it; kappa_b enters squared; bad values are
    refused synchronously."""
    prev = 0
    for t in (1e-4, 1e-8, 1e-11, 1e-13, 1e-15):
        S = gs.gram_config(1_000_000, 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT,
                           target_rel_err=t)["n_slices"]
        assert S >= prev, (t, S, prev)
        prev = S
    assert prev > gs.gram_config(1_000_000, 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT,
                                 target_rel_err=1e-4)["n_slices"]
    lo = gs.gram_config(1_000_000, 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT, kappa_b=10)["n_slices"]
    hi = gs.gram_config(1_000_000, 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT, kappa_b=1e5)["n_slices"]
    assert lo <= hi
    # an explicit count wins over the target
    assert gs.gram_config(1_000_000, 64, gs.GSVD_F64, gs.GSVD_GRAM_SPLIT, n_slices=4,
                          target_rel_err=1e-15)["n_slices"] == 4
    for bad in (dict(target_rel_err=-1.0), dict(kappa_b=-2.0), dict(target_rel_err=float("nan"))):
        o = gs.opts(gs.GSVD_F64, **bad)
        assert gs.gsvd_gram_config(1000, 4, ctypes.byref(o), None, None, None) == -3
        assert gs.gsvd_thin_workspace_size(1000, 4, ctypes.byref(o)) == 0


def test_auto_gram_form():
    """GSVD_GRAM_AUTO: the split form for FP64 A (the dd Gram is vector-unit bound), the
    plain form for FP32 A at n <= 128 (one exact FP64 matrix-core pass beats five int8
    digit planes), per the tuning table; PLAIN when no slice count meets the target."""
    assert gs.gram_config(1_000_000, 64, gs.GSVD_F64)["n_slices"] > 0
    assert gs.gram_config(2_000_000, 512, gs.GSVD_F64)["n_slices"] > 0
    assert gs.gram_config(4_000_000, 128, gs.GSVD_F32)["n_slices"] == 0
    assert gs.gram_config(1_000_000, 64, gs.GSVD_F64, target_rel_err=1e-30)["n_slices"] == 0
    # workspace sizes follow the resolved form
    o_auto = gs.opts(gs.GSVD_F64)
    o_split = gs.opts(gs.GSVD_F64, gs.GSVD_GRAM_SPLIT)
    assert (gs.gsvd_thin_workspace_size(1_000_000, 64, ctypes.byref(o_auto)) ==
            gs.gsvd_thin_workspace_size(1_000_000, 64, ctypes.byref(o_split)))


@fake_pointers
def test_noalloc_rejects_oversized_and_bad_arguments():
    """gsvd_thin_noalloc refuses, before touching any device, a problem whose workspace
    exceeds its fixed array (GSVD_ERR_SCRATCH) and bad arguments (-k)."""
    assert gs.gsvd_noalloc_max_bytes() == 64 << 20
    o = gs.opts(gs.GSVD_F64)
    assert gs.gsvd_thin_workspace_size(2_000_000, 512, ctypes.byref(o)) > 64 << 20
    rc = gs.gsvd_thin_noalloc(2_000_000, 512, FAKE, 2_000_000, FAKE, FAKE, 512, FAKE, 2_000_000,
                              FAKE, ctypes.byref(o), None)
    assert rc == gs.GSVD_ERR_SCRATCH == -102
    assert "scratch" in gs.gsvd_status_string(rc)
    assert gs.gsvd_thin_noalloc(100, 8, None, 100, FAKE, FAKE, 8, FAKE, 100, FAKE,
                                ctypes.byref(o), None) == -3
    assert gs.gsvd_thin_noalloc(100, 8, FAKE, 100, FAKE, FAKE, 8, FAKE, 100, None,
                                ctypes.byref(o), None) == -10
    assert gs.gsvd_thin_noalloc(100, 8, FAKE, 100, FAKE, FAKE, 8, FAKE, 100, FAKE, None,
                                None) == -11


@fake_pointers
def test_cholqr_arguments():
    o = gs.opts(gs.GSVD_F64)
    assert gs.gsvd_cholqr_workspace_size(1000, 64, ctypes.byref(o)) % 256 == 0
    assert gs.gsvd_cholqr_workspace_size(1000, 64, ctypes.byref(o)) > 2 * 64 * 64 * 8
    a = dict(m=100, n=8, A=FAKE, lda=100, Q=FAKE, ldq=100, R=FAKE, ldr=8, work=FAKE,
             wb=1 << 40, info=FAKE)
    for k, v, code in (("m", 0, -1), ("n", 0, -2), ("A", None, -3), ("lda", 50, -4),
                       ("Q", None, -5), ("ldq", 50, -6), ("R", None, -7), ("ldr", 7, -8),
                       ("work", FAKE + 8, -9), ("wb", 10, -10), ("info", None, -11)):
        b = dict(a)
        b[k] = v
        rc = gs.gsvd_cholqr(b["m"], b["n"], b["A"], b["lda"], b["Q"], b["ldq"], b["R"], b["ldr"],
                            b["work"], b["wb"], b["info"], ctypes.byref(o), None)
        assert rc == code, (k, rc, code)

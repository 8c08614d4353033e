#!/usr/bin/env python3
"""Benchmark: thin-SVD throughput of the Gram-based mixed precision method on one MI355X.

One step = one call of gsvd_thin (Gram in the higher precision, eigensolver, U = A V
Sigma^-1) on an input already resident in HBM.

Headline workload: the largest single-GPU configuration, FP64 A = B D, m = 2,000,000,
n = 512 (8.2 GB), kappa(B) = 1e3, kappa(D) = 1e12 (log-spaced), in the form the
library chooses (GSVD_GRAM_AUTO: the int8 operand-split Gram with the slice count the
default accuracy target asks for; the default eigensolver: the double-double two-sided
Jacobi stage on Algorithm 2's basis), with the plain double-double Gram form beside it.
Prints one JSON line.

    value         = thin-SVD GFLOP/s = (m n (n + 1) + 2 m n^2) / t_step
    gram_hbm_gbps = (m n w + n^2 8) / t_gram (the metric's second figure)
    roofline      = the dominant kernel of the step (U = A W, urecover_wide_kernel, one
                    launch per step: 2 m n^2 flops on the FP64 matrix cores); the Gram
                    stage's own roofline is reported beside it (gram_roofline)
    cpu_baseline  = the CPU oracle (dd Gram + dd two-sided Jacobi + dd U) on the first
                    rows of the same matrix

Accuracy is checked after all timed legs (no oracle work overlaps a timed region): sigma
against the oracle's SVD of the n x n factor of A, ||U^T U - I||_F exactly (torch FP64
products of 18-bit pieces, independent of the library), the residual on sampled rows.

Other legs (each skippable):
    tall    = FP64 m = 1e6, n = 64, kappa(B) = 100: plain vs the chosen form
    fp32    = FP32 m = 4e6, n = 128, kappa(B) = 1e2: plain vs split at every slice count,
              sigma error against the oracle per slice count
    batched = 512 FP64 problems of uneven shape through gsvd_thin_batched (eager and
              graph-replayed) vs 512 gsvd_thin calls
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "thin-SVD GFLOP/s & Gram HBM GB/s at σ rel-err tol; split/batched vs plain"
# MI355X datasheet peaks
FP64_VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # FP64 lane-operations per second, 1 per FMA
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBPS = 8000.0
INT8_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak (POP/s x 1e-12)
PEAKS_JSON = os.path.join(ROOT, "profiles", "peaks_mi355x.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=2_000_000, help="rows of the headline workload")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle accuracy checks")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-rows", type=int, default=20_000,
                    help="rows of A the CPU oracle processes for the baseline")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain form of the headline workload")
    ap.add_argument("--no-tall", action="store_true",
                    help="skip the FP64 m = 1e6, n = 64 leg")
    ap.add_argument("--tall-m", type=int, default=1_000_000)
    ap.add_argument("--tall-steps", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched leg (512 FP64 problems of uneven shape)")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32 leg (m = 4e6, n = 128, sigma error per slice count)")
    ap.add_argument("--f32-m", type=int, default=4_000_000)
    ap.add_argument("--f32-steps", type=int, default=5)
    ap.add_argument("--only", choices=("tall", "fp32", "batched"), default="",
                    help="one secondary leg alone, for profiling: prints that leg's record "
                         "(not the benchmark line)")
    ap.add_argument("--only-headline", action="store_true",
                    help="the headline workload only (no other legs, checks or CPU baseline): "
                         "the command the committed kernel profiles were taken with")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB buffer 3 times (calibrates the HBM byte counters)")
    a = ap.parse_args()
    if a.only_headline:
        a.no_check = a.no_cpu = a.no_tall = a.no_batched = a.no_fp32 = a.no_plain = True
    return a


def copy_probe(mib: int) -> None:
    """Plain device-to-device copies of a known size: under rocprofv3 --pmc the FETCH_SIZE and
    WRITE_SIZE of these dispatches give the factor that turns the counters into bytes."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: 3 copies of {mib} MiB")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash(*names) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_11953_amd", "csrc")
    for f in names:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path: str, m: int, n: int, sources):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated by plain copies), if it was taken on the
    current kernel source and this shape."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != source_hash(*sources) or t.get("m") != m or t.get("n") != n:
        return None
    return t.get("bytes_per_launch")


def measured_peaks():
    """Ceilings measured on this part by the committed probe (profiles/peaks_mi355x.json,
    written by paper_2603_11953_amd/peaks.py), or {}."""
    try:
        with open(PEAKS_JSON) as f:
            return json.load(f).get("peaks", {})
    except (OSError, ValueError):
        return {}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def timed_on(torch, stream, fn, k, w_):
    """Average ms of fn over k calls after w_ warm-up calls, events on `stream`."""
    for _ in range(w_):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(k):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / k


def measure_thin(torch, gs, dA, gram_mode, steps, warmup, stream, log_fn, n_slices=0,
                 eig=0, u_fp32_mfma=False):
    """Time gsvd_thin on the column-major device matrix dA (working precision = its dtype,
    the default eigensolver unless ``eig`` names one), and its three stages through
    gsvd_gram, gsvd_eig and gsvd_u_recover (same kernels, same shapes)."""
    import ctypes
    m, n = int(dA.shape[0]), int(dA.shape[1])
    lda = int(dA.stride(1))
    dev = dA.device
    dt = dA.dtype
    w = gs.GSVD_F64 if dt == torch.float64 else gs.GSVD_F32
    sp = ctypes.c_void_p(int(stream.cuda_stream))
    o = gs.opts(w, gram_mode, eig, n_slices=n_slices, u_fp32_mfma=u_fp32_mfma)
    ob = ctypes.byref(o)
    cfg = gs.gram_config(m, n, w, gram_mode, n_slices=n_slices)
    S = torch.empty(n, dtype=dt, device=dev)
    V = gs.colmajor_empty(n, n, dt, dev)
    U = gs.colmajor_empty(m, n, dt, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    work = gs.workspace(gs.gsvd_thin_workspace_size(m, n, ob), dev)

    def step():
        rc = gs.gsvd_thin(m, n, dA.data_ptr(), lda, S.data_ptr(), V.data_ptr(), n, U.data_ptr(),
                          m, work.data_ptr(), work.numel(), info.data_ptr(), ob, sp)
        if rc != 0:
            raise RuntimeError(f"gsvd_thin: {rc} {gs.gsvd_status_string(rc)}")

    Mhi = gs.colmajor_empty(n, n, torch.float64, dev)
    Mlo = gs.colmajor_empty(n, n, torch.float64, dev)
    Wm = gs.colmajor_empty(n, n, dt, dev)
    gwork = gs.workspace(gs.gsvd_gram_workspace_size(m, n, ob), dev)
    ewn = gs.gsvd_eig_workspace_size(n, ob)
    ework = gs.workspace(ewn, dev) if ewn else None
    S2, V2, info2 = torch.empty_like(S), torch.empty_like(V), torch.zeros_like(info)
    U2 = torch.empty_like(U)

    def ph_gram():
        assert gs.gsvd_gram(m, n, dA.data_ptr(), lda, Mhi.data_ptr(), Mlo.data_ptr(), n,
                            gwork.data_ptr(), gwork.numel(), ob, sp) == 0

    def ph_eig():
        assert gs.gsvd_eig(n, Mhi.data_ptr(), Mlo.data_ptr(), n, S2.data_ptr(), V2.data_ptr(), n,
                           Wm.data_ptr(), n, info2.data_ptr(),
                           ework.data_ptr() if ework is not None else None,
                           ework.numel() if ework is not None else 0, ob, sp) == 0

    def ph_u():
        assert gs.gsvd_u_recover(m, n, dA.data_ptr(), lda, Wm.data_ptr(), n, U2.data_ptr(), m,
                                 ob, sp) == 0

    ms_step = timed_on(torch, stream, step, steps, warmup)
    ms_gram = timed_on(torch, stream, ph_gram, steps, 1)
    ms_eig = timed_on(torch, stream, ph_eig, steps, 1)
    ms_u = timed_on(torch, stream, ph_u, steps, 1)
    form = f"split-int8-S{cfg['n_slices']}" if cfg["n_slices"] else "plain"
    log_fn(f"{form} m={m} n={n} {dt}: step "
           f"{ms_step:.4f} ms, gram {ms_gram:.4f} eig {ms_eig:.4f} u {ms_u:.4f}")
    del U2, gwork, ework, work
    return dict(ms_step=ms_step, ms_gram=ms_gram, ms_eig=ms_eig, ms_u=ms_u, S=S, V=V, U=U,
                info=info, form=form, n_slices=cfg["n_slices"])


def fp32_leg(args, torch, gs, g, log_fn):
    """The FP32 workload: A = B D stored in FP32, m = 4e6, n = 128, kappa(B) = 1e2,
    kappa(D) = 1e6 (log-spaced).  FP64-accumulated plain Gram against the split Gram at every
    slice count 1..8, each with the default eigensolver and the default U (BF16 operand split);
    the plain form also with U on the FP32 matrix cores.  ||U^T U - I|| is taken exactly after
    each run (outside its timed region);
    the oracle (dd SVD of the stored FP32 matrix) runs after every timed leg."""
    from tests.exact_gram import orth_exact
    spec = g.spec_tall_f32(m=args.f32_m)
    spec.w1 = "gauss"
    dev = torch.device("cuda:0")
    t0 = time.time()
    dA, _ = g.make_a_device(spec, dev)
    torch.cuda.synchronize()
    m, n = spec.m, spec.n
    log_fn(f"fp32: generated A {m}x{n} on the GPU in {time.time() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    runs = [("plain", gs.GSVD_GRAM_PLAIN, 0, False), ("plain-u-fp32mfma", gs.GSVD_GRAM_PLAIN, 0, True)]
    runs += [(f"split-S{S}", gs.GSVD_GRAM_SPLIT, S, False) for S in range(1, 9)]
    flops = m * n * (n + 1) + 2 * m * n * n
    out = {"m": m, "n": n,
           "default_form": gs.gram_config(m, n, gs.GSVD_F32)["n_slices"] or "plain",
           "default_split_slices": gs.gram_config(m, n, gs.GSVD_F32,
                                                  gs.GSVD_GRAM_SPLIT)["n_slices"]}
    sig = {}
    for name, gram, S, ufp32 in runs:
        r = measure_thin(torch, gs, dA, gram, args.f32_steps, 1, stream, log_fn, S,
                         u_fp32_mfma=ufp32)
        orth = orth_exact(r["U"].double())
        sig[name] = r["S"].cpu().numpy().astype(np.float64)
        out[name] = {"ms_per_step": round(r["ms_step"], 4), "ms_gram": round(r["ms_gram"], 4),
                     "value_gflops": round(flops / (r["ms_step"] * 1e-3) / 1e9, 1),
                     "ms_u": round(r["ms_u"], 4), "info": int(r["info"].item()), "u_orth": orth}
        del r
    out["_A_host"] = np.asfortranarray(dA.t().contiguous().cpu().numpy().T)
    out["_sig"] = sig
    del dA
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def fp32_check(out, log_fn):
    from oracle import ref
    A_host, sig = out.pop("_A_host"), out.pop("_sig")
    oracle = ref.svd(A_host)
    n = out["n"]
    u = 2.0 ** -24
    tol = 50 * n * u * oracle.kappa_b
    out.update({"workload": f"FP32 A=BD m={out['m']} n={n} kappa(B)=1e2 kappa(D)=1e6 "
                            "(log-spaced); FP64-accumulated plain Gram vs split int8-slice Gram "
                            "per slice count, the default eigensolver, U on the BF16 matrix cores "
                            "(exact 3-piece operand split; FP32 matrix cores beside it)",
                "kappa_b_oracle": oracle.kappa_b, "sigma_tol_50nu_kappaB": tol,
                "orth_tol_50nu": 50 * n * u})
    for name, Sn in sig.items():
        err = float(ref.sigma_rel_err(Sn, oracle).max())
        o = out[name]
        o["sigma_max_rel_err"] = err
        o["meets_tol"] = bool((o["info"] & 0xFF) == 0 and err <= tol and o["u_orth"] <= 50 * n * u)
        log_fn(f"fp32 {name}: {o}")
    return out


def _accuracy(gs, ref, torch, A_rows, rows, r, oracle, n, u, m):
    """sigma against the oracle, ||U^T U - I||_F exact (torch FP64 products of 18-bit
    pieces), residual on the sampled rows, with the paper's tolerances."""
    from tests.exact_gram import orth_exact
    Sn = r["S"].cpu().numpy().astype(np.float64)
    Vn = r["V"].t().contiguous().cpu().numpy().T.astype(np.float64)
    U64 = r["U"] if r["U"].dtype == torch.float64 else r["U"].double()
    orth = orth_exact(U64)
    idx = torch.from_numpy(rows).to(r["U"].device)
    U_s = np.asfortranarray(r["U"].index_select(0, idx).cpu().numpy())
    resid = ref.resid(A_rows, U_s, Sn.astype(A_rows.dtype), Vn.astype(A_rows.dtype))
    err = float(ref.sigma_rel_err(Sn, oracle).max())
    kb = oracle.kappa_b
    acc = {"info": int(r["info"].item()), "sigma_max_rel_err": err,
           "sigma_tol_50nu_kappaB": 50 * n * u * kb, "u_orth": orth,
           "orth_tol_50nu": 50 * n * u, "orth_50nu_kappaB": 50 * n * u * kb,
           "resid_sampled_rows": resid, "kappa_b_oracle": kb}
    acc["u_orth_meets_50nu"] = bool(orth <= 50 * n * u)
    acc["meets_tol"] = bool((acc["info"] & 0xFF) == 0 and err <= acc["sigma_tol_50nu_kappaB"]
                            and orth <= 50 * n * u and resid <= 50 * n * u)
    return acc


def headline_leg(args, torch, gs, g, log_fn):
    """FP64 A = B D, m = 2e6, n = 512, kappa(B) = 1e3, kappa(D) = 1e12 (log-spaced): the
    library's chosen form (AUTO) timed over --steps steps, the plain form beside it.

    A = W1 Y is built on the GPU with W1 orthonormal (QR of a seeded Gaussian), so its
    singular values are those of the 512 x 512 factor Y up to the rounding of the product
    (a columnwise relative perturbation of order u, far inside the tolerance); the oracle
    computes sigma(Y) and kappa(B) in double-double, after the timed regions."""
    spec = g.spec_large_f64(m=args.m)
    spec.w1 = "qr"
    dev = torch.device("cuda:0")
    t0 = time.time()
    dA, Y = g.make_a_device(spec, dev)
    torch.cuda.synchronize()
    m, n = spec.m, spec.n
    log_fn(f"headline: generated A {m}x{n} on the GPU in {time.time() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    res = {"auto": measure_thin(torch, gs, dA, gs.GSVD_GRAM_AUTO, args.steps, args.warmup,
                                stream, log_fn)}
    if not args.no_plain:
        res["plain"] = measure_thin(torch, gs, dA, gs.GSVD_GRAM_PLAIN, max(2, args.steps // 3),
                                    1, stream, log_fn)
    # the vendor library's FP64 GEMM on U's shape (A times an n x n matrix): the matrix-core
    # rate a tuned GEMM sustains on this part, the reference ceiling for U
    Wr = torch.randn(n, n, dtype=dA.dtype, device=dev)
    vendor_ms = timed_on(torch, stream, lambda: torch.matmul(dA, Wr), 5, 2)
    del Wr
    torch.cuda.empty_cache()
    log_fn(f"headline: vendor FP64 GEMM on U's shape {vendor_ms:.3f} ms")
    return dict(spec=spec, dA=dA, Y=Y, res=res, m=m, n=n, vendor_gemm_ms=vendor_ms)


def headline_check(H, torch, gs, log_fn):
    """The headline's accuracy, after every timed leg."""
    from oracle import ref
    m, n = H["m"], H["n"]
    t0 = time.time()
    oracle = ref.svd(H["Y"])
    rows = np.unique(np.random.default_rng(1).integers(0, m, 4000))
    A_rows = np.asfortranarray(
        H["dA"].index_select(0, torch.from_numpy(rows).to(H["dA"].device)).cpu().numpy())
    out = {}
    for form, r in H["res"].items():
        out[form] = _accuracy(gs, ref, torch, A_rows, rows,
                              r, oracle, n, 2.0 ** -53, m)
        log_fn(f"headline {form} accuracy: {out[form]}")
    log_fn(f"headline oracle + checks {time.time() - t0:.1f}s")
    return out


def tall_leg(args, torch, gs, g, log_fn):
    """FP64 A = B D, m = 1e6, n = 64, kappa(B) = 100, kappa(D) = 1e10 (shuffled columns):
    plain vs the chosen form, stage times; accuracy after all timed legs."""
    spec = g.spec_tall_f64(m=args.tall_m)
    t0 = time.time()
    A = g.make_a(spec)
    log_fn(f"tall: generated A {A.shape} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t()
    stream = torch.cuda.current_stream()
    res = {"plain": measure_thin(torch, gs, dA, gs.GSVD_GRAM_PLAIN, args.tall_steps, 3, stream,
                                 log_fn),
           "auto": measure_thin(torch, gs, dA, gs.GSVD_GRAM_AUTO, args.tall_steps, 3, stream,
                                log_fn),
           "alg2_plain": measure_thin(torch, gs, dA, gs.GSVD_GRAM_PLAIN, args.tall_steps, 3,
                                      stream, log_fn, eig=gs.GSVD_EIG_CHOL_JACOBI1)}
    return dict(A=A, dA=dA, res=res, m=spec.m, n=spec.n)


def tall_summary(T, torch, gs, log_fn, check):
    m, n = T["m"], T["n"]
    flops = m * n * (n + 1) + 2 * m * n * n
    gram_bytes = m * n * 8 + n * n * 8
    out = {"workload": f"FP64 A=BD m={m} n={n} kappa(B)=1e2 kappa(D)=1e10 (log-spaced, columns "
                       "shuffled)"}
    for k, r in T["res"].items():
        out[k] = {"form": r["form"], "eig": "alg2" if k == "alg2_plain" else "jacobi2-dd",
                  "ms_per_step": round(r["ms_step"], 4),
                  "value_gflops": round(flops / (r["ms_step"] * 1e-3) / 1e9, 1),
                  "gram_hbm_gbps": round(gram_bytes / (r["ms_gram"] * 1e-3) / 1e9, 1),
                  "phases_ms": {"gram": round(r["ms_gram"], 4), "eig": round(r["ms_eig"], 4),
                                "u": round(r["ms_u"], 4)}}
    dd_ops = 10 * m * n * (n + 1) // 2
    out["plain"]["gram_alu_frac"] = round(dd_ops / (T["res"]["plain"]["ms_gram"] * 1e-3) / 1e12
                                          / FP64_VALU_PEAK_TOPS, 4)
    out["auto_speedup_vs_plain"] = round(T["res"]["plain"]["ms_step"] /
                                         T["res"]["auto"]["ms_step"], 3)
    if check:
        from oracle import ref
        oracle = ref.svd(T["A"])
        rows = np.unique(np.random.default_rng(0).integers(0, m, 20000))
        for k, r in T["res"].items():
            out[k]["accuracy"] = _accuracy(gs, ref, torch, np.asfortranarray(T["A"][rows]),
                                           rows, r, oracle, n, 2.0 ** -53, m)
            log_fn(f"tall {k} accuracy {out[k]['accuracy']}")
    return out


def batched_leg(args, torch, gs, g, log_fn):
    """The batched workload: 512 FP64 problems A = B D, m ~ U[1e4, 2e5], n from
    {16, 32, 48, 64, 96}, kappa(B) log-U[10, 1e3], kappa(D) log-U[1e4, 1e12].  One
    gsvd_thin_batched call (eager and replayed from a captured HIP graph) against the
    same 512 problems through 512 gsvd_thin calls on the same stream, for the plain and
    the split Gram.  Accuracy is checked after both forms are timed, on every n = 16
    problem with kappa(B) > 300 (where 50 n u kappa(B) is far above the kappa(B)-free
    orthogonality target) and a few others."""
    import ctypes
    from concurrent.futures import ThreadPoolExecutor

    specs = g.batch_specs()
    t0 = time.time()
    with ThreadPoolExecutor(16) as ex:
        As = list(ex.map(g.make_a, specs))
    log_fn(f"batched: generated {len(As)} problems ({sum(A.nbytes for A in As) / 1e9:.1f} GB) "
           f"in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    dAs = [torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t() for A in As]
    flops = sum(A.shape[0] * A.shape[1] * (A.shape[1] + 1) + 2 * A.shape[0] * A.shape[1] ** 2
                for A in As)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(int(stream.cuda_stream))

    def timed(fn, k, w_):
        return timed_on(torch, stream, fn, k, w_)

    out = {"problems": len(As), "flop": flops}
    corner = [k for k, sp_ in enumerate(specs) if sp_.n == 16 and sp_.kappa_b > 300]
    sample = sorted(set(corner + [0, 1, 2] +
                        [int(np.argmax([A.shape[1] * 1e7 + A.shape[0] for A in As]))]))
    batches = {}
    for form, gram in (("plain", gs.GSVD_GRAM_PLAIN), ("split", gs.GSVD_GRAM_SPLIT)):
        b = gs.Batch(dAs, gram=gram)
        ms_b = timed(lambda: b.run(stream), args.batched_steps, 1)
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(stream)
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                b.run(s)
        stream.wait_stream(s)
        torch.cuda.synchronize()
        ms_g = timed(graph.replay, args.batched_steps, 1)
        o = gs.opts(gs.GSVD_F64, gram)
        ob = ctypes.byref(o)
        wsz = max(gs.gsvd_thin_workspace_size(A.shape[0], A.shape[1], ob) for A in As)
        work = gs.workspace(wsz, dev)
        info1 = torch.zeros(len(As), dtype=torch.int32, device=dev)

        def seq():
            for k, A in enumerate(dAs):
                m, n = A.shape
                rc = gs.gsvd_thin(m, n, A.data_ptr(), m, b.S[k].data_ptr(), b.V[k].data_ptr(), n,
                                  b.U[k].data_ptr(), m, work.data_ptr(), work.numel(),
                                  info1[k:].data_ptr(), ob, sp)
                if rc != 0:
                    raise RuntimeError(f"gsvd_thin {rc}")

        ms_s = timed(seq, max(1, args.batched_steps // 2), 1)
        out[form] = {
            "ms_batched": round(ms_b, 4), "ms_graph_replay": round(ms_g, 4),
            "ms_sequential_512_calls": round(ms_s, 4),
            "value_batched_gflops": round(flops / (min(ms_b, ms_g) * 1e-3) / 1e9, 2),
            "speedup_vs_sequential": round(ms_s / min(ms_b, ms_g), 3),
        }
        log_fn(f"batched {form}: {ms_b:.3f} ms eager, {ms_g:.3f} ms graph, sequential {ms_s:.3f} "
               "ms")
        del graph, work
        batches[form] = b
        torch.cuda.synchronize()
    out["split_speedup_vs_plain"] = round(
        min(out["plain"]["ms_batched"], out["plain"]["ms_graph_replay"]) /
        min(out["split"]["ms_batched"], out["split"]["ms_graph_replay"]), 3)
    out["_check"] = dict(As=As, batches=batches, sample=sample, corner=corner)
    return out


def batched_check(out, torch, log_fn):
    from oracle import ref
    chk = out.pop("_check")
    As, sample = chk["As"], chk["sample"]
    orc = {k: ref.svd(As[k]) for k in sample}
    u = 2.0 ** -53
    for form, b in chk["batches"].items():
        b.run()
        torch.cuda.synchronize()
        info = b.info.cpu().numpy()
        errs, orths, ok = [], [], bool(np.all((info & 0xFF) == 0))
        for k in sample:
            A = As[k]
            n = A.shape[1]
            S = b.S[k].cpu().numpy()
            U = np.asfortranarray(b.U[k].t().contiguous().cpu().numpy().T)
            e = float(ref.sigma_rel_err(S, orc[k]).max())
            ort = ref.orth(U)
            errs.append(e)
            orths.append(ort)
            ok = ok and e <= 50 * n * u * orc[k].kappa_b and ort <= 50 * n * u
        out[form].update({
            "info_failures": int(np.sum((info & 0xFF) != 0)),
            "info_warnings": int(np.sum((info & ~0xFF) != 0)),
            "sample": {"problems": sample, "corner_n16_kappaB_gt_300": chk["corner"],
                       "sigma_max_rel_err": max(errs),
                       "u_orth_over_50nu_max": max(o / (50 * As[k].shape[1] * u)
                                                   for o, k in zip(orths, sample))},
            "meets_tol": ok})
        log_fn(f"batched {form} check: {out[form]['sample']} ok={ok}")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: use --gpus 1 "
                                   "(the row-split multi-GPU design is described, not built)"}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import torch

    import paper_2603_11953_amd as gs
    from gen import matrices as g

    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.only:  # one secondary leg alone (profiling runs)
        leg = {"tall": tall_leg, "fp32": fp32_leg, "batched": batched_leg}[args.only]
        r = leg(args, torch, gs, g, log)
        print(json.dumps({args.only: {k: v for k, v in r.items() if not k.startswith("_")}},
                         default=str))
        return

    # ---- timed legs (no oracle work runs while any of them is timed)
    H = headline_leg(args, torch, gs, g, log)
    legs = {}
    if not args.no_tall:
        legs["tall"] = tall_leg(args, torch, gs, g, log)
    if not args.no_fp32:
        legs["fp32"] = fp32_leg(args, torch, gs, g, log)
    if not args.no_batched:
        legs["batched"] = batched_leg(args, torch, gs, g, log)

    m, n = H["m"], H["n"]
    auto = H["res"]["auto"]
    flops = m * n * (n + 1) + 2 * m * n * n
    gram_bytes = m * n * 8 + n * n * 8

    def phases(r):
        return {"gram": round(r["ms_gram"], 4), "eig": round(r["ms_eig"], 4),
                "u": round(r["ms_u"], 4)}

    # the dominant kernel: U = A W (urecover_wide_kernel), one launch per step, timed alone
    # on the library's stream by the gsvd_u_recover phase
    u_flops = 2 * m * n * n
    u_bytes = 2 * m * n * 8 + n * n * 8
    u_tf = u_flops / (auto["ms_u"] * 1e-3) / 1e12
    peaks = measured_peaks()
    roof = {"kernel": "urecover_wide_kernel (U = A W, FP64 matrix cores)", "bound": "mfma",
            "achieved": round(u_tf, 2), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(u_tf / FP64_MFMA_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(os.path.join(ROOT, "profiles",
                                                     "urecover_wide_m2e6_n512_traffic.json"),
                                        m, n, ("urecover_wide.hip",)),
            "algorithmic": f"{u_flops} flops = 2 m n^2 per launch; {u_bytes} bytes "
                           "(A read, U written, W)",
            "ms_per_launch": round(auto["ms_u"], 4),
            "hbm_gbps": round(u_bytes / (auto["ms_u"] * 1e-3) / 1e9, 1)}
    if H.get("vendor_gemm_ms"):
        vend = u_flops / (H["vendor_gemm_ms"] * 1e-3) / 1e12
        roof["measured_peak"] = round(vend, 2)
        roof["measured_peak_source"] = ("the vendor FP64 GEMM (torch.matmul) on U's shape, "
                                        "timed in this run")
        roof["frac_of_measured_peak"] = round(u_tf / vend, 4)
    if "fp64_mfma_tflops" in peaks:
        roof["probe_peak"] = peaks["fp64_mfma_tflops"]
    S_ = auto["n_slices"]
    if S_:
        i8 = 2 * m * (n * (n + 1) // 2) * (S_ * (S_ + 1) // 2)
        ach = i8 / (auto["ms_gram"] * 1e-3) / 1e12
        gram_roof = {"stage": "split Gram (sw_slice + sw_syrk + sw_reduce)", "bound": "mfma",
                     "achieved": round(ach, 1), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                     "frac": round(ach / INT8_PEAK_TOPS, 4),
                     "algorithmic": f"{i8} int8 ops = 2 m n(n+1)/2 S(S+1)/2, S = {S_}"}
        if "int8_mfma_tops" in peaks:
            gram_roof["measured_peak"] = peaks["int8_mfma_tops"]
            gram_roof["frac_of_measured_peak"] = round(ach / peaks["int8_mfma_tops"], 4)
    else:
        dd_ops = 10 * m * n * (n + 1) // 2
        ach = dd_ops / (auto["ms_gram"] * 1e-3) / 1e12
        gram_roof = {"stage": "plain dd Gram", "bound": "alu", "achieved": round(ach, 2),
                     "peak": round(FP64_VALU_PEAK_TOPS, 2), "unit": "T lane-op/s",
                     "frac": round(ach / FP64_VALU_PEAK_TOPS, 4)}
    result = {
        "metric": METRIC,
        "value": round(flops / (auto["ms_step"] * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(auto["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"FP64 A=BD m={m} n={n} kappa(B)=1e3 kappa(D)=1e12 (log-spaced), the "
                        "largest single-GPU configuration; the library's chosen form: "
                        f"{auto['form']} Gram (GSVD_GRAM_AUTO at the default accuracy target), "
                        "double-double two-sided Jacobi stage on an FP64 preconditioner's basis, "
                        "FP64 MFMA U",
            "m": m, "n": n, "gram": auto["form"], "eig": "jacobi2-dd (default)",
        },
        "gram_hbm_gbps": round(gram_bytes / (auto["ms_gram"] * 1e-3) / 1e9, 2),
        "phases_ms": phases(auto),
        "roofline": roof,
        "gram_roofline": gram_roof,
    }
    if "plain" in H["res"]:
        pl = H["res"]["plain"]
        result["plain"] = {"form": pl["form"], "ms_per_step": round(pl["ms_step"], 4),
                           "value": round(flops / (pl["ms_step"] * 1e-3) / 1e9, 2),
                           "gram_hbm_gbps": round(gram_bytes / (pl["ms_gram"] * 1e-3) / 1e9, 2),
                           "phases_ms": phases(pl),
                           "gram_alu_frac": round(10 * m * n * (n + 1) // 2 /
                                                  (pl["ms_gram"] * 1e-3) / 1e12 /
                                                  FP64_VALU_PEAK_TOPS, 4)}
        result["speedup_vs_plain"] = round(pl["ms_step"] / auto["ms_step"], 3)
        result["gram_speedup_vs_plain"] = round(pl["ms_gram"] / auto["ms_gram"], 3)

    # ---- checks and CPU work, after every timed region
    if not args.no_check:
        acc = headline_check(H, torch, gs, log)
        result["accuracy"] = acc["auto"]
        if "plain" in acc:
            result["plain"]["accuracy"] = acc["plain"]
    if "tall" in legs:
        result["tall"] = tall_summary(legs["tall"], torch, gs, log, not args.no_check)
    if "fp32" in legs:
        result["fp32"] = fp32_check(legs["fp32"], log) if not args.no_check else {
            k: v for k, v in legs["fp32"].items() if not k.startswith("_")}
    if "batched" in legs:
        result["batched"] = batched_check(legs["batched"], torch, log) if not args.no_check else {
            k: v for k, v in legs["batched"].items() if not k.startswith("_")}

    if not args.no_cpu:
        from oracle import ref
        rows = min(args.cpu_rows, m)
        As = np.asfortranarray(
            H["dA"][:rows].cpu().numpy())
        t2 = time.perf_counter()
        o2 = ref.svd(As, want_kappa=False)
        ref.u_rows_dd(As, o2.V_hi, o2.V_lo, o2.sigma_hi, o2.sigma_lo)
        tc = time.perf_counter() - t2
        fl_s = rows * n * (n + 1) + 2 * rows * n * n
        result["cpu_baseline"] = {
            "value": round(fl_s / tc / 1e9, 4),
            "unit": "GFLOP/s",
            "cores": ref.num_threads(),
            "cpu": cpu_model(),
            "kind": "oracle",
            "sample": f"first {rows} of {m} rows of the headline matrix: dd Gram + dd two-sided "
                      f"Jacobi (n = {n}) + dd U, {tc:.1f} s",
        }
        log(f"cpu baseline {result['cpu_baseline']}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

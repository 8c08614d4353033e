"""Tune the library's launch shapes and slice counts on the GPU in use.

Writes ``csrc/tune_table.inc`` (the rows behind ``tune_slab_rows`` and
``tune_eps``); rebuild the library afterwards (``python
paper_2603_11953_amd/build.py``).

Slab height (rows of A per Gram workgroup).  For every working precision, Gram
form (plain / split), call kind (one problem / batched), n bucket and m bucket,
the Gram stage is timed through the C-ABI over a ladder of slab heights (fixed
powers of two, and for single problems the heights giving 128, 256, 384 and 512
slabs) on
seeded Gaussian inputs (each height over at least 10 ms of work, best of three
passes that alternate over the ladder), and the fastest height is kept.

Error of the split Gram per slice count.  For each working precision and n
bucket the split Gram of seeded A = B D test matrices (the paper's recipe,
kappa(B) = kappa_ref, strongly graded D) is compared with the plain
higher-precision Gram of the same matrices, for every slice count S; the worst
scaled error eps(S) = max |dM_ij| / sqrt(M_ii M_jj) over the seeds goes into the
table.  The library picks S per call from it: a perturbation with
|dM_ij| <= eps sqrt(M_ii M_jj) moves each sigma_i by a relative
n eps kappa(B)^2 / 2 at most, so a requested sigma accuracy (default
50 n u kappa(B)) is met, with a factor 16 of margin, by the smallest S with
eps(S) <= target / (8 n kappa(B)^2).

Run on the GPU:  python -m paper_2603_11953_amd.autotune [--quick] [--write]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TABLE = os.path.join(HERE, "csrc", "tune_table.inc")

N_BUCKETS = (16, 32, 64, 96, 128)
# (tuning size, upper edge) of each m bucket: tuned near the bucket's middle
M_BUCKETS = ((20_000, 50_000), (160_000, 500_000), (1_000_000, 2_000_000), (4_000_000, 2**62))
SINGLE_LADDER = (0, 256, 512, 1024, 2048, 4096, 8192)
BATCH_LADDER = (512, 1024, 2048, 4096, 8192, 16384)
SLICE_N_BUCKETS = N_BUCKETS + (256, 512)  # the wide split form too
KAPPA_REF = {1: 1e3, 0: 1e2}  # FP64 working: kappa(B) up to 1e3; FP32 working: 1e2


def _gs():
    sys.path.insert(0, ROOT)
    import paper_2603_11953_amd as gs
    return gs


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _best(fns, quick):
    """Fastest of several launch shapes: each is timed over at least 10 ms of
    work (5 ms with --quick), and the passes over the shapes alternate, so a
    clock or cache transient does not favour one shape; the best pass counts."""
    target = 5.0 if quick else 10.0
    reps = {}
    for k, fn in fns.items():
        once = _time(fn, 2)
        reps[k] = max(5, min(2000, int(target / max(once, 1e-3))))
    best = {k: float("inf") for k in fns}
    for _ in range(2 if quick else 3):
        for k, fn in fns.items():
            best[k] = min(best[k], _time(fn, reps[k]))
    k = min(best, key=best.get)
    return k, best[k]


def _gram_fn(gs, A, Mhi, Mlo, work, o):
    m, n = A.shape
    ob = ctypes.byref(o)

    def f():
        rc = gs.gsvd_gram(m, n, A.data_ptr(), m, Mhi.data_ptr(), Mlo.data_ptr(), n,
                          work.data_ptr(), work.numel(), ob, gs._stream(None))
        if rc != 0:
            raise RuntimeError(f"gsvd_gram {rc}")
    return f


def tune_single(gs, quick):
    import torch
    rows = []
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(11953)
    for working, dt in ((1, torch.float64), (0, torch.float32)):
        for gram in (gs.GSVD_GRAM_PLAIN, gs.GSVD_GRAM_SPLIT):
            for n in N_BUCKETS:
                for m, m_edge in (M_BUCKETS[:2] if quick else M_BUCKETS):
                    A = torch.randn(n, m, device=dev, dtype=dt, generator=gen).t()
                    Mhi = torch.empty(n, n, device=dev, dtype=torch.float64)
                    Mlo = torch.empty_like(Mhi)
                    fns, works = {}, []
                    # besides the fixed ladder, heights that give 128 j slabs, so
                    # that the workgroups fill whole rounds of the 256 CUs
                    ladder = sorted(set(SINGLE_LADDER) | {-(-m // (128 * j)) for j in (1, 2, 3, 4)})
                    for slab in ladder:
                        if slab and slab > m:
                            continue
                        o = gs.opts(working, gram, slab_rows=slab)
                        need = gs.gsvd_gram_workspace_size(m, n, ctypes.byref(o))
                        works.append(gs.workspace(need, dev))
                        fns[slab] = _gram_fn(gs, A, Mhi, Mlo, works[-1], o)
                    best = _best(fns, quick)
                    del fns, works
                    S_used = (gs.gram_config(m, n, working, gram)["n_slices"]
                              if gram == gs.GSVD_GRAM_SPLIT else 0)
                    rows.append(dict(working=working, gram=gram, batched=0, n_max=n, m_max=m_edge,
                                     slab_rows=best[0], ms=round(best[1], 4), m_tuned=m,
                                     slices=S_used))
                    print(f"[tune] single w={working} gram={gram} n<={n} m={m}: slab {best[0]} "
                          f"({best[1]:.3f} ms)", flush=True)
                    del A
    return rows


def tune_batched(gs, quick):
    import torch
    rows = []
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev).manual_seed(11954)
    count = 16 if quick else 48
    for working, dt in ((1, torch.float64), (0, torch.float32)):
        for gram in (gs.GSVD_GRAM_PLAIN, gs.GSVD_GRAM_SPLIT):
            for n in N_BUCKETS:
                if working == 1 and n > 96:
                    continue  # the FP64 eigensolver stops at n = 96
                ms_ = torch.randint(10_000, 200_001, (count,), generator=torch.Generator().manual_seed(n))
                As = [torch.randn(n, int(m), device=dev, dtype=dt, generator=gen).t() for m in ms_]
                batches = {slab: gs.Batch(As, gram=gram, want_u=False, slab_rows=slab)
                           for slab in BATCH_LADDER}
                best = _best({slab: b.run for slab, b in batches.items()}, quick)
                del batches
                S_used = (gs.gram_config(100_000, n, working, gram)["n_slices"]
                          if gram == gs.GSVD_GRAM_SPLIT else 0)
                rows.append(dict(working=working, gram=gram, batched=1, n_max=n, m_max=2**62,
                                 slab_rows=best[0], ms=round(best[1], 4), slices=S_used))
                print(f"[tune] batched w={working} gram={gram} n<={n}: slab {best[0]} "
                      f"({best[1]:.3f} ms for {count} problems)", flush=True)
                del As
    return rows


def tune_slices(gs, quick):
    """Smallest slice count meeting the Gram accuracy budget with a factor-16 margin."""
    import numpy as np
    import torch
    from gen import matrices as g
    rows = []
    dev = torch.device("cuda:0")
    for working, dt in ((1, "f64"), (0, "f32")):
        u = 2.0 ** -53 if working == 1 else 2.0 ** -24
        kref = KAPPA_REF[working]
        budget = 50 * u / kref
        smax = 12 if working == 1 else 8
        for n in (N_BUCKETS[:3] if quick else SLICE_N_BUCKETS):
            worst = np.zeros(smax + 1)
            for seed in range(1 if quick else 3):
                A = g.make_a(g.MatrixSpec(m=100_000, n=n, kappa_b=kref,
                                          kappa_d=1e12 if working == 1 else 1e6, mode_b=3, mode_d=5,
                                          seed=12_000 + 31 * n + seed, dtype=dt, shuffle=True,
                                          w1="gauss"))
                dA = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t()
                m = A.shape[0]
                Mhi = torch.empty(n, n, device=dev, dtype=torch.float64)
                Mlo = torch.empty_like(Mhi)
                o = gs.opts(working, gs.GSVD_GRAM_PLAIN)
                work = gs.workspace(gs.gsvd_gram_workspace_size(m, n, ctypes.byref(o)), dev)
                _gram_fn(gs, dA, Mhi, Mlo, work, o)()
                torch.cuda.synchronize()
                ref = Mhi.cpu().numpy() + Mlo.cpu().numpy()
                d = np.sqrt(np.diag(Mhi.cpu().numpy()))
                for S in range(1, smax + 1):
                    o = gs.opts(working, gs.GSVD_GRAM_SPLIT, n_slices=S)
                    work = gs.workspace(gs.gsvd_gram_workspace_size(m, n, ctypes.byref(o)), dev)
                    Sh, Sl = torch.empty_like(Mhi), torch.empty_like(Mhi)
                    _gram_fn(gs, dA, Sh, Sl, work, o)()
                    torch.cuda.synchronize()
                    diff = (Sh.cpu().numpy() - Mhi.cpu().numpy()) + (Sl.cpu().numpy() - Mlo.cpu().numpy())
                    eps = float(np.max(np.abs(diff) / np.outer(d, d)))
                    worst[S] = max(worst[S], eps)
            ok = [S for S in range(1, smax + 1) if worst[S] <= budget / 16]
            pick = ok[0] if ok else smax
            rows.append(dict(working=working, n_max=n, slices=pick,
                             eps=[float(f"{e:.3g}") for e in worst[1:]], budget=budget))
            print(f"[tune] slices w={working} n<={n}: eps(S) = "
                  + " ".join(f"{S}:{worst[S]:.1e}" for S in range(1, smax + 1))
                  + f"; budget {budget:.1e} -> S = {pick}", flush=True)
    return rows


def render_slices(slice_rows):
    names = {1: "GSVD_F64", 0: "GSVD_F32"}
    out = ["static const TuneEps kTuneEps[] = {"]
    for r in slice_rows:
        eps = ", ".join(f"{e:.3g}" for e in (list(r["eps"]) + [0.0] * 12)[:12])
        out.append(f"    {{{names[r['working']]}, {r['n_max']}, {{{eps}}}}},")
    out.append("};")
    return out


def render(slab_rows, slice_rows, meta, slab_text=None):
    # the largest m bucket of each (precision, form, kind, n) also covers every taller matrix
    top = {}
    for r in slab_rows:
        k = (r["working"], r["gram"], r["batched"], r["n_max"])
        top[k] = max(top.get(k, 0), r["m_max"])
    for r in slab_rows:
        if r["m_max"] == top[(r["working"], r["gram"], r["batched"], r["n_max"])]:
            r["m_max"] = 2**62
    names = {1: "GSVD_F64", 0: "GSVD_F32"}
    grams = {1: "GSVD_GRAM_PLAIN", 2: "GSVD_GRAM_SPLIT"}
    out = ["// Generated by paper_2603_11953_amd/autotune.py -- do not edit by hand.",
           f"// {meta}"]
    if slab_text is not None:  # slab heights kept from the previous table
        out.append(slab_text)
    else:
        out.append("static const TuneSlab kTuneSlab[] = {")
        for r in slab_rows:
            m_max = "INT64_MAX" if r["m_max"] >= 2**62 else str(r["m_max"])
            note = f"{r['ms']} ms at m = {r['m_tuned']}" if "m_tuned" in r else f"{r['ms']} ms"
            out.append(f"    {{{names[r['working']]}, {grams[r['gram']]}, {r['batched']}, "
                       f"{r['n_max']}, {m_max}, {r['slab_rows']}, {r['ms']}, "
                       f"{r.get('slices', 0)}}},  // {note}")
        out.append("};")
    out += render_slices(slice_rows)
    return "\n".join(out) + "\n"


def _slab_block(path):
    """The kTuneSlab block of an existing table, verbatim."""
    txt = open(path).read()
    a = txt.index("static const TuneSlab kTuneSlab[]")
    b = txt.index("};", a) + 2
    return txt[a:b]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--quick", action="store_true", help="fewer sizes and repetitions")
    ap.add_argument("--write", action="store_true", help="write the table (to --out)")
    ap.add_argument("--out", default=TABLE, help="table path (default: the library's csrc)")
    ap.add_argument("--json", default="", help="also dump the measurements to this file")
    ap.add_argument("--slices-only", action="store_true",
                    help="measure only the split Gram error per slice count; keep the slab "
                         "heights of the current table")
    args = ap.parse_args()
    gs = _gs()
    t0 = time.time()
    slab_text = _slab_block(TABLE) if args.slices_only else None
    slab_rows = [] if args.slices_only else tune_single(gs, args.quick) + tune_batched(gs, args.quick)
    slice_rows = tune_slices(gs, args.quick)
    import torch
    meta = (f"{torch.cuda.get_device_name(0)}; {'quick' if args.quick else 'full'} run"
            f"{' (slice counts; slab heights kept)' if args.slices_only else ''}, "
            f"{time.time() - t0:.0f} s")
    text = render(slab_rows, slice_rows, meta, slab_text)
    print(text)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"slab": slab_rows, "slices": slice_rows, "meta": meta}, f, indent=1)
    if args.write:
        with open(args.out, "w") as f:
            f.write(text)
        print(f"[tune] wrote {args.out}; rebuild the library to use it")


if __name__ == "__main__":
    main()

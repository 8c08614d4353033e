"""The batched entry point (gsvd_thin_batched): parity with the oracle problem by problem,
bitwise agreement with one-at-a-time gsvd_thin at the same slab height, per-problem info
codes, and replay of a captured HIP graph."""
import numpy as np
import pytest

from gen import matrices as g
from oracle import ref
from tests.helpers import check_thin, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _specs(seed, dtype, ns, count, m_hi):
    """Uneven shapes: ragged m (not multiples of the slab or tile heights), mixed n."""
    rng = g.rng_for(seed)
    out = []
    for i in range(count):
        n = int(ns[i % len(ns)])
        m = int(rng.integers(max(n, 1), m_hi))
        kb = float(10 ** rng.uniform(1, 2.5))
        kd = float(10 ** rng.uniform(2, 10))
        out.append(g.MatrixSpec(m=m, n=n, kappa_b=kb, kappa_d=kd, mode_b=3, mode_d=3,
                                seed=seed + 7 * i, dtype=dtype, shuffle=True, w1="gauss"))
    return out


def _run(As, **kw):
    import paper_2603_11953_amd as gs
    dev = [to_dev(A) for A in As]
    b = gs.Batch(dev, **kw)
    b.run()
    _torch().cuda.synchronize()
    S = [to_np(t) for t in b.S]
    V = [to_np(t) for t in b.V]
    U = [to_np(t) for t in b.U] if b.U is not None else None
    return S, V, U, b.info.cpu().numpy()


CASES = [
    ("f64", (1, 5, 16, 17, 33, 48, 64, 96), 9000, "plain"),
    ("f64", (3, 16, 31, 64, 80, 96), 9000, "split"),
    ("f32", (2, 16, 47, 64, 100, 128), 9000, "plain"),
    ("f32", (8, 16, 33, 96, 128), 9000, "split"),
]


@pytest.mark.parametrize("dt,ns,m_hi,form", CASES, ids=[f"{c[0]}-{c[3]}" for c in CASES])
def test_batched_parity_with_oracle(dt, ns, m_hi, form):
    import paper_2603_11953_amd as gs
    specs = _specs(4100 + len(ns), dt, ns, 2 * len(ns), m_hi)
    As = [g.make_a(s) for s in specs]
    gram = gs.GSVD_GRAM_SPLIT if form == "split" else gs.GSVD_GRAM_PLAIN
    say("batched parity", dt, form, [A.shape for A in As])
    S, V, U, info = _run(As, gram=gram)
    assert np.all(info == 0), info
    for k, A in enumerate(As):
        o = ref.svd(A)
        check_thin(A, S[k], V[k], U[k], o, label=f"{dt} {form} problem {k} {A.shape}")


@pytest.mark.parametrize("dt,form,slab", [("f64", "plain", 640), ("f64", "split", 256),
                                          ("f32", "plain", 1000), ("f32", "split", 512)])
def test_batched_equals_single_calls(dt, form, slab):
    """Same kernels, same slab height: every problem's S, V, U are bitwise those of gsvd_thin
    (FP32 working: the batched call forms U on the FP32 matrix cores, the single call's
    GSVD_U_FP32_MFMA form)."""
    import paper_2603_11953_amd as gs
    gram = gs.GSVD_GRAM_SPLIT if form == "split" else gs.GSVD_GRAM_PLAIN
    specs = _specs(5200, dt, (4, 16, 40, 64, 96), 7, 7000)
    As = [g.make_a(s) for s in specs]
    say("batched vs single", dt, form, slab)
    S, V, U, info = _run(As, gram=gram, slab_rows=slab)
    assert np.all(info == 0), info
    for k, A in enumerate(As):
        s1, v1, u1, i1 = gs.thin(to_dev(A), gram=gram, slab_rows=slab, u_fp32_mfma=dt == "f32")
        _torch().cuda.synchronize()
        assert int(i1.item()) == 0
        assert np.array_equal(to_np(s1), S[k]), k
        assert np.array_equal(to_np(v1), V[k]), k
        assert np.array_equal(to_np(u1), U[k]), k


@pytest.mark.parametrize("form", ["plain", "split"])
def test_batched_info_codes_per_problem(form):
    import paper_2603_11953_amd as gs
    specs = _specs(6100, "f64", (10, 24, 10, 24, 7), 5, 3000)
    As = [g.make_a(s) for s in specs]
    As[1][:, 3] = 0.0          # rank deficient: info 1
    As[2][17, 2] = np.nan      # non-finite: info 3
    As[4][5, 6] = np.inf       # non-finite: info 3
    As = [np.asfortranarray(A) for A in As]
    say("batched info codes", form)
    S, V, U, info = _run(As, gram=gs.GSVD_GRAM_SPLIT if form == "split" else gs.GSVD_GRAM_PLAIN)
    assert list(info) == [0, 1, 3, 0, 3], info
    for k in (0, 3):
        check_thin(As[k], S[k], V[k], U[k], ref.svd(As[k]), label=f"problem {k}")


def test_batched_sigma_only():
    specs = _specs(6200, "f32", (16, 64, 128), 3, 5000)
    As = [g.make_a(s) for s in specs]
    say("batched want_u=False")
    S, V, U, info = _run(As, want_u=False)
    assert U is None and np.all(info == 0)
    for k, A in enumerate(As):
        o = ref.svd(A)
        assert ref.sigma_rel_err(S[k].astype(np.float64), o).max() <= \
            50 * A.shape[1] * 2.0 ** -24 * o.kappa_b


def test_batched_graph_replay():
    """Capture one batched call in a HIP graph; every replay, with eager work and new input
    values in between, reproduces the eager call on the current inputs bitwise."""
    import paper_2603_11953_amd as gs
    torch = _torch()
    specs = _specs(6300, "f64", (16, 33, 64, 96), 6, 20_000)
    As = [g.make_a(s) for s in specs]
    dev = [to_dev(A) for A in As]
    b = gs.Batch(dev, gram=gs.GSVD_GRAM_SPLIT)
    say("batched graph capture")
    b.run()
    torch.cuda.synchronize()
    ref0 = [t.clone() for t in b.S + b.V + b.U]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            b.run(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in b.S + b.V + b.U:
            t.zero_()
        b.info.fill_(-1)
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()  # unrelated eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.all(b.info == 0)
        for t, r in zip(b.S + b.V + b.U, ref0):
            assert torch.equal(t, r), rep
    # new values in the same input buffers: the replay reads them
    As2 = [g.make_a(g.MatrixSpec(m=s.m, n=s.n, kappa_b=20, kappa_d=1e3, seed=s.seed + 1,
                                 w1="gauss")) for s in specs]
    for d, A in zip(dev, As2):
        d.copy_(to_dev(A))
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    got = [t.clone() for t in b.S + b.V + b.U]
    b.run()
    torch.cuda.synchronize()
    for t, r in zip(b.S + b.V + b.U, got):
        assert torch.equal(t, r)
    for k, A in enumerate(As2):
        check_thin(A, to_np(b.S[k]), to_np(b.V[k]), to_np(b.U[k]), ref.svd(A), label=f"g{k}")


def test_batched_workload_sample_full_sizes():
    """The batched workload's own recipe at full size (first 24 problems: m up to 2e5,
    n in {16, ..., 96}), every problem checked against the oracle."""
    specs = g.batch_specs()[:24]
    As = [g.make_a(s) for s in specs]
    for form in ("plain", "split"):
        import paper_2603_11953_amd as gs
        say("batched workload sample", form, sum(A.size for A in As))
        S, V, U, info = _run(As, gram=gs.GSVD_GRAM_SPLIT if form == "split" else gs.GSVD_GRAM_PLAIN)
        assert np.all(info == 0), info
        for k, A in enumerate(As):
            rows = np.random.default_rng(k).integers(0, A.shape[0], 2000)
            check_thin(A, S[k], V[k], U[k], ref.svd(A), rows=rows, label=f"{form} {k} {A.shape}")

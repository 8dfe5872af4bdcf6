"""Batches of uneven mixtures (ctfiss_batch_*) against single contexts.

A batch runs, per mixture, the iteration a single context runs on the same
launch shape with its NMF steps as separate launches (CTFISS_UNFUSED_NMF):
the W update per bin, the NMF steps per workgroup in the same order, so its
images must equal those single-context images bit for bit.  Mixtures drawn
as the batched workload are also checked against the FP64 oracle directly.
"""
import numpy as np
import pytest

from datagen import random_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (F, T, M, D, N, K, taps): several launch shapes, two mixtures of one shape
SHAPES = [
    (9, 40, 2, 2, 2, 3, (2, 2)),
    (7, 100, 3, 1, 2, 2, (2, 1)),
    (5, 313, 3, 4, 2, 4, (6, 6)),
    (11, 70, 4, 2, 3, 3, (3, 3, 2)),
    (9, 40, 2, 2, 2, 3, (2, 2)),
    (4, 500, 2, 2, 2, 5, (2, 2)),
    (3, 700, 2, 4, 2, 3, (4, 4)),
]


def _problems(precision, seed0=20):
    rd = torch.float32 if precision == "fp32" else torch.float64
    cd = torch.complex64 if precision == "fp32" else torch.complex128
    out = []
    for i, (F, T, M, D, N, K, taps) in enumerate(SHAPES):
        X, B0, V0 = random_problem(F, T, M, N, K, seed0 + i, scale_spread=0.5)
        out.append((torch.from_numpy(X).to("cuda", cd), torch.from_numpy(B0).to("cuda", rd),
                    torch.from_numpy(V0).to("cuda", rd)))
    return out


def _single(precision, rule, probs, splits):
    from paper_2510_02382_amd import Separator
    imgs = []
    for (F, T, M, D, N, K, taps), (X, B, V) in zip(SHAPES, probs):
        sep = Separator(F, T, M, D, N, K, taps, precision=precision, rule=rule)
        sep.set_input(X)
        sep.set_state(B=B, V=V)
        for n in splits:
            sep.iterate(n)
        imgs.append(sep.source_images())
        assert sep.status() == 0
        sep.close()
    return imgs


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_single_contexts(precision, monkeypatch):
    """The batch runs each mixture's NMF steps as separate launches over all mixtures; a single
    context does the same with CTFISS_UNFUSED_NMF (by default its bins form 1/lambda and the
    basis update themselves, which changes only the order of some sums)."""
    from paper_2510_02382_amd import BatchSeparator
    monkeypatch.setenv("CTFISS_UNFUSED_NMF", "1")
    probs = _problems(precision)
    ref = _single(precision, "iss", probs, (4, 3))
    bs = BatchSeparator(SHAPES, precision=precision)
    bs.set_input([p[0] for p in probs])
    bs.set_state(B=[p[1] for p in probs], V=[p[2] for p in probs])
    bs.iterate(4)
    bs.iterate(3)  # the carried demixed rows and the pending rescale cross calls as in a context
    got = bs.source_images()
    assert bs.status() == (-1, 0)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert torch.equal(a, b), f"mixture {i}: max |diff| {float((a - b).abs().max())}"
    bs.close()


def test_batch_ip_rule_runs_per_mixture():
    from paper_2510_02382_amd import BatchSeparator
    probs = _problems("fp64", seed0=40)
    ref = _single("fp64", "ip", probs, (3,))
    bs = BatchSeparator(SHAPES, precision="fp64", rule="ip")
    bs.set_input([p[0] for p in probs])
    bs.set_state(B=[p[1] for p in probs], V=[p[2] for p in probs])
    bs.iterate(3)
    for a, b in zip(bs.source_images(), ref):
        assert torch.equal(a, b)
    bs.close()


def test_batch_reports_the_faulting_mixture():
    from paper_2510_02382_amd import BatchSeparator
    probs = _problems("fp32", seed0=60)
    X3 = probs[3][0].clone()
    X3[0, 2, 5] = complex(float("nan"), 0.0)
    bs = BatchSeparator(SHAPES, precision="fp32")
    bs.set_input([p[0] if i != 3 else X3 for i, p in enumerate(probs)])
    bs.set_state(B=[p[1] for p in probs], V=[p[2] for p in probs])
    bs.iterate(1)
    mix, code = bs.status()
    assert mix == 3 and code != 0
    bs.close()


def test_batch_rejects_wrong_tensors():
    from paper_2510_02382_amd import BatchSeparator
    probs = _problems("fp32", seed0=80)
    bs = BatchSeparator(SHAPES, precision="fp32")
    with pytest.raises(ValueError):
        bs.set_input([p[0] for p in probs][:-1])
    with pytest.raises(ValueError):
        bs.set_input([p[0].to(torch.complex128) for p in probs])
    bs.close()


# ------------------------------------------------------------------ against the oracle
# Mixtures drawn as the batched workload (3-12 s, N in {2, 3}, M = N + 1, D in {4, 8},
# RT60 0.3-1.0 s, STFT 1024/256, K = 10, 50 iterations); draws 0-4 and 9 (Mbar = 32,
# 12, 24, 16, 16, 32; T = 540, 315, 191, 451, 331, 704), each cut to 10 bins so that the
# oracle finishes in seconds.
BATCH_DRAWS = (0, 1, 2, 3, 4, 9)


def _workload_slices(draws, f0=60, nf=10):
    from datagen import batched_workloads, init_nmf, make_mixture
    wls = batched_workloads(max(draws) + 1, 7)
    out = []
    for i in draws:
        w = wls[i]
        X = np.ascontiguousarray(make_mixture(w, 1000 + i).X[:, f0:f0 + nf, :])
        B0, V0 = init_nmf(w.N, nf, w.K, w.T, 1000 + i)
        out.append((w, X, B0, V0))
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_of_workload_mixtures_matches_oracle(precision):
    """A batch of uneven mixtures against the FP64 oracle run mixture by mixture on the
    original FP64 data: every source image within 1e-4 (FP32; the accuracy target) or 1e-9
    (FP64) after the workload's 50 iterations."""
    from oracle import ctf_iss as o
    from oracle import threaded as oth
    from paper_2510_02382_amd import BatchSeparator
    from parity import elem_err, record, rel
    # FP64 batches take one workgroup per bin: the Mbar = 32 draws (T = 540, 704) need a team in FP64
    draws = BATCH_DRAWS if precision == "fp32" else (1, 2, 3, 4)
    items = _workload_slices(draws)
    rd = torch.float32 if precision == "fp32" else torch.float64
    cd = torch.complex64 if precision == "fp32" else torch.complex128
    shapes = [(X.shape[1], w.T, w.M, w.D, w.N, w.K, w.row_taps) for w, X, B0, V0 in items]
    bs = BatchSeparator(shapes, precision=precision)
    Xs = [torch.from_numpy(X).to("cuda", cd) for w, X, B0, V0 in items]
    bs.set_input(Xs)
    bs.set_state(B=[torch.from_numpy(B0).to("cuda", rd) for w, X, B0, V0 in items],
                 V=[torch.from_numpy(V0).to("cuda", rd) for w, X, B0, V0 in items])
    n_iter = items[0][0].n_iter
    bs.iterate(n_iter)
    C = [c.cpu().numpy() for c in bs.source_images()]
    assert bs.status() == (-1, 0)
    bs.close()
    tol = 1e-4 if precision == "fp32" else 1e-9
    for i, (w, X, B0, V0) in zip(draws, items):
        W, _, _ = oth.run(X, w.D, w.row_taps, B0, V0, n_iter)
        Cr = o.source_images(W, X, w.D, w.row_taps)
        Cg = C[draws.index(i)]
        for n in range(w.N):
            e = rel(Cg[n], Cr[n])
            record(f"batch_vs_oracle[{precision}]", draw=i, source=n, rel=e,
                   elem=elem_err(Cg[n:n + 1], Cr[n:n + 1], "C"))
            assert e < tol, (i, n, e)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_graph_replays_equal_eager(precision):
    """Graph mode: the first iterate(n) call of a batch captures its launches, later calls replay
    them.  Three replays, each after eager work on the device and a synchronisation, with a new
    state set in between, give the eager images bit for bit."""
    from paper_2510_02382_amd import BatchSeparator
    probs = _problems(precision, seed0=90)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = BatchSeparator(SHAPES, precision=precision, stream=stream)
        eager.set_input([p[0] for p in probs])
        eager.set_state(B=[p[1] for p in probs], V=[p[2] for p in probs])
        eager.iterate(3)
        eager.iterate(2)
        ref = [c.clone() for c in eager.source_images()]
        stream.synchronize()
        eager.close()
        bs = BatchSeparator(SHAPES, precision=precision, stream=stream)
        bs.set_graph(True)
        bs.set_input([p[0] for p in probs])
        for replay in range(4):
            bs.set_state(B=[p[1] for p in probs], V=[p[2] for p in probs])
            bs.iterate(3)  # captured on the first pass (carried Y not valid), replayed after
            bs.iterate(2)  # likewise with the carried Y valid
            got = bs.source_images()
            junk = torch.randn(1 << 20, device="cuda")  # eager work between replays
            (junk * 2).sum().item()
            stream.synchronize()
            assert bs.status() == (-1, 0)
            for i, (a, b_) in enumerate(zip(got, ref)):
                assert torch.equal(a, b_), (replay, i)
        bs.close()

"""Graph mode (ctfiss_set_graph): iterate() calls replayed from captured HIP
graphs give the same results, bit for bit, as the launches they were captured
from.  Each replay is separated by eager work of the same context (set_state,
source images) and of torch, and by synchronisations, and every replay is
checked, as replays after the first are where graphs go wrong if anything in
them does not replay faithfully."""
import numpy as np
import pytest

from test_gpu_parity import as_device, make_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(case, precision, graph, stream, splits, reps=3):
    from paper_2510_02382_amd import Separator
    X, B0, V0, W0, D, taps = make_case(case, seed=31)
    M, F, T = X.shape
    out = []
    with torch.cuda.stream(stream):
        sep = Separator(F, T, M, D, len(taps), B0.shape[-1], taps, precision=precision, stream=stream)
        if graph:
            sep.set_graph(True)
        sep.set_input(as_device(X, precision))
        B, V = as_device(B0, precision), as_device(V0, precision)
        for rep in range(reps):
            sep.set_state(B=B, V=V)
            for n in splits:
                sep.iterate(n)
            junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
            C = sep.source_images()
            W, Bo, Vo = sep.state()
            stream.synchronize()
            out.append((C.cpu().numpy(), W.cpu().numpy(), Bo.cpu().numpy(), Vo.cpu().numpy(), sep.status()))
            del junk
        sep.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64", "mixed"])
@pytest.mark.parametrize("case", ["c0_like", "ragged", "three_src"])
def test_graph_replays_equal_eager_launches(case, precision):
    stream = torch.cuda.Stream()
    splits = (3, 2, 2)  # the second call of 2 replays the (2, carried Y valid) graph
    eager = _run(case, precision, False, stream, splits)
    graph = _run(case, precision, True, stream, splits)
    for rep, (e, g) in enumerate(zip(eager, graph)):
        assert g[4] == 0 and e[4] == 0
        for k in range(4):
            np.testing.assert_array_equal(g[k], e[k], err_msg=f"replay {rep}, output {k}")


def test_graph_mode_rejects_null_stream_and_team_launches(monkeypatch):
    from paper_2510_02382_amd import Separator
    from paper_2510_02382_amd import binding as b
    X, B0, V0, W0, D, taps = make_case("ragged", seed=32)
    M, F, T = X.shape
    sep = Separator(F, T, M, D, len(taps), B0.shape[-1], taps, precision="fp32",
                    stream=torch.cuda.default_stream())
    if sep.stream.cuda_stream == 0:
        with pytest.raises(b.CtfissError) as e:
            sep.set_graph(True)
        assert e.value.status == b.CTFISS_E_UNSUPPORTED
    sep.close()
    monkeypatch.setenv("CTFISS_PLAN", "32,4,2,3")
    stream = torch.cuda.Stream()
    sep = Separator(F, T, M, D, len(taps), B0.shape[-1], taps, precision="fp32", stream=stream)
    with pytest.raises(b.CtfissError) as e:
        sep.set_graph(True)
    assert e.value.status == b.CTFISS_E_UNSUPPORTED
    sep.close()


def test_graph_follows_a_new_input():
    """set_input with another tensor drops the captured graphs (they hold the old pointer)."""
    from paper_2510_02382_amd import Separator
    X, B0, V0, W0, D, taps = make_case("three_src", seed=33)
    M, F, T = X.shape
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ref = Separator(F, T, M, D, len(taps), B0.shape[-1], taps, precision="fp64", stream=stream)
        sep = Separator(F, T, M, D, len(taps), B0.shape[-1], taps, precision="fp64", stream=stream)
        sep.set_graph(True)
        B, V = as_device(B0, "fp64"), as_device(V0, "fp64")
        X1 = as_device(X, "fp64")
        X2 = as_device(X[:, :, ::-1].copy(), "fp64")
        for Xi in (X1, X2):
            for s in (ref, sep):
                s.set_input(Xi)
                s.set_state(B=B, V=V)
                s.iterate(3)
            stream.synchronize()
            assert torch.equal(ref.source_images(), sep.source_images())
        ref.close()
        sep.close()

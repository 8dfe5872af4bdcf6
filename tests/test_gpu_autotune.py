"""Measured launch-shape choice (ctfiss_autotune): the chosen plan is one of
the shapes that fit, the state is left as it was, the separation with the
tuned plan still matches the FP64 oracle, and a later context of the same
shape starts with the tuned plan."""
import numpy as np
import pytest

from test_gpu_parity import TOL1, as_device, gpu_run, make_case, oracle_run, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _fresh_plans():
    """Tuned plans are cached per process: leave none behind for the other tests."""
    from paper_2510_02382_amd import binding as b
    b.ctfiss_clear_tuned_plans()
    yield
    b.ctfiss_clear_tuned_plans()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", ["c1_like", "long_frames", "three_src"])
def test_autotune_keeps_state_and_parity(case, precision, monkeypatch):
    from paper_2510_02382_amd import Separator
    monkeypatch.delenv("CTFISS_PLAN", raising=False)
    X, B0, V0, W0, D, taps = make_case(case, seed=41)
    M, F, T = X.shape
    K = B0.shape[-1]
    sep = Separator(F, T, M, D, len(taps), K, taps, precision=precision)
    sep.set_input(as_device(X, precision))
    sep.set_state(B=as_device(B0, precision), V=as_device(V0, precision), W=as_device(W0, precision))
    before = [t.cpu().numpy() for t in sep.state()]
    plan = sep.autotune(trials=2)
    after = [t.cpu().numpy() for t in sep.state()]
    for a, b_ in zip(after, before):
        np.testing.assert_array_equal(a, b_)
    assert sep.status() == 0
    G, cpl, rpl, team = plan
    assert G in (16, 32, 64) and rpl in (1, 2) and team >= 1 and G * cpl * team >= T
    sep.iterate(1)
    W, B, V = (t.cpu().numpy() for t in sep.state())
    C = sep.source_images().cpu().numpy()
    sep.close()
    r = oracle_run(X, D, taps, B0, V0, W0, 1, precision)
    for k, g in (("W", W), ("B", B), ("V", V), ("C", C)):
        assert rel(g, r[k]) < TOL1[precision], (k, rel(g, r[k]))
    # a new context of this shape starts with the tuned plan
    sep2 = Separator(F, T, M, D, len(taps), K, taps, precision=precision)
    assert sep2.plan() == plan
    sep2.close()

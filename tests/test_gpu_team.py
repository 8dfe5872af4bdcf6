"""Team launches of the ISS W update against the FP64 oracle.

A bin whose rows and frames do not fit one workgroup (Mbar = 64 with T ~ 1000,
the precision workload) is split by frames over a team of workgroups that add
their partial frame sums in member order.  The split is forced on small shapes
through CTFISS_PLAN ("G,CPL,RPL,P"), so that uneven slices, slices barely
longer than the tap halo, both activation rules and the carried demixed rows
across calls are covered at sizes the oracle finishes in seconds; the long
Mbar = 64 shape takes the team path by itself.

Tolerances are those of the single-workgroup parity tests (relative Frobenius
norm per output): 1e-4 for FP32, 1e-11 for FP64 after one iteration, ten
times that after three.
"""
import numpy as np
import pytest

from test_gpu_parity import TOL1, gpu_run, make_case, oracle_run, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# case -> (FP32 team plan, FP64 team plan); the last field is the team size
FORCED = {
    "ragged": ("32,4,2,3", "16,4,2,3"),      # T = 100: slices 34, 34, 32; Mbar = 6
    "three_src": ("16,8,1,3", "16,4,1,3"),   # T = 150: three sources, Lmax - 1 = 2
    "max_rows": ("16,8,1,4", "16,4,1,4"),    # Mbar = 64, T = 100: slices of 25 >= Lmax - 1 = 21
    "c1_like": ("16,8,1,3", "16,8,1,3"),     # T = 313: slices 105, 105, 103
}


def _plan(case, precision):
    return FORCED[case][0 if precision == "fp32" else 1]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", list(FORCED))
def test_forced_team_matches_oracle(case, precision, monkeypatch):
    monkeypatch.setenv("CTFISS_PLAN", _plan(case, precision))
    X, B0, V0, W0, D, taps = make_case(case, seed=11)
    g = gpu_run(X, D, taps, B0, V0, W0, 1, precision)
    r = oracle_run(X, D, taps, B0, V0, W0, 1, precision)
    assert g["status"] == 0
    for k in ("W", "B", "V", "C"):
        assert rel(g[k], r[k]) < TOL1[precision], (k, rel(g[k], r[k]))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", ["ragged", "max_rows"])
def test_forced_team_carried_rows_across_calls(case, precision, monkeypatch):
    """iterate(2) then iterate(1): the second call starts from the carried Y
    slices each member wrote, with the pending rescale applied."""
    monkeypatch.setenv("CTFISS_PLAN", _plan(case, precision))
    X, B0, V0, W0, D, taps = make_case(case, seed=12)
    g = gpu_run(X, D, taps, B0, V0, W0, 3, precision, splits=[2, 1])
    r = oracle_run(X, D, taps, B0, V0, W0, 3, precision)
    assert g["status"] == 0
    for k in ("W", "B", "V", "C"):
        assert rel(g[k], r[k]) < 10 * TOL1[precision], (k, rel(g[k], r[k]))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_forced_team_paper_tap0_rule(precision, monkeypatch):
    monkeypatch.setenv("CTFISS_PLAN", _plan("three_src", precision))
    X, B0, V0, W0, D, taps = make_case("three_src", seed=13)
    g = gpu_run(X, D, taps, B0, V0, W0, 2, precision, "iss", "paper_tap0")
    r = oracle_run(X, D, taps, B0, V0, W0, 2, precision, "iss", "paper_tap0")
    for k in ("W", "B", "V"):
        assert rel(g[k], r[k]) < 10 * TOL1[precision], (k, rel(g[k], r[k]))


def test_team_and_single_workgroup_agree(monkeypatch):
    """The same bins through one workgroup and through a team of four differ
    only in the order of the frame sums."""
    X, B0, V0, W0, D, taps = make_case("max_rows", seed=14)
    single = gpu_run(X, D, taps, B0, V0, W0, 2, "fp64")
    monkeypatch.setenv("CTFISS_PLAN", _plan("max_rows", "fp64"))
    team = gpu_run(X, D, taps, B0, V0, W0, 2, "fp64")
    for k in ("W", "B", "V", "C"):
        assert rel(team[k], single[k]) < 1e-11, (k, rel(team[k], single[k]))


# Mbar = 64 with the precision workload's frame count: no single-workgroup
# plan exists, so the context takes a team plan by itself.
LONG = (3, 938, 4, 16, (22, 21, 21), 30)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_long_signal_mbar64_matches_oracle(precision, monkeypatch):
    import test_gpu_parity as tp
    monkeypatch.delenv("CTFISS_PLAN", raising=False)
    monkeypatch.setitem(tp.CASES, "long_mbar64", LONG)
    X, B0, V0, W0, D, taps = make_case("long_mbar64", seed=15)
    g = gpu_run(X, D, taps, B0, V0, W0, 1, precision)
    r = oracle_run(X, D, taps, B0, V0, W0, 1, precision)
    assert g["status"] == 0
    for k in ("W", "B", "V", "C"):
        assert rel(g[k], r[k]) < TOL1[precision], (k, rel(g[k], r[k]))


def test_team_plans_are_iss_only_and_not_batched(monkeypatch):
    from paper_2510_02382_amd import BatchSeparator
    from paper_2510_02382_amd import binding as b
    X, B0, V0, W0, D, taps = make_case("ragged", seed=16)
    monkeypatch.setenv("CTFISS_PLAN", "16,4,1,3")
    with pytest.raises(b.CtfissError) as e:
        gpu_run(X, D, taps, B0, V0, W0, 1, "fp64", rule="ip")
    assert e.value.status == b.CTFISS_E_UNSUPPORTED
    monkeypatch.delenv("CTFISS_PLAN")
    F, T, M, D_, tp_, K = LONG
    with pytest.raises(b.CtfissError) as e:
        BatchSeparator([(F, T, M, D_, len(tp_), K, tp_)], precision="fp32")
    assert e.value.status == b.CTFISS_E_UNSUPPORTED

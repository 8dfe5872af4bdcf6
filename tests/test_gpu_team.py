"""Team launches of the ISS W update against the FP64 oracle.

A bin whose rows and frames do not fit one workgroup (Mbar = 64 with T ~ 1000,
the precision workload) is split by frames over a team of workgroups that add
their partial frame sums in member order.  The split is forced on small shapes
through CTFISS_PLAN ("G,CPL,RPL,P"), so that uneven slices, slices barely
longer than the tap halo, both activation rules and the carried demixed rows
across calls are covered at sizes the oracle finishes in seconds; the long
Mbar = 64 shape takes the team path by itself.

Tolerances are those of the single-workgroup parity tests (relative Frobenius
norm and element-wise per group, tests/parity.py) after one iteration, ten
times those after three.
"""
import numpy as np
import pytest

from parity import check_outputs, elem_err, record
from test_gpu_parity import ELEM1, TOL1, gpu_run, make_case, oracle_run, rel

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
    check_outputs(None, g, r, TOL1[precision], ELEM1[precision])


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
    check_outputs(None, g, r, 10 * TOL1[precision], 10 * ELEM1[precision])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_forced_team_paper_tap0_rule(precision, monkeypatch):
    monkeypatch.setenv("CTFISS_PLAN", _plan("three_src", precision))
    X, B0, V0, W0, D, taps = make_case("three_src", seed=13)
    g = gpu_run(X, D, taps, B0, V0, W0, 2, precision, "iss", "paper_tap0")
    r = oracle_run(X, D, taps, B0, V0, W0, 2, precision, "iss", "paper_tap0")
    check_outputs(None, g, r, 10 * TOL1[precision], 10 * ELEM1[precision], keys=("W", "B", "V"))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_too_few_workgroups_for_a_team_are_raised_to_its_size(precision, monkeypatch):
    """CTFISS_WBLOCKS below the team size would leave a bin's members unable to run together;
    the library raises the count to the team size (here 3 workgroups for 7 bins x 3 members),
    and any count of at least one team gives the default launch's results bit for bit."""
    monkeypatch.setenv("CTFISS_PLAN", _plan("ragged", precision))
    X, B0, V0, W0, D, taps = make_case("ragged", seed=15)
    ref = gpu_run(X, D, taps, B0, V0, W0, 2, precision)
    monkeypatch.setenv("CTFISS_WBLOCKS", "1")
    g = gpu_run(X, D, taps, B0, V0, W0, 2, precision)
    assert g["status"] == 0 and ref["status"] == 0
    for k in ("W", "B", "V", "C"):
        assert np.array_equal(g[k], ref[k]), k


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
    check_outputs(None, g, r, TOL1[precision], ELEM1[precision])


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


# ------------------------------------------------------------------ 100 iterations at Mbar = 64
@pytest.fixture(scope="module")
def c3_slice():
    """Four bins of the 60 s precision-workload mixture (N = 3, M = 4, D = 16: Mbar = 64, taps
    22 + 21 + 21, T = 938, K = 30) and the FP64 oracle's 100 iterations on them."""
    from datagen import WORKLOADS, init_nmf, make_mixture
    from oracle import ctf_iss as o
    from oracle import threaded as oth
    wl = WORKLOADS["c3"]
    f0, nf = 600, 4
    X = np.ascontiguousarray(make_mixture(wl, 0).X[:, f0:f0 + nf, :])
    B0, V0 = init_nmf(wl.N, nf, wl.K, wl.T, 0)
    W, B, V = oth.run(X, wl.D, wl.row_taps, B0, V0, wl.n_iter)
    return X, B0, V0, wl, dict(W=W, B=B, V=V, C=o.source_images(W, X, wl.D, wl.row_taps))


@pytest.mark.parametrize("precision", ["mixed", "fp32", "fp64", "mixed_bf16"])
def test_mbar64_slice_100_iterations_against_oracle(c3_slice, precision, monkeypatch):
    """The team launch over a whole run of the precision workload's shape (four bins): every
    source image against the FP64 oracle on the original data.  Mixed precision meets the 1e-4
    target, mixed precision with bfloat16 NMF contractions the 1e-2 target; plain FP32 is held
    to what it measures (1.8e-4: its W takes 64 FP32-rounded rank-one updates per iteration);
    FP64 to 1e-9."""
    monkeypatch.delenv("CTFISS_PLAN", raising=False)
    X, B0, V0, wl, r = c3_slice
    g = gpu_run(X, wl.D, wl.row_taps, B0, V0, None, wl.n_iter, precision)
    assert g["status"] == 0
    tol = {"mixed": 1e-4, "fp32": 1e-3, "fp64": 1e-9, "mixed_bf16": 1e-2}[precision]
    for n in range(wl.N):
        e = rel(g["C"][n], r["C"][n])
        record(source=n, rel=e, elem=elem_err(g["C"][n:n + 1], r["C"][n:n + 1], "C"))
        assert e < tol, (n, e)


# ------------------------------------------------------------------ the whole precision workload
@pytest.mark.parametrize("precision,tol", [("mixed", 1e-4), ("mixed_bf16", 1e-2)])
def test_c3_whole_run_matches_oracle_images(precision, tol):
    """The precision workload at full size, as the benchmark runs it (60 s mixture, F = 2049,
    T = 938, Mbar = 64 in team launches, K = 30, 100 iterations from W = I): the source images
    of 16 bins spread over the band against the FP64 oracle's whole run of the same seeded
    mixture (tests/golden/c3_oracle_images.npz, written by make_c3_reference.py from the
    oracle only), per source within the targets (mixed 1e-4, bfloat16 NMF contractions 1e-2)."""
    import os
    from datagen import WORKLOADS, init_nmf, make_mixture
    from paper_2510_02382_amd import Separator
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle_images.npz")
    ref = np.load(path)
    bins, Cref = ref["bins"], ref["images"].astype(np.complex128)
    wl = WORKLOADS["c3"]
    assert int(ref["n_iter"]) == wl.n_iter
    X = make_mixture(wl, 0).X
    B0, V0 = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
    sep = Separator(wl.F, wl.T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision=precision)
    assert sep.plan()[3] > 1  # team launches
    sep.set_input(torch.from_numpy(X).to("cuda", torch.complex64))
    sep.set_state(B=torch.from_numpy(B0).to("cuda", torch.float32), V=torch.from_numpy(V0).to("cuda", torch.float32))
    sep.iterate(wl.n_iter)
    C = sep.source_images()[:, :, torch.as_tensor(bins, device="cuda"), :].cpu().numpy().astype(np.complex128)
    assert sep.status() == 0
    sep.close()
    for n in range(wl.N):
        e = rel(C[n], Cref[n])
        record(f"c3_whole_run[{precision}]", source=n, rel=e, elem=elem_err(C[n:n + 1], Cref[n:n + 1], "C"))
        assert e < tol, (n, e)

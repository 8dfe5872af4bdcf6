"""Mixed precision (CTFISS_MIXED) against the FP64 oracle.

The mixed path keeps the FP32 data, frame sums and NMF kernels and updates the
rows of W in FP64 registers during the ISS sweep.  One iteration is held to
the FP32 tolerance on every case; over 100 iterations of a mixture it must
stay well inside it (a pure FP32 sweep loses about an order of magnitude more
there, since W takes Mbar FP32-rounded rank-one updates per iteration).
"""
import numpy as np
import pytest

from parity import check_outputs, elem_err, record
from test_gpu_parity import (ELEM1, TOL1, gpu_run, make_case, mixture_slice, oracle_run, rel)
from oracle import ctf_iss as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("case", ["d1_tiny", "single_row", "ragged", "three_src", "short_T", "c1_like",
                                  "long_frames", "max_rows"])
def test_mixed_one_iteration_matches_oracle(case):
    X, B0, V0, W0, D, taps = make_case(case, seed=21)
    g = gpu_run(X, D, taps, B0, V0, W0, 1, "mixed")
    r = oracle_run(X, D, taps, B0, V0, W0, 1, "fp32")  # the oracle on the complex64/float32 inputs
    assert g["status"] == 0
    check_outputs(None, g, r, TOL1["fp32"], ELEM1["fp32"])


def test_mixed_paper_tap0_and_carried_rows():
    X, B0, V0, W0, D, taps = make_case("three_src", seed=22)
    g = gpu_run(X, D, taps, B0, V0, W0, 3, "mixed", "iss", "paper_tap0", splits=[2, 1])
    r = oracle_run(X, D, taps, B0, V0, W0, 3, "fp32", "iss", "paper_tap0")
    check_outputs(None, g, r, 10 * TOL1["fp32"], 10 * ELEM1["fp32"], keys=("W", "B", "V"))


def test_mixed_trajectory_c1_slice_100_iterations():
    """100 iterations on 12 bins of the long-reverberation mixture: the mixed
    path's images against the FP64 oracle, and against the FP32 path's."""
    X, B0, V0, wl = mixture_slice("c1", 300, 12)
    gm = gpu_run(X, wl.D, wl.row_taps, B0, V0, None, wl.n_iter, "mixed", "iss")
    g32 = gpu_run(X, wl.D, wl.row_taps, B0, V0, None, wl.n_iter, "fp32", "iss")
    W, B, V = o.run(X, wl.D, wl.row_taps, B0, V0, wl.n_iter, rule=o.ISS)
    C = o.source_images(W, X, wl.D, wl.row_taps)
    assert gm["status"] == 0
    em = [rel(gm["C"][n], C[n]) for n in range(wl.N)]
    e32 = [rel(g32["C"][n], C[n]) for n in range(wl.N)]
    assert max(em) < 2e-5, (em, e32)
    assert max(em) < max(e32), (em, e32)


# Mbar = 64 with T = 938: the frame-split team launch in mixed precision.
def test_mixed_long_signal_mbar64_matches_oracle(monkeypatch):
    import test_gpu_parity as tp
    monkeypatch.setitem(tp.CASES, "long_mbar64", (3, 938, 4, 16, (22, 21, 21), 30))
    X, B0, V0, W0, D, taps = make_case("long_mbar64", seed=23)
    g = gpu_run(X, D, taps, B0, V0, W0, 1, "mixed")
    r = oracle_run(X, D, taps, B0, V0, W0, 1, "fp32")
    assert g["status"] == 0
    check_outputs(None, g, r, TOL1["fp32"], ELEM1["fp32"])


def test_mixed_is_single_context_iss_only():
    from paper_2510_02382_amd import BatchSeparator
    from paper_2510_02382_amd import binding as b
    X, B0, V0, W0, D, taps = make_case("ragged", seed=24)
    with pytest.raises(b.CtfissError) as e:
        gpu_run(X, D, taps, B0, V0, W0, 1, "mixed", rule="ip")
    assert e.value.status == b.CTFISS_E_UNSUPPORTED
    M, F, T = X.shape
    with pytest.raises(b.CtfissError) as e:
        BatchSeparator([(F, T, M, D, len(taps), B0.shape[-1], taps)], precision="mixed")
    assert e.value.status == b.CTFISS_E_UNSUPPORTED

"""Seeded input generators: shapes, determinism, STFT pair, workload table."""
import numpy as np

from datagen import WORKLOADS, balanced_taps, init_nmf, istft, make_mixture, stft


def test_stft_istft_roundtrip_and_frame_count():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4000))
    S = stft(x, 256, 64)
    assert S.shape == (2, 129, 1 + 4000 // 64)
    np.testing.assert_allclose(istft(S, 256, 64, 4000), x, atol=1e-12)


def test_workload_shapes():
    assert (WORKLOADS["c0"].F, WORKLOADS["c0"].T, WORKLOADS["c0"].mbar) == (513, 251, 12)
    assert (WORKLOADS["c1"].F, WORKLOADS["c1"].T, WORKLOADS["c1"].mbar) == (1025, 313, 24)
    assert WORKLOADS["c1"].row_taps == (12, 12)
    assert WORKLOADS["c0_d1"].row_taps == (2, 1)
    assert balanced_taps(64, 3) == (22, 21, 21)
    assert WORKLOADS["P8"].row_taps == (4, 4)


def test_mixture_is_seeded():
    wl = WORKLOADS["c0"]
    a = make_mixture(wl, 3).X
    b = make_mixture(wl, 3).X
    c = make_mixture(wl, 4).X
    assert a.shape == (3, 513, 251)
    np.testing.assert_array_equal(a, b)
    assert not np.allclose(a, c)
    B0, V0 = init_nmf(2, 513, 10, 251, 3)
    assert B0.shape == (2, 513, 10) and V0.shape == (2, 10, 251)
    assert B0.min() >= 0.1 and V0.max() <= 1.0

"""Host checks of the separation-quality helpers used by the ISS/IP study."""
import numpy as np

from paper_2510_02382_amd.study import best_permutation_sdr, sdr_db


def test_sdr_closed_forms():
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((3, 5, 7)) + 1j * rng.standard_normal((3, 5, 7))
    assert sdr_db(ref, ref) == float("inf")
    # zero estimate: error power equals signal power -> 0 dB
    assert abs(sdr_db(ref, np.zeros_like(ref))) < 1e-12
    # estimate scaled by (1 - a): error = a ref -> -20 log10(a)
    assert abs(sdr_db(ref, 0.9 * ref) - 20.0) < 1e-9


def test_permutation_is_resolved():
    rng = np.random.default_rng(1)
    img = rng.standard_normal((2, 2, 4, 6)) + 1j * rng.standard_normal((2, 2, 4, 6))
    est = img[::-1] * 0.9  # swapped sources, each at 20 dB
    mean, per = best_permutation_sdr(img, est)
    assert abs(mean - 20.0) < 1e-9 and all(abs(v - 20.0) < 1e-9 for v in per)


def test_ctf_images_sum_to_the_mixture():
    """The images of a mixture drawn from Eq. (2) add up to the mixture, and each one is the
    filtered, delayed source it is defined as (checked at one bin by direct summation)."""
    import numpy as np

    from datagen import ctf_mixture
    from paper_2510_02382_amd.study import ctf_images
    taps = (2, 1)
    X, Ht, S = ctf_mixture(4, 9, 2, taps, 2, 5)
    C = ctf_images(Ht, S, taps)
    assert np.allclose(C.sum(axis=0), X, atol=1e-12)
    f, t = 2, 5
    direct = Ht[f, :, 0] * S[0, f, t] + Ht[f, :, 1] * S[0, f, t - 1]
    assert np.allclose(C[0, :, f, t], direct, atol=1e-12)

"""Pins of the FP64 PyTorch forward used for reference gradients (CPU).

* Its forward equals the NumPy oracle's (W, B, V and the images) on a case
  with stacked frames and uneven taps, under both activation rules: the two
  are written separately, so a dropped term or a wrong shift in either would
  show here.
* Its autograd gradients of the image MSE with respect to the mixture and the
  initial bases match central finite differences of the same forward, under
  both activation rules.
"""
import numpy as np
import pytest
import torch

from datagen import random_problem, rng_for
from oracle import ctf_iss as o
from oracle import ctf_iss_torch as ot


def _case(F, T, M, D, taps, K, seed):
    X, B0, V0 = random_problem(F, T, M, len(taps), K, seed, scale_spread=0.5)
    return X, B0, V0


@pytest.mark.parametrize("vrule", [o.ALL_TAPS, o.PAPER_TAP0])
def test_torch_forward_matches_numpy_oracle(vrule):
    F, T, M, D, taps, K = 3, 23, 2, 3, (4, 2), 3
    X, B0, V0 = _case(F, T, M, D, taps, K, 5)
    W, B, V = o.run(X, D, taps, B0, V0, 4, vrule=vrule)
    C = o.source_images(W, X, D, taps)
    Ct, Wt, Bt, Vt = ot.forward(torch.from_numpy(X), torch.from_numpy(B0), torch.from_numpy(V0), D, taps, 4,
                                vrule=vrule)
    for a, b in ((Wt, W), (Bt, B), (Vt, V), (Ct, C)):
        a = a.detach().numpy()
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12


def test_torch_tap_power_matches_index_loops():
    rng = rng_for(9)
    F, T, taps = 2, 7, (3, 2)
    Y = rng.standard_normal((F, 5, T)) + 1j * rng.standard_normal((F, 5, T))
    P = ot.tap_power(torch.from_numpy(Y), taps).numpy()
    rows = [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1)]
    for n in range(2):
        for f in range(F):
            for s in range(T):
                ref = sum(abs(Y[f, r, s + l]) ** 2 for r, (m, l) in enumerate(rows) if m == n and s + l < T)
                assert abs(P[n, f, s] - ref) < 1e-12
    c = ot.tap_count(taps, T).numpy()
    assert list(c[0]) == [3, 3, 3, 3, 3, 2, 1] and list(c[1]) == [2, 2, 2, 2, 2, 2, 1]


def test_torch_rules_differ():
    """The two activation rules give different activations once a source has more than one tap."""
    F, T, M, D, taps, K = 3, 23, 2, 3, (4, 2), 3
    X, B0, V0 = (torch.from_numpy(a) for a in _case(F, T, M, D, taps, K, 5))
    Va = ot.forward(X, B0, V0, D, taps, 1, vrule=ot.ALL_TAPS)[3]
    Vp = ot.forward(X, B0, V0, D, taps, 1, vrule=ot.PAPER_TAP0)[3]
    assert float((Va - Vp).abs().max()) > 1e-3 * float(Va.abs().max())


@pytest.mark.parametrize("vrule", [ot.ALL_TAPS, ot.PAPER_TAP0])
@pytest.mark.parametrize("seed", [0, 1])
def test_torch_gradients_match_central_differences(seed, vrule):
    F, T, M, D, taps, K, n_iter = 2, 12, 2, 2, (3, 1), 2, 3
    X, B0, V0 = _case(F, T, M, D, taps, K, 30 + seed)
    rng = rng_for(40 + seed)
    target = rng.standard_normal((len(taps), M, F, T)) + 1j * rng.standard_normal((len(taps), M, F, T))
    tg = torch.from_numpy(target)

    def loss(Xn, Bn):
        C = ot.forward(torch.from_numpy(Xn), torch.from_numpy(Bn), torch.from_numpy(V0), D, taps, n_iter,
                       vrule=vrule)[0]
        return float(ot.mse(C, tg))

    Xt = torch.from_numpy(X).requires_grad_(True)
    Bt = torch.from_numpy(B0).requires_grad_(True)
    C = ot.forward(Xt, Bt, torch.from_numpy(V0), D, taps, n_iter, vrule=vrule)[0]
    ot.mse(C, tg).backward()
    gX, gB = Xt.grad.numpy(), Bt.grad.numpy()
    dX = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
    dB = rng.standard_normal(B0.shape) * B0
    h = 1e-6
    fd_x = (loss(X + h * dX, B0) - loss(X - h * dX, B0)) / (2 * h)
    fd_b = (loss(X, B0 + h * dB) - loss(X, B0 - h * dB)) / (2 * h)
    an_x = float(np.sum(np.real(np.conj(gX) * dX)))
    an_b = float(np.sum(gB * dB))
    assert abs(an_x - fd_x) <= 1e-6 * abs(fd_x), (an_x, fd_x)
    assert abs(an_b - fd_b) <= 1e-6 * abs(fd_b), (an_b, fd_b)

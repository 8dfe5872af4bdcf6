"""FP64 PyTorch (CPU) forward of the unrolled CTF-MNMF-ISS iterations, for
reference gradients by automatic differentiation.

TEST INFRASTRUCTURE ONLY, like the NumPy oracle next to it: only the
test-suite may import it.  It is written separately from the NumPy oracle
(it imports nothing from it) so that the two pin each other, and its
autograd gradients are pinned against central finite differences.

The computation is the one the NumPy oracle documents, with the same
readings: ISS sweep with rows r ascending (Eqs. (11), (16); numerator
w_p^H Q_p w_r, z_r = 1 - d_r^{-1/2}), delayed variances dropped before frame 0,
basis update Eq. (17), activation update over all taps of a source (the
majorise-minimise step of Eq. (5); vrule "all_taps") or over tap 0 only
(Eq. (18) as printed; vrule "paper_tap0"), factor floor after each multiplicative
update, rescale Eqs. (19)-(21), and source images by projection back
(Eq. (24) with H = W^{-1}).  The loss is the mean over all elements of
|c - c_target|^2.
"""
from __future__ import annotations

import torch

FLOOR = 1e-8
ALL_TAPS = "all_taps"
PAPER_TAP0 = "paper_tap0"


def stacked(X, D):
    """xbar[f, d*M + m, t] = x[m, f, t - d], zero for t < d (Eq. (3) with D stacked frames)."""
    M, F, T = X.shape
    blocks = []
    for d in range(D):
        shifted = torch.cat([torch.zeros(M, F, d, dtype=X.dtype), X[:, :, :T - d]], dim=2)
        blocks.append(shifted.permute(1, 0, 2))  # [F, M, T]
    return torch.cat(blocks, dim=1)


def rows_of(taps):
    out = []
    for n, L in enumerate(taps):
        out += [(n, l) for l in range(L)]
    return out


def weights(lam, taps):
    """phi[f, r, t] = 1 / lambda[n, f, t - l] for row r = (n, l), 0 for t < l."""
    N, F, T = lam.shape
    rows = []
    for n, l in rows_of(taps):
        rows.append(torch.cat([torch.zeros(F, l, dtype=lam.dtype), 1.0 / lam[n, :, :T - l]], dim=1))
    return torch.stack(rows, dim=1)


def tap_power(Y, taps):
    """P[n, f, s] = sum over the taps l of source n of |y_(n,l)[s + l]|^2 (s + l < T)."""
    F, Mb, T = Y.shape
    P = [torch.zeros(F, T, dtype=torch.float64) for _ in taps]
    for r, (n, l) in enumerate(rows_of(taps)):
        a = Y[:, r, l:].abs() ** 2
        P[n] = P[n] + torch.cat([a, torch.zeros(F, l, dtype=torch.float64)], dim=1)
    return torch.stack(P)


def tap_count(taps, T):
    """c[n, s] = number of taps l of source n with s + l < T."""
    s = torch.arange(T, dtype=torch.float64)
    return torch.stack([torch.clamp(T - s, max=float(L)) for L in taps])


def iss_sweep(W, Y, phi):
    T = Y.shape[-1]
    Mb = W.shape[1]
    for r in range(Mb):
        yr = Y[:, r, :]
        wr = W[:, r, :]
        d = (phi * (yr.abs() ** 2)[:, None, :]).sum(-1) / T                 # [F, Mb]
        a = (phi * Y * yr.conj()[:, None, :]).sum(-1) / T                    # [F, Mb]
        own = torch.zeros(Mb, dtype=torch.bool)
        own[r] = True
        z = torch.where(own[None, :], (1.0 - d.rsqrt()).to(a.dtype), a / d)
        W = W - z[:, :, None] * wr[:, None, :]
        Y = Y - z[:, :, None] * yr[:, None, :]
    return W, Y


def tap0_power(Y, taps):
    """P0[n, f, s] = |y_(n,0)[s]|^2, the power of the first tap row of each source."""
    first = [sum(taps[:n]) for n in range(len(taps))]
    return torch.stack([Y[:, r, :].abs() ** 2 for r in first])


def iteration(W, B, V, Xb, taps, floor=FLOOR, vrule=ALL_TAPS):
    N, F, K = B.shape
    T = Xb.shape[-1]
    lam = B @ V
    W, Y = iss_sweep(W, W @ Xb, weights(lam, taps))
    P = tap_power(Y, taps)
    c = tap_count(taps, T)
    # bases, Eq. (17): sums over s of P v / lambda^2 and c v / lambda
    num = (P / lam ** 2) @ V.transpose(1, 2)
    den = (c[:, None, :] / lam) @ V.transpose(1, 2)
    B = torch.clamp(B * torch.sqrt(num / den), min=floor)
    # activations with the new bases: sums over f of b P / lambda^2 and b c / lambda, with
    # P the tap-0 power and c = 1 under Eq. (18) as printed
    if vrule == PAPER_TAP0:
        P, c = tap0_power(Y, taps), torch.ones_like(c)
    lam = B @ V
    num = B.transpose(1, 2) @ (P / lam ** 2)
    den = B.transpose(1, 2) @ (c[:, None, :] / lam)
    V = torch.clamp(V * torch.sqrt(num / den), min=floor)
    # rescale, Eqs. (19)-(21)
    mu = torch.sqrt((Y.abs() ** 2).mean(dim=(0, 2)))
    W = W / mu[None, :, None]
    first = [sum(taps[:n]) for n in range(len(taps))]
    B = B / (mu[first] ** 2)[:, None, None]
    return W, B, V


def images(W, Xb, taps, M):
    """c[n, m, f, t] = sum over the rows r of source n of H[m, r] y_r[t], H = W^{-1}."""
    H = torch.linalg.inv(W)
    Y = W @ Xb
    out = []
    r0 = 0
    for L in taps:
        out.append((H[:, :M, r0:r0 + L] @ Y[:, r0:r0 + L, :]).permute(1, 0, 2))
        r0 += L
    return torch.stack(out)


def forward(X, B0, V0, D, taps, n_iter, floor=FLOOR, vrule=ALL_TAPS):
    """Images after n_iter iterations from W = I (Sec. V-A), B0, V0."""
    M, F, T = X.shape
    Xb = stacked(X, D)
    Mb = Xb.shape[1]
    W = torch.eye(Mb, dtype=torch.complex128).expand(F, Mb, Mb)
    B, V = B0, V0
    for _ in range(n_iter):
        W, B, V = iteration(W, B, V, Xb, taps, floor, vrule)
    return images(W, Xb, taps, M), W, B, V


def mse(C, target):
    return ((C - target).abs() ** 2).mean()

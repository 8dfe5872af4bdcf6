"""Pins of the CPU oracle against the mathematics of the paper, not against itself.

Each test checks the oracle with something independent of its own code: brute
force loops over the paper's index sums on tiny inputs, closed forms derived
from the equations, finite-difference stationarity, the matrix determinant
lemma checked with a library determinant, a library generalised eigensolver,
library matrix inverses, and separation of a noiseless mixture with known
mixing drawn from the CTF model of Eq. (2).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

from datagen import ctf_mixture, random_problem, rng_for
from oracle import ctf_iss as o


# ------------------------------------------------------------------ helpers
def brute_Q(X, D, taps, lam, r):
    """Weighted covariance of Eq. (8) for row r of one bin, by explicit loops.

    X: [M, T] complex (one bin), lam: [N, T].  Builds each stacked frame from
    its definition and accumulates xbar xbar^H / lambda_{n, t - l}.
    """
    M, T = X.shape
    src = [n for n, L in enumerate(taps) for _ in range(L)]
    tap = [l for L in taps for l in range(L)]
    Mb = M * D
    Q = np.zeros((Mb, Mb), dtype=complex)
    for t in range(T):
        if t - tap[r] < 0:
            continue
        xb = np.zeros(Mb, dtype=complex)
        for d in range(D):
            for m in range(M):
                if t - d >= 0:
                    xb[d * M + m] = X[m, t - d]
        Q += np.outer(xb, np.conj(xb)) / lam[src[r], t - tap[r]]
    return Q / T


def w_cost(W, Qs, T):
    """W-dependent part of Eq. (5) for one bin given the Q_r of Eq. (8): T (sum_r w_r^H Q_r w_r) - 2T log|det W|."""
    tot = 0.0
    for r, Q in enumerate(Qs):
        w = np.conj(W[r])            # column vector w_r (row r of W is w_r^H)
        tot += np.real(np.conj(w) @ Q @ w)
    return T * tot - 2 * T * np.log(np.abs(np.linalg.det(W)))


def tiny(F=2, T=17, M=2, D=2, taps=(3, 1), K=2, seed=0, spread=0.5):
    X, B0, V0 = random_problem(F, T, M, len(taps), K, seed, scale_spread=spread)
    rng = rng_for(seed + 7)
    Mb = M * D
    W = np.eye(Mb) + 0.3 * (rng.standard_normal((F, Mb, Mb)) + 1j * rng.standard_normal((F, Mb, Mb)))
    return X, B0, V0, W


# ------------------------------------------------------------------ row map and view
def test_row_map_and_stacked_view_brute():
    taps = (3, 1, 2)
    src, tap = o.row_map(taps)
    for n, L in enumerate(taps):
        for l in range(L):
            r = sum(taps[:n]) + l          # flattened index below Eq. (10), 0-based
            assert src[r] == n and tap[r] == l
    assert list(o.first_row(taps)) == [0, 3, 4]
    X, _, _ = random_problem(3, 9, 2, 2, 1, 1)
    D = 3
    Xb = o.stacked_view(X, D)
    for f, t, d, m in itertools.product(range(3), range(9), range(D), range(2)):
        expect = X[m, f, t - d] if t - d >= 0 else 0.0
        assert Xb[f, d * 2 + m, t] == expect


def test_nll_matches_brute_force_sum():
    X, B0, V0, W = tiny()
    taps, D = (3, 1), 2
    F, T = X.shape[1:]
    lam = np.einsum("nfk,nkt->nft", B0, V0)
    Xb = o.stacked_view(X, D)
    src = [n for n, L in enumerate(taps) for _ in range(L)]
    tap = [l for L in taps for l in range(L)]
    tot = 0.0
    for f in range(F):
        for r in range(sum(taps)):
            for t in range(T):
                if t - tap[r] < 0:
                    continue
                y = W[f, r] @ Xb[f, :, t]          # w_r^H xbar, row r of W holds w_r^H
                lm = lam[src[r], f, t - tap[r]]
                tot += np.log(lm) + abs(y) ** 2 / lm
        tot -= 2 * T * np.log(abs(np.linalg.det(W[f])))
    assert o.nll(W, Xb, B0, V0, taps) == pytest.approx(tot, rel=1e-12)


# ------------------------------------------------------------------ ISS
def _iss_setup(seed=0):
    X, B0, V0, W = tiny(seed=seed)
    taps, D = (3, 1), 2
    lam = o.psd(B0, V0)
    Xb = o.stacked_view(X, D)
    phi = o.row_weights(lam, taps)
    return X, B0, V0, W, taps, D, lam, Xb, phi


@pytest.mark.parametrize("r", [0, 2, 3])
def test_iss_step_is_stationary_point(r):
    """Finite-difference gradient of the ISS sub-objective, Eq. (12), vanishes at the oracle's z."""
    X, B0, V0, W, taps, D, lam, Xb, phi = _iss_setup()
    T = X.shape[-1]
    f = 1
    Qs = [brute_Q(X[:, f], D, taps, lam[:, f], p) for p in range(sum(taps))]
    _, _, z = o.iss_step(W, o.demix(W, Xb), phi, r)
    z = z[f]
    wr_row = W[f, r].copy()

    def cost(zv):
        return w_cost(W[f] - np.outer(zv, wr_row), Qs, T)

    h = 1e-6
    for p in range(len(z)):
        for step in (h, 1j * h):
            e = np.zeros_like(z)
            e[p] = step
            g = (cost(z + e) - cost(z - e)) / (2 * h)
            assert abs(g) < 1e-4 * T, (p, step, g)
    # The product order printed in Eq. (16), w_r^H Q_p w_p, is the conjugate of the stationary
    # numerator; at that z the gradient does not vanish (whenever z_p is not real).
    wr = np.conj(wr_row)
    zp = z.copy()
    for p in range(len(z)):
        if p != r:
            zp[p] = (np.conj(wr) @ Qs[p] @ np.conj(W[f, p])) / np.real(np.conj(wr) @ Qs[p] @ wr)
            np.testing.assert_allclose(zp[p], np.conj(z[p]), rtol=1e-10)
    p_off = int(np.argmax(np.abs(np.imag(zp))))
    e = np.zeros_like(z)
    e[p_off] = 1j * h
    assert abs((cost(zp + e) - cost(zp - e)) / (2 * h)) > 1e-2


def test_iss_decrease_equals_closed_form():
    """Measured NLL drop of one ISS step equals T * sum_f [sum_{p!=r} |a_p|^2/d_p + d_r - 1 - log d_r].

    With lambda fixed, the W part of Eq. (5) is T sum_p w_p^H Q_p w_p - 2T log|det W|.  Row p != r
    changes by -|a_p|^2/d_p with a_p = w_p^H Q_p w_r, d_p = w_r^H Q_p w_r; row r becomes
    |1 - z_r|^2 d_r = 1 and the log-det term changes by -2 log|1 - z_r| = log d_r.
    a_p and d_p are taken from explicitly built Q matrices, not from the oracle.
    """
    X, B0, V0, W, taps, D, lam, Xb, phi = _iss_setup(seed=3)
    T = X.shape[-1]
    F = X.shape[1]
    for r in range(sum(taps)):
        before = o.nll(W, Xb, B0, V0, taps)
        predicted = 0.0
        for f in range(F):
            Qs = [brute_Q(X[:, f], D, taps, lam[:, f], p) for p in range(sum(taps))]
            wr = np.conj(W[f, r])
            for p, Q in enumerate(Qs):
                d = np.real(np.conj(wr) @ Q @ wr)
                if p == r:
                    predicted += d - 1 - np.log(d)
                else:
                    a = W[f, p] @ Q @ wr           # w_p^H Q_p w_r
                    predicted += abs(a) ** 2 / d
        Y = o.demix(W, Xb)
        W2, Y2, _ = o.iss_step(W, Y, phi, r)
        np.testing.assert_allclose(Y2, o.demix(W2, Xb), rtol=0, atol=1e-10)
        after = o.nll(W2, Xb, B0, V0, taps)
        assert before - after == pytest.approx(T * predicted, rel=1e-8, abs=1e-8)
        assert after <= before + 1e-9
        W = W2


def test_iss_determinant_lemma():
    """log|det W| after a step = before + log|1 - z_r| (matrix determinant lemma, Eq. (13))."""
    X, B0, V0, W, taps, D, lam, Xb, phi = _iss_setup(seed=5)
    for r in range(sum(taps)):
        W2, _, z = o.iss_step(W, o.demix(W, Xb), phi, r)
        _, ld1 = np.linalg.slogdet(W)
        _, ld2 = np.linalg.slogdet(W2)
        np.testing.assert_allclose(ld2, ld1 + np.log(np.abs(1 - z[:, r])), rtol=0, atol=1e-11)
        W = W2


def test_iss_single_row_normalises():
    """Mbar = 1: the update reduces to w <- w / sqrt(d) with d the weighted power."""
    X, B0, V0 = random_problem(3, 11, 1, 1, 2, 4)
    W = np.full((3, 1, 1), 1.7 - 0.4j)
    lam = o.psd(B0, V0)
    phi = o.row_weights(lam, (1,))
    Xb = o.stacked_view(X, 1)
    W2, Y2, _ = o.iss_step(W, o.demix(W, Xb), phi, 0)
    y = W[:, 0, 0][:, None] * X[0]
    d = np.mean(np.abs(y) ** 2 / lam[0], axis=-1)
    np.testing.assert_allclose(W2[:, 0, 0], W[:, 0, 0] / np.sqrt(d), rtol=1e-13)


def test_iss_converges_to_head_and_generalised_eigenvectors():
    """Frozen lambda, Mbar = 2: repeated ISS sweeps reach the stationary (HEAD) conditions
    W Q_r w_r = e_r, and each row is a generalised eigenvector of (Q_1, Q_2) (scipy eigh)."""
    X, B0, V0 = random_problem(2, 200, 2, 2, 2, 11, scale_spread=0.7)
    taps, D = (1, 1), 1
    lam = o.psd(B0, V0)
    Xb = o.stacked_view(X, D)
    phi = o.row_weights(lam, taps)
    W = np.tile(np.eye(2, dtype=complex), (2, 1, 1))
    Y = o.demix(W, Xb)
    for _ in range(300):
        W, Y = o.iss_sweep(W, Y, phi)
    for f in range(2):
        Qs = [brute_Q(X[:, f], D, taps, lam[:, f], r) for r in range(2)]
        for r in range(2):
            col = W[f] @ Qs[r] @ np.conj(W[f, r])
            np.testing.assert_allclose(col, np.eye(2)[r], atol=1e-8)
        _, vecs = scipy.linalg.eigh(Qs[0], Qs[1])
        for r in range(2):
            w = np.conj(W[f, r])
            cos = max(abs(np.vdot(vecs[:, i], w)) / (np.linalg.norm(vecs[:, i]) * np.linalg.norm(w))
                      for i in range(2))
            assert cos == pytest.approx(1.0, abs=1e-8)


# ------------------------------------------------------------------ IP
def test_ip_step_matches_explicit_inverse_and_head():
    """IP, Eqs. (9)-(10): solve equals the explicit inverse; after the update of row r,
    W Q_r w_r = e_r exactly; the NLL does not increase."""
    X, B0, V0, W, taps, D, lam, Xb, phi = _iss_setup(seed=2)
    for r in range(sum(taps)):
        before = o.nll(W, Xb, B0, V0, taps)
        W2 = o.ip_step(W, Xb, phi, r)
        for f in range(X.shape[1]):
            Q = brute_Q(X[:, f], D, taps, lam[:, f], r)
            u = np.linalg.inv(W[f] @ Q)[:, r]
            u = u / np.sqrt(np.real(np.conj(u) @ Q @ u))
            np.testing.assert_allclose(W2[f, r], np.conj(u), rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(W2[f] @ Q @ np.conj(W2[f, r]), np.eye(sum(taps))[r], atol=1e-10)
        assert o.nll(W2, Xb, B0, V0, taps) <= before + 1e-9
        W = W2


# ------------------------------------------------------------------ NMF updates
def brute_update_B(B, V, Y, taps):
    N, F, K = B.shape
    T = V.shape[-1]
    lam = np.zeros((N, F, T))
    for n, f, t in itertools.product(range(N), range(F), range(T)):
        lam[n, f, t] = sum(B[n, f, k] * V[n, k, t] for k in range(K))
    out = B.copy()
    for n, f, k in itertools.product(range(N), range(F), range(K)):
        num = den = 0.0
        for t in range(T):
            for l in range(taps[n]):
                if t - l < 0:
                    continue
                y = Y[f, sum(taps[:n]) + l, t]
                num += abs(y) ** 2 * V[n, k, t - l] / lam[n, f, t - l] ** 2
                den += V[n, k, t - l] / lam[n, f, t - l]
        out[n, f, k] = B[n, f, k] * np.sqrt(num / den)
    return out


def brute_update_V(B, V, Y, taps, tap0):
    N, F, K = B.shape
    T = V.shape[-1]
    lam = np.einsum("nfk,nkt->nft", B, V)
    out = V.copy()
    for n, k, t in itertools.product(range(N), range(K), range(T)):
        num = den = 0.0
        for f in range(F):
            for l in range(1 if tap0 else taps[n]):
                if t + l >= T:
                    continue
                y = Y[f, sum(taps[:n]) + l, t + l]
                num += abs(y) ** 2 * B[n, f, k] / lam[n, f, t] ** 2
                den += B[n, f, k] / lam[n, f, t]
        out[n, k, t] = V[n, k, t] * np.sqrt(num / den)
    return out


def test_mu_updates_match_brute_force_sums():
    X, B0, V0, W = tiny(F=2, T=7, seed=9)
    taps = (3, 1)
    Y = o.demix(W, o.stacked_view(X, 2))
    np.testing.assert_allclose(o.update_B(B0, V0, Y, taps, floor=0.0), brute_update_B(B0, V0, Y, taps), rtol=1e-12)
    for vr, tap0 in ((o.ALL_TAPS, False), (o.PAPER_TAP0, True)):
        np.testing.assert_allclose(o.update_V(B0, V0, Y, taps, vr, floor=0.0),
                                   brute_update_V(B0, V0, Y, taps, tap0), rtol=1e-12)


@pytest.mark.parametrize("floor", [0.0, 1e-8, 0.3])
def test_mu_updates_monotone_and_nonnegative(floor):
    """MM guarantee: each update (ALL_TAPS) does not increase Eq. (5); the clamp to the floor is
    the exact minimiser of the auxiliary over the box, so this holds with an active floor too."""
    for seed in range(4):
        X, B, V, W = tiny(F=3, T=40, seed=seed)
        taps, D = (3, 1), 2
        Xb = o.stacked_view(X, D)
        Y = o.demix(W, Xb)
        for _ in range(5):
            c0 = o.nll(W, Xb, B, V, taps)
            B = o.update_B(B, V, Y, taps, floor)
            c1 = o.nll(W, Xb, B, V, taps)
            V = o.update_V(B, V, Y, taps, o.ALL_TAPS, floor)
            c2 = o.nll(W, Xb, B, V, taps)
            assert c1 <= c0 + 1e-9 * abs(c0) and c2 <= c1 + 1e-9 * abs(c1)
            assert B.min() >= floor and V.min() >= floor and B.min() > 0


def test_paper_tap0_equals_all_taps_with_single_taps():
    X, B0, V0 = random_problem(3, 12, 2, 2, 2, 21)
    W = np.tile(np.eye(2, dtype=complex), (3, 1, 1))
    Y = o.demix(W, o.stacked_view(X, 1))
    np.testing.assert_array_equal(o.update_V(B0, V0, Y, (1, 1), o.PAPER_TAP0),
                                  o.update_V(B0, V0, Y, (1, 1), o.ALL_TAPS))


def test_rescale_gives_unit_row_power():
    X, B0, V0, W = tiny(seed=13)
    taps, D = (3, 1), 2
    Xb = o.stacked_view(X, D)
    Y = o.demix(W, Xb)
    W2, B2, mu = o.rescale(W, B0, Y, taps)
    Y2 = o.demix(W2, Xb)
    np.testing.assert_allclose(np.mean(np.abs(Y2) ** 2, axis=(0, 2)), 1.0, rtol=1e-12)
    np.testing.assert_allclose(B2[0] * mu[0] ** 2, B0[0], rtol=1e-13)
    np.testing.assert_allclose(B2[1] * mu[3] ** 2, B0[1], rtol=1e-13)


def test_full_iteration_does_not_increase_cost_before_rescale():
    """W update, then b, then v: the NLL is non-increasing at every stage (rescale excluded)."""
    X, B, V, _ = tiny(F=3, T=30, seed=17)
    taps, D = (3, 1), 2
    Xb = o.stacked_view(X, D)
    W = np.tile(np.eye(4, dtype=complex), (3, 1, 1))
    for rule in (o.ISS, o.IP):
        Wc, Bc, Vc = W.copy(), B.copy(), V.copy()
        for _ in range(4):
            c0 = o.nll(Wc, Xb, Bc, Vc, taps)
            phi = o.row_weights(o.psd(Bc, Vc), taps)
            if rule == o.ISS:
                Wc, Y = o.iss_sweep(Wc, o.demix(Wc, Xb), phi)
            else:
                Wc, Y = o.ip_sweep(Wc, Xb, phi)
            c1 = o.nll(Wc, Xb, Bc, Vc, taps)
            Bc = o.update_B(Bc, Vc, Y, taps)
            Vc = o.update_V(Bc, Vc, Y, taps)
            c2 = o.nll(Wc, Xb, Bc, Vc, taps)
            assert c1 <= c0 + 1e-9 * abs(c0) and c2 <= c1 + 1e-9 * abs(c1)
            Wc, Bc, _ = o.rescale(Wc, Bc, Y, taps)


# ------------------------------------------------------------------ source images
@pytest.mark.parametrize("D,taps", [(1, (2, 1)), (2, (3, 1))])
def test_projection_back_equals_mwf_and_sums_to_mixture(D, taps):
    M = sum(taps) // D
    X, B0, V0 = random_problem(2, 6, M, len(taps), 2, 31)
    rng = rng_for(32)
    Mb = M * D
    W = np.eye(Mb) + 0.4 * (rng.standard_normal((2, Mb, Mb)) + 1j * rng.standard_normal((2, Mb, Mb)))
    C = o.source_images(W, X, D, taps)
    np.testing.assert_allclose(C, o.mwf_images(W, X, D, taps, B0, V0), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(C.sum(axis=0), X, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------ known mixing
@pytest.mark.parametrize("rule", [o.ISS, o.IP])
def test_noiseless_known_mixing_is_separated(rule):
    """Data drawn from Eq. (2) with a square extended mixing matrix: W_f Htilde_f becomes a
    scaled permutation in every bin (row dominance near 1)."""
    taps = (2, 1)
    for seed in (0, 1):
        X, Ht, _ = ctf_mixture(6, 400, 2, taps, 2, seed)
        rng = rng_for(seed + 100)
        B0 = rng.uniform(0.1, 1, (2, 6, 2))
        V0 = rng.uniform(0.1, 1, (2, 2, 400))
        W, _, _ = o.run(X, 1, taps, B0, V0, 200, rule=rule)
        P = np.abs(W @ Ht) ** 2
        dom = P.max(-1) / P.sum(-1)
        assert np.median(dom) > 0.98 and dom.min() > 0.5
        for f in range(6):
            assert sorted(np.argmax(P[f], -1)) == [0, 1, 2]


def test_threaded_driver_equals_serial_oracle():
    """oracle.threaded runs the W update of bin chunks on a thread pool and the rest of each
    iteration on the whole arrays; per bin it is ctf_iss.run's arithmetic (both rules)."""
    from oracle import threaded as th
    X, B0, V0 = random_problem(7, 40, 2, 2, 3, 5, scale_spread=0.5)
    for rule in (o.ISS, o.IP):
        W1, B1, V1 = o.run(X, 2, (2, 2), B0, V0, 4, rule=rule)
        W2, B2, V2 = th.run(X, 2, (2, 2), B0, V0, 4, rule=rule, workers=3, chunk=2)
        for a, b in ((W1, W2), (B1, B2), (V1, V2)):
            assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))

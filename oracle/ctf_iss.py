"""Plain FP64 CPU oracle of CTF-MNMF with ISS (and IP) demixing updates.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the CPU-baseline leg of the benchmark may import or call anything here; the
product path (the HIP library and its Python binding) never does, and shares
no code with this module.

Everything is complex128 / float64 and written in the order of the paper
(Xie et al., "Accelerated Convolutive Transfer Function-Based Multichannel NMF
Using Iterative Source Steering", APSIPA ASC 2025).  The paper's indices are
i (frequency bin) and j (frame); here they are f and t, both 0-based.  The
flattened row index r of the extended demixing matrix is 0-based as well.

Readings of points the paper leaves open (each is applied identically by the
GPU path):
  * Frame stacking: an observation may stack D delayed frames,
    xbar_{f,t}[d*M + m] = x_{m,f,t-d} (zero before the first frame), giving
    Mbar = M*D "virtual microphones".  D = 1 is exactly the paper's square
    model (sum of taps = M, Sec. II).
  * Delayed variances before the first frame: a term whose delayed index
    t - l is negative is dropped from the cost, Q, the MU sums (weight 0),
    while the 1/T normalisation of Q is kept.
  * ISS numerator: the closed form of Eq. (16) is used with the numerator
    w_p^H Q_p w_r, the stationary point of the ISS sub-objective Eq. (12)
    with respect to z_p^*; the printed order of the product is its conjugate.
  * The p = r branch of Eq. (16) takes the real positive root,
    z_r = 1 - (w_r^H Q_r w_r)^{-1/2}.
  * Activation update: ALL_TAPS (default) sums every tap of a source, which
    is the majorise-minimise step of Eq. (5); PAPER_TAP0 is Eq. (18) as
    printed (tap 0 only).  They coincide when a source has one tap.
  * The sum over l in Eq. (17) runs over the taps of source n (0..L_n-1).
  * Update order inside one iteration: W (all rows r ascending) -> b -> v ->
    rescale, with lambda recomputed from the current b, v before each update.
  * Rescaling, Eqs. (19)-(21): W row (n,l) is divided by mu_{n,l} and b_n by
    mu_{n,0}^2, as printed.
  * Factor floor: the paper states no safeguard.  With stacked frames the
    per-bin demixing matrix has many more coefficients than the frames can
    pin down, a row can null a frame exactly and the likelihood is unbounded
    below along lambda -> 0 (both ISS and IP reach it within about 30
    iterations on reverberant mixtures).  After each multiplicative update the
    factors are therefore clamped, b, v >= floor (default 1e-8).  The MM
    auxiliary function of Eq. (17)/(18) is convex in each factor, so the clamp
    is its exact minimiser over the box {b, v >= floor} and the update stays a
    descent step.  floor = 0 reproduces the printed update.
  * Source images, Eq. (24): with a square invertible H = W^{-1} the
    multichannel Wiener filter reduces exactly to projection back,
    c_n = H_n y_n; with D > 1 the first M rows (the undelayed block) are
    returned.
"""
from __future__ import annotations

import numpy as np

ISS = "iss"
FLOOR = 1e-8
IP = "ip"
ALL_TAPS = "all_taps"
PAPER_TAP0 = "paper_tap0"


# ------------------------------------------------------------ index maps
def row_map(taps):
    """Flattened row index r <-> (source n, tap l), Sec. III-A-1 (below Eq. (10)).

    r = L_1 + ... + L_{n-1} + l (0-based), i.e. source-major, tap-minor.
    Returns integer arrays src[r], tap[r].
    """
    src, tap = [], []
    for n, L in enumerate(taps):
        for l in range(L):
            src.append(n)
            tap.append(l)
    return np.asarray(src, dtype=np.int64), np.asarray(tap, dtype=np.int64)


def first_row(taps):
    """Row index of tap 0 of each source."""
    return np.concatenate([[0], np.cumsum(taps)[:-1]]).astype(np.int64)


def stacked_view(X, D):
    """Observation vectors, Eq. (3), with D stacked delayed frames.

    X: [M, F, T] complex.  Returns xbar [F, M*D, T] with
    xbar[f, d*M + m, t] = X[m, f, t - d] for t >= d and 0 otherwise.
    """
    X = np.asarray(X, dtype=np.complex128)
    M, F, T = X.shape
    Xb = np.zeros((F, M * D, T), dtype=np.complex128)
    for d in range(D):
        Xb[:, d * M:(d + 1) * M, d:] = np.transpose(X[:, :, :T - d], (1, 0, 2))
    return Xb


# ------------------------------------------------------------ source model
def psd(B, V):
    """NMF source variance lambda_{n,f,t} = sum_k b_{n,f,k} v_{n,k,t} (Sec. II).

    B: [N, F, K], V: [N, K, T] -> [N, F, T].
    """
    return np.matmul(B, V)


def row_weights(lam, taps):
    """Inverse delayed variance of each demixed row, phi[f, r, t] = 1 / lambda_{n(r), f, t - l(r)}.

    Row r = (n, l) at frame t is modelled with variance lambda_{n, f, t-l}
    (Sec. II, source model; Eq. (8)).  Frames t < l get weight 0.
    """
    N, F, T = lam.shape
    src, tap = row_map(taps)
    phi = np.zeros((F, len(src), T))
    for r in range(len(src)):
        l = tap[r]
        phi[:, r, l:] = 1.0 / lam[src[r], :, :T - l]
    return phi


def demix(W, Xb):
    """y_{r,f,t} = w_{r,f}^H xbar_{f,t}, Eq. (4).  W[f, r, :] holds the row w_r^H."""
    return np.matmul(W, Xb)


# ------------------------------------------------------------ W update: ISS
def iss_step(W, Y, phi, r):
    """One rank-1 ISS update of every bin for row r, Eqs. (11) and (16).

    With Q_p the weighted covariance of Eq. (8), the sub-problem coefficients
    are evaluated in the demixed domain:
        d_p = w_r^H Q_p w_r = (1/T) sum_t phi_p |y_r|^2,
        a_p = w_p^H Q_p w_r = (1/T) sum_t phi_p y_p conj(y_r),
    z_p = a_p / d_p for p != r and z_r = 1 - d_r^{-1/2}; then
    W <- W - z w_r^H and Y <- Y - z y_r with the pre-update row r.
    Returns (W, Y, z) with z [F, Mbar].
    """
    T = Y.shape[-1]
    yr = Y[:, r, :].copy()
    wr = W[:, r, :].copy()
    d = np.einsum("fpt,ft->fp", phi, np.abs(yr) ** 2) / T
    a = np.matmul(phi * Y, np.conj(yr)[:, :, None])[:, :, 0] / T
    z = a / d
    z[:, r] = 1.0 - 1.0 / np.sqrt(d[:, r])
    W = W - z[:, :, None] * wr[:, None, :]
    Y = Y - z[:, :, None] * yr[:, None, :]
    return W, Y, z


def iss_sweep(W, Y, phi):
    """ISS updates for r = 0 .. Mbar-1 in ascending order (Sec. III-A-1)."""
    for r in range(W.shape[1]):
        W, Y, _ = iss_step(W, Y, phi, r)
    return W, Y


# ------------------------------------------------------------ W update: IP
def weighted_cov(Xb, phi_r):
    """Q_{r,f} = (1/T) sum_t xbar xbar^H / lambda_{n,f,t-l}, Eq. (8).  Returns [F, Mbar, Mbar]."""
    T = Xb.shape[-1]
    return np.matmul(Xb * phi_r[:, None, :], np.conj(np.swapaxes(Xb, 1, 2))) / T


def ip_step(W, Xb, phi, r):
    """Iterative-projection update of row r in every bin, Eqs. (9) and (10).

    u = (W Q_r)^{-1} e_r, then u <- u (u^H Q_r u)^{-1/2}; row r of W becomes u^H.
    """
    F, Mb, _ = W.shape
    Q = weighted_cov(Xb, phi[:, r, :])
    e = np.zeros((F, Mb, 1), dtype=np.complex128)
    e[:, r, 0] = 1.0
    u = np.linalg.solve(np.matmul(W, Q), e)[:, :, 0]
    s = np.real(np.einsum("fi,fij,fj->f", np.conj(u), Q, u))
    u = u / np.sqrt(s)[:, None]
    W = W.copy()
    W[:, r, :] = np.conj(u)
    return W


def ip_sweep(W, Xb, phi):
    """IP updates for r = 0 .. Mbar-1, then the demixed signals of the final W."""
    for r in range(W.shape[1]):
        W = ip_step(W, Xb, phi, r)
    return W, demix(W, Xb)


# ------------------------------------------------------------ Lambda update
def update_B(B, V, Y, taps, floor=FLOOR):
    """Multiplicative update of the bases, Eq. (17), then the factor floor.

    b_{n,f,k} <- b * sqrt( sum_t sum_l |y_{n,f,t,l}|^2 v_{n,k,t-l} lambda^{-2}_{n,f,t-l}
                          / sum_t sum_l v_{n,k,t-l} lambda^{-1}_{n,f,t-l} ),
    l over the taps of source n, terms with t - l < 0 dropped; b <- max(b, floor).
    """
    lam = psd(B, V)
    T = Y.shape[-1]
    src, tap = row_map(taps)
    num = np.zeros_like(B)
    den = np.zeros_like(B)
    for r in range(len(src)):
        n, l = src[r], tap[r]
        A = np.abs(Y[:, r, l:]) ** 2              # |y_{n,f,t,l}|^2 for t = l .. T-1
        lam_d = lam[n][:, :T - l]                  # lambda_{n,f,t-l}
        v_d = V[n][:, :T - l]                      # v_{n,k,t-l}
        num[n] += (A / lam_d ** 2) @ v_d.T
        den[n] += (1.0 / lam_d) @ v_d.T
    return np.maximum(B * np.sqrt(num / den), floor)


def update_V(B, V, Y, taps, vrule=ALL_TAPS, floor=FLOOR):
    """Multiplicative update of the activations.

    PAPER_TAP0 is Eq. (18) as printed:
        v_{n,k,t} <- v * sqrt( sum_f |y_{n,f,t,0}|^2 b lambda^{-2}_{n,f,t} / sum_f b lambda^{-1}_{n,f,t} ).
    ALL_TAPS adds every tap l of source n whose frame t + l exists, i.e. all
    terms of Eq. (5) in which v_{n,k,t} appears (the majorise-minimise step).
    Then v <- max(v, floor).
    """
    lam = psd(B, V)
    T = Y.shape[-1]
    r0 = first_row(taps)
    num = np.zeros_like(V)
    den = np.zeros_like(V)
    for n, L in enumerate(taps):
        Bt = B[n].T                                 # [K, F]
        n_taps = 1 if vrule == PAPER_TAP0 else L
        for l in range(n_taps):
            A = np.abs(Y[:, r0[n] + l, l:]) ** 2   # |y_{n,f,t+l,l}|^2 for t = 0 .. T-1-l
            lam_t = lam[n][:, :T - l]
            num[n][:, :T - l] += Bt @ (A / lam_t ** 2)
            den[n][:, :T - l] += Bt @ (1.0 / lam_t)
    return np.maximum(V * np.sqrt(num / den), floor)


def rescale(W, B, Y, taps):
    """Scale normalisation, Eqs. (19)-(21).

    mu_{n,l} = sqrt( (1/(F T)) sum_{f,t} |y_{n,f,t,l}|^2 ); W row (n,l) /= mu_{n,l};
    b_n /= mu_{n,0}^2.  Returns (W, B, mu).
    """
    mu = np.sqrt(np.mean(np.abs(Y) ** 2, axis=(0, 2)))
    W = W / mu[None, :, None]
    r0 = first_row(taps)
    B = B / (mu[r0] ** 2)[:, None, None]
    return W, B, mu


# ------------------------------------------------------------ objective
def nll(W, Xb, B, V, taps):
    """Negative log-likelihood, Eq. (5), without the constant.

    sum_{f,t,n,l} ( log lambda_{n,f,t-l} + |y_{n,f,t,l}|^2 / lambda_{n,f,t-l} ) - 2 T sum_f log|det W_f|,
    terms with t - l < 0 dropped.
    """
    lam = psd(B, V)
    Y = demix(W, Xb)
    T = Y.shape[-1]
    src, tap = row_map(taps)
    total = 0.0
    for r in range(len(src)):
        n, l = src[r], tap[r]
        lam_d = lam[n][:, :T - l]
        total += float(np.sum(np.log(lam_d)) + np.sum(np.abs(Y[:, r, l:]) ** 2 / lam_d))
    _, logabsdet = np.linalg.slogdet(W)
    return total - 2.0 * T * float(np.sum(logabsdet))


# ------------------------------------------------------------ iteration
def iterate(W, B, V, Xb, taps, rule=ISS, vrule=ALL_TAPS, floor=FLOOR):
    """One iteration: W update (ISS or IP), b update, v update, rescale.  Returns (W, B, V, mu)."""
    lam = psd(B, V)
    phi = row_weights(lam, taps)
    if rule == ISS:
        W, Y = iss_sweep(W, demix(W, Xb), phi)
    elif rule == IP:
        W, Y = ip_sweep(W, Xb, phi)
    else:
        raise ValueError(rule)
    B = update_B(B, V, Y, taps, floor)
    V = update_V(B, V, Y, taps, vrule, floor)
    W, B, mu = rescale(W, B, Y, taps)
    return W, B, V, mu


def run(X, D, taps, B0, V0, n_iter, W0=None, rule=ISS, vrule=ALL_TAPS, floor=FLOOR, callback=None):
    """Run n_iter iterations from (W0, B0, V0); W0 = None is the identity (Sec. V-A).

    Returns (W [F, Mbar, Mbar], B [N, F, K], V [N, K, T]).
    callback(it, W, B, V) is called after every iteration when given.
    """
    Xb = stacked_view(X, D)
    F, Mb, _ = Xb.shape
    if int(sum(taps)) != Mb:
        raise ValueError("sum of taps must equal M*D")
    W = np.tile(np.eye(Mb, dtype=np.complex128), (F, 1, 1)) if W0 is None else np.array(W0, dtype=np.complex128)
    B = np.array(B0, dtype=np.float64)
    V = np.array(V0, dtype=np.float64)
    for it in range(n_iter):
        W, B, V, _ = iterate(W, B, V, Xb, taps, rule, vrule, floor)
        if callback is not None:
            callback(it, W, B, V)
    return W, B, V


# ------------------------------------------------------------ source images
def source_images(W, X, D, taps):
    """Spatial images by projection back, Eq. (24) with square invertible H = W^{-1}.

    c_{n,m,f,t} = sum_{l < L_n} H_f[m, (n,l)] y_{(n,l),f,t} for the M undelayed
    channels m.  Returns [N, M, F, T] complex128.
    """
    M = X.shape[0]
    Xb = stacked_view(X, D)
    H = np.linalg.inv(W)
    Y = demix(W, Xb)
    src, _ = row_map(taps)
    out = np.zeros((len(taps), M) + X.shape[1:], dtype=np.complex128)
    for n in range(len(taps)):
        rows = np.nonzero(src == n)[0]
        out[n] = np.transpose(np.matmul(H[:, :M, rows], Y[:, rows, :]), (1, 0, 2))
    return out


def mwf_images(W, X, D, taps, B, V):
    """Multichannel Wiener filter images, Eq. (24), evaluated literally per (f, t).

    c_n = H_n Lambda_n H_n^H (H Lambda H^H)^{-1} xbar with H = W^{-1} and the
    diagonal Lambda of delayed variances lambda_{n,f,t-l} (clamped to frame 0
    before the first frame).  Slow; for small inputs.  Returns [N, M, F, T].
    """
    M = X.shape[0]
    Xb = stacked_view(X, D)
    F, Mb, T = Xb.shape
    lam = psd(B, V)
    src, tap = row_map(taps)
    H = np.linalg.inv(W)
    out = np.zeros((len(taps), M, F, T), dtype=np.complex128)
    for f in range(F):
        for t in range(T):
            diag = np.array([lam[src[r], f, max(t - tap[r], 0)] for r in range(Mb)])
            Rx = H[f] @ np.diag(diag) @ np.conj(H[f]).T
            g = np.linalg.solve(Rx, Xb[f, :, t])
            for n in range(len(taps)):
                rows = np.nonzero(src == n)[0]
                Hn = H[f][:, rows]
                c = Hn @ np.diag(diag[rows]) @ np.conj(Hn).T @ g
                out[n, :, f, t] = c[:M]
    return out

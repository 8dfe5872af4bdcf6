"""Seeded synthetic inputs for the CTF-MNMF separation path.

This module only draws and shapes input data: random sources, room impulse
responses, time-domain mixing, additive noise and the STFT that turns the
mixture into the observation the separation path consumes.  It holds none of
the separation method's arithmetic (no demixing, no ISS/IP, no NMF update), so
both the GPU path and the CPU oracle may draw their inputs from it.

Stand-in notice: the paper evaluates on TIMIT speech convolved with RWCP room
impulse responses (Section V-A).  Neither is available here and neither is
reproduced: sources are complex Gaussian STFTs whose variances follow a random
NMF model, and impulse responses are exponentially decaying white noise at the
stated reverberation time.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.signal


def rng_for(seed: int) -> np.random.Generator:
    """PCG64 generator for one seed (every draw in this module goes through it)."""
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------- STFT pair
def hann(nfft: int) -> np.ndarray:
    """Periodic Hann analysis window of length nfft."""
    return scipy.signal.get_window("hann", nfft)


def n_frames(n_samples: int, hop: int) -> int:
    """Frame count of the centred STFT: one frame per hop plus the first."""
    return 1 + n_samples // hop


def stft(x: np.ndarray, nfft: int, hop: int) -> np.ndarray:
    """Centred STFT of real signals.

    x: [..., samples] real.  Returns [..., F, T] complex128 with F = nfft/2+1
    and T = 1 + samples // hop; the signal is zero padded by nfft/2 on both
    sides so that frame t is centred on sample t*hop.
    """
    x = np.asarray(x, dtype=np.float64)
    lead = x.shape[:-1]
    n = x.shape[-1]
    T = n_frames(n, hop)
    pad = nfft // 2
    need = (T - 1) * hop + nfft
    xp = np.zeros(lead + (need,), dtype=np.float64)
    xp[..., pad:pad + n] = x
    win = hann(nfft)
    idx = np.arange(T)[:, None] * hop + np.arange(nfft)[None, :]
    frames = xp[..., idx] * win                      # [..., T, nfft]
    spec = np.fft.rfft(frames, axis=-1)              # [..., T, F]
    return np.ascontiguousarray(np.swapaxes(spec, -1, -2))


def istft(S: np.ndarray, nfft: int, hop: int, length: int) -> np.ndarray:
    """Weighted overlap-add inverse of :func:`stft` ([..., F, T] -> [..., length])."""
    S = np.asarray(S)
    lead = S.shape[:-2]
    T = S.shape[-1]
    win = hann(nfft)
    frames = np.fft.irfft(np.swapaxes(S, -1, -2), n=nfft, axis=-1) * win   # [..., T, nfft]
    total = (T - 1) * hop + nfft
    out = np.zeros(lead + (total,), dtype=np.float64)
    norm = np.zeros(total, dtype=np.float64)
    for t in range(T):
        out[..., t * hop:t * hop + nfft] += frames[..., t, :]
        norm[t * hop:t * hop + nfft] += win * win
    norm[norm < 1e-10] = 1.0
    out = out / norm
    pad = nfft // 2
    return out[..., pad:pad + length]


# ------------------------------------------------------------- workloads
def balanced_taps(mbar: int, n_src: int) -> tuple[int, ...]:
    """Split mbar extended-demixing rows over n_src sources as evenly as possible.

    The first sources take the remainder, e.g. (3, 2) -> (2, 1) and
    (64, 3) -> (22, 21, 21).
    """
    base, rem = divmod(mbar, n_src)
    return tuple(base + (1 if n < rem else 0) for n in range(n_src))


@dataclass(frozen=True)
class Workload:
    """One synthetic reverberant-mixture workload.

    D is the number of stacked observation frames (the CTF tap count of the
    workload); the extended demixing matrix is (M*D) x (M*D) per bin and its
    rows are split over sources by ``taps``.
    """
    name: str
    fs: int
    dur: float
    nfft: int
    hop: int
    M: int
    N: int
    D: int
    K: int
    n_iter: int
    rt60: float
    rir_len: float
    snr_db: float = 30.0
    taps: tuple[int, ...] | None = None

    @property
    def F(self) -> int:
        return self.nfft // 2 + 1

    @property
    def n_samples(self) -> int:
        return int(round(self.dur * self.fs))

    @property
    def T(self) -> int:
        return n_frames(self.n_samples, self.hop)

    @property
    def mbar(self) -> int:
        return self.M * self.D

    @property
    def row_taps(self) -> tuple[int, ...]:
        return self.taps if self.taps is not None else balanced_taps(self.mbar, self.N)


WORKLOADS: dict[str, Workload] = {
    # FP64 single mixture: 4 s, STFT 1024/256, 3 mics, 2 sources, 4 taps, K=10, 30 iterations.
    "c0": Workload("c0", 16000, 4.0, 1024, 256, M=3, N=2, D=4, K=10, n_iter=30, rt60=0.6, rir_len=0.5),
    # Same mixture with no frame stacking: exactly the paper's square model (sum of taps = M).
    "c0_d1": Workload("c0_d1", 16000, 4.0, 1024, 256, M=3, N=2, D=1, K=10, n_iter=30, rt60=0.6, rir_len=0.5),
    # Long-reverb single mixture: 10 s, STFT 2048/512, 8 taps, K=20, 100 iterations.
    "c1": Workload("c1", 16000, 10.0, 2048, 512, M=3, N=2, D=8, K=20, n_iter=100, rt60=0.9, rir_len=0.9),
    # Precision workload: 60 s, STFT 4096/1024, 4 mics, 3 sources, 16 taps, K=30.
    "c3": Workload("c3", 16000, 60.0, 4096, 1024, M=4, N=3, D=16, K=30, n_iter=100, rt60=0.8, rir_len=0.8),
    # One mixture of the differentiation batch: 6 s, STFT 1024/256, 4 taps, K=10, 20 iterations.
    "c4": Workload("c4", 16000, 6.0, 1024, 256, M=3, N=2, D=4, K=10, n_iter=20, rt60=0.6, rir_len=0.5),
    # Paper shapes (Sec. V-A, Table I): 8 s, STFT 1024/256, K=3, 100 iterations, L_n = M/2.
    "P4": Workload("P4", 16000, 8.0, 1024, 256, M=4, N=2, D=1, K=3, n_iter=100, rt60=0.30, rir_len=0.30),
    "P6": Workload("P6", 16000, 8.0, 1024, 256, M=6, N=2, D=1, K=3, n_iter=100, rt60=0.47, rir_len=0.47),
    "P8": Workload("P8", 16000, 8.0, 1024, 256, M=8, N=2, D=1, K=3, n_iter=100, rt60=1.30, rir_len=1.30),
}


def batched_workloads(count: int, seed: int) -> list[Workload]:
    """Per-mixture draws of the batched workload (3-12 s, N in {2,3}, M=N+1, 4 or 8 taps)."""
    rng = rng_for(seed)
    out = []
    for i in range(count):
        dur = float(rng.uniform(3.0, 12.0))
        n_src = int(rng.integers(2, 4))
        D = int(rng.choice([4, 8]))
        rt60 = float(rng.uniform(0.3, 1.0))
        out.append(Workload(f"c2_{i}", 16000, dur, 1024, 256, M=n_src + 1, N=n_src, D=D, K=10,
                            n_iter=50, rt60=rt60, rir_len=rt60))
    return out


# ------------------------------------------------------------- drawing
def draw_sources(wl: Workload, rng: np.random.Generator) -> np.ndarray:
    """Time-domain sources [N, samples]: CN(0, B V) STFTs with Gamma(1,1) factors, then iSTFT."""
    F, T = wl.F, wl.T
    srcs = []
    for _ in range(wl.N):
        Bt = rng.gamma(1.0, 1.0, size=(F, wl.K))
        Vt = rng.gamma(1.0, 1.0, size=(wl.K, T))
        var = Bt @ Vt
        S = np.sqrt(var / 2.0) * (rng.standard_normal((F, T)) + 1j * rng.standard_normal((F, T)))
        srcs.append(istft(S, wl.nfft, wl.hop, wl.n_samples))
    return np.stack(srcs)


def draw_rirs(wl: Workload, rng: np.random.Generator) -> np.ndarray:
    """Impulse responses [M, N, taps]: white noise times exp(-6.9 tau / RT60)."""
    n = max(1, int(round(wl.rir_len * wl.fs)))
    tau = np.arange(n) / wl.fs
    env = np.exp(-6.9 * tau / wl.rt60)
    return rng.standard_normal((wl.M, wl.N, n)) * env


@dataclass
class Mixture:
    X: np.ndarray          # [M, F, T] complex128 observed STFT
    images: np.ndarray     # [N, M, F, T] complex128 STFT of each source's image at each mic
    wl: Workload


def make_mixture(wl: Workload, seed: int, with_images: bool = False) -> Mixture:
    """Convolve sources with impulse responses in the time domain, add white noise, STFT."""
    rng = rng_for(seed)
    s = draw_sources(wl, rng)
    h = draw_rirs(wl, rng)
    n = wl.n_samples
    img = np.zeros((wl.N, wl.M, n))
    for m in range(wl.M):
        for k in range(wl.N):
            img[k, m] = scipy.signal.fftconvolve(s[k], h[m, k])[:n]
    x = img.sum(axis=0)
    p_sig = float(np.mean(x ** 2))
    noise = rng.standard_normal(x.shape) * np.sqrt(p_sig / (10.0 ** (wl.snr_db / 10.0)))
    X = stft(x + noise, wl.nfft, wl.hop)
    images = stft(img, wl.nfft, wl.hop) if with_images else np.zeros((0,))
    return Mixture(X=X, images=images, wl=wl)


def init_nmf(N: int, F: int, K: int, T: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Initial NMF factors B0 [N, F, K] and V0 [N, K, T], uniform in (0.1, 1), from seed + 1."""
    rng = rng_for(seed + 1)
    B0 = rng.uniform(0.1, 1.0, size=(N, F, K))
    V0 = rng.uniform(0.1, 1.0, size=(N, K, T))
    return B0, V0


def random_problem(F: int, T: int, M: int, N: int, K: int, seed: int,
                   scale_spread: float = 0.0):
    """Small random observation X [M, F, T] (complex Gaussian) plus B0, V0 for unit tests.

    scale_spread > 0 multiplies each frame by exp(scale_spread * g), g ~ N(0, 1), to
    give the frame powers a realistic dynamic range.
    """
    rng = rng_for(seed)
    X = (rng.standard_normal((M, F, T)) + 1j * rng.standard_normal((M, F, T))) / np.sqrt(2.0)
    if scale_spread > 0:
        X = X * np.exp(scale_spread * rng.standard_normal((1, F, T)))
    B0, V0 = init_nmf(N, F, K, T, seed)
    return X, B0, V0


def ctf_mixture(F: int, T: int, N: int, taps: tuple[int, ...], K: int, seed: int):
    """Noiseless mixture drawn directly from the band-to-band CTF model, Eq. (2).

    Sources s_{n,f,t} ~ CN(0, b v) with Gamma(1,1) NMF factors; filters
    h_{m,n,f,l} ~ CN(0, 1) with M = sum(taps) microphones, so the extended mixing
    matrix of Eq. (3) is square.  Returns (X [M, F, T], Htilde [F, M, M], S [N, F, T])
    where column r = (n, l) of Htilde multiplies s_{n, t - l}.
    """
    rng = rng_for(seed)
    M = int(sum(taps))
    S = np.zeros((N, F, T), dtype=np.complex128)
    for n in range(N):
        var = rng.gamma(1.0, 1.0, size=(F, K)) @ rng.gamma(1.0, 1.0, size=(K, T))
        S[n] = np.sqrt(var / 2.0) * (rng.standard_normal((F, T)) + 1j * rng.standard_normal((F, T)))
    Ht = (rng.standard_normal((F, M, M)) + 1j * rng.standard_normal((F, M, M))) / np.sqrt(2.0)
    X = np.zeros((M, F, T), dtype=np.complex128)
    col = 0
    for n in range(N):
        for l in range(taps[n]):
            delayed = np.zeros((F, T), dtype=np.complex128)
            delayed[:, l:] = S[n, :, :T - l]
            X += np.einsum("fm,ft->mft", Ht[:, :, col], delayed)
            col += 1
    return X, Ht, S

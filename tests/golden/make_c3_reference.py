"""Writes c3_oracle_images.npz: the FP64 oracle's source images after the whole run of the
precision workload (60 s at 16 kHz, N = 3 sources, M = 4 microphones, RT60 0.8 s, STFT
4096/1024: F = 2049, T = 938; D = 16 stacked frames: Mbar = 64, taps 22 + 21 + 21; K = 30;
100 iterations from W = I), for 16 bins spread over the band.  Inputs: the seeded synthetic
mixture and initial factors of datagen (seed 0), as the benchmark's precision leg draws them.

Only datagen and oracle/ are called.  Run from the repository root:
    python tests/golden/make_c3_reference.py [--workers N]
(hours: ~3.7 h with 7 pool workers on an 8-core host, 80-210 s per iteration, since every
iteration's activation update needs all 2049 bins; the images are stored in complex64, i.e.
to ~6e-8 relative, well below the errors they are used to measure).
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from datagen import WORKLOADS, init_nmf, make_mixture  # noqa: E402
from oracle import ctf_iss as o  # noqa: E402
from oracle import threaded as oth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_images.npz")


def sample_bins(F: int, count: int = 16) -> np.ndarray:
    return np.linspace(8, F - 9, count).round().astype(np.int64)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=4, help="bins per task of the thread pool")
    args = ap.parse_args()
    wl = WORKLOADS["c3"]
    X = make_mixture(wl, 0).X
    B0, V0 = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
    t0 = time.time()

    def progress(it, W, B, V):
        print(f"iteration {it + 1}/{wl.n_iter}: {time.time() - t0:.0f} s", flush=True)

    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # one BLAS thread per pool worker
        W, _, _ = oth.run(X, wl.D, wl.row_taps, B0, V0, wl.n_iter, workers=args.workers, chunk=args.chunk,
                          callback=progress)
    bins = sample_bins(wl.F)
    C = o.source_images(W[bins], X[:, bins, :], wl.D, wl.row_taps)  # [N, M, bins, T]
    np.savez(OUT, bins=bins, images=C.astype(np.complex64), n_iter=wl.n_iter, seed=0,
             workload="c3: 60 s, N=3, M=4, RT60 0.8 s, STFT 4096/1024, D=16 (Mbar=64), K=30")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())

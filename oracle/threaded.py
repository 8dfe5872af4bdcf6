"""The FP64 oracle's iteration with its W update spread over host threads.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test-suite,
the package smoke check and the CPU-baseline leg of the benchmark may use it.

The W update of an iteration (the ISS sweep of Eqs. (11) and (16), or the IP
sweep of Eqs. (9)-(10)) acts on each frequency bin separately, and it is the
only step whose cost grows with Mbar^2 per bin and frame.  `run` below takes
the same steps as `ctf_iss.run`, in the same order, calling the same oracle
functions; it only hands the W update of contiguous chunks of bins to a pool
of threads (NumPy releases the interpreter lock inside its array loops), then
updates b, v and the scales on the whole arrays as `ctf_iss.iterate` does.
Per bin the arithmetic is that of `ctf_iss.run`; only the batch extent of the
array operations differs.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import ctf_iss as o


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _w_update(W, Xb, phi, rule):
    if rule == o.ISS:
        return o.iss_sweep(W, o.demix(W, Xb), phi)
    if rule == o.IP:
        return o.ip_sweep(W, Xb, phi)
    raise ValueError(rule)


def iterate(pool, chunks, W, B, V, Xb, taps, rule=o.ISS, vrule=o.ALL_TAPS, floor=o.FLOOR):
    """One iteration as ctf_iss.iterate, the W update of each bin chunk on the pool."""
    lam = o.psd(B, V)
    phi = o.row_weights(lam, taps)
    parts = list(pool.map(lambda c: _w_update(W[c[0]:c[1]], Xb[c[0]:c[1]], phi[c[0]:c[1]], rule), chunks))
    W = np.concatenate([p[0] for p in parts], axis=0)
    Y = np.concatenate([p[1] for p in parts], axis=0)
    B = o.update_B(B, V, Y, taps, floor)
    V = o.update_V(B, V, Y, taps, vrule, floor)
    W, B, mu = o.rescale(W, B, Y, taps)
    return W, B, V, mu


def run(X, D, taps, B0, V0, n_iter, W0=None, rule=o.ISS, vrule=o.ALL_TAPS, floor=o.FLOOR, callback=None,
        workers=None, chunk=None):
    """ctf_iss.run with the W update over `workers` threads (bins in chunks of `chunk`).

    Returns (W, B, V); callback(it, W, B, V) after every iteration when given.
    """
    Xb = o.stacked_view(X, D)
    F, Mb, _ = Xb.shape
    if int(sum(taps)) != Mb:
        raise ValueError("sum of taps must equal M*D")
    workers = workers or default_workers()
    if chunk is None:
        chunk = max(1, -(-F // (4 * workers)))
    chunks = [(f, min(F, f + chunk)) for f in range(0, F, chunk)]
    W = np.tile(np.eye(Mb, dtype=np.complex128), (F, 1, 1)) if W0 is None else np.array(W0, dtype=np.complex128)
    B = np.array(B0, dtype=np.float64)
    V = np.array(V0, dtype=np.float64)
    with ThreadPoolExecutor(max_workers=workers) as pool:
        for it in range(n_iter):
            W, B, V, _ = iterate(pool, chunks, W, B, V, Xb, taps, rule, vrule, floor)
            if callback is not None:
                callback(it, W, B, V)
    return W, B, V

"""Separation quality and run time of ISS against IP on synthetic stand-in data.

The shape of the paper's experiment (Sec. V, Table I): two sources, M = 4, 6
or 8 microphones, no frame stacking (D = 1) with L_n = M / 2 rows per source,
K = 3 bases, 100 iterations, STFT 1024/256 at 16 kHz, 8 s mixtures, and three
reverberation times.  The paper uses recorded speech and measured room
responses; here every source is synthetic (complex Gaussian STFTs with an NMF
variance) and every response is exponentially decaying noise, so the absolute
numbers are not the paper's and only the comparison between methods carries
over.

For each (M, RT60, seed) it separates the same mixture with the ISS rule
(FP32, ALL_TAPS and the printed tap-0 activation rule) and with the IP rule
(FP64 and FP32), all on the GPU through the C ABI, and reports
  * SDR per source: 10 log10(sum |c|^2 / sum |c - c_hat|^2) over microphones,
    bins and frames of the STFT images, with the source permutation that
    maximises the mean, and the same figure for the unprocessed mixture;
  * the GPU wall time of the 100 iterations (after one warm-up iteration).

Control: the same runs on mixtures drawn directly from the paper's own
convolutive model, Eq. (2) (datagen.ctf_mixture: complex Gaussian NMF sources,
random band-wise filters h_{m,n,f,l} with L_n = M / 2 taps per source, square
extended mixing, no noise), whose source images are known exactly and which
the demixing model can separate: there ISS and IP are compared where
separation succeeds, as the paper's Fig. 2 does on speech.

Usage: python -m paper_2510_02382_amd.study [--seeds 3] [--out FILE] [--no-control]
"""
from __future__ import annotations

import argparse
import dataclasses
import itertools
import json
import sys
import time

import numpy as np


def sdr_db(ref: np.ndarray, est: np.ndarray) -> float:
    err = float(np.sum(np.abs(ref - est) ** 2))
    if err == 0.0:
        return float("inf")
    return float(10.0 * np.log10(float(np.sum(np.abs(ref) ** 2)) / err))


def best_permutation_sdr(images: np.ndarray, est: np.ndarray) -> tuple[float, list]:
    """Mean SDR over sources for the best assignment of estimates to sources.
    images, est: [N, M, F, T]."""
    N = images.shape[0]
    best = None
    for perm in itertools.permutations(range(N)):
        vals = [sdr_db(images[n], est[perm[n]]) for n in range(N)]
        if best is None or np.mean(vals) > np.mean(best[1]):
            best = (perm, vals)
    return float(np.mean(best[1])), best[1]


def ctf_images(Ht: np.ndarray, S: np.ndarray, taps) -> np.ndarray:
    """Source images of a mixture drawn from Eq. (2): c_{n,m,f,t} = sum_l h_{m,(n,l),f} s_{n,f,t-l}
    (zero before the first frame).  Ht [F, M, Mbar] (column (n, l)), S [N, F, T] -> [N, M, F, T]."""
    F, M, _ = Ht.shape
    N, _, T = S.shape
    out = np.zeros((N, M, F, T), dtype=np.complex128)
    col = 0
    for n in range(N):
        for l in range(taps[n]):
            delayed = np.zeros((F, T), dtype=np.complex128)
            delayed[:, l:] = S[n, :, :T - l]
            out[n] += Ht[:, :, col].T[:, :, None] * delayed[None, :, :]
            col += 1
    return out


@dataclasses.dataclass
class _Mix:
    X: np.ndarray
    images: np.ndarray


def run_one(torch, Separator, wl, mix, B0, V0, precision, rule, vrule):
    dev = torch.device("cuda:0")
    cd = torch.complex64 if precision == "fp32" else torch.complex128
    rd = torch.float32 if precision == "fp32" else torch.float64
    sep = Separator(wl.F, wl.T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision=precision, rule=rule, vrule=vrule)
    X = torch.from_numpy(mix.X).to(dev, cd)
    B = torch.from_numpy(B0).to(dev, rd)
    V = torch.from_numpy(V0).to(dev, rd)
    sep.set_input(X)
    sep.set_state(B=B, V=V)
    sep.iterate(1)
    torch.cuda.synchronize()
    sep.set_state(B=B, V=V)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sep.iterate(wl.n_iter)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    C = sep.source_images().to(torch.complex128).cpu().numpy()
    status = sep.status()
    sep.close()
    return C, dt, status


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--mics", default="4,6,8")
    ap.add_argument("--rt60", default="0.30,0.47,1.30")
    ap.add_argument("--out", default=None, help="write one JSON line per run here")
    ap.add_argument("--no-control", action="store_true", help="skip the mixtures drawn from Eq. (2)")
    args = ap.parse_args(argv)

    import torch

    from datagen import WORKLOADS, ctf_mixture, init_nmf, make_mixture
    from paper_2510_02382_amd import Separator

    runs = [("iss_fp32", "fp32", "iss", "all_taps"), ("iss_fp32_tap0", "fp32", "iss", "paper_tap0"),
            ("iss_fp64", "fp64", "iss", "all_taps"), ("ip_fp64", "fp64", "ip", "all_taps"),
            ("ip_fp32", "fp32", "ip", "all_taps")]
    rows = []
    out = open(args.out, "w") if args.out else None
    for M in [int(m) for m in args.mics.split(",")]:
        base = WORKLOADS[f"P{M}"]
        for rt in [float(r) for r in args.rt60.split(",")]:
            wl = dataclasses.replace(base, name=f"P{M}_rt{rt:.2f}", rt60=rt, rir_len=rt)
            for seed in range(args.seeds):
                mix = make_mixture(wl, 100 * M + seed, with_images=True)
                B0, V0 = init_nmf(wl.N, wl.F, wl.K, wl.T, 100 * M + seed)
                sdr_in, _ = best_permutation_sdr(mix.images, np.broadcast_to(mix.X, mix.images.shape))
                rec = {"M": M, "rt60": rt, "seed": seed, "F": wl.F, "T": wl.T, "sdr_mixture": sdr_in}
                for name, prec, rule, vrule in runs:
                    C, dt, status = run_one(torch, Separator, wl, mix, B0, V0, prec, rule, vrule)
                    s, _ = best_permutation_sdr(mix.images, C) if status == 0 else (float("nan"), None)
                    rec[name] = {"sdr": s, "seconds": dt, "status": status}
                rows.append(rec)
                line = json.dumps(rec)
                print(line, flush=True)
                if out:
                    out.write(line + "\n")
    controls = []
    if not args.no_control:
        for M in [int(m) for m in args.mics.split(",")]:
            wl = dataclasses.replace(WORKLOADS[f"P{M}"], name=f"P{M}_ctf")
            for seed in range(args.seeds):
                X, Ht, S = ctf_mixture(wl.F, wl.T, wl.N, wl.row_taps, wl.K, 7000 + 100 * M + seed)
                mix = _Mix(X=X, images=ctf_images(Ht, S, wl.row_taps))
                B0, V0 = init_nmf(wl.N, wl.F, wl.K, wl.T, 7000 + 100 * M + seed)
                sdr_in, _ = best_permutation_sdr(mix.images, np.broadcast_to(mix.X, mix.images.shape))
                rec = {"control": "eq2", "M": M, "seed": seed, "F": wl.F, "T": wl.T, "sdr_mixture": sdr_in}
                for name, prec, rule, vrule in runs:
                    C, dt, status = run_one(torch, Separator, wl, mix, B0, V0, prec, rule, vrule)
                    sv, _ = best_permutation_sdr(mix.images, C) if status == 0 else (float("nan"), None)
                    rec[name] = {"sdr": sv, "seconds": dt, "status": status}
                controls.append(rec)
                line = json.dumps(rec)
                print(line, flush=True)
                if out:
                    out.write(line + "\n")
    if out:
        out.close()
    # summary per (M, RT60): mean over seeds
    print("\n| M | RT60 s | SDR mixture | ISS | ISS tap-0 | IP FP64 | IP FP32 | ISS FP32 ms | ISS FP64 ms | "
          "IP FP64 ms | IP/ISS time (FP64) |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for (M, rt), grp in itertools.groupby(rows, key=lambda r: (r["M"], r["rt60"])):
        grp = list(grp)
        def mean(key, field="sdr"):
            v = [g[key][field] for g in grp if g[key]["status"] == 0]
            return float(np.mean(v)) if v else float("nan")
        sm = float(np.mean([g["sdr_mixture"] for g in grp]))
        t_iss, t_iss64, t_ip = mean("iss_fp32", "seconds"), mean("iss_fp64", "seconds"), mean("ip_fp64", "seconds")
        print(f"| {M} | {rt:.2f} | {sm:.2f} | {mean('iss_fp32'):.2f} | {mean('iss_fp32_tap0'):.2f} | "
              f"{mean('ip_fp64'):.2f} | {mean('ip_fp32'):.2f} | {t_iss * 1e3:.1f} | {t_iss64 * 1e3:.1f} | "
              f"{t_ip * 1e3:.1f} | {t_ip / t_iss64:.2f} |")
    if controls:
        print("\nControl, mixtures drawn from Eq. (2) (no noise, square extended mixing):")
        print("\n| M | SDR mixture | ISS | ISS tap-0 | ISS FP64 | IP FP64 | IP FP32 |")
        print("|---|---|---|---|---|---|---|")
        for M, grp in itertools.groupby(controls, key=lambda r: r["M"]):
            grp = list(grp)
            def cmean(key):
                v = [g[key]["sdr"] for g in grp if g[key]["status"] == 0]
                return float(np.mean(v)) if v else float("nan")
            print(f"| {M} | {float(np.mean([g['sdr_mixture'] for g in grp])):.2f} | {cmean('iss_fp32'):.2f} | "
                  f"{cmean('iss_fp32_tap0'):.2f} | {cmean('iss_fp64'):.2f} | {cmean('ip_fp64'):.2f} | "
                  f"{cmean('ip_fp32'):.2f} |")
    return 0


if __name__ == "__main__":
    sys.exit(main())

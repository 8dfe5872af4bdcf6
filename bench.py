"""Throughput benchmark of the CTF-MNMF-ISS hot path on one MI355X.

Workload (single mixture, long reverberation): 10 s at 16 kHz, N=2 sources,
M=3 microphones, RT60 0.9 s, STFT 2048/512 (F=1025, T=313), D=8 stacked frames
(Mbar=24 rows, 12 taps per source), K=20 NMF bases, 100 iterations, complex64
data with FP32 arithmetic.  One step is one whole separation: identity
initialisation, 100 iterations (ISS sweep, basis and activation updates,
rescale) and the source images, with every input already in HBM.

value = F*T*iterations / second of the FP32 ISS path.  Alongside, the same
mixture is separated by the mixed-precision and FP64 ISS paths and by the IP
baseline.  The FP64 CPU oracle then runs all 100 iterations of the same
mixture (its W update over bin chunks on a pool of host threads): every GPU
path's images are compared with it per source (the accuracy field; the FP32
target is 1e-4), and its wall time is the cpu_baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6         # MI355X published FP64 vector and matrix peak
# Runtime reduction of ISS against IP that the paper reports for its 4, 6 and 8 microphone
# setups on a laptop CPU (Sec. V-B): context for the same ratio measured here, not a target.
PAPER_REDUCTION = {"P4": 0.41, "P6": 0.51, "P8": 0.33}
PEAK_HBM_TBS = 8.0              # MI355X published HBM3E bandwidth
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_iss_c1_traffic.json")
KERNEL_SOURCES = ["paper_2510_02382_amd/csrc/iter_impl.hpp", "paper_2510_02382_amd/csrc/common.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def iss_flops_per_unit(Mbar: int) -> float:
    """Algorithmic flops of the ISS W update per bin, frame and iteration: the demix
    y = W xbar, 8 Mbar^2, and the sweep, 20 Mbar^2 (per row pair and step: a_p 10, d_p 2,
    rank-1 update 8) -- 28 Mbar^2 in all."""
    return 28 * Mbar * Mbar


def iss_executed_flops_per_unit(Mbar: int, n_iter: int) -> float:
    """Flops the kernel executes per unit, averaged over the launches of one n_iter-iteration
    run: the sweep every iteration, the demix on the first only (later iterations carry Y,
    whose rows get the same operations as W's)."""
    return 20 * Mbar * Mbar + 8 * Mbar * Mbar / n_iter


def iss_bytes_per_unit(M: int, N: int, Mbar: int, T: int) -> float:
    """HBM bytes the FP32 ISS W update must move per bin, frame and iteration with a bin's
    rows resident on chip: X read (8 M), 1/lambda in and P out (8 N), W in and out
    (16 Mbar^2 / T)."""
    return 8 * M + 8 * N + 16 * Mbar * Mbar / T


def cpu_info() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_config(sep, X, B0, V0, n_iter):
    sep.set_input(X)
    sep.set_state(B=B0, V=V0)
    sep.iterate(n_iter)
    return sep.source_images()


def time_path(torch, Separator, wl, Xc, B0, V0, precision, rule, steps, warmup, profile=0):
    sep = Separator(wl.F, wl.T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision=precision, rule=rule)
    rd = torch.float64 if precision == "fp64" else torch.float32
    cd = torch.complex128 if precision == "fp64" else torch.complex64
    X = Xc.to(cd).contiguous()
    B = B0.to(rd).contiguous()
    V = V0.to(rd).contiguous()
    for _ in range(warmup):
        run_config(sep, X, B, V, wl.n_iter)
    torch.cuda.synchronize()
    if profile:
        sep.set_profiling(profile)
    t0 = time.perf_counter()
    for _ in range(steps):
        C = run_config(sep, X, B, V, wl.n_iter)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = sep.status()
    stats = {k: sep.kernel_stats(k) for k in range(7)} if profile else None
    sep.close()
    return dt, C, status, stats


def oracle_reference(wl, X, B0, V0, rule="iss"):
    """The FP64 oracle's whole run of the workload (all iterations, original FP64 data), the W
    update of bin chunks over a pool of host threads with BLAS pinned to one thread each.
    Returns (images, wall seconds, threads)."""
    from threadpoolctl import threadpool_limits

    from oracle import ctf_iss as o
    from oracle import threaded as oth
    workers = oth.default_workers()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        W, _, _ = oth.run(X, wl.D, wl.row_taps, B0, V0, wl.n_iter, rule=o.ISS if rule == "iss" else o.IP,
                          workers=workers)
        dt = time.perf_counter() - t0
    return o.source_images(W, X, wl.D, wl.row_taps), dt, workers


def per_source_err(C, Cref):
    import numpy as np
    C = np.asarray(C, dtype=np.complex128)
    return [float(np.linalg.norm(C[n] - Cref[n]) / np.linalg.norm(Cref[n])) for n in range(Cref.shape[0])]


def batched_bench(args) -> int:
    """256 uneven mixtures (3-12 s, N in {2, 3}, M = N + 1, D in {4, 8}, RT60 0.3-1.0 s, STFT
    1024/256, K = 10, 50 iterations) separated as one batch in FP32, against the same
    mixtures separated one context at a time (FP32 and FP64 ISS) and against FP64 IP (on a
    subset, per unit of work).  value = sum of F*T*iterations / second of the batch."""
    import torch

    from datagen import batched_workloads, init_nmf, make_mixture
    from paper_2510_02382_amd import BatchSeparator, Separator

    wls = batched_workloads(args.batch, 7)
    log(f"batched workload: {len(wls)} mixtures, T {min(w.T for w in wls)}-{max(w.T for w in wls)}, "
        f"Mbar {sorted(set(w.mbar for w in wls))}; drawing mixtures")
    dev = torch.device("cuda:0")
    X32, X64, B32, B64, V32, V64, shapes = [], [], [], [], [], [], []
    for i, w in enumerate(wls):
        mix = make_mixture(w, 1000 + i)
        B0, V0 = init_nmf(w.N, w.F, w.K, w.T, 1000 + i)
        X64.append(torch.from_numpy(mix.X).to(dev))
        X32.append(X64[-1].to(torch.complex64))
        B64.append(torch.from_numpy(B0).to(dev))
        B32.append(B64[-1].float())
        V64.append(torch.from_numpy(V0).to(dev))
        V32.append(V64[-1].float())
        shapes.append((w.F, w.T, w.M, w.D, w.N, w.K, w.row_taps))
        if (i + 1) % 64 == 0:
            log(f"  {i + 1} mixtures drawn")
    n_iter = wls[0].n_iter
    units = sum(w.F * w.T for w in wls) * n_iter

    stream = torch.cuda.Stream(device=dev)

    def run_batch(graph=False):
        bs = BatchSeparator(shapes, precision="fp32", stream=stream)
        if graph:
            bs.set_graph(True)  # the first iterate() captures, the others replay
        bs.set_input(X32)
        for _ in range(max(args.warmup, 1 if graph else 0)):
            bs.set_state(B=B32, V=V32)
            bs.iterate(n_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bs.set_state(B=B32, V=V32)
            bs.iterate(n_iter)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / args.steps
        Cb = bs.source_images()
        stb = bs.status()
        bs.close()
        return dtb, Cb, stb

    from paper_2510_02382_amd import binding as _b
    _b.ctfiss_clear_tuned_plans()
    with torch.cuda.stream(stream):
        dt_eager, C32e, st_e = run_batch(graph=False)
        dt, C32, st = run_batch(graph=True)
    graph_equals_eager = all(torch.equal(a, b) for a, b in zip(C32, C32e))
    value = units / dt
    log(f"batched FP32 ISS: eager {dt_eager * 1e3:.1f} ms, graph replay {dt * 1e3:.1f} ms per batch, "
        f"{value:.4e} F*T*it/s, status {st}, replay == eager: {graph_equals_eager}")
    tuned = None
    if args.autotune:
        # one context per distinct tuning key (Mbar, M, D, N, largest tap count, T rounded up to 32),
        # tuned on that mixture's data; the batch then starts from the cached plans
        t0 = time.perf_counter()
        seen = {}
        for i, w in enumerate(wls):
            key = (w.mbar, w.M, w.D, w.N, max(w.row_taps), (w.T + 31) // 32)
            if key in seen:
                continue
            sp = Separator(*shapes[i], precision="fp32")
            sp.set_input(X32[i])
            sp.set_state(B=B32[i], V=V32[i])
            seen[key] = sp.autotune(trials=3)
            sp.close()
        t_tune = time.perf_counter() - t0
        with torch.cuda.stream(stream):
            dtt, _, stt = run_batch(graph=True)
        tuned = {"ms": dtt * 1e3, "value": units / dtt, "keys_tuned": len(seen), "tuning_seconds": t_tune,
                 "status": list(stt)}
        log(f"autotuned ({len(seen)} shapes in {t_tune:.1f} s): {dtt * 1e3:.1f} ms per batch "
            f"({units / dtt:.4e} F*T*it/s)")
        _b.ctfiss_clear_tuned_plans()

    from paper_2510_02382_amd.binding import CtfissError

    def single(precision, rule, idx):
        """Separate mixtures idx one context at a time; mixtures whose shape this precision
        does not support are skipped.  Returns (seconds, images by index, status, units run)."""
        Xs, Bs, Vs = (X32, B32, V32) if precision == "fp32" else (X64, B64, V64)
        seps, ran = [], []
        for i in idx:
            F, T, M, D, N, K, taps = shapes[i]
            try:
                sp = Separator(F, T, M, D, N, K, taps, precision=precision, rule=rule)
            except CtfissError:
                continue
            sp.set_input(Xs[i])
            seps.append(sp)
            ran.append(i)
        idx = ran
        for i, sp in zip(idx, seps):  # warm-up
            sp.set_state(B=Bs[i], V=Vs[i])
            sp.iterate(1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i, sp in zip(idx, seps):
            sp.set_state(B=Bs[i], V=Vs[i])
            sp.iterate(n_iter)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        imgs = {i: sp.source_images() for i, sp in zip(idx, seps)}
        stat = max(sp.status() for sp in seps)
        for sp in seps:
            sp.close()
        return el, imgs, stat, sum(wls[i].F * wls[i].T for i in idx) * n_iter

    allidx = list(range(len(wls)))
    if args.no_side:
        print(json.dumps({"metric": "F·T·iters/s of a batch of uneven mixtures (batched FP32 ISS)", "value": value,
                          "unit": "F·T·iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": f"{len(wls)} uneven mixtures, 50 iterations"},
                          "autotuned_batch": tuned}), flush=True)
        return 0
    dt32, _, st32, u32 = single("fp32", "iss", allidx)
    log(f"single-context FP32 ISS: {dt32 * 1e3:.1f} ms, status {st32}")
    dt64, C64, st64, u64 = single("fp64", "iss", allidx)
    log(f"single-context FP64 ISS on {len(C64)} mixtures (the others exceed the FP64 kernel's limits): "
        f"{dt64 * 1e3:.1f} ms, status {st64}")
    sub = allidx[: min(32, len(allidx))]
    dtip, _, stip, uip = single("fp64", "ip", sub)
    log(f"single-context FP64 IP on the first {len(sub)} mixtures: {dtip * 1e3:.1f} ms, status {stip}")
    rel = max(float(torch.linalg.norm((C32[i].to(torch.complex128) - C64[i]).flatten())
                    / torch.linalg.norm(C64[i].flatten())) for i in C64)
    out = {
        "metric": "F·T·iters/s of a batch of uneven mixtures (batched FP32 ISS)",
        "value": value,
        "unit": "F·T·iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(wls)} mixtures: 3-12 s, N in {{2,3}}, M = N + 1, D in {{4,8}}, RT60 0.3-1.0 s, "
                               "STFT 1024/256, K = 10, 50 iterations", "mixtures": len(wls),
                   "sum_FT": sum(w.F * w.T for w in wls), "iterations": n_iter},
        "eager_ms_per_step": dt_eager * 1e3, "graph_equals_eager": graph_equals_eager,
        "hw_queues": args.hw_queues,
        "side_by_side": {
            "single_fp32_iss": {"value": u32 / dt32, "ms": dt32 * 1e3, "status": st32},
            "single_fp64_iss": {"value": u64 / dt64, "ms": dt64 * 1e3, "mixtures": len(C64), "status": st64},
            "single_fp64_ip": {"value": uip / dtip, "ms": dtip * 1e3, "mixtures": len(sub), "status": stip},
            "speedup_vs_single_fp64_iss": value / (u64 / dt64),
            "speedup_vs_single_fp32_iss": value / (u32 / dt32),
            "speedup_vs_single_fp64_ip": value / (uip / dtip),
            "batched_fp32_images_max_rel_err_vs_fp64_iss": rel,
            "autotuned_batch": tuned,
        },
        "status": list(st),
    }
    print(json.dumps(out), flush=True)
    return 0


def exchange_cost(args) -> int:
    """Price of the team exchange at c3, on correct kernels only.  A team member of the c3 W update
    (P workgroups per bin, each holding S = ceil(T/P) frames of every row) does what the
    single-workgroup kernel of the same launch shape does on a bin of S frames, plus the exchange
    of its partial sums with the other members (one round per ISS step) and the halo and row
    powers after the sweep.  Timed: (a) the mixed-precision team launch on the c3 mixture, (b) the
    single-workgroup kernel of the member's shape (CTFISS_PLAN=G,CPL,RPL) on that mixture cut to its
    first S frames with its bins repeated P times, i.e. as many workgroup items of the same shape
    as the team launch, none of which exchanges.  (a) - (b) per launch is the exchange."""
    import numpy as np
    import torch

    from datagen import WORKLOADS, init_nmf, make_mixture
    from paper_2510_02382_amd import Separator

    wl = WORKLOADS["c3"]
    n_iter = 20
    mix = make_mixture(wl, 0)
    B0n, V0n = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
    dev = torch.device("cuda:0")

    def launch_us(F, T, X, B0, V0, plan=None):
        if plan:  # the member's shape, with the NMF steps as launches of their own as in a team
            os.environ["CTFISS_PLAN"] = plan
            os.environ["CTFISS_UNFUSED_NMF"] = "1"
        try:
            sep = Separator(F, T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision="mixed", rule="iss")
        finally:
            os.environ.pop("CTFISS_PLAN", None)
            os.environ.pop("CTFISS_UNFUSED_NMF", None)
        shape = sep.plan()
        Xd = torch.from_numpy(X).to(dev, torch.complex64)
        Bd = torch.from_numpy(B0).to(dev, torch.float32)
        Vd = torch.from_numpy(V0).to(dev, torch.float32)
        run_config(sep, Xd, Bd, Vd, 2)  # warm-up
        torch.cuda.synchronize()
        sep.set_profiling(1)
        run_config(sep, Xd, Bd, Vd, n_iter)
        n, ms = sep.kernel_stats(0)
        st = sep.status()
        sep.close()
        return ms / max(n, 1) * 1e3, shape, st

    log("team launch on the c3 mixture")
    team_us, (G, cpl, rpl, P), st_team = launch_us(wl.F, wl.T, mix.X, B0n, V0n)
    if P <= 1:
        log("the default c3 plan is not a team plan: nothing to price")
        return 1
    S = -(-wl.T // P)
    Xs = np.ascontiguousarray(np.tile(mix.X[:, :, :S], (1, P, 1)))
    Bs = np.ascontiguousarray(np.tile(B0n, (1, P, 1)))
    Vs = np.ascontiguousarray(V0n[:, :, :S])
    log(f"single-workgroup launches of the member shape ({G}, {cpl}, {rpl}) on {P * wl.F} bins of {S} frames")
    single_us, shape1, st_single = launch_us(P * wl.F, S, Xs, Bs, Vs, plan=f"{G},{cpl},{rpl}")
    assert shape1[3] == 1 and shape1[:3] == (G, cpl, rpl), shape1
    out = {"workload": "c3 team exchange", "team_plan": [G, cpl, rpl, P], "member_frames": S,
           "items_per_launch": P * wl.F, "team_launch_us": team_us, "no_exchange_launch_us": single_us,
           "exchange_us_per_launch": team_us - single_us,
           "exchange_share": (team_us - single_us) / team_us,
           "status": [st_team, st_single], "iterations_timed": n_iter}
    print(json.dumps(out), flush=True)
    return 0


def precision_bench(args) -> int:
    """Long-signal workload with Mbar = 64: 60 s at 16 kHz, N=3, M=4, RT60 0.8 s, STFT 4096/1024
    (F=2049, T=938), D=16 stacked frames (taps 22+21+21), K=30, 100 iterations.  A bin's 64 rows x
    938 frames exceed one workgroup, so the W update runs as teams of workgroups splitting each
    bin's frames.  The mixed-precision path (FP32 data and frame sums, FP64 W rows) is timed
    (value); the mixed path with bfloat16 NMF contractions, the FP32 and the FP64 paths run
    alongside on the same mixture, and every path's images are compared, on 16 sampled bins,
    with the FP64 oracle's images of the whole run (tests/golden/c3_oracle_images.npz)."""
    import torch

    from datagen import WORKLOADS, init_nmf, make_mixture
    from paper_2510_02382_amd import Separator

    wl = WORKLOADS["c3"]
    log(f"workload c3: F={wl.F} T={wl.T} M={wl.M} D={wl.D} Mbar={wl.mbar} taps={wl.row_taps} K={wl.K} "
        f"iters={wl.n_iter}")
    mix = make_mixture(wl, 0)
    B0n, V0n = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
    dev = torch.device("cuda:0")
    Xc = torch.from_numpy(mix.X).to(dev)
    B0 = torch.from_numpy(B0n).to(dev)
    V0 = torch.from_numpy(V0n).to(dev)
    units = wl.F * wl.T * wl.n_iter
    log("timing mixed-precision ISS (FP32 data and sums, FP64 W rows)")
    dt, Cm, stm, stats = time_path(torch, Separator, wl, Xc, B0, V0, "mixed", "iss", args.steps, args.warmup,
                                   profile=1)
    value = units * args.steps / dt
    n_iss, ms_iss = stats[0]
    avg_iss_ms = ms_iss / max(n_iss, 1)
    flops_launch = wl.F * wl.T * iss_flops_per_unit(wl.mbar)
    achieved = flops_launch / (avg_iss_ms * 1e-3) / 1e12
    _, _, _, allstats = time_path(torch, Separator, wl, Xc, B0, V0, "mixed", "iss", 1, 0, profile=-1)
    names = ["w_update_iss", "v_partial", "v_update_mu", "final_rescale", "images", "lambda", "basis_update"]
    kernel_ms = {names[i]: allstats[i][1] / max(allstats[i][0], 1) for i in range(7)}
    log(f"mixed ISS: {dt / args.steps * 1e3:.3f} ms/step, {value:.4e} F·T·it/s, W update avg "
        f"{avg_iss_ms * 1e3:.1f} us ({achieved:.1f} TFLOP/s), status {stm}")
    side = {}
    images = {"iss_mixed": Cm}
    if not args.no_side:
        log("timing mixed ISS with bfloat16 NMF contractions")
        dtb, Cb, stb, _ = time_path(torch, Separator, wl, Xc, B0, V0, "mixed_bf16", "iss", args.side_steps, 1)
        log("timing FP32 ISS")
        dt32, C32, st32, _ = time_path(torch, Separator, wl, Xc, B0, V0, "fp32", "iss", args.side_steps, 1)
        log("timing FP64 ISS")
        dt64, C64, st64, _ = time_path(torch, Separator, wl, Xc, B0, V0, "fp64", "iss", args.side_steps, 1)
        images.update({"iss_mixed_bf16": Cb, "iss_fp32": C32, "iss_fp64": C64})
        side["iss_mixed_bf16"] = {"value": units * args.side_steps / dtb, "ms_per_step": dtb / args.side_steps * 1e3,
                                  "status": stb}
        side["iss_fp32"] = {"value": units * args.side_steps / dt32, "ms_per_step": dt32 / args.side_steps * 1e3,
                            "status": st32}
        side["iss_fp64"] = {"value": units * args.side_steps / dt64, "ms_per_step": dt64 / args.side_steps * 1e3,
                            "status": st64}
        side["speedup_iss_mixed_vs_fp64"] = value / side["iss_fp64"]["value"]
        log(f"mixed + bf16 NMF: {dtb / args.side_steps * 1e3:.3f} ms/step; FP32 ISS: {dt32 / args.side_steps * 1e3:.3f} "
            f"ms/step; FP64 ISS: {dt64 / args.side_steps * 1e3:.3f} ms/step")
    # accuracy: every path's images on the sampled bins against the FP64 oracle's whole run
    # (tests/golden/make_c3_reference.py wrote them, calling only the oracle)
    accuracy = None
    ref_path = os.path.join(ROOT, "tests", "golden", "c3_oracle_images.npz")
    if os.path.exists(ref_path):
        import numpy as np
        ref = np.load(ref_path)
        bins, Cref = ref["bins"], ref["images"].astype(np.complex128)
        accuracy = {"reference": f"FP64 oracle, {int(ref['n_iter'])} ISS iterations of the full mixture, images of "
                                 f"{len(bins)} bins spread over the band (stored to complex64 precision)",
                    "targets": {"iss_mixed": 1e-4, "iss_fp32": 1e-4, "iss_mixed_bf16": 1e-2}, "per_source_rel_err": {}}
        for k, C in images.items():
            g = C[:, :, torch.as_tensor(bins, device=C.device), :].cpu().numpy()
            accuracy["per_source_rel_err"][k] = per_source_err(g, Cref)
            log(f"  {k}: per-source error vs oracle {accuracy['per_source_rel_err'][k]}")
    out = {
        "metric": "F·T·iters/s ISS vs IP vs FP64-ISS at rel err ≤1e-4; HBM GB/s fraction",
        "value": value, "unit": "F·T·iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (W rows f64)", "data": "synthetic",
        "config": {"workload": "c3 single mixture: 60 s, N=3, M=4, RT60 0.8 s, STFT 4096/1024, D=16 stacked frames "
                               "(Mbar=64, taps 22+21+21), K=30, 100 iterations, CTF-MNMF-ISS, bins split over "
                               "teams of workgroups",
                   "F": wl.F, "T": wl.T, "Mbar": wl.mbar, "K": wl.K, "iterations": wl.n_iter},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": None,
                     "kernel": "k_iss_team (mixed precision W update, each bin's frames split over a team of "
                               "workgroups)",
                     "avg_launch_us": avg_iss_ms * 1e3, "flops_per_launch": flops_launch},
        "kernel_avg_ms": kernel_ms, "status": stm, "accuracy": accuracy, "side_by_side": side, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def adjoint_bench(args) -> int:
    """Differentiation workload: 32 mixtures of 6 s (N=2, M=3, STFT 1024/256: F=513, T=376, D=4
    stacked frames: Mbar=12, taps 6+6, K=10), 20 unrolled iterations, loss = mean squared error of
    the source images against the known synthetic images.  One step = forward and reverse pass
    (ctfiss_backward) of all 32 mixtures, one context per mixture, spread over --streams streams,
    in complex64 (value) and in FP64 (alongside).  Mixture 0's gradients of both are checked
    against the FP64 PyTorch autograd reference on the host, which is also timed there as the
    CPU baseline."""
    import torch

    from datagen import WORKLOADS, init_nmf, make_mixture
    from paper_2510_02382_amd.autograd import separate

    wl = WORKLOADS["c4"]
    nmix = args.batch if args.batch != 256 else 32
    log(f"workload c4: {nmix} mixtures, F={wl.F} T={wl.T} M={wl.M} D={wl.D} Mbar={wl.mbar} taps={wl.row_taps} "
        f"K={wl.K} iters={wl.n_iter}")
    dev = torch.device("cuda:0")
    mixes = []
    for i in range(nmix):
        m = make_mixture(wl, 1000 + i, with_images=True)
        B0, V0 = init_nmf(wl.N, wl.F, wl.K, wl.T, 1000 + i)
        mixes.append((torch.from_numpy(m.X).to(dev), torch.from_numpy(B0).to(dev), torch.from_numpy(V0).to(dev),
                      torch.from_numpy(m.images).to(dev)))

    # the mixtures are independent: round-robin over a few streams (default
    # priority) so that their launches overlap; each backward runs on the
    # stream of its forward
    streams = [torch.cuda.Stream(device=dev) for _ in range(max(1, args.streams))]

    # the inputs in each precision, resident before timing
    typed = {cd: [(X.to(cd), B0.to(rd), V0.to(rd), img.to(cd)) for X, B0, V0, img in mixes]
             for cd, rd in ((torch.complex64, torch.float32), (torch.complex128, torch.float64))}

    def step(cd=torch.complex128, sample=None, check=False):
        out = None
        cur = torch.cuda.current_stream(dev)
        for st in streams:
            st.wait_stream(cur)
        for i, (X, B0, V0, img) in enumerate(typed[cd] if sample is None else typed[cd][:sample]):
            st = streams[i % len(streams)]
            with torch.cuda.stream(st):
                Xg = X.clone().requires_grad_(True)
                Bg = B0.clone().requires_grad_(True)
                C = separate(Xg, Bg, V0, wl.D, wl.row_taps, wl.n_iter, check=check)
                loss = ((C - img).abs() ** 2).mean()
                loss.backward()
                if i == 0:
                    out = (loss, Xg.grad, Bg.grad)
        for st in streams:
            cur.wait_stream(st)
        return (float(out[0].detach()), out[1], out[2])

    def timed_steps(cd):
        for _ in range(args.warmup):
            step(cd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fst = step(cd)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, fst

    dt, first = timed_steps(torch.complex64)
    dt64, first64 = timed_steps(torch.complex128)
    # the timed steps leave the device status unread (a read synchronises); one more step
    # per precision reads it after every forward and reverse pass and raises on a fault
    step(torch.complex64, check=True)
    step(torch.complex128, check=True)
    torch.cuda.synchronize()
    units = nmix * wl.F * wl.T * wl.n_iter
    value = units / dt
    # forward alone, for the split
    t0 = time.perf_counter()
    with torch.no_grad():
        for X, B0, V0, img in mixes:
            separate(X, B0, V0, wl.D, wl.row_taps, wl.n_iter)
    torch.cuda.synchronize()
    dt_fwd = time.perf_counter() - t0
    log(f"forward + reverse, complex64: {dt * 1e3:.1f} ms per step of {nmix} mixtures ({value:.3e} F·T·it/s); "
        f"FP64: {dt64 * 1e3:.1f} ms; FP64 forward alone {dt_fwd * 1e3:.1f} ms")
    cpu = None
    check = None
    if not args.no_cpu_baseline:
        from oracle import ctf_iss_torch as ot
        X, B0, V0, img = mixes[0]
        Xt = X.cpu().clone().requires_grad_(True)
        Bt = B0.cpu().clone().requires_grad_(True)
        nthreads = torch.get_num_threads()
        t0 = time.perf_counter()
        C = ot.forward(Xt, Bt, V0.cpu(), wl.D, wl.row_taps, wl.n_iter)[0]
        loss = ot.mse(C, img.cpu())
        loss.backward()
        dtc = time.perf_counter() - t0
        import numpy as np

        def errs(fst):
            gx = fst[1].cpu().numpy().astype(np.complex128)
            gb = fst[2].cpu().numpy().astype(np.float64)
            return {"loss": fst[0],
                    "gX_rel_err": float(np.linalg.norm(gx - Xt.grad.numpy()) / np.linalg.norm(Xt.grad.numpy())),
                    "gB0_rel_err": float(np.linalg.norm(gb - Bt.grad.numpy()) / np.linalg.norm(Bt.grad.numpy()))}
        check = {"mixture": 0, "loss_reference": float(loss), "complex64": errs(first), "fp64": errs(first64)}
        cpu = {"value": wl.F * wl.T * wl.n_iter / dtc, "unit": "F·T·iters/s (forward + reverse)", "cores": nthreads,
               "kind": "oracle", "sample": f"mixture 0 of the batch: FP64 PyTorch autograd forward and reverse on the "
                                           f"host, {nthreads} threads, {dtc:.1f} s"}
        log(f"autograd reference on the host: {dtc:.1f} s for one mixture; gradient errors {check}")
    out = {
        "metric": "F·T·iters/s ISS vs IP vs FP64-ISS at rel err ≤1e-4; HBM GB/s fraction",
        "value": value, "unit": "F·T·iters/s (forward + reverse)", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c4 differentiation: {nmix} mixtures of 6 s, N=2, M=3, STFT 1024/256, D=4 "
                               f"(Mbar=12, taps 6+6), K=10, 20 unrolled iterations, image MSE loss, gradients "
                               f"w.r.t. the mixture STFT and the initial bases",
                   "F": wl.F, "T": wl.T, "Mbar": wl.mbar, "K": wl.K, "iterations": wl.n_iter, "mixtures": nmix},
        "fp64_ms_per_step": dt64 * 1e3, "fp64_forward_ms_per_step": dt_fwd * 1e3, "streams": len(streams),
        "hw_queues": args.hw_queues, "gradient_check": check, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def c0_bench(args) -> int:
    """The small FP64 workload: 4 s, N = 2, M = 3, STFT 1024/256 (F = 513, T = 251), K = 10, 30
    iterations, with D = 4 stacked frames (Mbar = 12, taps 6 + 6) and, alongside, D = 1 (Mbar = 3,
    taps 2 + 1).  FP64 ISS with graph replay is `value` (an iteration is tens of microseconds, so
    launches matter); FP64 ISS eager, FP64 IP and FP32 ISS are timed alike beside it, every path's
    images are compared with the FP64 oracle of its rule, and the oracle is timed on all host threads
    (bin chunks) and on one thread."""
    import torch
    from threadpoolctl import threadpool_limits

    from datagen import WORKLOADS, init_nmf, make_mixture
    from oracle import ctf_iss as o
    from paper_2510_02382_amd import Separator

    dev = torch.device("cuda:0")
    lines = {}
    for name in ("c0", "c0_d1"):
        wl = WORKLOADS[name]
        log(f"workload {wl.name}: F={wl.F} T={wl.T} M={wl.M} Mbar={wl.mbar} taps={wl.row_taps} K={wl.K} "
            f"iters={wl.n_iter}")
        mix = make_mixture(wl, 0)
        B0n, V0n = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
        Xc = torch.from_numpy(mix.X).to(dev)
        B0d, V0d = torch.from_numpy(B0n).to(dev), torch.from_numpy(V0n).to(dev)
        units = wl.F * wl.T * wl.n_iter
        stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(stream):
            sep = Separator(wl.F, wl.T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision="fp64", stream=stream)
            sep.set_graph(True)
            sep.set_input(Xc)
            for _ in range(args.warmup + 1):
                sep.set_state(B=B0d, V=V0d)
                sep.iterate(wl.n_iter)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                sep.set_state(B=B0d, V=V0d)
                sep.iterate(wl.n_iter)
                Cg = sep.source_images()
            stream.synchronize()
            dtg = (time.perf_counter() - t0) / args.steps
            stg = sep.status()
            sep.close()
        log(f"FP64 ISS, graph replay: {dtg * 1e3:.3f} ms per separation, status {stg}")
        side, images = {}, {"iss_fp64_graph": Cg}
        for prec, rule in (("fp64", "iss"), ("fp64", "ip"), ("fp32", "iss")):
            dt, Cp, st, _ = time_path(torch, Separator, wl, Xc, B0d, V0d, prec, rule, args.side_steps, 1)
            key = f"{rule}_{prec}"
            side[key] = {"value": units * args.side_steps / dt, "ms_per_step": dt / args.side_steps * 1e3,
                         "status": st}
            images[key] = Cp
            log(f"{key}: {dt / args.side_steps * 1e3:.3f} ms per separation, status {st}")
        side["speedup_iss_fp64_vs_ip_fp64"] = side["ip_fp64"]["ms_per_step"] / side["iss_fp64"]["ms_per_step"]
        accuracy, cpu = None, None
        if not args.no_cpu_baseline:
            accuracy = {"reference": f"FP64 oracle, {wl.n_iter} iterations of the same rule on the original FP64 "
                                     f"data", "target_fp64": 1e-9, "target_fp32": 1e-4, "per_source_rel_err": {}}
            for rule in ("iss", "ip"):
                Cref, dto, workers = oracle_reference(wl, mix.X, B0n, V0n, rule)
                log(f"  oracle {rule.upper()}: {dto:.1f} s on {workers} threads")
                for key, Cp in images.items():
                    if key.startswith(rule):
                        accuracy["per_source_rel_err"][key] = per_source_err(Cp.cpu().numpy(), Cref)
                if rule == "iss":
                    with threadpool_limits(limits=1):
                        t0 = time.perf_counter()
                        o.run(mix.X, wl.D, wl.row_taps, B0n, V0n, wl.n_iter, rule=o.ISS)
                        dt1 = time.perf_counter() - t0
                    log(f"  oracle ISS, one thread: {dt1:.1f} s")
                    cpu = {"value": units / dto, "unit": "F·T·iters/s", "cores": workers, "kind": "oracle",
                           "sample": f"all {wl.n_iter} ISS iterations of the mixture (F={wl.F}, T={wl.T}, "
                                     f"Mbar={wl.mbar}) in FP64 NumPy, the W update of bin chunks on {workers} "
                                     f"threads, BLAS on 1 thread each; {dto:.1f} s",
                           "one_thread_value": units / dt1, "one_thread_s": dt1,
                           "cpu_model": cpu_info(), "os_cpu_count": os.cpu_count()}
                else:
                    cpu["ip_oracle_value"] = units / dto
        lines[name] = {
            "value": units / dtg, "ms_per_step": dtg * 1e3, "status": stg,
            "config": {"workload": f"{name}: 4 s, N=2, M=3, RT60 0.6 s, STFT 1024/256, D={wl.D} stacked frames "
                                   f"(Mbar={wl.mbar}, taps {'+'.join(map(str, wl.row_taps))}), K={wl.K}, "
                                   f"{wl.n_iter} iterations, FP64, graph replay",
                       "F": wl.F, "T": wl.T, "Mbar": wl.mbar, "K": wl.K, "iterations": wl.n_iter},
            "side_by_side": side, "accuracy": accuracy, "cpu_baseline": cpu}
    main_line = lines["c0"]
    out = {
        "metric": "F·T·iters/s ISS vs IP vs FP64-ISS at rel err ≤1e-4; HBM GB/s fraction",
        "value": main_line["value"], "unit": "F·T·iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_line["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": main_line["config"], "status": main_line["status"], "side_by_side": main_line["side_by_side"],
        "accuracy": main_line["accuracy"], "cpu_baseline": main_line["cpu_baseline"], "d1_variant": lines["c0_d1"],
    }
    print(json.dumps(out), flush=True)
    return 0


def small_bench(args) -> int:
    """The paper's experimental shape (Sec. V-A, Table I): 8 s at 16 kHz, N=2, M = 4/6/8 microphones,
    no frame stacking (Mbar = M, L_n = M / 2), STFT 1024/256 (F=513, T=501), K=3, 100 iterations.  At
    these sizes an iteration is a few tens of microseconds of kernels, so launches matter: the FP32
    ISS path is timed eagerly and with graph replay (ctfiss_set_graph).  Beside it, ISS and IP in
    FP32 and FP64 are timed the same way as one another (eager, input and state set every step), for
    the ISS-vs-IP runtime reduction the paper reports at these shapes; the FP64 oracle runs both
    rules on the original data (the accuracy of every path, and the CPU baseline)."""
    import torch

    from datagen import WORKLOADS, init_nmf, make_mixture
    from paper_2510_02382_amd import Separator

    wl = WORKLOADS[args.workload]
    log(f"workload {wl.name}: F={wl.F} T={wl.T} M={wl.M} Mbar={wl.mbar} taps={wl.row_taps} K={wl.K} "
        f"iters={wl.n_iter}")
    dev = torch.device("cuda:0")
    X = torch.from_numpy(make_mixture(wl, 0).X).to(dev).to(torch.complex64)
    B0n, V0n = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
    B0 = torch.from_numpy(B0n).to(dev).float()
    V0 = torch.from_numpy(V0n).to(dev).float()
    stream = torch.cuda.Stream(device=dev)
    res = {}
    for graph in (False, True):
        with torch.cuda.stream(stream):
            sep = Separator(wl.F, wl.T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision="fp32", stream=stream)
            if graph:
                sep.set_graph(True)
            sep.set_input(X)
            for _ in range(args.warmup + 1):
                sep.set_state(B=B0, V=V0)
                sep.iterate(wl.n_iter)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                sep.set_state(B=B0, V=V0)
                sep.iterate(wl.n_iter)
                C = sep.source_images()
            stream.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            res["graph" if graph else "eager"] = {"ms_per_step": dt * 1e3, "status": sep.status(), "C": C}
            sep.close()
        log(f"{'graph' if graph else 'eager'}: {dt * 1e3:.3f} ms per separation ({wl.n_iter} iterations)")
    same = bool(torch.equal(res["eager"]["C"], res["graph"]["C"]))
    units = wl.F * wl.T * wl.n_iter

    # ISS against IP at the paper's shape, each path timed the same way (eager launches; every
    # step sets the input and the state, iterates and forms the images), in FP32 and FP64
    mix = make_mixture(wl, 0)
    Xc = torch.from_numpy(mix.X).to(dev)
    B0d, V0d = torch.from_numpy(B0n).to(dev), torch.from_numpy(V0n).to(dev)
    side, images = {}, {}
    if not args.no_side:
        for prec, rule in (("fp32", "iss"), ("fp32", "ip"), ("fp64", "iss"), ("fp64", "ip")):
            dt, Cp, st, _ = time_path(torch, Separator, wl, Xc, B0d, V0d, prec, rule, args.side_steps, 1)
            key = f"{rule}_{prec}"
            side[key] = {"value": units * args.side_steps / dt, "ms_per_step": dt / args.side_steps * 1e3,
                         "status": st}
            images[key] = Cp
            log(f"{key}: {dt / args.side_steps * 1e3:.3f} ms per separation, status {st}")
        # counted only where both paths ran without a latched fault (FP32 IP can latch the
        # singular-system fault; its images are then not a separation)
        side["runtime_reduction_iss_vs_ip"] = {
            pr: (1.0 - side[f"iss_{pr}"]["ms_per_step"] / side[f"ip_{pr}"]["ms_per_step"])
            if side[f"iss_{pr}"]["status"] == 0 and side[f"ip_{pr}"]["status"] == 0 else None
            for pr in ("fp32", "fp64")}
        side["paper_runtime_reduction_iss_vs_ip"] = {
            "value": PAPER_REDUCTION.get(wl.name), "hardware": "laptop CPU (AMD Ryzen 7 5800H), paper Sec. V-A",
            "note": "the paper's relative figure for this microphone count (Sec. V-B, Fig. 3), context only"}
    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        accuracy = {"reference": f"FP64 oracle, {wl.n_iter} iterations of the same rule on the original FP64 data",
                    "target": 1e-4, "per_source_rel_err": {}}
        for rule in ("iss", "ip"):
            if rule == "ip" and (args.no_ip_oracle or args.no_side):
                continue
            log(f"FP64 oracle ({rule.upper()}), all iterations of the mixture, bin chunks over host threads")
            Cref, dto, workers = oracle_reference(wl, mix.X, B0n, V0n, rule)
            log(f"  oracle {rule.upper()}: {dto:.1f} s on {workers} threads")
            for key, Cp in list(images.items()) + ([("iss_fp32_graph", res["graph"]["C"])] if rule == "iss" else []):
                if key.startswith(rule):
                    ok = side.get(key, {"status": 0})["status"] == 0
                    accuracy["per_source_rel_err"][key] = per_source_err(Cp.cpu().numpy(), Cref) if ok else None
            if rule == "iss":
                cpu = {"value": units / dto, "unit": "F·T·iters/s", "cores": workers, "kind": "oracle",
                       "sample": f"all {wl.n_iter} ISS iterations of the mixture (F={wl.F}, T={wl.T}, "
                                 f"Mbar={wl.mbar}) in FP64 NumPy, the W update of bin chunks on {workers} threads, "
                                 f"BLAS on 1 thread each; {dto:.1f} s",
                       "cpu_model": cpu_info(), "os_cpu_count": os.cpu_count()}
            else:
                cpu["ip_oracle_value"] = units / dto
        errs = accuracy["per_source_rel_err"]
        accuracy["iss_fp32_meets_target"] = max(errs["iss_fp32_graph"]) <= 1e-4
    out = {
        "metric": "F·T·iters/s ISS vs IP vs FP64-ISS at rel err ≤1e-4; HBM GB/s fraction",
        "value": units / (res["graph"]["ms_per_step"] * 1e-3), "unit": "F·T·iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["graph"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"paper shape {wl.name}: 8 s, N=2, M={wl.M}, no frame stacking (Mbar={wl.mbar}), "
                               f"STFT 1024/256, K={wl.K}, {wl.n_iter} iterations, graph replay",
                   "F": wl.F, "T": wl.T, "Mbar": wl.mbar, "K": wl.K, "iterations": wl.n_iter},
        "eager_ms_per_step": res["eager"]["ms_per_step"], "graph_equals_eager": same,
        "status": res["graph"]["status"], "side_by_side": side, "accuracy": accuracy, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side-steps", type=int, default=2, help="timed steps of the FP64 and IP paths")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle (then no accuracy against the oracle either)")
    ap.add_argument("--no-ip-oracle", action="store_true", help="skip the IP oracle run (c1)")
    ap.add_argument("--no-side", action="store_true", help="time only the FP32 ISS path")
    ap.add_argument("--batched", action="store_true",
                    help="time the batch of uneven mixtures instead of the single long mixture")
    ap.add_argument("--batch", type=int, default=256, help="mixtures in --batched mode")
    ap.add_argument("--autotune", action="store_true",
                    help="--batched: also time the batch after tuning the launch shape of every distinct shape")
    ap.add_argument("--streams", type=int, default=8, help="c4: streams the mixtures are spread over")
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="hardware queues the HIP runtime opens for this process (GPU_MAX_HW_QUEUES, at most "
                         "32); default 16 for c4 (mixtures spread over several streams), else the runtime's own")
    ap.add_argument("--workload", choices=["c0", "c1", "c3", "c4", "P4", "P6", "P8"], default="c1",
                    help="c3: the 60 s, Mbar = 64 mixture (team launches) instead of the 10 s, Mbar = 24 one; "
                         "c4: forward and reverse pass of 32 mixtures (gradients); P4/P6/P8: the paper's "
                         "shapes, eager and graph replay")
    ap.add_argument("--exchange-cost", action="store_true",
                    help="c3: time the team launch against single-workgroup launches of the member's shape "
                         "on as many items without exchange")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs one mixture on one GPU; --gpus must be 1 "
              "(the bin-sharded multi-GPU path is a design, not built)", file=sys.stderr)
        return 2

    # streams beyond the runtime's hardware queues (4 by default) share queues and so run
    # their kernels one after another; set before the runtime starts.  The differentiation
    # workload's 8 streams gain from 16 queues (277 -> 255 ms per step); the batch's graph
    # replay does not (934 -> 960 ms), so it keeps the runtime's own count
    q = args.hw_queues if args.hw_queues is not None else (16 if args.workload == "c4" and not args.batched else 0)
    if q > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(q, 32))
    args.hw_queues = os.environ.get("GPU_MAX_HW_QUEUES")

    import torch

    if args.batched:
        return batched_bench(args)
    if args.workload == "c3":
        return exchange_cost(args) if args.exchange_cost else precision_bench(args)
    if args.workload == "c4":
        return adjoint_bench(args)
    if args.workload in ("P4", "P6", "P8"):
        return small_bench(args)
    if args.workload == "c0":
        return c0_bench(args)

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "copies": 3}))
        return 0

    from datagen import WORKLOADS, init_nmf, make_mixture
    from paper_2510_02382_amd import Separator

    wl = WORKLOADS["c1"]
    log(f"workload c1: F={wl.F} T={wl.T} M={wl.M} D={wl.D} Mbar={wl.mbar} taps={wl.row_taps} K={wl.K} "
        f"iters={wl.n_iter}")
    mix = make_mixture(wl, 0)
    B0n, V0n = init_nmf(wl.N, wl.F, wl.K, wl.T, 0)
    dev = torch.device("cuda:0")
    Xc = torch.from_numpy(mix.X).to(dev)
    B0 = torch.from_numpy(B0n).to(dev)
    V0 = torch.from_numpy(V0n).to(dev)
    units = wl.F * wl.T * wl.n_iter

    log("timing FP32 ISS (HIP events around the W-update kernel)")
    dt, C32, st32, stats = time_path(torch, Separator, wl, Xc, B0, V0, "fp32", "iss", args.steps, args.warmup,
                                     profile=1)
    value = units * args.steps / dt
    n_iss, ms_iss = stats[0]
    avg_iss_ms = ms_iss / max(n_iss, 1)
    units_launch = wl.F * wl.T
    flops_launch = units_launch * iss_flops_per_unit(wl.mbar)
    exec_flops_launch = units_launch * iss_executed_flops_per_unit(wl.mbar, wl.n_iter)
    bytes_launch = units_launch * iss_bytes_per_unit(wl.M, wl.N, wl.mbar, wl.T)
    achieved = flops_launch / (avg_iss_ms * 1e-3) / 1e12
    log("per-kernel breakdown (separate profiled steps, every kernel timed)")
    _, _, _, allstats = time_path(torch, Separator, wl, Xc, B0, V0, "fp32", "iss", 1, 0, profile=-1)
    names = ["w_update_iss", "v_partial", "v_update_mu", "final_rescale", "images", "lambda", "basis_update"]
    kernel_ms = {names[i]: allstats[i][1] / max(allstats[i][0], 1) for i in range(7)}
    probe = Separator(wl.F, wl.T, wl.M, wl.D, wl.N, wl.K, wl.row_taps, precision="fp32", rule="iss")
    nmf_path = probe.nmf_path()  # (1/lambda + basis update in the W update: 0/1/2, one-launch activation update)
    probe.close()
    log(f"FP32 ISS: {dt / args.steps * 1e3:.3f} ms/step, {value:.4e} F·T·it/s, k_iss avg {avg_iss_ms * 1e3:.1f} us "
        f"({achieved:.1f} TFLOP/s), status {st32}")

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
    hbm_bytes = traffic if traffic is not None else bytes_launch
    hbm_gbs = hbm_bytes / (avg_iss_ms * 1e-3) / 1e9

    side = {}
    images = {"iss_fp32": C32}
    if not args.no_side:
        log("timing FP64 ISS")
        dt64, C64, st64, _ = time_path(torch, Separator, wl, Xc, B0, V0, "fp64", "iss", args.side_steps, 1)
        side["iss_fp64"] = {"value": units * args.side_steps / dt64, "ms_per_step": dt64 / args.side_steps * 1e3,
                            "status": st64}
        images["iss_fp64"] = C64
        log(f"FP64 ISS: {dt64 / args.side_steps * 1e3:.3f} ms/step")
        log("timing mixed-precision ISS")
        dtm, Cm, stm, _ = time_path(torch, Separator, wl, Xc, B0, V0, "mixed", "iss", args.side_steps, 1)
        side["iss_mixed"] = {"value": units * args.side_steps / dtm, "ms_per_step": dtm / args.side_steps * 1e3,
                             "status": stm}
        images["iss_mixed"] = Cm
        log(f"mixed ISS: {dtm / args.side_steps * 1e3:.3f} ms/step")
        log("timing FP64 IP")
        dtip, Cip, stip, ipstats = time_path(torch, Separator, wl, Xc, B0, V0, "fp64", "ip", args.side_steps, 1,
                                             profile=1)
        n_ip, ms_ip = ipstats[0]
        avg_ip_ms = ms_ip / max(n_ip, 1)
        ip_flops_launch = units_launch * wl.mbar * (4 * wl.mbar ** 2 + 11 * wl.mbar ** 3 / wl.T + 8 * wl.mbar)
        side["ip_fp64"] = {"value": units * args.side_steps / dtip, "ms_per_step": dtip / args.side_steps * 1e3,
                           "status": stip, "k_ip_avg_us": avg_ip_ms * 1e3,
                           "k_ip_tflops": ip_flops_launch / (avg_ip_ms * 1e-3) / 1e12,
                           "k_ip_frac_fp64_peak": ip_flops_launch / (avg_ip_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        images["ip_fp64"] = Cip
        log(f"FP64 IP: {dtip / args.side_steps * 1e3:.3f} ms/step, status {stip}")
        log("timing FP32 IP")
        dtip32, _, stip32, _ = time_path(torch, Separator, wl, Xc, B0, V0, "fp32", "ip", 1, 0)
        side["ip_fp32"] = {"value": units / dtip32, "ms_per_step": dtip32 * 1e3, "status": stip32,
                           "note": "FP32 IP latches the singular-system fault on this mixture; not counted"
                           if stip32 else "ok"}
        side["speedup_iss_fp32_vs_ip_fp64"] = value / side["ip_fp64"]["value"]
        side["speedup_iss_fp64_vs_ip_fp64"] = side["iss_fp64"]["value"] / side["ip_fp64"]["value"]

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        log("FP64 oracle (ISS), all iterations of the full mixture, bin chunks over host threads")
        Cref, dto, workers = oracle_reference(wl, mix.X, B0n, V0n, "iss")
        log(f"  oracle ISS: {dto:.1f} s on {workers} threads")
        accuracy = {"reference": f"FP64 oracle, {wl.n_iter} ISS iterations of the full mixture on the original FP64 "
                                 f"data", "target": 1e-4, "per_source_rel_err": {}}
        for k in ("iss_fp32", "iss_mixed", "iss_fp64"):
            if k in images:
                accuracy["per_source_rel_err"][k] = per_source_err(images[k].cpu().numpy(), Cref)
        accuracy["iss_fp32_meets_target"] = max(accuracy["per_source_rel_err"]["iss_fp32"]) <= 1e-4
        cpu = {"value": units / dto, "unit": "F·T·iters/s", "cores": workers, "kind": "oracle",
               "sample": f"all {wl.n_iter} ISS iterations of the full mixture (F={wl.F}, T={wl.T}, Mbar={wl.mbar}) "
                         f"in FP64 NumPy: the oracle's functions, the W update of bin chunks on a pool of {workers} "
                         f"threads, BLAS on 1 thread each; {dto:.1f} s",
               "cpu_model": cpu_info(), "os_cpu_count": os.cpu_count()}
        if "ip_fp64" in images and not args.no_ip_oracle:
            log("FP64 oracle (IP), all iterations of the full mixture")
            Cref_ip, dtoi, _ = oracle_reference(wl, mix.X, B0n, V0n, "ip")
            log(f"  oracle IP: {dtoi:.1f} s")
            accuracy["per_source_rel_err"]["ip_fp64_vs_ip_oracle"] = per_source_err(images["ip_fp64"].cpu().numpy(),
                                                                                    Cref_ip)
            cpu["ip_oracle_value"] = units / dtoi

    out = {
        "metric": "F·T·iters/s ISS vs IP vs FP64-ISS at rel err ≤1e-4; HBM GB/s fraction",
        "value": value,
        "unit": "F·T·iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c1 single mixture: 10 s, N=2, M=3, RT60 0.9 s, STFT 2048/512, D=8 stacked frames "
                               "(Mbar=24, taps 12+12), K=20, 100 iterations, CTF-MNMF-ISS",
                   "F": wl.F, "T": wl.T, "Mbar": wl.mbar, "K": wl.K, "iterations": wl.n_iter},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": traffic,
                     "kernel": "k_iss (W update: ISS sweep on the carried Y + tap-aligned powers, one launch per "
                               "iteration; with nmf_path[0] > 0 each bin also forms its 1/lambda and basis update)",
                     "nmf_path": list(nmf_path),
                     "iteration_us": dt / args.steps / wl.n_iter * 1e6,
                     "frac_iteration": flops_launch / (dt / args.steps / wl.n_iter) / 1e12 / PEAK_FP32_VALU_TFLOPS,
                     "avg_launch_us": avg_iss_ms * 1e3, "flops_per_launch": flops_launch,
                     "flops_per_unit": iss_flops_per_unit(wl.mbar), "units_per_launch": units_launch,
                     "executed_flops_per_launch": exec_flops_launch,
                     "frac_executed": exec_flops_launch / (avg_iss_ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "hbm_gbs": hbm_gbs, "hbm_frac": hbm_gbs / (PEAK_HBM_TBS * 1e3),
                     "hbm_bytes_source": "rocprofv3 counters (FETCH_SIZE, WRITE_SIZE)" if traffic is not None
                     else "algorithmic bytes"},
        "kernel_avg_ms": kernel_ms,
        "status": st32,
        "accuracy": accuracy,
        "side_by_side": side,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

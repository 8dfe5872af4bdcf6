"""Seeded synthetic input generators shared by the GPU path's tests/bench and the CPU oracle.

Holds no arithmetic of the separation method itself."""
from .synth import (WORKLOADS, Mixture, Workload, balanced_taps, batched_workloads, ctf_mixture,
                    init_nmf, istft, make_mixture, n_frames, random_problem, rng_for, stft)

__all__ = ["WORKLOADS", "Mixture", "Workload", "balanced_taps", "batched_workloads", "ctf_mixture",
           "init_nmf", "istft", "make_mixture", "n_frames", "random_problem", "rng_for", "stft"]

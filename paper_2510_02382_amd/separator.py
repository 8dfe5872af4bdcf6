"""Tensor-level wrapper over the C ABI: one context, its workspace and bound buffers."""
from __future__ import annotations

import numpy as np
import torch

from . import binding as b

_PREC = {"fp32": b.CTFISS_FP32, "fp64": b.CTFISS_FP64, "mixed": b.CTFISS_MIXED, "mixed_bf16": b.CTFISS_MIXED_BF16}
_RULE = {"iss": b.CTFISS_RULE_ISS, "ip": b.CTFISS_RULE_IP}
_VRULE = {"all_taps": b.CTFISS_VRULE_ALL_TAPS, "paper_tap0": b.CTFISS_VRULE_PAPER_TAP0}


class Separator:
    """CTF-MNMF separation of one mixture on one GPU.

    X [M, F, T] complex (complex64 for fp32 and mixed, complex128 for fp64) on the device;
    W [F, Mbar, Mbar] complex, B [N, F, K] and V [N, K, T] real.  All work is
    enqueued on `stream` (default: torch's current stream when the object is made).
    """

    def __init__(self, F, T, M, D, N, K, taps, precision="fp32", rule="iss", vrule="all_taps", floor=1e-8,
                 device="cuda", stream=None):
        self.F, self.T, self.M, self.D, self.N, self.K = int(F), int(T), int(M), int(D), int(N), int(K)
        self.taps = tuple(int(x) for x in taps)
        self.Mbar = self.M * self.D
        self.precision = precision
        self.rdtype = torch.float64 if precision == "fp64" else torch.float32
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._shape = b.make_shape(F, T, M, D, N, K, self.taps)
        nbytes = b.ctfiss_workspace_size(self._shape, _PREC[precision])
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        self.ctx = b.ctfiss_create(self._shape, _PREC[precision], _RULE[rule], _VRULE[vrule], floor,
                                   self.workspace, self.stream)
        self._X = None

    def _check(self, t, shape, dtype, name):
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {self.device}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")

    def set_input(self, X: torch.Tensor) -> None:
        self._check(X, (self.M, self.F, self.T), self.cdtype, "X")
        self._X = X
        b.ctfiss_set_input(self.ctx, X)

    def set_state(self, B: torch.Tensor, V: torch.Tensor, W: torch.Tensor | None = None) -> None:
        self._check(B, (self.N, self.F, self.K), self.rdtype, "B")
        self._check(V, (self.N, self.K, self.T), self.rdtype, "V")
        if W is not None:
            self._check(W, (self.F, self.Mbar, self.Mbar), self.cdtype, "W")
        b.ctfiss_set_state(self.ctx, W, B, V)

    def iterate(self, n_iter: int, trace: bool = False):
        """Enqueue n_iter iterations.  trace=True: returns the objective of Eq. (5) after every
        iteration (a float64 NumPy array; the call then synchronises)."""
        if not trace:
            b.ctfiss_iterate(self.ctx, n_iter)
            return None
        out = np.empty(int(n_iter), dtype=np.float64)
        b.ctfiss_iterate(self.ctx, n_iter, out)
        return out

    def plan(self):
        """(G, frames per lane, rows per group, workgroups per bin) of the W update."""
        return b.ctfiss_get_plan(self.ctx)

    def nmf_path(self):
        """(fused, v_one_launch) of ctfiss_get_nmf_path: where 1/lambda and the basis update run
        (0 own launches, 1 in the W update with the activations in LDS, 2 read from device
        memory) and whether the activation update is one launch."""
        return b.ctfiss_get_nmf_path(self.ctx)

    def autotune(self, trials: int = 3):
        """Time every fitting launch shape of the W update on this context's data and keep the
        fastest (ctfiss_autotune; cached for later contexts of the shape).  Returns plan()."""
        scratch = torch.empty(b.ctfiss_autotune_scratch_size(self.ctx), dtype=torch.uint8, device=self.device)
        if scratch.data_ptr() % 256:
            raise RuntimeError("scratch allocation is not 256-byte aligned")
        b.ctfiss_autotune(self.ctx, trials, scratch)
        return self.plan()

    def set_graph(self, enable: bool = True) -> None:
        """Replay captured HIP graphs for iterate() (ctfiss_set_graph); needs a non-NULL stream."""
        b.ctfiss_set_graph(self.ctx, enable)

    def state(self):
        W = torch.empty((self.F, self.Mbar, self.Mbar), dtype=self.cdtype, device=self.device)
        B = torch.empty((self.N, self.F, self.K), dtype=self.rdtype, device=self.device)
        V = torch.empty((self.N, self.K, self.T), dtype=self.rdtype, device=self.device)
        b.ctfiss_get_state(self.ctx, W, B, V)
        return W, B, V

    def source_images(self) -> torch.Tensor:
        C = torch.empty((self.N, self.M, self.F, self.T), dtype=self.cdtype, device=self.device)
        b.ctfiss_source_images(self.ctx, C)
        return C

    def nll(self) -> float:
        return b.ctfiss_nll(self.ctx)

    def status(self) -> int:
        """0 if no device fault was latched, else the device fault code (synchronises)."""
        return b.ctfiss_sync_status(self.ctx)[1]

    def set_profiling(self, mask) -> None:
        """mask: bit i times kernel class i (see ctfiss_set_profiling); True = all, False = none."""
        if mask is True:
            mask = -1
        elif mask is False:
            mask = 0
        b.ctfiss_set_profiling(self.ctx, int(mask))

    def kernel_stats(self, which: int):
        return b.ctfiss_kernel_stats(self.ctx, which)

    def check(self) -> None:
        """Raise CtfissError(CTFISS_E_NUMERIC) if a device fault is latched (synchronises)."""
        st, code = b.ctfiss_sync_status(self.ctx)
        if st != b.CTFISS_OK:
            raise b.CtfissError(st, f"device fault {code}")

    def backward(self, n_iter: int, B0: torch.Tensor, V0: torch.Tensor, gC: torch.Tensor):
        """Gradients (gX, gB0, gV0) of a real loss through W = I, (B0, V0), n_iter
        iterations and the source images, given gC = dL/dC (ctfiss_backward; FP32, FP64 or
        mixed, ISS, either activation rule).  The input bound by set_input is X.  Enqueued
        without waiting: a numeric fault stays latched for status() / check()."""
        self._check(B0, (self.N, self.F, self.K), self.rdtype, "B0")
        self._check(V0, (self.N, self.K, self.T), self.rdtype, "V0")
        self._check(gC, (self.N, self.M, self.F, self.T), self.cdtype, "gC")
        nbytes = b.ctfiss_adjoint_workspace_size(self._shape, _PREC[self.precision], n_iter)
        aws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if aws.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        gX = torch.empty((self.M, self.F, self.T), dtype=self.cdtype, device=self.device)
        gB0 = torch.empty_like(B0)
        gV0 = torch.empty_like(V0)
        b.ctfiss_backward(self.ctx, n_iter, B0, V0, gC, gX, gB0, gV0, aws)
        return gX, gB0, gV0

    def close(self) -> None:
        if self.ctx is not None:
            b.ctfiss_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSeparator:
    """CTF-MNMF separation of many mixtures of uneven shape on one GPU (ctfiss_batch_*).

    shapes: list of (F, T, M, D, N, K, taps).  Mixture i takes tensors of the
    shapes a Separator of shapes[i] takes.  Each iteration runs every mixture;
    per launch shape the W update is one persistent launch over all bins of all
    those mixtures, and each NMF step is one launch over all mixtures.
    """

    def __init__(self, shapes, precision="fp32", rule="iss", vrule="all_taps", floor=1e-8, device="cuda",
                 stream=None):
        self.shapes = [(int(F), int(T), int(M), int(D), int(N), int(K), tuple(int(x) for x in taps))
                       for (F, T, M, D, N, K, taps) in shapes]
        self.precision = precision
        self.rdtype = torch.float64 if precision == "fp64" else torch.float32
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._shapes = [b.make_shape(*sh) for sh in self.shapes]
        nbytes = b.ctfiss_batch_workspace_size(self._shapes, _PREC[precision])
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        self.batch = b.ctfiss_batch_create(self._shapes, _PREC[precision], _RULE[rule], _VRULE[vrule], floor,
                                           self.workspace, self.stream)
        self._X = None

    def _check(self, ts, shape_fn, dtype, name):
        if len(ts) != len(self.shapes):
            raise ValueError(f"{name}: expected {len(self.shapes)} tensors, got {len(ts)}")
        for i, (t, sh) in enumerate(zip(ts, self.shapes)):
            want = shape_fn(*sh)
            if t.device != self.device or t.dtype != dtype or tuple(t.shape) != want or not t.is_contiguous():
                raise ValueError(f"{name}[{i}]: expected contiguous {dtype} {want} on {self.device}, got "
                                 f"{t.dtype} {tuple(t.shape)} on {t.device}")

    def set_input(self, X) -> None:
        self._check(X, lambda F, T, M, D, N, K, taps: (M, F, T), self.cdtype, "X")
        self._X = list(X)
        b.ctfiss_batch_set_input(self.batch, self._X)

    def set_state(self, B, V, W=None) -> None:
        self._check(B, lambda F, T, M, D, N, K, taps: (N, F, K), self.rdtype, "B")
        self._check(V, lambda F, T, M, D, N, K, taps: (N, K, T), self.rdtype, "V")
        if W is not None:
            self._check(W, lambda F, T, M, D, N, K, taps: (F, M * D, M * D), self.cdtype, "W")
        b.ctfiss_batch_set_state(self.batch, W, B, V)

    def iterate(self, n_iter: int) -> None:
        b.ctfiss_batch_iterate(self.batch, n_iter)

    def set_graph(self, enable: bool = True) -> None:
        """Replay captured HIP graphs for iterate() (ctfiss_batch_set_graph); needs a non-NULL stream."""
        b.ctfiss_batch_set_graph(self.batch, enable)

    def source_images(self):
        C = [torch.empty((N, M, F, T), dtype=self.cdtype, device=self.device)
             for (F, T, M, D, N, K, taps) in self.shapes]
        b.ctfiss_batch_source_images(self.batch, C)
        return C

    def status(self) -> tuple[int, int]:
        """(mixture, code) of the first mixture with a latched device fault, or (-1, 0) (synchronises)."""
        _, mix, code = b.ctfiss_batch_sync_status(self.batch)
        return mix, code

    def close(self) -> None:
        if self.batch is not None:
            b.ctfiss_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

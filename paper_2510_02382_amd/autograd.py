"""torch.autograd.Function over the unrolled separation (forward and reverse on the GPU).

    C = separate(X, B0, V0, D, taps, n_iter, vrule="all_taps")

runs W = I, (B0, V0), n_iter CTF-MNMF-ISS iterations (activation update over all
taps of a source, or over tap 0 as Eq. (18) prints it: vrule "paper_tap0") and the source images
through the C ABI (FP64 contexts for complex128 inputs, FP32 for complex64, or the mixed
path for complex64 with precision="mixed": its forward keeps the sweep's W rows in FP64, its
reverse pass runs the FP32 adjoint kernels),
and its backward calls ctfiss_backward,
whose hand-written adjoint kernels re-run the forward with the state saved per
iteration and reverse it.  Gradients flow to X (complex [M, F, T]), B0 and V0.
"""
from __future__ import annotations

import torch

from .separator import Separator


class _Separate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, B0, V0, D, taps, n_iter, floor, check, vrule, precision):
        M, F, T = X.shape
        N, _, K = B0.shape
        if precision is None:
            precision = "fp32" if X.dtype == torch.complex64 else "fp64"
        sep = Separator(F, T, M, D, N, K, taps, precision=precision, vrule=vrule, floor=floor, device=X.device)
        Xc, Bc, Vc = X.detach().contiguous(), B0.detach().contiguous(), V0.detach().contiguous()
        sep.set_input(Xc)
        sep.set_state(B=Bc, V=Vc)
        sep.iterate(n_iter)
        C = sep.source_images()
        if check:
            sep.check()
        ctx.sep = sep
        ctx.n_iter = n_iter
        ctx.check = check
        ctx.save_for_backward(Xc, Bc, Vc)
        return C

    @staticmethod
    def backward(ctx, gC):
        Xc, Bc, Vc = ctx.saved_tensors
        sep = ctx.sep
        sep.set_input(Xc)
        gX, gB0, gV0 = sep.backward(ctx.n_iter, Bc, Vc, gC.contiguous())
        try:
            if ctx.check:
                sep.check()
        finally:
            sep.close()
        return gX, gB0, gV0, None, None, None, None, None, None, None


def separate(X: torch.Tensor, B0: torch.Tensor, V0: torch.Tensor, D: int, taps, n_iter: int,
             floor: float = 1e-8, check: bool = True, vrule: str = "all_taps",
             precision: str | None = None) -> torch.Tensor:
    """Source images [N, M, F, T] after n_iter iterations, differentiable in X, B0, V0 (complex128 /
    float64 tensors run in FP64, complex64 / float32 in FP32).  check=True: the forward and the
    backward each read the device status word and raise CtfissError on a latched numeric fault
    (a synchronisation each); check=False leaves both asynchronous (faults then go unreported).
    precision: None (from the dtype), or "mixed" for complex64 / float32 inputs."""
    if precision not in (None, "mixed"):
        raise ValueError("precision is None (from the dtype) or 'mixed'")
    if precision == "mixed" and X.dtype != torch.complex64:
        raise ValueError("the mixed path takes complex64 / float32 inputs")
    return _Separate.apply(X, B0, V0, int(D), tuple(int(t) for t in taps), int(n_iter), float(floor), bool(check),
                           str(vrule), precision)

"""Thin Python binding of the C ABI in include/ctfiss.h.

Functions carry the C names and only marshal arguments: torch tensors supply
device pointers and the current HIP stream, every computation runs in the HIP
library.  There is no CPU fallback: importing this module on a machine where
libctfiss.so was not built raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctfiss.so")

CTFISS_OK = 0
CTFISS_E_ARG = -1
CTFISS_E_SHAPE = -2
CTFISS_E_UNSUPPORTED = -3
CTFISS_E_WORKSPACE = -4
CTFISS_E_ORDER = -5
CTFISS_E_HIP = -6
CTFISS_E_NUMERIC = -7
CTFISS_E_TOO_LARGE = -8

CTFISS_FP32, CTFISS_FP64, CTFISS_MIXED, CTFISS_MIXED_BF16 = 0, 1, 2, 3
CTFISS_RULE_ISS, CTFISS_RULE_IP = 0, 1
CTFISS_VRULE_ALL_TAPS, CTFISS_VRULE_PAPER_TAP0 = 0, 1

EXPORTS = (
    "ctfiss_workspace_size", "ctfiss_create", "ctfiss_set_input", "ctfiss_set_state", "ctfiss_iterate",
    "ctfiss_get_state", "ctfiss_source_images", "ctfiss_nll", "ctfiss_sync_status", "ctfiss_destroy",
    "ctfiss_status_string", "ctfiss_set_profiling", "ctfiss_kernel_stats",
    "ctfiss_batch_workspace_size", "ctfiss_batch_create", "ctfiss_batch_set_input", "ctfiss_batch_set_state",
    "ctfiss_batch_iterate", "ctfiss_batch_source_images", "ctfiss_batch_sync_status", "ctfiss_batch_destroy",
    "ctfiss_adjoint_workspace_size", "ctfiss_backward", "ctfiss_set_graph", "ctfiss_get_plan", "ctfiss_get_nmf_path", "ctfiss_autotune",
    "ctfiss_autotune_scratch_size", "ctfiss_clear_tuned_plans", "ctfiss_separate_noalloc", "ctfiss_batch_set_graph",
)


class CtfissError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {ctfiss_status_string(status)} ({status})")


class Shape(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int32), ("T", ctypes.c_int32), ("M", ctypes.c_int32), ("D", ctypes.c_int32),
                ("N", ctypes.c_int32), ("K", ctypes.c_int32), ("taps", ctypes.POINTER(ctypes.c_int32))]


def load_library(path: str = _LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first (python -m paper_2510_02382_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "ctfiss_workspace_size": ([ctypes.POINTER(Shape), i32, ctypes.POINTER(sz)], i32),
        "ctfiss_create": ([ctypes.POINTER(Shape), i32, i32, i32, ctypes.c_double, vp, sz, vp,
                           ctypes.POINTER(vp)], i32),
        "ctfiss_set_input": ([vp, vp], i32),
        "ctfiss_set_state": ([vp, vp, vp, vp], i32),
        "ctfiss_iterate": ([vp, i32, ctypes.POINTER(ctypes.c_double)], i32),
        "ctfiss_get_state": ([vp, vp, vp, vp], i32),
        "ctfiss_source_images": ([vp, vp], i32),
        "ctfiss_nll": ([vp, ctypes.POINTER(ctypes.c_double)], i32),
        "ctfiss_sync_status": ([vp, ctypes.POINTER(i32)], i32),
        "ctfiss_destroy": ([vp], i32),
        "ctfiss_status_string": ([i32], ctypes.c_char_p),
        "ctfiss_set_profiling": ([vp, i32], i32),
        "ctfiss_kernel_stats": ([vp, i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)], i32),
        "ctfiss_batch_workspace_size": ([ctypes.POINTER(Shape), i32, i32, ctypes.POINTER(sz)], i32),
        "ctfiss_batch_create": ([ctypes.POINTER(Shape), i32, i32, i32, i32, ctypes.c_double, vp, sz, vp,
                                 ctypes.POINTER(vp)], i32),
        "ctfiss_batch_set_input": ([vp, ctypes.POINTER(vp)], i32),
        "ctfiss_batch_set_state": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)], i32),
        "ctfiss_batch_iterate": ([vp, i32], i32),
        "ctfiss_batch_set_graph": ([vp, i32], i32),
        "ctfiss_batch_source_images": ([vp, ctypes.POINTER(vp)], i32),
        "ctfiss_batch_sync_status": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "ctfiss_batch_destroy": ([vp], i32),
        "ctfiss_adjoint_workspace_size": ([ctypes.POINTER(Shape), i32, i32, ctypes.POINTER(sz)], i32),
        "ctfiss_backward": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, sz], i32),
        "ctfiss_set_graph": ([vp, i32], i32),
        "ctfiss_get_nmf_path": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "ctfiss_get_plan": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
                            i32),
        "ctfiss_autotune_scratch_size": ([vp, ctypes.POINTER(sz)], i32),
        "ctfiss_autotune": ([vp, i32, vp, sz], i32),
        "ctfiss_clear_tuned_plans": ([], i32),
        "ctfiss_separate_noalloc": ([ctypes.POINTER(Shape), i32, i32, i32, ctypes.c_double, vp, vp, vp, vp, i32, vp,
                                     vp, vp, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = load_library()


def _check(status: int, where: str) -> None:
    if status != CTFISS_OK:
        raise CtfissError(status, where)


def make_shape(F, T, M, D, N, K, taps):
    arr = (ctypes.c_int32 * len(taps))(*[int(x) for x in taps])
    sh = Shape(int(F), int(T), int(M), int(D), int(N), int(K), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)))
    sh._taps_keepalive = arr
    return sh


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def ctfiss_status_string(status: int) -> str:
    return _lib.ctfiss_status_string(int(status)).decode()


def ctfiss_workspace_size(shape: Shape, precision: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ctfiss_workspace_size(ctypes.byref(shape), int(precision), ctypes.byref(out)), "ctfiss_workspace_size")
    return int(out.value)


def ctfiss_create(shape: Shape, precision: int, rule: int, vrule: int, floor: float, workspace: torch.Tensor,
                  stream=None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(_lib.ctfiss_create(ctypes.byref(shape), int(precision), int(rule), int(vrule), float(floor),
                              _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream),
                              ctypes.byref(ctx)), "ctfiss_create")
    return ctx


def ctfiss_set_input(ctx, X: torch.Tensor) -> None:
    _check(_lib.ctfiss_set_input(ctx, _ptr(X)), "ctfiss_set_input")


def ctfiss_set_state(ctx, W, B, V) -> None:
    _check(_lib.ctfiss_set_state(ctx, _ptr(W), _ptr(B), _ptr(V)), "ctfiss_set_state")


def ctfiss_iterate(ctx, n_iter: int, nll_host=None) -> None:
    """nll_host: None, or a C-contiguous float64 NumPy array of n_iter entries that receives the
    objective after every iteration."""
    ptr = None
    if nll_host is not None:
        if nll_host.dtype.name != "float64" or not nll_host.flags.c_contiguous or nll_host.size < int(n_iter):
            raise ValueError("nll_host: expected a C-contiguous float64 array of n_iter entries")
        ptr = nll_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(_lib.ctfiss_iterate(ctx, int(n_iter), ptr), "ctfiss_iterate")


def ctfiss_get_state(ctx, W, B, V) -> None:
    _check(_lib.ctfiss_get_state(ctx, _ptr(W), _ptr(B), _ptr(V)), "ctfiss_get_state")


def ctfiss_source_images(ctx, C: torch.Tensor) -> None:
    _check(_lib.ctfiss_source_images(ctx, _ptr(C)), "ctfiss_source_images")


def ctfiss_nll(ctx) -> float:
    out = ctypes.c_double(0.0)
    _check(_lib.ctfiss_nll(ctx, ctypes.byref(out)), "ctfiss_nll")
    return float(out.value)


def ctfiss_sync_status(ctx) -> tuple[int, int]:
    code = ctypes.c_int32(0)
    st = _lib.ctfiss_sync_status(ctx, ctypes.byref(code))
    if st not in (CTFISS_OK, CTFISS_E_NUMERIC):
        raise CtfissError(st, "ctfiss_sync_status")
    return st, int(code.value)


def ctfiss_destroy(ctx) -> None:
    _check(_lib.ctfiss_destroy(ctx), "ctfiss_destroy")


def ctfiss_set_profiling(ctx, mask: int) -> None:
    """mask: bit i times kernel class i; -1 times all, 0 disables."""
    _check(_lib.ctfiss_set_profiling(ctx, int(mask)), "ctfiss_set_profiling")


def ctfiss_kernel_stats(ctx, which: int) -> tuple[int, float]:
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(_lib.ctfiss_kernel_stats(ctx, int(which), ctypes.byref(n), ctypes.byref(ms)), "ctfiss_kernel_stats")
    return int(n.value), float(ms.value)


def ctfiss_get_plan(ctx) -> tuple[int, int, int, int]:
    v = [ctypes.c_int32(0) for _ in range(4)]
    _check(_lib.ctfiss_get_plan(ctx, *[ctypes.byref(x) for x in v]), "ctfiss_get_plan")
    return tuple(int(x.value) for x in v)


def ctfiss_get_nmf_path(ctx) -> tuple[int, int]:
    """(fused: 0 separate launches, 1 in the W update with activations in LDS, 2 likewise from
    device memory; 1 if the activation update is one launch)."""
    v = [ctypes.c_int32(0) for _ in range(2)]
    _check(_lib.ctfiss_get_nmf_path(ctx, *[ctypes.byref(x) for x in v]), "ctfiss_get_nmf_path")
    return tuple(int(x.value) for x in v)


def ctfiss_autotune_scratch_size(ctx) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ctfiss_autotune_scratch_size(ctx, ctypes.byref(out)), "ctfiss_autotune_scratch_size")
    return int(out.value)


def ctfiss_autotune(ctx, trials: int, scratch: torch.Tensor) -> None:
    _check(_lib.ctfiss_autotune(ctx, int(trials), _ptr(scratch), scratch.numel() * scratch.element_size()),
           "ctfiss_autotune")


def ctfiss_clear_tuned_plans() -> None:
    _check(_lib.ctfiss_clear_tuned_plans(), "ctfiss_clear_tuned_plans")


def ctfiss_set_graph(ctx, enable: bool) -> None:
    _check(_lib.ctfiss_set_graph(ctx, 1 if enable else 0), "ctfiss_set_graph")


def ctfiss_adjoint_workspace_size(shape: Shape, precision: int, n_iter: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ctfiss_adjoint_workspace_size(ctypes.byref(shape), int(precision), int(n_iter), ctypes.byref(out)),
           "ctfiss_adjoint_workspace_size")
    return int(out.value)


def ctfiss_backward(ctx, n_iter: int, B0, V0, gC, gX, gB0, gV0, aws: torch.Tensor) -> None:
    _check(_lib.ctfiss_backward(ctx, int(n_iter), _ptr(B0), _ptr(V0), _ptr(gC), _ptr(gX), _ptr(gB0), _ptr(gV0),
                                _ptr(aws), aws.numel() * aws.element_size()), "ctfiss_backward")


def ctfiss_separate_noalloc(shape: Shape, precision: int, rule: int, vrule: int, floor: float, X, W0, B0, V0,
                            n_iter: int, C, W, B, V, status, stream=None) -> None:
    _check(_lib.ctfiss_separate_noalloc(ctypes.byref(shape), int(precision), int(rule), int(vrule), float(floor),
                                        _ptr(X), _ptr(W0), _ptr(B0), _ptr(V0), int(n_iter), _ptr(C), _ptr(W),
                                        _ptr(B), _ptr(V), _ptr(status), _stream(stream)),
           "ctfiss_separate_noalloc")


# ------------------------------------------------------------------ batches
def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))(*[None if t is None else int(t.data_ptr()) for t in tensors])
    return arr


def _shape_array(shapes):
    arr = (Shape * len(shapes))(*shapes)
    arr._keepalive = [sh._taps_keepalive for sh in shapes]
    return arr


def ctfiss_batch_workspace_size(shapes, precision: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ctfiss_batch_workspace_size(_shape_array(shapes), len(shapes), int(precision), ctypes.byref(out)),
           "ctfiss_batch_workspace_size")
    return int(out.value)


def ctfiss_batch_create(shapes, precision: int, rule: int, vrule: int, floor: float, workspace: torch.Tensor,
                        stream=None) -> ctypes.c_void_p:
    b = ctypes.c_void_p()
    _check(_lib.ctfiss_batch_create(_shape_array(shapes), len(shapes), int(precision), int(rule), int(vrule),
                                    float(floor), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                    _stream(stream), ctypes.byref(b)), "ctfiss_batch_create")
    return b


def ctfiss_batch_set_input(b, X) -> None:
    _check(_lib.ctfiss_batch_set_input(b, _ptr_array(X)), "ctfiss_batch_set_input")


def ctfiss_batch_set_state(b, W, B, V) -> None:
    _check(_lib.ctfiss_batch_set_state(b, None if W is None else _ptr_array(W), _ptr_array(B), _ptr_array(V)),
           "ctfiss_batch_set_state")


def ctfiss_batch_iterate(b, n_iter: int) -> None:
    _check(_lib.ctfiss_batch_iterate(b, int(n_iter)), "ctfiss_batch_iterate")


def ctfiss_batch_set_graph(b, enable: bool) -> None:
    _check(_lib.ctfiss_batch_set_graph(b, 1 if enable else 0), "ctfiss_batch_set_graph")


def ctfiss_batch_source_images(b, C) -> None:
    _check(_lib.ctfiss_batch_source_images(b, _ptr_array(C)), "ctfiss_batch_source_images")


def ctfiss_batch_sync_status(b) -> tuple[int, int, int]:
    mix = ctypes.c_int32(-1)
    code = ctypes.c_int32(0)
    st = _lib.ctfiss_batch_sync_status(b, ctypes.byref(mix), ctypes.byref(code))
    if st not in (CTFISS_OK, CTFISS_E_NUMERIC):
        raise CtfissError(st, "ctfiss_batch_sync_status")
    return st, int(mix.value), int(code.value)


def ctfiss_batch_destroy(b) -> None:
    _check(_lib.ctfiss_batch_destroy(b), "ctfiss_batch_destroy")

"""C-ABI library on the CPU: it loads, exports every declared entry point, and
rejects bad arguments before touching the GPU (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctfiss.h")
LIB = os.path.join(ROOT, "paper_2510_02382_amd", "libctfiss.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(ctfiss_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def binding():
    if not os.path.exists(LIB):
        from paper_2510_02382_amd import build
        build.build(verbose=False)
    from paper_2510_02382_amd import binding
    return binding


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ctfiss_create", "ctfiss_set_input", "ctfiss_set_state", "ctfiss_iterate",
                     "ctfiss_get_state", "ctfiss_source_images", "ctfiss_nll", "ctfiss_sync_status",
                     "ctfiss_destroy", "ctfiss_workspace_size", "ctfiss_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ctfiss_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(binding.EXPORTS) == set(declared_functions())


def test_shape_validation_without_gpu(binding):
    b = binding
    ok = b.make_shape(1025, 313, 3, 8, 2, 20, (12, 12))
    assert b.ctfiss_workspace_size(ok, b.CTFISS_FP32) > 0
    assert b.ctfiss_workspace_size(ok, b.CTFISS_FP64) > b.ctfiss_workspace_size(ok, b.CTFISS_FP32)
    cases = [
        ((1025, 313, 3, 8, 2, 20, (12, 11)), b.CTFISS_E_SHAPE),      # taps do not sum to M*D
        ((0, 313, 3, 8, 2, 20, (12, 12)), b.CTFISS_E_SHAPE),
        ((10, 0, 3, 1, 2, 2, (2, 1)), b.CTFISS_E_SHAPE),
        ((10, 10, 3, 1, 2, 2, (3, 0)), b.CTFISS_E_SHAPE),            # a source without taps
        ((10, 10, 3, 30, 2, 2, (45, 45)), b.CTFISS_E_UNSUPPORTED),   # Mbar = 90 > 64
        ((10, 10, 3, 1, 2, 65, (2, 1)), b.CTFISS_E_UNSUPPORTED),     # K > 64
    ]
    for args, code in cases:
        with pytest.raises(b.CtfissError) as e:
            b.ctfiss_workspace_size(b.make_shape(*args), b.CTFISS_FP32)
        assert e.value.status == code, args
    with pytest.raises(b.CtfissError) as e:
        b.ctfiss_workspace_size(ok, 7)
    assert e.value.status == b.CTFISS_E_ARG


def test_create_rejects_bad_arguments_before_hip(binding):
    b = binding
    lib = b._lib
    sh = b.make_shape(8, 20, 2, 1, 2, 3, (1, 1))
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(256)  # never dereferenced: every call below fails validation first
    assert lib.ctfiss_create(ctypes.byref(sh), 0, 5, 0, 1e-8, fake, 1 << 20, None, ctypes.byref(ctx)) == b.CTFISS_E_ARG
    assert lib.ctfiss_create(ctypes.byref(sh), 0, 0, 9, 1e-8, fake, 1 << 20, None, ctypes.byref(ctx)) == b.CTFISS_E_ARG
    assert lib.ctfiss_create(ctypes.byref(sh), 0, 0, 0, -1.0, fake, 1 << 20, None, ctypes.byref(ctx)) == b.CTFISS_E_ARG
    assert lib.ctfiss_create(ctypes.byref(sh), 0, 0, 0, 1e-8, None, 1 << 20, None, ctypes.byref(ctx)) == b.CTFISS_E_ARG
    assert lib.ctfiss_create(ctypes.byref(sh), 0, 0, 0, 1e-8, fake, 16, None, ctypes.byref(ctx)) == b.CTFISS_E_WORKSPACE
    assert lib.ctfiss_create(ctypes.byref(sh), 0, 0, 0, 1e-8, ctypes.c_void_p(257), 1 << 20, None,
                             ctypes.byref(ctx)) == b.CTFISS_E_WORKSPACE
    bad = b.make_shape(8, 20, 2, 1, 2, 3, (2, 1))
    assert lib.ctfiss_create(ctypes.byref(bad), 0, 0, 0, 1e-8, fake, 1 << 20, None, ctypes.byref(ctx)) == b.CTFISS_E_SHAPE
    for fn in ("ctfiss_iterate", "ctfiss_destroy", "ctfiss_sync_status"):
        args = {"ctfiss_iterate": (None, 1, None), "ctfiss_destroy": (None,), "ctfiss_sync_status": (None, None)}[fn]
        assert getattr(lib, fn)(*args) == b.CTFISS_E_ARG
    for code in range(-8, 1):
        assert b.ctfiss_status_string(code) != "unknown status"


def test_noalloc_rejects_shapes_beyond_its_scratch_before_hip(binding):
    """ctfiss_separate_noalloc checks the workspace of the shape against its static scratch
    (96 MiB) before any HIP call: the 60 s, Mbar = 64 shape needs ~1.2 GiB."""
    b = binding
    lib = b._lib
    fake = ctypes.c_void_p(256)  # never dereferenced
    big = b.make_shape(2049, 938, 4, 16, 3, 30, (22, 21, 21))
    assert b.ctfiss_workspace_size(big, b.CTFISS_FP32) > (96 << 20)
    st = lib.ctfiss_separate_noalloc(ctypes.byref(big), 0, 0, 0, 1e-8, fake, None, fake, fake, 1, fake, None, None,
                                     None, None, None)
    assert st == b.CTFISS_E_TOO_LARGE
    small = b.make_shape(8, 20, 2, 1, 2, 3, (1, 1))
    assert lib.ctfiss_separate_noalloc(ctypes.byref(small), 0, 0, 0, 1e-8, None, None, fake, fake, 1, fake, None, None,
                                       None, None, None) == b.CTFISS_E_ARG
    assert lib.ctfiss_separate_noalloc(ctypes.byref(small), 0, 0, 0, 1e-8, fake, None, fake, fake, -1, fake, None,
                                       None, None, None, None) == b.CTFISS_E_ARG
    bad = b.make_shape(8, 20, 2, 1, 2, 3, (2, 1))
    assert lib.ctfiss_separate_noalloc(ctypes.byref(bad), 0, 0, 0, 1e-8, fake, None, fake, fake, 1, fake, None, None,
                                       None, None, None) == b.CTFISS_E_SHAPE

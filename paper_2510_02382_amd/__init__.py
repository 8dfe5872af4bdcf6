"""MI355X-native CTF-MNMF-ISS: HIP kernels for gfx950 behind the C ABI of include/ctfiss.h.

The library (libctfiss.so) is built in-tree by paper_2510_02382_amd.build; the
Python side only marshals arguments.  `Separator` and `BatchSeparator` are
imported lazily so that the package can be imported (e.g. to build it) before
the library exists.
"""
import importlib
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctfiss.so")


def __getattr__(name):
    if name in ("Separator", "BatchSeparator"):
        return getattr(importlib.import_module(".separator", __name__), name)
    raise AttributeError(name)

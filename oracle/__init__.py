"""CPU oracle (FP64 NumPy) of CTF-MNMF-ISS and its IP baseline.

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library or its Python binding."""
from . import ctf_iss

__all__ = ["ctf_iss"]

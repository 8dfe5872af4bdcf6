"""Error measures of the parity tests and a recorder of the values they measure.

rel(): relative Frobenius norm of a whole array.
elem_err(): element-wise error scaled per group -- the largest |g - r| within
each group of elements divided by the RMS of the reference over that group,
maximised over the groups.  The groups are the natural units of each output:
W per bin (its Mbar x Mbar entries), B per (source, bin) (its K bases), V per
(source, basis) (its T frames), C per (source, microphone, bin) (its T frames).
A wrong low-energy bin or a wrong boundary frame then fails the check even
where the whole-array norm is dominated by high-energy bins.

Every measured value is kept in RECORDS; when CTFISS_PARITY_LOG names a file,
the test session writes them there as JSON at its end (tests/conftest.py).
"""
from __future__ import annotations

import os

import numpy as np

RECORDS: list[dict] = []

GROUP_AXES = {"W": (1, 2), "B": (2,), "V": (2,), "C": (3,)}


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def elem_err(g, r, key: str) -> float:
    g = np.asarray(g)
    r = np.asarray(r)
    axes = GROUP_AXES[key]
    d = np.abs(g - r).max(axis=axes)
    rms = np.sqrt(np.mean(np.abs(r) ** 2, axis=axes))
    return float((d / np.maximum(rms, 1e-300)).max())


def current_test() -> str:
    return os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0].split("::")[-1]


def record(test: str | None = None, **values) -> None:
    RECORDS.append({"test": test or current_test(),
                    **{k: (float(v) if isinstance(v, (float, np.floating)) else v) for k, v in values.items()}})


def check_outputs(test: str | None, g: dict, r: dict, tol_norm: float, tol_elem: float,
                  keys=("W", "B", "V", "C")) -> None:
    """rel() and elem_err() of each output within its tolerance (values recorded under `test`,
    default the running test's name)."""
    for k in keys:
        rn, re = rel(g[k], r[k]), elem_err(g[k], r[k], k)
        record(test, output=k, rel=rn, elem=re, tol_rel=tol_norm, tol_elem=tol_elem)
        assert rn < tol_norm, (k, "rel", rn)
        assert re < tol_elem, (k, "elem", re)

"""Norms and bars shared by the GPU parity tests.

Every comparison reports, per field, the relative 2-norm ||a - b|| / ||b|| and
the relative max-norm max|a - b| / max|b|; a bar holds only if both are within
it.  Bars: FP64 storage 1e-12, FP32 storage 1e-5 (phi, u and P); the 16-bit
deviation modes carry their own, derived from their quantisation."""
import numpy as np

FIELDS = ("phi", "ux", "uy", "P")
BAR = {"fp64": 1e-12, "fp32": 1e-5}


def rel(a, b):
    n = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / n) if n > 0 else float(np.linalg.norm(a - b))


def relmax(a, b):
    n = np.abs(b).max()
    return float(np.abs(a - b).max() / n) if n > 0 else float(np.abs(a - b).max())


def errors(got, ref, names=FIELDS):
    """{name: (2-norm, max-norm)} for matching sequences of fields."""
    return {n: (rel(a, b), relmax(a, b)) for n, a, b in zip(names, got, ref)}


def fmt(errs):
    return " ".join(f"{k}={v[0]:.2e}/{v[1]:.2e}" for k, v in errs.items())


def check(errs, bar, names=None):
    """Assert both norms of every named field (all by default) within bar."""
    for k in (names or errs):
        e2, emax = errs[k]
        assert e2 <= bar and emax <= bar, (k, e2, emax, bar)

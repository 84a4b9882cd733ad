"""Parity measures shared by the GPU tests.

Two measures, both against the FP64 oracle and both held to the same bar:
  rel      ||x - x_ref||_2 / ||x_ref||_2 over the whole complex vector;
  max_rel  max_i |x_i - x_ref_i| / max_i |x_ref_i|, which a localised error
           (one bad tile or split of a large output) cannot hide under.
"""
import numpy as np

TOL = {"fp32": 1e-4, "bf16": 2e-3, "fp16": 2e-3}
PRECS = ["fp32", "bf16", "fp16"]


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def max_rel(a, b):
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if a.size else 0.0


def check(a, b, tol, what=""):
    """Assert both measures are below tol; return them for printing."""
    e, em = rel(a, b), max_rel(a, b)
    assert e < tol and em < tol, (what, e, em, tol)
    return e, em


def horizon(dev, tol, lookahead=2):
    """Rounding horizon of a CG trajectory from a probe's deviation per
    iterate (dev[k - 1] for iterate k): the last iterate k such that the
    probe stays within tol / 4 at every iterate up to k + lookahead.  The
    lookahead keeps the horizon off the iterates where the trajectory starts
    to depend on rounding: there one rounding pattern can leave it an
    iterate or two before another."""
    n = len(dev)
    first_out = next((j for j in range(n) if dev[j] > tol / 4), n)  # 0-based index of the first iterate beyond
    return n if first_out == n else max(0, first_out - lookahead)


def spread(dev, lookahead=2):
    """A probe's deviation as a bound past the horizon: at iterate k the
    largest deviation up to iterate k + lookahead (the same allowance for a
    trajectory that leaves an iterate or two earlier than the probe's)."""
    dev = np.asarray(dev, dtype=np.float64)
    return np.array([dev[:min(len(dev), k + 1 + lookahead)].max() for k in range(len(dev))])

"""Comparison helpers shared by the GPU parity tests.

`assert_close(x, ref, tol)` checks a result against its reference two ways:
normwise, ||x - ref||_2 <= tol ||ref||_2, and componentwise,
|x_i - ref_i| <= tol max(|ref_i|, rms(ref)) for every entry.  The
componentwise floor at the root-mean-square entry keeps entries that are
near zero from demanding a relative accuracy that no rounding order can give,
while entries at or above the typical size are held to `tol` relative to
themselves (tighter than the normwise bound by up to sqrt(len)).
"""
import numpy as np


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def comp_err(a, b):
    """Largest |a_i - b_i| / max(|b_i|, rms(b))."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    rms = float(np.sqrt(np.mean(b * b)))
    scale = np.maximum(np.abs(b), rms)
    return float(np.max(np.abs(a - b) / scale))


def assert_close(a, b, tol, what=""):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    assert np.all(np.isfinite(a)), f"{what}: non-finite entries"
    r = rel(a, b)
    c = comp_err(a, b)
    assert r <= tol, f"{what}: normwise {r:.3e} > {tol:.1e}"
    assert c <= tol, f"{what}: componentwise {c:.3e} > {tol:.1e}"

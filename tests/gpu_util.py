"""Helpers shared by the GPU parity tests (comparison metrics only)."""
import numpy as np


def rel_err(a, b):
    """max|a-b| / max|b| (global-normalised error of one field)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    s = np.max(np.abs(b))
    if s == 0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - b)) / s)


def assert_close(a, b, rtol, atol_frac, name="", mask=None):
    """|a-b| <= rtol |b| + atol_frac max|b|, element by element (over mask)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if mask is not None:
        a = a[..., mask] if a.shape[-mask.ndim:] == mask.shape else a[mask]
        b = b[..., mask] if b.shape[-mask.ndim:] == mask.shape else b[mask]
    scale = np.max(np.abs(b)) if b.size else 0.0
    bad = np.abs(a - b) > rtol * np.abs(b) + atol_frac * scale
    if np.any(bad):
        i = np.argmax(np.abs(a - b) - rtol * np.abs(b))
        raise AssertionError(f"{name}: {int(bad.sum())} of {bad.size} elements differ; worst "
                             f"a={a.flat[i]!r} b={b.flat[i]!r} (rel_err {rel_err(a, b):.3e})")

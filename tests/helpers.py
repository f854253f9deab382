"""Shared test helpers (input plumbing only; no solver arithmetic)."""
import numpy as np


def rand_orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b)
    n = np.linalg.norm(b)
    return d / n if n > 0 else d


def max_rel(a, b):
    """Element-wise check: max_i |a_i - b_i| / max_i |b_i| (every entry counts,
    unlike the Frobenius ratio of ``rel``)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.size == 0:
        return 0.0
    m = np.max(np.abs(b))
    d = np.max(np.abs(a - b))
    return d / m if m > 0 else d

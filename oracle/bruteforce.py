"""Exhaustive Max-Cut for tiny graphs -- TEST INFRASTRUCTURE ONLY.

Enumerates every partition of n <= 22 vertices (vertex 0 fixed to +1, which a
global flip makes free) and evaluates the Max-Cut objective of Eq. (6),
cut(s) = 1/4 sum_{a,b} A_ab (1 - s_a s_b) with A = -J (Eq. 4), directly.
"""
from __future__ import annotations

import numpy as np


def maxcut(J: np.ndarray, chunk_bits: int = 16):
    """Return (best cut, one optimal spin vector) of the couplings J (dense, symmetric)."""
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    if n > 22:
        raise ValueError("brute force is limited to 22 vertices")
    if n <= 1:
        return 0.0, np.ones(n, dtype=np.int8)
    A = -J
    total = 1 << (n - 1)
    best = -np.inf
    best_s = None
    step = 1 << min(chunk_bits, n - 1)
    bits = np.arange(n - 1, dtype=np.int64)
    for start in range(0, total, step):
        codes = np.arange(start, min(start + step, total), dtype=np.int64)
        rest = 1 - 2 * ((codes[:, None] >> bits[None, :]) & 1)      # +1 / -1
        S = np.concatenate([np.ones((codes.shape[0], 1), dtype=np.int64), rest], axis=1)
        Sf = S.astype(np.float64)
        # sum_{a,b} A_ab (1 - s_a s_b) = sum(A) - s^T A s
        quad = np.einsum("ka,ab,kb->k", Sf, A, Sf)
        cut = 0.25 * (A.sum() - quad)
        k = int(np.argmax(cut))
        if cut[k] > best:
            best = float(cut[k])
            best_s = S[k].astype(np.int8)
    return best, best_s

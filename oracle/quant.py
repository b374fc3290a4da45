"""Software round-to-nearest-even quantizers -- TEST INFRASTRUCTURE ONLY.

Written from the format definitions: IEEE binary16 (10 fraction bits, emin
-14), bfloat16 (7 fraction bits, emin -126) and OCP FP8 E4M3 (3 fraction bits,
emin -6, largest finite 448, no infinities; out-of-range values saturate to
+-448).  Every conversion rounds the FP64 input once, directly to the target.
The per-row FP8 scale is s_i = RNE_f32(max_j |J_ij| / 448) and the stored code
is RNE_e4m3(J_ij / s_i) with the quotient taken in FP64.
"""
from __future__ import annotations

import numpy as np

_FORMATS = {
    # fraction bits, min normal exponent, max finite, saturate on overflow
    "f16": (10, -14, 65504.0, False),
    "bf16": (7, -126, float.fromhex("0x1.fep127"), False),
    "e4m3": (3, -6, 448.0, True),
    "f32": (23, -126, float.fromhex("0x1.fffffep127"), False),
}


def round_to(fmt: str, v) -> np.ndarray:
    """Round FP64 values to the nearest representable value of ``fmt`` (ties to even)."""
    p, emin, vmax, sat = _FORMATS[fmt]
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    m, ex = np.frexp(a)                 # a = m * 2^ex, m in [0.5, 1)
    e = np.maximum(ex - 1, emin)        # unbiased exponent (subnormals share emin)
    quantum = np.ldexp(1.0, (e - p).astype(np.int64))
    k = np.rint(a / quantum)            # exact scaling by a power of two; rint = ties-to-even
    r = k * quantum
    over = r > vmax
    if sat:
        r = np.where(over, vmax, r)
    else:
        r = np.where(over, np.inf, r)
    r = np.where(a == 0, 0.0, r)
    return np.copysign(r, v)


def rowscale_e4m3(J: np.ndarray):
    """Per-row scale (f32) and codes (as their FP64 values) for a dense J."""
    J = np.asarray(J, dtype=np.float64)
    rmax = np.abs(J).max(axis=1)
    scale = round_to("f32", rmax / 448.0)
    safe = np.where(scale > 0, scale, 1.0)
    q = round_to("e4m3", J / safe[:, None])
    q = np.where(scale[:, None] > 0, q, 0.0)
    return scale, q


def e4m3_bits(v) -> np.ndarray:
    """Bit patterns of values already representable in E4M3."""
    v = np.asarray(v, dtype=np.float64)
    sign = np.signbit(v).astype(np.uint8) << 7
    a = np.abs(v)
    out = np.zeros(v.shape, dtype=np.uint8)
    m, ex = np.frexp(a)
    e = ex - 1
    normal = (a >= 2.0 ** -6)
    exp_field = np.where(normal, e + 7, 0)
    frac = np.where(normal, np.rint((a / np.ldexp(1.0, e) - 1.0) * 8), np.rint(a / 2.0 ** -9))
    out = (exp_field.astype(np.int64) << 3) | frac.astype(np.int64)
    out = np.where(a == 0, 0, out)
    return (out.astype(np.uint8) | sign).astype(np.uint8)

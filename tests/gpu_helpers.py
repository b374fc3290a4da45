"""Shared helpers of the GPU tests: workloads to device tensors, GPU graphs, bounds."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2603_25762_amd as qh
from oracle import quant


def device_reads(w):
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    return d


def gpu_graph(w, kind="read_signed", dtype="f32", linkage_k=10, band_limit=0, with_alpha=True):
    d = device_reads(w)
    return qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"],
                          kind=kind, dtype=dtype, alpha=d["alpha"] if with_alpha else None,
                          linkage_k=linkage_k, band_limit=band_limit)


def oracle_graph(w, kind="read_signed", linkage_k=10):
    return oracle.build_graph(w, kind, linkage_k)


def snp_abs_terms(w, linkage_k=10):
    """Per-entry sum of |pair terms| of Eq. (14): the oracle graph of the same reads with
    every allele made concordant with the initial haplotype (all terms then share a sign)."""
    allele = w.init_h1[w.snp].copy()
    M = oracle.encode(w.snp, allele, w.init_h1)
    g = oracle.snp_graph(w.n_snp, w.frag_ptr, w.snp, M, w.phred, w.alpha, linkage_k)
    return np.abs(g.dense())


def step_bounds(J_abs_xabs, x, y, p, dt, c0, a0=1.0, rel=1e-5):
    """Elementwise tolerance of one FP32 step against the FP64 reference."""
    S = np.abs(y) + (abs(a0 - p) * np.abs(x) + c0 * J_abs_xabs) * dt
    tol_y = rel * S
    tol_x = rel * (np.abs(x) + a0 * dt * S)
    return tol_x, tol_y


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def cpu(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


# Unit roundoff of the 16-bit copy of x the dense 16/8-bit product multiplies (binary16 for
# F16 and FP8 tiles, bfloat16 for BF16 tiles), and the absolute error bound below binary16's
# normal range (its subnormal spacing 2^-24, halved).
COPY_UNIT = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
COPY_ABS = {"f16": 2.0 ** -25, "bf16": 0.0}


def far_mask(n, band_limit):
    """Entries of the long-range part of a SNP graph built with ``band_limit``: |i - j| above it."""
    i = np.arange(n)
    return np.abs(i[:, None] - i[None, :]) > band_limit


def step_with_rounded_copy(J, x, y, p, dt, c0, a0=1.0, fmt=None, walls=True, discrete=False, field=None,
                           lr_band=None):
    """The precision form's step as the 16/8-bit kernels compute it, in FP64: the coupling
    product multiplies the copy of x rounded to ``fmt`` (binary16 or bfloat16, round to
    nearest even; dense storage), or, with ``lr_band`` (16-bit SNP storage built with that
    band limit), the long-range entries multiply x rounded to binary16 and the band x itself.
    The update keeps x and y unrounded.  A model of the kernels, kept in the tests: the
    oracle's step (oracle.bsb_step_dense) is the unrounded definition."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if discrete or (fmt is None and lr_band is None):
        return oracle.bsb_step_dense(J, x, y, p, dt, c0, a0, walls=walls, discrete=discrete, field=field)
    J = np.asarray(J, dtype=np.float64)
    if lr_band is not None:
        far = far_mask(J.shape[0], lr_band)
        z = np.where(far, 0.0, J) @ x + np.where(far, J, 0.0) @ quant.round_to("f16", x)
    else:
        z = J @ quant.round_to(fmt, x)
    if field is not None:
        z = z + np.asarray(field, dtype=np.float64)[:, None]
    y2 = y + (-(a0 - p) * x + c0 * z) * dt
    x2 = x + a0 * y2 * dt
    if not walls:
        return x2, y2
    wall = np.abs(x2) > 1.0
    return np.where(wall, np.sign(x2), x2), np.where(wall, 0.0, y2)

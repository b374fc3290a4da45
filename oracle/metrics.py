"""Phasing accuracy metrics (Methods, "Evaluation metrics of haplotype phasing").

TEST INFRASTRUCTURE ONLY.  Haplotypes are allele vectors (0/1); -1 marks an
unphased SNP, which the metrics skip.
"""
from __future__ import annotations

from typing import Optional

import numpy as np


def _blocks(h1: np.ndarray, block: Optional[np.ndarray]):
    h1 = np.asarray(h1)
    if block is None:
        block = np.zeros(h1.shape[0], dtype=np.int64)
    block = np.asarray(block)
    phased = (h1 >= 0) & (block >= 0)
    for b in np.unique(block[phased]):
        idx = np.nonzero(phased & (block == b))[0]
        yield idx


def switch_error(h1, truth, block=None) -> float:
    """Switches between consecutive phased SNPs of a block / (n - 1) pairs."""
    h1 = np.asarray(h1); truth = np.asarray(truth)
    sw = 0
    pairs = 0
    for idx in _blocks(h1, block):
        if idx.shape[0] < 2:
            continue
        rel = h1[idx] == truth[idx]
        sw += int(np.count_nonzero(rel[1:] != rel[:-1]))
        pairs += idx.shape[0] - 1
    return sw / pairs if pairs else 0.0


def switch_count(h1, truth, block=None) -> int:
    h1 = np.asarray(h1); truth = np.asarray(truth)
    sw = 0
    for idx in _blocks(h1, block):
        rel = h1[idx] == truth[idx]
        sw += int(np.count_nonzero(rel[1:] != rel[:-1]))
    return sw


def hamming_error(h1, truth, block=None, literal: bool = True) -> float:
    """Mismatching phased alleles / phased SNPs.

    literal=True compares against ``truth`` as given (the paper's worked example);
    literal=False takes, per block, the better of the two orientations.
    """
    h1 = np.asarray(h1); truth = np.asarray(truth)
    mis = 0
    n = 0
    for idx in _blocks(h1, block):
        m = int(np.count_nonzero(h1[idx] != truth[idx]))
        mis += m if literal else min(m, idx.shape[0] - m)
        n += idx.shape[0]
    return mis / n if n else 0.0


def haplotype_n50(h1, block, pos) -> int:
    """Haplotype N50 (Methods, evaluation metrics): a block is the set of phased SNPs that
    share a block label, its size the genomic span pos[last] - pos[first] + 1 in bp;
    ranked by size, descending, the N50 is the size at which the running sum first
    reaches half the total span.  0 when nothing is phased."""
    pos = np.asarray(pos)
    spans = sorted((int(pos[idx[-1]] - pos[idx[0]] + 1) for idx in _blocks(h1, block)), reverse=True)
    total = sum(spans)
    run = 0
    for s in spans:
        run += s
        if 2 * run >= total:
            return s
    return 0


def phasing_completeness(h1, block=None) -> float:
    """Phased heterozygous sites over all heterozygous sites of the input."""
    h1 = np.asarray(h1)
    n = h1.shape[0]
    phased = sum(idx.shape[0] for idx in _blocks(h1, block))
    return phased / n if n else 0.0


def snp_completeness(h1, n_true: int, block=None) -> float:
    """Phased heterozygous SNPs over the true heterozygous variants of the reference."""
    phased = sum(idx.shape[0] for idx in _blocks(h1, block))
    return phased / n_true if n_true else 0.0

"""Seeded synthetic phasing workloads.

This module only draws inputs: SNP positions, a planted haplotype pair, reads
with their observed alleles and Phred qualities, and the random initial
haplotype assignment.  It holds none of the phasing method's arithmetic (no
encoding, no graph weights, no solver); both the GPU library and the CPU oracle
take its output as their input.
"""
from .workloads import (  # noqa: F401
    Workload, Batch, read_tiny, read_mhc, snp_chrom, snp_porec, batched_blocks,
    snp_small, read_small, by_name, CONFIGS, CHROM_GAP_BP, workload_hash, batch_hash, stratified_subset,
)

"""GPU-vs-oracle parity at the full sizes of the benchmark workloads, in the launch
configurations bench.py times.

Expected values come from tests/golden/*_reference.json, written by
tests/golden/make_reference_cuts.py from the FP64 oracle alone (same seed, replicas and
schedule); each file carries the hash of the synthetic inputs it was made from, checked
first.  Contract: best cut within 0.1 % of the oracle's and equal switch error on the
planted haplotypes; SNP weights (Eqs. 9-14) on sampled rows within 1e-12 of the summed
|pair terms| (the full graphs are too large to compare densely).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2603_25762_amd as qh
import synth
from oracle import metrics
from gpu_helpers import cpu, device_reads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def reference(name):
    return json.load(open(os.path.join(GOLDEN, f"{name}_reference.json")))


def gap(ref, got):
    return (ref - got) / abs(ref)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    qh.load()
    yield
    torch.cuda.synchronize()


def snp_rows_match(g, w, rows):
    """Rows of the GPU's FP64 master against the oracle's Eq. (14) weights: |diff| <= 1e-12 of
    the entry's summed |pair terms| (the oracle graph of the same reads with every allele made
    concordant, whose terms then all share one sign)."""
    go = oracle.build_graph(w, "snp_llr")
    allele = w.init_h1[w.snp].copy()
    Ma = oracle.encode(w.snp, allele, w.init_h1)
    gabs = oracle.snp_graph(w.n_snp, w.frag_ptr, w.snp, Ma, w.phred, w.alpha)
    for u in rows:
        got = cpu(g.export_rows(int(u), int(u) + 1))[0]
        want = np.zeros_like(got)
        bound = np.zeros_like(got)
        a, b = go.row_ptr[u], go.row_ptr[u + 1]
        want[go.col[a:b]] = go.val[a:b]
        a, b = gabs.row_ptr[u], gabs.row_ptr[u + 1]
        bound[gabs.col[a:b]] = np.abs(gabs.val[a:b])
        assert np.all(np.abs(got - want) <= 1e-12 * bound), u
    return go


@pytest.mark.parametrize("name", ["snp_chrom", "snp_porec"])
def test_snp_chromosome_full_size(name):
    """C3 (250,000 SNPs, FP16 band) and C4 (plus 600,000 Pore-C contacts, BF16 band + long-range
    CSR, band limit 64): sampled rows of the weights, then the whole solve (R = 64, 3,000 /
    4,000 steps, autotuned step kernel) and one parity round against the oracle's."""
    ref = reference(name)
    w = synth.snp_chrom() if name == "snp_chrom" else synth.snp_porec()
    assert synth.workload_hash(w) == ref["hash"], "inputs changed: regenerate the reference"
    d = device_reads(w)
    dtype, band = ("f16", 0) if name == "snp_chrom" else ("bf16", 64)
    g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="snp_llr",
                       dtype=dtype, alpha=d["alpha"], band_limit=band)
    inf = g.info()
    assert inf["n"] == ref["n"] and inf["n_comp"] == ref["n_comp"]
    # nonzero count: Eq. (14) sums that cancel leave FP64 residue whose exact zero depends on
    # the order of the additions; a handful of entries may differ in being zero
    assert abs(inf["nnz"] - ref["nnz"]) <= 1e-5 * ref["nnz"]
    rng = np.random.default_rng(5)
    rows = list(rng.choice(inf["n"], 40, replace=False)) + [0, inf["n"] - 1]
    if name == "snp_porec":
        assert inf["longrange_nnz"] > 1_000_000
        deg = np.diff(oracle.build_graph(w, "snp_llr").row_ptr)
        rows += list(np.argsort(deg)[-8:])              # the hub rows with the most contacts
    snp_rows_match(g, w, rows)
    r = qh.bsb_solve(g, ref["replicas"], ref["steps"], dt=ref["dt"], seed=ref["seed"])
    cut = float(cpu(r["best_cut"])[0])
    assert gap(ref["best_cut"], cut) <= 1e-3
    h1, blk = qh.phase(g, r["best_spins"])
    assert metrics.switch_error(cpu(h1), w.truth, cpu(blk)) == ref["switch_error"]
    g.free()


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_read_mhc_full_size(dtype):
    """C2 (8,000 reads, dense BF16 tiles as the benchmark runs it, and FP16; R = 256, 2,000
    steps, autotuned plan)."""
    ref = reference("read_mhc")
    w = synth.read_mhc()
    assert synth.workload_hash(w) == ref["hash"], "inputs changed: regenerate the reference"
    d = device_reads(w)
    g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="read_signed",
                       dtype=dtype)
    assert g.info()["nnz"] == ref["nnz"]
    r = qh.bsb_solve(g, ref["replicas"], ref["steps"], dt=ref["dt"], seed=ref["seed"])
    cut = float(cpu(r["best_cut"])[0])
    assert gap(ref["best_cut"], cut) <= 1e-3
    h1, blk = qh.phase(g, r["best_spins"])
    assert metrics.switch_error(cpu(h1), w.truth, cpu(blk)) == ref["switch_error"]
    g.free()


def test_batched_full_size_subset():
    """C5: all 3,000 blocks (dense FP8 read blocks, BF16 SNP blocks) in one batched solve
    (R = 32, 500 steps, per-step plan replayed from a captured hipGraph, as the benchmark
    runs it); the stratified 5 % subset of blocks the oracle solved: every block's best cut
    within 0.1 % and its switch error equal."""
    ref = reference("batched")
    batch = synth.batched_blocks()
    assert synth.batch_hash(batch) == ref["hash"], "inputs changed: regenerate the reference"
    assert [b["block"] for b in ref["blocks"]] == synth.stratified_subset(batch)
    gs = []
    for i, w in enumerate(batch.blocks):
        d = device_reads(w)
        kind = "read_signed" if i % 2 == 0 else "snp_llr"
        gs.append(qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind=kind,
                                 dtype=w.solve["dtype"], alpha=d["alpha"] if kind == "snp_llr" else None))
    r = qh.bsb_solve_batched(gs, ref["replicas"], ref["steps"], dt=ref["dt"], seed=ref["seed"], use_graph=True)
    bc = cpu(r["best_cut"])
    off = r["vertex_offset"]
    for blk in ref["blocks"]:
        b = blk["block"]
        assert gs[b].info()["nnz"] == blk["nnz"] or blk["kind"] == "snp_llr"
        assert gap(blk["best_cut"], float(bc[b])) <= 1e-3, b
        h1, bl = qh.phase(gs[b], r["best_spins"][int(off[b]):int(off[b + 1])])
        assert metrics.switch_error(cpu(h1), batch.blocks[b].truth, cpu(bl)) == blk["switch_error"], b
    for g in gs:
        g.free()

"""Pins of the oracle's phasing (Eqs. 7-8, 15-17), metrics and quantizers."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import metrics, quant


# ---------------------------------------------------------------- metrics

def test_metrics_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "metrics_example.json")) as f:
        ex = json.load(f)
    h = np.array([int(c) for c in ex["inferred"]])
    t = np.array([int(c) for c in ex["reference"]])
    assert metrics.switch_error(h, t) == ex["switch_error"]
    assert metrics.switch_count(h, t) == ex["switch_count"]
    assert metrics.hamming_error(h, t, literal=True) == ex["hamming_error"]
    assert metrics.hamming_error(h, t, literal=False) == pytest.approx(2 / 5)


def test_metrics_skip_unphased_and_blocks():
    h = np.array([0, 1, -1, 1, 0, 0])
    t = np.array([0, 1, 0, 0, 1, 1])
    blk = np.array([0, 0, 0, 1, 1, 1])
    # block 0 phased {0,1}: no switch; block 1 {3,4,5}: rel F,F,F no switch
    assert metrics.switch_error(h, t, blk) == 0.0
    assert metrics.switch_error(h, t) == pytest.approx(1 / 4)



def test_n50_and_completeness_by_hand():
    """Evaluation metrics (Methods): N50 over block spans, phasing and SNP completeness."""
    pos = np.array([0, 10, 99, 200, 249, 300, 329, 400, 419, 500])
    # blocks: {0,1,2} span 100; {3,4} span 50; {5,6} span 30; {7,8} span 20; SNP 9 unphased
    h1 = np.array([0, 1, 1, 0, 0, 1, 0, 1, 1, -1])
    blk = np.array([0, 0, 0, 1, 1, 2, 2, 3, 3, 4])
    # spans 100, 50, 30, 20 (total 200): the running sum reaches 100 at the first block
    assert metrics.haplotype_n50(h1, blk, pos) == 100
    # spans 40, 30, 20, 10 (total 100): 40 < 50, 70 >= 50
    pos2 = np.array([0, 39, 100, 129, 200, 219, 300, 309])
    assert metrics.haplotype_n50(np.zeros(8, int), np.repeat(np.arange(4), 2), pos2) == 30
    # block labels are arbitrary and -1 marks an unphased SNP (like h1 = -1)
    blk3 = np.array([7, 7, 7, 2, 2, 9, 9, 4, 4, -1])
    assert metrics.haplotype_n50(h1, blk3, pos) == 100
    assert metrics.phasing_completeness(h1, blk) == pytest.approx(0.9)
    assert metrics.snp_completeness(h1, 12, blk) == pytest.approx(9 / 12)
    assert metrics.haplotype_n50(-np.ones(4, int), np.zeros(4, int), np.arange(4)) == 0
    assert metrics.phasing_completeness(np.zeros(0, int)) == 0.0


def test_bench_phasing_report_equals_oracle_metrics():
    """bench.py's own phasing report (switch error, orientation-free Hamming error, phased
    fraction, N50) against the oracle's metrics on random phasings with ragged blocks."""
    import bench
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(1, 400))
        truth = rng.integers(0, 2, n)
        h1 = np.where(rng.random(n) < 0.1, -1, rng.integers(0, 2, n))
        blk = np.sort(rng.integers(-1, max(2, n // 30), n))
        pos = np.cumsum(rng.integers(1, 500, n))
        r = bench.phasing_errors(h1, blk, truth, pos)
        assert r["switch_error"] == pytest.approx(metrics.switch_error(h1, truth, blk), abs=1e-15)
        assert r["hamming_error_min"] == pytest.approx(metrics.hamming_error(h1, truth, blk, literal=False),
                                                       abs=1e-15)
        assert r["phased_fraction"] == pytest.approx(metrics.phasing_completeness(h1, blk), abs=1e-15)
        assert r["haplotype_n50_bp"] == metrics.haplotype_n50(h1, blk, pos)


# ---------------------------------------------------------------- Eqs. (7)-(8) voting

def vote_case(c1p, c1m, c2p, c2m, init=0):
    """One SNP covered by fragments with the given per-subset support counts."""
    frags = [(1, +1)] * c1p + [(1, -1)] * c1m + [(-1, +1)] * c2p + [(-1, -1)] * c2m
    n = len(frags)
    frag_ptr = np.arange(n + 1, dtype=np.int64)
    snp = np.zeros(n, dtype=np.int32)
    M = np.array([m for _, m in frags], dtype=np.int8)
    s = np.array([sf for sf, _ in frags], dtype=np.int8)
    comp = np.zeros(n, dtype=np.int32)
    h1, blk = oracle.phase_vote(1, frag_ptr, snp, M, s, comp, np.array([init], dtype=np.uint8))
    return int(h1[0])


@pytest.mark.parametrize("init", [0, 1])
def test_vote_branches(init):
    H1, H2 = init, 1 - init
    # concordant majorities, S1 has the larger differential: S1 keeps its majority
    assert vote_case(5, 1, 3, 2, init) == H1
    assert vote_case(1, 5, 2, 3, init) == H2
    # concordant, S2 larger: S2 keeps its majority, S1 takes the complement
    assert vote_case(3, 2, 6, 1, init) == H2
    assert vote_case(2, 3, 1, 6, init) == H1
    # concordant with equal differentials: S1 wins
    assert vote_case(4, 1, 3, 0, init) == H1
    # opposing majorities: the +1 subset takes H1
    assert vote_case(4, 1, 0, 3, init) == H1
    assert vote_case(0, 3, 4, 1, init) == H2
    # only one subset has a majority
    assert vote_case(3, 1, 2, 2, init) == H1
    assert vote_case(0, 0, 3, 1, init) == H2
    assert vote_case(1, 1, 1, 3, init) == H1
    # filtered: equal support in both subsets, or no coverage
    assert vote_case(2, 2, 1, 1, init) == -1
    assert vote_case(0, 0, 0, 0, init) == -1


def test_read_phasing_planted_twin_is_exact():
    w = synth.read_tiny(error=0.0)
    g = oracle.build_graph(w, "read_signed")
    r = oracle.solve(g, R=16, steps=1000, dt=0.5, seed=4, integer=True)
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    h1, blk = oracle.phase_vote(w.n_snp, w.frag_ptr, w.snp, M, r["best"], r["comp"], w.init_h1)
    assert metrics.switch_error(h1, w.truth, blk) == 0.0
    assert metrics.hamming_error(h1, w.truth, blk, literal=False) == 0.0


# ---------------------------------------------------------------- Eqs. (15)-(17)

def test_parity_hand():
    comp = np.array([0, 0, 0, 0, 1, 1, -1], dtype=np.int32)
    s = np.array([1, -1, 1, 1, 1, -1, 1], dtype=np.int8)
    init = np.array([0, 0, 1, 1, 0, 1, 0], dtype=np.uint8)
    h1, blk = oracle.phase_parity(comp, 2, s, init)
    # comp 0: S_min = {1} -> SNP 1 swaps; comp 1 tie -> s = -1 swaps (SNP 5)
    assert h1.tolist() == [0, 1, 1, 1, 0, 0, -1]
    assert blk.tolist() == [0, 0, 0, 0, 1, 1, -1]


def test_snp_phasing_planted_twin_is_exact():
    w = synth.snp_small(8, n_snp=600, error=0.0)
    g = oracle.build_graph(w, "snp_llr")
    r = oracle.solve(g, R=32, steps=600, dt=0.5, seed=5)
    h1, blk = oracle.phase_parity(r["comp"], r["n_comp"], r["best"], w.init_h1)
    assert metrics.switch_error(h1, w.truth, blk) == 0.0


def test_flip_crossing_cut_identity():
    """cut_{w'}(t) = cut_w(t*s) - cut_w(s) for the sign-flipped graph of Eq. (15)."""
    w = synth.snp_small(9, n_snp=120)
    g = oracle.build_graph(w, "snp_llr")
    rng = np.random.default_rng(1)
    s = np.where(rng.random(g.n) < 0.5, 1, -1).astype(np.int8)
    g2 = oracle.flip_crossing(g, s)
    comp = np.zeros(g.n, dtype=np.int32)
    for _ in range(5):
        t = np.where(rng.random(g.n) < 0.5, 1, -1).astype(np.int8)
        lhs = oracle.cuts(g2, comp, 1, t).sum()
        rhs = oracle.cuts(g, comp, 1, (t * s).astype(np.int8)).sum() - oracle.cuts(g, comp, 1, s).sum()
        assert lhs == pytest.approx(rhs, abs=1e-9)


# ---------------------------------------------------------------- quantizers

def test_f16_matches_ieee_library_cast():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-5, 5000), rng.normal(0, 3e4, 5000),
                        (np.arange(-2048, 2049) + 0.5), [65504.0, 65519.9, 65520.0, 6e-8, 3e-8, 0.0]])
    got = quant.round_to("f16", v)
    ref = v.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, ref)


def test_bf16_patterns_and_library_cast():
    assert quant.round_to("bf16", 1.0 + 2.0 ** -8) == 1.0                 # tie -> even
    assert quant.round_to("bf16", 1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even
    assert quant.round_to("bf16", 1.0 / 3.0) == float.fromhex("0x1.56p-2")
    rng = np.random.default_rng(1)
    v32 = rng.normal(0, 10, 50000).astype(np.float32).astype(np.float64)   # exact in f32
    ref = torch.from_numpy(v32.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(quant.round_to("bf16", v32), ref)
    # integers up to 256 are exact
    ints = np.arange(-256, 257, dtype=np.float64)
    assert np.array_equal(quant.round_to("bf16", ints), ints)


def test_e4m3_patterns_saturation_and_library_cast():
    r = lambda x: float(quant.round_to("e4m3", x))
    assert r(1.0) == 1.0 and r(448.0) == 448.0 and r(500.0) == 448.0 and r(-1e9) == -448.0
    assert r(2.0 ** -9) == 2.0 ** -9            # smallest subnormal
    assert r(2.0 ** -10) == 0.0                 # tie between 0 and 2^-9 -> even (0)
    assert r(3 * 2.0 ** -10) == 2.0 ** -8       # tie between 1 and 2 quanta -> even
    assert r(17.0) == 16.0 and r(19.0) == 20.0  # ties at spacing 2 -> even mantissa
    assert quant.e4m3_bits(np.array([1.0, 448.0, -2.0 ** -9, 0.5])).tolist() == [0x38, 0x7E, 0x81, 0x30]
    rng = np.random.default_rng(2)
    v = rng.uniform(-440, 440, 40000)
    v32 = v.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(v32.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(quant.round_to("e4m3", v32), ref)


def test_rowscale_e4m3_bounds():
    rng = np.random.default_rng(3)
    J = rng.integers(-45, 46, size=(40, 40)).astype(np.float64)
    scale, q = quant.rowscale_e4m3(J)
    assert np.all(np.abs(q) <= 448.0)
    rel = np.abs(scale[:, None] * q - J) / np.maximum(np.abs(J), 1e-30)
    assert np.all(rel[J != 0] <= 2.0 ** -4 + 1e-6)   # half an ulp at 3 fraction bits


def test_refinement_gauge_identity_and_monotone():
    """Eqs. (15)-(17): the partition implied by the flip counters has, on the original graph,
    exactly the sum of the per-round cuts; every applied round adds a positive cut; the switch
    error does not exceed the single-round parity phasing."""
    w = synth.snp_small(24, n_snp=1500, error=0.0)
    g = oracle.build_graph(w, "snp_llr")
    single = oracle.solve(g, 32, 600, 0.5, seed=1)
    h1s, bs = oracle.phase_parity(single["comp"], single["n_comp"], single["best"], w.init_h1)
    rr = oracle.refine(g, w.init_h1, 32, 600, 0.5, seed=1, max_rounds=15)
    S = np.where(rr["flips"] % 2 == 1, -1, 1).astype(np.int8)
    assert oracle.cuts(g, rr["comp"], rr["n_comp"], S).sum() == pytest.approx(sum(rr["round_cuts"]), rel=1e-12)
    assert all(c > 0 for c in rr["round_cuts"]) and rr["rounds"] >= 1
    assert rr["round_cuts"][0] == pytest.approx(single["best_cut"], rel=1e-12)
    assert metrics.switch_error(rr["h1"], w.truth, rr["block"]) <= metrics.switch_error(h1s, w.truth, bs)
    # the haplotype of round one alone is the single parity round
    r1 = oracle.refine(g, w.init_h1, 32, 600, 0.5, seed=1, max_rounds=1)
    assert np.array_equal(r1["h1"], h1s)

"""Pins of the oracle's encoding and graph construction (Eqs. 1-3, 9-14).

Every expected value here comes from a route other than the oracle's own code:
a dense-matrix identity, exact rational arithmetic, or a structural property of
planted (error-free) reads.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def dense_M(w):
    """Dense fragment x SNP ternary matrix, built independently of the oracle."""
    M = np.zeros((w.n_frag, w.n_snp), dtype=np.int64)
    rows = np.repeat(np.arange(w.n_frag), np.diff(w.frag_ptr))
    M[rows, w.snp] = np.where(w.allele == w.init_h1[w.snp], 1, -1)
    return M


# ---------------------------------------------------------------- Eq. (1)

def test_encode_hand_example():
    # SNP 0: H1 carries allele 0; SNP 1: H1 carries 1; SNP 2: H1 carries 1.
    init_h1 = np.array([0, 1, 1], dtype=np.uint8)
    snp = np.array([0, 1, 2, 0], dtype=np.int32)
    allele = np.array([0, 0, 1, 1], dtype=np.uint8)
    M = oracle.encode(snp, allele, init_h1)
    assert M.tolist() == [1, -1, 1, -1]


# ---------------------------------------------------------------- Eqs. (2)-(3)

@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("kind", ["signed", "conflict"])
def test_read_graph_matches_matrix_identity(seed, kind):
    w = synth.read_small(seed, n_snp=90, n_reads=45, span=(5, 30))
    Md = dense_M(w)
    P = Md @ Md.T                      # agree - disagree per pair
    Q = np.abs(Md) @ np.abs(Md).T      # shared SNPs per pair
    np.fill_diagonal(P, 0)
    np.fill_diagonal(Q, 0)
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    g = oracle.read_graph(w.n_snp, w.frag_ptr, w.snp, M, kind)
    if kind == "signed":
        expect = P
    else:
        expect = -((Q - P) // 2)       # J = -A, A = number of disagreeing shared SNPs
    assert np.array_equal(g.dense(), expect.astype(np.float64))
    # structural pairs are exactly the co-covered pairs
    struct = np.zeros_like(Q, dtype=bool)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    struct[rows, g.col] = True
    assert np.array_equal(struct, Q > 0)


def test_read_graph_planted_twin():
    w = synth.read_small(7, n_snp=120, n_reads=50, span=(10, 40), error=0.0)
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    g = oracle.read_graph(w.n_snp, w.frag_ptr, w.snp, M, "signed")
    Md = np.abs(dense_M(w))
    overlap = Md @ Md.T
    np.fill_diagonal(overlap, 0)
    same = (w.origin[:, None] == w.origin[None, :])
    assert np.array_equal(g.dense(), np.where(same, overlap, -overlap).astype(np.float64))
    gc = oracle.read_graph(w.n_snp, w.frag_ptr, w.snp, M, "conflict")
    assert np.array_equal(-gc.dense(), np.where(same, 0, overlap).astype(np.float64))


# ---------------------------------------------------------------- Eqs. (9)-(14)

def exact_llr(Qu, Qv):
    """log10(P_cis / P_trans) with P_cis, P_trans in exact rationals."""
    qu = 1 - Fraction(1, 10) ** Fraction(Qu, 10) if Qu % 10 == 0 else None
    qv = 1 - Fraction(1, 10) ** Fraction(Qv, 10) if Qv % 10 == 0 else None
    assert qu is not None and qv is not None
    p_cis = qu * qv + (1 - qu) * (1 - qv)
    p_trans = qu * (1 - qv) + (1 - qu) * qv
    return math.log10(p_cis.numerator) - math.log10(p_cis.denominator) - (
        math.log10(p_trans.numerator) - math.log10(p_trans.denominator))


def one_fragment(snps, alleles, quals, init, n_snp, alpha=None):
    frag_ptr = np.array([0, len(snps)], dtype=np.int64)
    snp = np.array(snps, dtype=np.int32)
    allele = np.array(alleles, dtype=np.uint8)
    phred = np.array(quals, dtype=np.uint8)
    init_h1 = np.array(init, dtype=np.uint8)
    M = oracle.encode(snp, allele, init_h1)
    return oracle.snp_weights(n_snp, frag_ptr, snp, M, phred,
                            None if alpha is None else np.array([alpha]), 10), M


def test_snp_graph_three_snp_fragment_exact():
    # one fragment, SNPs 0,1,2 with Q = 20, 30, 10; M = (+1, -1, +1)
    g, M = one_fragment([0, 1, 2], [0, 0, 1], [20, 30, 10], [0, 1, 1], 3)
    assert M.tolist() == [1, -1, 1]
    D = g.dense()
    Q = [20, 30, 10]
    for u in range(3):
        for v in range(3):
            if u == v:
                assert D[u, v] == 0.0
                continue
            sgn = M[u] * M[v]
            expect = -sgn * exact_llr(Q[u], Q[v]) / (3 - 1)
            assert D[u, v] == pytest.approx(expect, rel=1e-13, abs=0)
    # P_cis / P_trans for Q = 10, 20 is 0.892 / 0.108 (hand): q = 0.9, 0.99
    assert -D[0, 2] * 2 * 1 == pytest.approx(math.log10(0.99 * 0.9 + 0.01 * 0.1) - math.log10(0.99 * 0.1 + 0.01 * 0.9), rel=1e-14)
    assert math.isclose(10 ** (-D[0, 2] * 2), 892 / 108, rel_tol=1e-13)


def test_snp_graph_alpha_linear_and_duplicate_doubles():
    init8 = [0, 0, 0, 1, 1, 1, 1, 0]
    g1, _ = one_fragment([1, 3, 4, 6], [0, 1, 1, 0], [20, 40, 30, 10], init8, 8)
    g3, _ = one_fragment([1, 3, 4, 6], [0, 1, 1, 0], [20, 40, 30, 10], init8, 8, alpha=0.3)
    assert np.allclose(g3.dense(), 0.3 * g1.dense(), rtol=1e-15, atol=0)
    # the same fragment twice doubles every weight
    frag_ptr = np.array([0, 4, 8], dtype=np.int64)
    snp = np.array([1, 3, 4, 6] * 2, dtype=np.int32)
    allele = np.array([0, 1, 1, 0] * 2, dtype=np.uint8)
    phred = np.array([20, 40, 30, 10] * 2, dtype=np.uint8)
    init = np.array(init8, dtype=np.uint8)
    M = oracle.encode(snp, allele, init)
    g2 = oracle.snp_weights(8, frag_ptr, snp, M, phred, None, 10)
    assert np.array_equal(g2.dense(), 2.0 * g1.dense())


def test_snp_graph_sign_rule_and_symmetry():
    w = synth.snp_small(11, n_snp=300, error=0.06)
    g = oracle.build_graph(w, "snp_llr")
    D = g.dense()
    assert np.array_equal(D, D.T)
    assert np.all(np.diag(D) == 0)
    # single fragment: sgn(w_uv) = -M_u M_v
    g1, M = one_fragment([0, 2, 5, 7, 9], [0, 1, 1, 0, 1], [7, 15, 40, 25, 30],
                         [0, 0, 0, 0, 1, 1, 1, 1, 0, 0], 10)
    D1 = g1.dense()
    idx = [0, 2, 5, 7, 9]
    for a in range(5):
        for b in range(5):
            if a != b:
                assert np.sign(D1[idx[a], idx[b]]) == -M[a] * M[b]


def test_snp_graph_drops_low_quality_and_counts_kept():
    # Q = 3 observation is dropped: |S| = 2 after dropping, so the weight is not halved
    g, M = one_fragment([0, 1, 2], [0, 0, 0], [20, 3, 20], [0, 0, 0], 3)
    D = g.dense()
    assert D[0, 1] == 0.0 and D[1, 2] == 0.0
    assert D[0, 2] == pytest.approx(-exact_llr(20, 20) / 1, rel=1e-13)


@pytest.mark.parametrize("k", [1, 3, 5, 8, 10])
def test_snp_graph_linkage_depth_pair_count(k):
    n = 12
    snps = list(range(n))
    frag_ptr = np.array([0, n], dtype=np.int64)
    snp = np.array(snps, dtype=np.int32)
    allele = np.zeros(n, dtype=np.uint8)
    phred = np.full(n, 30, dtype=np.uint8)
    init = np.zeros(n, dtype=np.uint8)
    M = oracle.encode(snp, allele, init)
    g = oracle.snp_weights(n, frag_ptr, snp, M, phred, None, k)
    L = (k * (n - 1)) // 10
    expect_pairs = sum(min(L, n - 1 - a) for a in range(n))
    assert g.nnz_struct == 2 * expect_pairs
    D = g.dense()
    for u in range(n):
        for v in range(n):
            if u != v:
                assert (D[u, v] != 0) == (abs(u - v) <= L)


def test_snp_graph_planted_twin_is_frustration_free():
    w = synth.snp_small(5, n_snp=400, error=0.0)
    g = oracle.build_graph(w, "snp_llr")          # Ising J = -w
    t = np.where(w.init_h1 == w.truth, 1, -1)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    nz = g.val != 0
    # the planted frame satisfies every coupling: sgn(J_uv) = t_u t_v
    assert np.all(np.sign(g.val[nz]) == t[rows[nz]] * t[g.col[nz]])
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    wts = oracle.snp_weights(w.n_snp, w.frag_ptr, w.snp, M, w.phred, w.alpha, 10)
    assert np.array_equal(wts.val, -g.val)


def test_components_bfs():
    # two triangles and an isolated vertex
    D = np.zeros((7, 7))
    for a, b in [(0, 1), (1, 2), (0, 2), (4, 5), (5, 6)]:
        D[a, b] = D[b, a] = -1.0
    rows, cols = np.nonzero(D)
    rp = np.zeros(8, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    g = oracle.CSR(7, rp, cols, D[rows, cols])
    comp, nc = oracle.components(g)
    assert nc == 2
    assert comp.tolist() == [0, 0, 0, -1, 1, 1, 1]

"""Pins of the oracle's Ising / Max-Cut, bSB, selection and greedy pass (Eqs. 4-6).

Exact optima come from exhaustive enumeration (<= 16 vertices), from graphs with
a textbook optimum (complete bipartite graphs, rings) and from frustration-free
planted twins; the bSB step is pinned by its J = 0 closed form, a two-spin
system and the wall invariants; SplitMix64 by its published test vector.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import bruteforce


def csr_from_dense(D):
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    mask = D != 0
    np.fill_diagonal(mask, False)
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return oracle.CSR(n, np.cumsum(rp), cols, D[rows, cols])


def random_graph(seed, n, density=0.5, integer=True):
    rng = np.random.default_rng(seed)
    D = np.zeros((n, n))
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < density:
                v = float(rng.integers(-5, 6)) if integer else rng.normal()
                D[a, b] = D[b, a] = v
    return D


# ---------------------------------------------------------------- brute force itself

def test_bruteforce_triangle_and_path():
    # unit antiferromagnetic triangle (A = 1): best cut 2
    J = -np.ones((3, 3)); np.fill_diagonal(J, 0)
    best, s = bruteforce.maxcut(J)
    assert best == 2.0
    # path of 4 with A = 1: all edges cut
    J = np.zeros((4, 4))
    for a in range(3):
        J[a, a + 1] = J[a + 1, a] = -1
    assert bruteforce.maxcut(J)[0] == 3.0


# ---------------------------------------------------------------- Eqs. (4)-(6)

def test_cut_energy_identity_and_flip_invariance():
    D = random_graph(3, 30, 0.3, integer=False)
    g = csr_from_dense(D)
    rng = np.random.default_rng(0)
    s = np.where(rng.random((30, 8)) < 0.5, 1, -1).astype(np.int8)
    comp = np.zeros(30, dtype=np.int32)
    cut = oracle.cuts(g, comp, 1, s)[:, 0]
    E = oracle.energy(g, s)
    A_sum = -D.sum()
    assert np.allclose(cut, 0.25 * A_sum - 0.5 * E, rtol=0, atol=1e-10)
    # explicit pair sum: cut = sum_{a<b, s_a != s_b} A_ab
    for r in range(8):
        direct = sum(-D[a, b] for a in range(30) for b in range(a + 1, 30) if s[a, r] != s[b, r])
        assert cut[r] == pytest.approx(direct, abs=1e-10)
    assert np.array_equal(oracle.cuts(g, comp, 1, -s), oracle.cuts(g, comp, 1, s))


@pytest.mark.parametrize("seed,n,integer", [(1, 10, True), (2, 12, True), (3, 14, True),
                                            (4, 12, False), (5, 14, False), (6, 16, False)])
def test_bsb_greedy_hits_bruteforce_optimum(seed, n, integer):
    D = random_graph(seed, n, 0.6, integer)
    g = csr_from_dense(D)
    opt, _ = bruteforce.maxcut(D)
    r = oracle.solve(g, R=64, steps=1000, dt=0.5, seed=seed, integer=integer)
    assert r["best_cut"] == pytest.approx(opt, abs=1e-9)


@pytest.mark.parametrize("m,n", [(3, 4), (5, 5), (7, 9)])
def test_complete_bipartite_optimum(m, n):
    N = m + n
    D = np.zeros((N, N))
    D[:m, m:] = -1.0
    D[m:, :m] = -1.0
    r = oracle.solve(csr_from_dense(D), R=32, steps=800, dt=0.5, seed=1, integer=True)
    assert r["best_cut"] == m * n


@pytest.mark.parametrize("n", [10, 11, 40, 41])
def test_ring_optimum(n):
    D = np.zeros((n, n))
    for a in range(n):
        b = (a + 1) % n
        D[a, b] = D[b, a] = -1.0
    r = oracle.solve(csr_from_dense(D), R=32, steps=1500, dt=0.5, seed=2, integer=True)
    assert r["best_cut"] == (n if n % 2 == 0 else n - 1)


def test_planted_read_twin_optimum():
    w = synth.read_tiny(error=0.0)
    g = oracle.build_graph(w, "read_signed")
    r = oracle.solve(g, R=16, steps=1000, dt=0.5, seed=3, integer=True)
    # frustration-free: optimum = sum over pairs of max(A_ab, 0), A = -J
    assert r["best_cut"] == np.maximum(-g.val, 0).sum() / 2
    # and the planted partition attains it
    s = np.where(w.origin == 0, 1, -1).astype(np.int8)
    comp, nc = oracle.components(g)
    assert oracle.cuts(g, comp, nc, s).sum() == r["best_cut"]


# ---------------------------------------------------------------- bSB dynamics

def test_bsb_step_closed_form_zero_coupling():
    g = csr_from_dense(np.zeros((2, 2)))
    x = np.array([[0.05, -0.08]], dtype=np.float64).repeat(2, 0).copy()
    y = np.array([[-0.02, 0.01]], dtype=np.float64).repeat(2, 0).copy()
    oracle.bsb_run(g, x, y, np.array([0.3]), dt=0.5, c0_=0.7, a0=1.0)
    # y' = y - (a0 - p) dt x ; x' = x + a0 dt y'
    assert y[0, 0] == pytest.approx(-0.02 - 0.7 * 0.5 * 0.05, abs=1e-16)
    assert x[0, 0] == pytest.approx(0.05 + 0.5 * (-0.0375), abs=1e-16)
    assert x[0, 0] == pytest.approx(0.03125, abs=1e-16)
    assert y[0, 1] == pytest.approx(0.01 + 0.7 * 0.5 * 0.08, abs=1e-16)
    assert x[0, 1] == pytest.approx(-0.08 + 0.5 * 0.038, abs=1e-16)


def test_bsb_step_coupling_and_wall():
    D = np.array([[0.0, 2.0], [2.0, 0.0]])
    g = csr_from_dense(D)
    x = np.array([[0.9], [0.5]])
    y = np.array([[0.5], [0.0]])
    oracle.bsb_run(g, x, y, np.array([1.0]), dt=0.5, c0_=0.25, a0=1.0)
    # vertex 0: y = 0.5 + (0 + 0.25*2*0.5)*0.5 = 0.625 ; x = 0.9 + 0.3125 > 1 -> wall
    assert x[0, 0] == 1.0 and y[0, 0] == 0.0
    # vertex 1: y = 0 + 0.25*2*0.9*0.5 = 0.225 ; x = 0.5 + 0.1125
    assert y[1, 0] == pytest.approx(0.225, abs=1e-16)
    assert x[1, 0] == pytest.approx(0.6125, abs=1e-16)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_two_spin_alignment(sign):
    g = csr_from_dense(np.array([[0.0, sign], [sign, 0.0]]))
    r = oracle.solve(g, R=16, steps=400, dt=0.5, seed=9, greedy_pass=False)
    s = r["spins"]
    assert np.all(s[0] == (s[1] if sign > 0 else -s[1]))


def test_bsb_wall_invariants_and_resume():
    w = synth.read_small(21, n_snp=150, n_reads=40, span=(10, 40))
    g = oracle.build_graph(w, "read_signed")
    c0 = oracle.c0(g)
    pump = oracle.pump_linear(300)
    x, y = oracle.init_state(5, g.n, 8)
    for k in range(300):
        x_prev = x.copy()
        oracle.bsb_run(g, x, y, pump, 0.5, c0, 1.0, k, k + 1)
        assert np.all(np.abs(x) <= 1.0)
        clamped = np.abs(x) == 1.0
        assert np.all(y[clamped] == 0.0)
    xa, ya = oracle.init_state(5, g.n, 8)
    oracle.bsb_run(g, xa, ya, pump, 0.5, c0, 1.0, 0, 300)
    assert np.array_equal(xa, x) and np.array_equal(ya, y)
    xb, yb = oracle.init_state(5, g.n, 8)
    oracle.bsb_run(g, xb, yb, pump, 0.5, c0, 1.0, 0, 170)
    oracle.bsb_run(g, xb, yb, pump, 0.5, c0, 1.0, 170, 300)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)


def test_c0_complete_graph():
    n = 9
    D = -np.ones((n, n)); np.fill_diagonal(D, 0)
    assert oracle.c0(csr_from_dense(D)) == pytest.approx(0.5 / np.sqrt(n), rel=1e-15)


def test_pump_linear_endpoints():
    p = oracle.pump_linear(5)
    assert p.tolist() == [0.0, 0.25, 0.5, 0.75, 1.0]


def test_splitmix64_published_vector(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64_vector.json")) as f:
        ref = json.load(f)
    got = [oracle.splitmix64(ref["seed"], k) for k in range(len(ref["outputs"]))]
    assert got == [int(v) for v in ref["outputs"]]


def test_init_uses_counter_layout():
    x, y = oracle.init_state(77, 5, 3)
    assert np.all(np.abs(x) <= 0.1) and np.all(np.abs(y) <= 0.1)
    for i in range(5):
        for r in range(3):
            c = 2 * (r * 5 + i)
            ux = (oracle.splitmix64(77, c) >> 11) * 2.0 ** -53
            uy = (oracle.splitmix64(77, c + 1) >> 11) * 2.0 ** -53
            assert x[i, r] == 0.2 * ux - 0.1
            assert y[i, r] == 0.2 * uy - 0.1


# ---------------------------------------------------------------- selection, greedy

def test_select_per_component_ties_and_orientation():
    # components: {0,1,2} -> 0, {3,4} -> 1, vertex 5 isolated
    comp = np.array([0, 0, 0, 1, 1, -1], dtype=np.int32)
    s = np.array([[1, -1, 1], [-1, -1, 1], [1, 1, -1], [-1, 1, 1], [1, 1, -1], [-1, 1, -1]],
                 dtype=np.int8)
    cut = np.array([[2.0, 1.0], [5.0, 3.0], [5.0, 3.0]])    # [r, c]
    best, br = oracle.select(comp, 2, s, cut)
    assert br.tolist() == [1, 1]                 # ties go to the lowest replica
    # component 0 from replica 1: (-1,-1,1) oriented so vertex 0 is +1
    assert best[:3].tolist() == [1, 1, -1]
    assert best[3:5].tolist() == [1, 1]          # (1, 1) from replica 1
    assert best[5] == 1


def test_greedy_monotone_and_one_flip_optimal():
    for seed in range(5):
        D = random_graph(100 + seed, 60, 0.15, integer=(seed % 2 == 0))
        g = csr_from_dense(D)
        rng = np.random.default_rng(seed)
        s0 = np.where(rng.random(60) < 0.5, 1, -1).astype(np.int8)
        comp = np.zeros(60, dtype=np.int32)
        c_before = oracle.cuts(g, comp, 1, s0).sum()
        eps = oracle.greedy_eps(g, integer=(seed % 2 == 0))
        s1, rounds = oracle.greedy(g, s0, eps)
        c_after = oracle.cuts(g, comp, 1, s1).sum()
        assert c_after >= c_before
        # gains of every single flip, computed from the dense matrix
        A = -D
        gains = s1 * (A @ s1.astype(np.float64))
        assert gains.max() <= eps + 1e-12
        assert rounds >= 0


def test_greedy_independent_set_rule_hand():
    # path 0-1-2 with A = (1, 1) and all spins equal: gains 1, 2, 1.
    D = np.zeros((3, 3)); D[0, 1] = D[1, 0] = -1; D[1, 2] = D[2, 1] = -1
    g = csr_from_dense(D)
    s, rounds = oracle.greedy(g, np.array([1, 1, 1], dtype=np.int8), 0.0)
    # round 1 flips only the middle vertex (largest gain among neighbours): cut 2 = optimum
    assert s.tolist() == [1, -1, 1] and rounds == 1


def test_dense_step_helper_matches_c_step():
    w = synth.read_small(31, n_snp=100, n_reads=30, span=(10, 30))
    g = oracle.build_graph(w, "read_signed")
    x, y = oracle.init_state(3, g.n, 4)
    x2, y2 = oracle.bsb_step_dense(g.dense(), x, y, 0.37, 0.5, oracle.c0(g), 1.0)
    pump = np.array([0.0, 0.37])
    oracle.bsb_run(g, x, y, pump, 0.5, oracle.c0(g), 1.0, 1, 2)
    assert np.allclose(x2, x, rtol=0, atol=1e-15) and np.allclose(y2, y, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- discrete variant (dSB)

def test_dsb_step_by_hand_and_sign_of_zero():
    """dSB takes sgn(x_j) in the coupling (sgn(0) = +1), the rest of the step unchanged."""
    D = np.array([[0.0, 2.0, -1.0], [2.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    g = csr_from_dense(D)
    x = np.array([[0.3], [0.0], [-0.2]])
    y = np.array([[0.1], [0.0], [0.05]])
    oracle.bsb_run(g, x, y, np.array([0.4]), dt=0.5, c0_=0.5, a0=1.0, discrete=True)
    # vertex 0: z = 2 sgn(0) - sgn(-0.2) = 3 ; y = 0.1 + (-0.6*0.3 + 0.5*3)*0.5 = 0.76 ; x = 0.3 + 0.38
    assert y[0, 0] == pytest.approx(0.76, abs=1e-15) and x[0, 0] == pytest.approx(0.68, abs=1e-15)
    # vertex 1: z = 2 sgn(0.3) = 2 ; y = 0 + (0 + 0.5*2)*0.5 = 0.5 ; x = 0 + 0.25
    assert y[1, 0] == pytest.approx(0.5, abs=1e-15) and x[1, 0] == pytest.approx(0.25, abs=1e-15)
    # vertex 2: z = -sgn(0.3) = -1 ; y = 0.05 + (-0.6*-0.2 - 0.5)*0.5 = -0.14 ; x = -0.2 - 0.07
    assert y[2, 0] == pytest.approx(-0.14, abs=1e-15) and x[2, 0] == pytest.approx(-0.27, abs=1e-15)


def test_dsb_equals_bsb_without_coupling_and_dense_helper():
    g0 = csr_from_dense(np.zeros((3, 3)))
    xa, ya = oracle.init_state(4, 3, 8)
    xb, yb = xa.copy(), ya.copy()
    pump = oracle.pump_linear(50)
    oracle.bsb_run(g0, xa, ya, pump, 0.5, 0.3, 1.0)
    oracle.bsb_run(g0, xb, yb, pump, 0.5, 0.3, 1.0, discrete=True)
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    w = synth.read_small(32, n_snp=100, n_reads=30, span=(10, 30))
    g = oracle.build_graph(w, "read_signed")
    x, y = oracle.init_state(3, g.n, 4)
    x2, y2 = oracle.bsb_step_dense(g.dense(), x, y, 0.37, 0.5, oracle.c0(g), 1.0, discrete=True)
    oracle.bsb_run(g, x, y, np.array([0.0, 0.37]), 0.5, oracle.c0(g), 1.0, 1, 2, discrete=True)
    assert np.allclose(x2, x, rtol=0, atol=1e-15) and np.allclose(y2, y, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed,n,integer", [(1, 10, True), (2, 14, True), (5, 14, False)])
def test_dsb_greedy_hits_bruteforce_optimum(seed, n, integer):
    D = random_graph(seed, n, 0.6, integer)
    g = csr_from_dense(D)
    opt, _ = bruteforce.maxcut(D)
    r = oracle.solve(g, R=64, steps=1000, dt=0.5, seed=seed, integer=integer, discrete=True)
    assert r["best_cut"] == pytest.approx(opt, abs=1e-9)


# ---------------------------------------------------------------- deformation field h

def test_field_step_by_hand_zero_coupling():
    """With J = 0 the field is the whole coupling force: y' = y + (-(a0 - p) x + c0 h) dt."""
    g = csr_from_dense(np.zeros((2, 2)))
    x = np.array([[0.05], [-0.08]])
    y = np.array([[-0.02], [0.01]])
    oracle.bsb_run(g, x, y, np.array([0.3]), dt=0.5, c0_=0.5, a0=1.0, field=np.array([0.4, -1.0]))
    # vertex 0: y = -0.02 + (-0.7*0.05 + 0.5*0.4)*0.5 = 0.0625 ; x = 0.05 + 0.03125
    assert y[0, 0] == pytest.approx(0.0625, abs=1e-16) and x[0, 0] == pytest.approx(0.08125, abs=1e-16)
    # vertex 1: y = 0.01 + (0.7*0.08 - 0.5)*0.5 = -0.212 ; x = -0.08 - 0.106
    assert y[1, 0] == pytest.approx(-0.212, abs=1e-15) and x[1, 0] == pytest.approx(-0.186, abs=1e-15)


@pytest.mark.parametrize("discrete", [False, True])
def test_field_equals_coupling_to_a_clamped_spin(discrete):
    """h_i acts as a coupling J_i,a = h_i to an extra spin held at x_a = +1: stepping the
    graph with that vertex appended (and re-clamped before every step) gives the field
    run bit for bit, its coupling being the last term of every row's sum."""
    rng = np.random.default_rng(7)
    n, R, steps = 24, 8, 60
    D = random_graph(3, n, 0.4, integer=False)
    h = rng.normal(size=n) * 0.8
    h[::5] = 0.0                                   # some vertices without a field
    g = csr_from_dense(D)
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = D
    A[:n, n] = A[n, :n] = h
    ga = csr_from_dense(A)
    pump = oracle.pump_linear(steps)
    c0 = oracle.c0(g)
    x, y = oracle.init_state(9, n, R)
    oracle.bsb_run(g, x, y, pump, 0.5, c0, 1.0, discrete=discrete, field=h)
    xa, ya = oracle.init_state(9, n + 1, R)
    xa[:n], ya[:n] = oracle.init_state(9, n, R)
    for k in range(steps):
        xa[n], ya[n] = 1.0, 0.0
        oracle.bsb_run(ga, xa, ya, pump, 0.5, c0, 1.0, k, k + 1, discrete=discrete)
    assert np.array_equal(x, xa[:n]) and np.array_equal(y, ya[:n])
    # the dense helper's field agrees with the sparse run for one step
    x0, y0 = oracle.init_state(2, n, R)
    x2, y2 = oracle.bsb_step_dense(D, x0, y0, 0.4, 0.5, c0, 1.0, discrete=discrete, field=h)
    oracle.bsb_run(g, x0, y0, np.array([0.0, 0.4]), 0.5, c0, 1.0, 1, 2, discrete=discrete, field=h)
    assert np.allclose(x2, x0, rtol=0, atol=1e-15) and np.allclose(y2, y0, rtol=0, atol=1e-15)


def test_field_zero_and_mirror_symmetry():
    """h = 0 is the plain step; (x, y, h) -> (-x, -y, -h) mirrors the whole trajectory."""
    D = random_graph(5, 30, 0.3, integer=False)
    g = csr_from_dense(D)
    pump = oracle.pump_linear(200)
    xa, ya = oracle.init_state(1, 30, 16)
    xb, yb = xa.copy(), ya.copy()
    oracle.bsb_run(g, xa, ya, pump, 0.5, oracle.c0(g), 1.0)
    oracle.bsb_run(g, xb, yb, pump, 0.5, oracle.c0(g), 1.0, field=np.zeros(30))
    assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
    h = np.random.default_rng(4).normal(size=30)
    xp, yp = oracle.init_state(6, 30, 16)
    xm, ym = -xp, -yp
    oracle.bsb_run(g, xp, yp, pump, 0.5, oracle.c0(g), 1.0, field=h)
    oracle.bsb_run(g, xm, ym, pump, 0.5, oracle.c0(g), 1.0, field=-h)
    assert np.array_equal(xm, -xp) and np.array_equal(ym, -yp)


def test_dominant_field_fixes_the_ground_state():
    """When |h_i| exceeds sum_j |J_ij| the Ising energy -x'Jx/2 - h'x is lowest at
    x = sgn(h) (each spin's field outweighs every coupling), and bSB reaches it in
    every replica."""
    D = random_graph(11, 20, 0.5, integer=False)
    g = csr_from_dense(D)
    rng = np.random.default_rng(12)
    sgn = np.where(rng.random(20) < 0.5, -1.0, 1.0)
    h = sgn * (np.abs(D).sum(axis=1) + 0.5)
    r = oracle.solve(g, 32, 400, 0.5, seed=2, greedy_pass=False, field=h)
    assert np.array_equal(r["spins"], np.repeat(sgn.astype(np.int8)[:, None], 32, axis=1))
    # and by brute force no other spin vector has lower field energy
    n = 12
    Ds, hs = D[:n, :n], h[:n]
    best, arg = None, None
    for m in range(1 << n):
        s = np.array([1.0 if (m >> i) & 1 else -1.0 for i in range(n)])
        e = -0.5 * s @ Ds @ s - hs @ s
        if best is None or e < best:
            best, arg = e, s
    assert np.array_equal(arg, sgn[:n])


def test_deformed_refinement_properties():
    """Adaptive deformation of the refinement: without a negative cut nothing changes; on
    weights gauge-flipped around a good partition (where the one-sided partition is near
    optimal, so rough spins cut negatively) the deformed attempts run, the applied cut
    never drops, and the flip counters still carry exactly the sum of the applied cuts."""
    w = synth.snp_small(24, n_snp=800)
    g = oracle.build_graph(w, "snp_llr")
    plain = oracle.refine(g, w.init_h1, 32, 300, 0.5, seed=1, max_rounds=1)
    deformed = oracle.refine(g, w.init_h1, 32, 300, 0.5, seed=1, max_rounds=1, deform=0.5, deform_tries=3)
    assert plain["round_cuts"][0] > 0 and deformed["deformed"] == 0
    assert np.array_equal(plain["flips"], deformed["flips"]) and plain["round_cuts"] == deformed["round_cuts"]
    # later rounds, whose weights are already near a good partition, do get stuck
    later = oracle.refine(g, w.init_h1, 32, 300, 0.5, seed=1, max_rounds=4, deform=0.5, deform_tries=3)
    g2 = oracle.flip_crossing(g, oracle.solve(g, 16, 600, 0.5, seed=1)["best"])
    a = oracle.refine(g2, w.init_h1, 16, 2, 0.5, seed=3, max_rounds=2, greedy_pass=False)
    b = oracle.refine(g2, w.init_h1, 16, 2, 0.5, seed=3, max_rounds=2, greedy_pass=False, deform=0.5,
                      deform_tries=4)
    assert a["deformed"] == 0 and b["deformed"] >= 1
    assert sum(b["round_cuts"][:1]) >= sum(a["round_cuts"][:1])
    for rr in (a, b, plain, later):
        gg = g if rr is plain or rr is later else g2
        S = np.where(rr["flips"] % 2 == 1, -1, 1).astype(np.int8)
        total = oracle.cuts(gg, rr["comp"], rr["n_comp"], S).sum()
        assert total == pytest.approx(sum(rr["round_cuts"]), rel=1e-12, abs=1e-9)
    # the field of attempt a draws right after the initial state's draws of the round
    n, R = 5, 4
    h = oracle.deformation_field(77, n, R, 2, 3.0)
    k0 = 2 * n * R + n
    u = np.array([(oracle.splitmix64(77, k0 + i) >> 11) * 2.0 ** -53 for i in range(n)])
    assert np.array_equal(h, 3.0 * (2.0 * u - 1.0)) and np.all(np.abs(h) <= 3.0)


def test_eval_every_readouts():
    """Readouts every m steps (the best of many samples over one run).  Pins: the energy of
    every readout is -1/2 s'Js of that readout's signs, which equals W - 2 cut (Eq. 5,
    W = -1/2 sum J) for every replica; one readout after the last step (m = 0, or m at least
    the step count) is the plain solve; more readouts never lower the selected cut of any
    component (the last readout is among them); the merge keeps, per component, the largest
    cut over all readouts, which brute enumeration over (readout, replica) confirms."""
    w = synth.read_tiny()
    g = oracle.build_graph(w, "read_signed")
    comp, nc = oracle.components(g)
    W = -0.5 * float(g.val.sum())
    plain = oracle.solve(g, 16, 300, 0.5, seed=5, integer=True, greedy_pass=False)
    same = oracle.solve(g, 16, 300, 0.5, seed=5, integer=True, greedy_pass=False, eval_every=300)
    assert np.array_equal(plain["best"], same["best"]) and plain["selected_cut"] == same["selected_cut"]
    assert plain["energy"].shape == (1, 16) and same["eval_steps"] == [300]
    ev = oracle.solve(g, 16, 300, 0.5, seed=5, integer=True, greedy_pass=False, eval_every=70)
    assert ev["eval_steps"] == [70, 140, 210, 280, 300] and ev["energy"].shape == (5, 16)
    assert np.array_equal(ev["x"], plain["x"])                     # readouts leave the run alone
    # energies against W - 2 cut, readout by readout
    x, y = oracle.init_state(5, g.n, 16)
    pump = oracle.pump_linear(300)
    k = 0
    best_by_comp = np.full(nc, -np.inf)
    for e, k1 in enumerate(ev["eval_steps"]):
        oracle.bsb_run(g, x, y, pump, 0.5, oracle.c0(g), 1.0, k, k1)
        k = k1
        s = oracle.signs(x)
        cut = oracle.cuts(g, comp, nc, s)
        assert np.allclose(ev["energy"][e], W - 2.0 * cut.sum(axis=1), rtol=0, atol=1e-9)
        best_by_comp = np.maximum(best_by_comp, cut.max(axis=0))
    assert ev["selected_cut"] == pytest.approx(float(best_by_comp.sum()), abs=1e-9)
    assert ev["selected_cut"] >= plain["selected_cut"]
    got = oracle.cuts(g, comp, nc, ev["best"])[0]
    assert np.allclose(got, best_by_comp, atol=1e-9)
    # orientation: the lowest vertex of every component reads +1
    for c in range(nc):
        assert ev["best"][np.nonzero(comp == c)[0][0]] == 1


def test_merge_best_ties_go_to_the_earlier_readout():
    """Two readouts with equal cuts: the first one's spins are kept (hand case on a
    two-component graph)."""
    D = np.zeros((4, 4))
    D[0, 1] = D[1, 0] = -1.0          # J = -1: the cut of edge (0, 1) is 1 when split
    D[2, 3] = D[3, 2] = -2.0
    g = csr_from_dense(D)
    comp, nc = oracle.components(g)
    s1 = np.array([[1], [-1], [1], [1]], dtype=np.int8)     # comp 0 cut 1, comp 1 cut 0
    s2 = np.array([[-1], [1], [1], [-1]], dtype=np.int8)    # comp 0 cut 1 (mirror), comp 1 cut 2
    best, bc, br = oracle.merge_best(g, comp, nc, [s1, s2])
    assert list(bc) == [1.0, 2.0]
    assert list(best) == [1, -1, 1, -1]

"""GPU-vs-oracle parity of the gfx950 library, called through its C ABI.

Every expected value comes from ``oracle/`` (or the paper): graph weights
(bit-exact for integer kinds, <= 1e-12 of the summed |terms| for the SNP
log-likelihood weights), stored number formats (bit-exact against the oracle's
software rounding), one bSB step (<= 1e-5 of the step's own magnitude), the
FP64 readout (exact for integer weights), phasing (exact), and the final best
cut of a whole solve (<= 0.1 % below the FP64 oracle, equal switch error).
"""
import ctypes
import json

import numpy as np
import pytest
import torch

import oracle
import paper_2603_25762_amd as qh
import synth
from oracle import metrics, quant
from gpu_helpers import (COPY_ABS, COPY_UNIT, cpu, device_reads, f32, far_mask, gpu_graph, oracle_graph,
                         snp_abs_terms, step_bounds, step_with_rounded_copy)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    qh.load()
    yield
    torch.cuda.synchronize()


FMT = {"f32": None, "f16": "f16", "bf16": "bf16", "fp8": "f16"}


def stored_J(J, dtype):
    if dtype == "f32":
        return quant.round_to("f32", J)
    if dtype == "fp8":
        scale, q = quant.rowscale_e4m3(J)
        return scale[:, None] * q
    return quant.round_to(dtype, J)


# ----------------------------------------------------------------------------- graphs

READ_CASES = {
    "tiny": lambda: synth.read_tiny(),
    "ragged300": lambda: synth.read_small(5, n_snp=400, n_reads=300, span=(10, 60)),
    "sparse_many_comps": lambda: synth.read_small(6, n_snp=2000, n_reads=130, span=(3, 12)),
    # reads plus Pore-C contact fragments, which the read-based method merges unweighted
    "porec_merged": lambda: synth.snp_porec(43, n_snp=600, n_edges=500, zipf_s=1.0),
}


@pytest.mark.parametrize("kind", ["read_signed", "read_conflict"])
@pytest.mark.parametrize("case", list(READ_CASES))
def test_read_graph_bit_exact(kind, case):
    w = READ_CASES[case]()
    g = gpu_graph(w, kind)
    go = oracle_graph(w, kind)
    info = g.info()
    assert info["n"] == go.n and info["integer_weights"] == 1
    assert np.array_equal(cpu(g.export_rows(0, go.n)), go.dense())
    comp, nc = oracle.components(go)
    assert info["n_comp"] == nc
    assert np.array_equal(cpu(g.components()), comp)
    assert info["nnz"] == go.nnz
    assert info["c0_auto"] == pytest.approx(oracle.c0(go), rel=1e-15)
    if case == "porec_merged":
        # Pore-C fragments join the read graph without their down-weighting factor
        assert np.any(w.alpha != 1.0)
        g1 = gpu_graph(w, kind, with_alpha=False)
        assert torch.equal(g1.export_rows(0, go.n), g.export_rows(0, go.n))


def _oracle_read_row(w, kind, p):
    """Row p of the oracle's read graph from the oracle run on read p and the reads sharing a
    SNP with it (an entry (p, q) depends on reads p and q alone), mapped back to all reads."""
    fp, snp = w.frag_ptr, w.snp
    owner = np.repeat(np.arange(len(fp) - 1), np.diff(fp))
    qs = np.unique(owner[np.isin(snp, snp[fp[p]:fp[p + 1]])])
    lens = np.diff(fp)[qs]
    sub_fp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    take = np.concatenate([np.arange(fp[q], fp[q + 1]) for q in qs])
    M = oracle.encode(snp[take], w.allele[take], w.init_h1)
    go = oracle.read_graph(w.n_snp, sub_fp, snp[take], M, "signed" if kind == "read_signed" else "conflict")
    i = int(np.searchsorted(qs, p))
    row = np.zeros(len(fp) - 1)
    b, e = go.row_ptr[i], go.row_ptr[i + 1]
    row[qs[go.col[b:e]]] = go.val[b:e]
    return row


@pytest.mark.parametrize("n_reads,kind", [(20000, "read_signed"), (40000, "read_conflict")])
def test_read_graph_large_fragment_counts(n_reads, kind):
    """Eqs. (2)-(3) past the row kernel's small-LDS case: 20,000 reads need 80 KB of LDS per
    row (the large-LDS launch), 40,000 go past its limit to the per-SNP kernel with global
    atomics.  Sampled rows of the FP64 master equal the oracle's bit for bit (each from the
    oracle on the reads that share a SNP with the row's read); at 20,000 reads the whole
    oracle graph also gives the nonzero count and the components."""
    w = synth.read_small(61, n_snp=4000, n_reads=n_reads, span=(2, 6))
    g = gpu_graph(w, kind)
    n = g.info()["n"]
    assert n == n_reads and g.info()["integer_weights"] == 1
    rng = np.random.default_rng(5)
    for r in sorted({0, 1, n // 3, n // 2, n - 2, n - 1, *rng.integers(0, n, 24).tolist()}):
        assert np.array_equal(cpu(g.export_rows(r, r + 1))[0], _oracle_read_row(w, kind, r)), r
    if n_reads <= 20000:
        go = oracle_graph(w, kind)
        assert g.info()["nnz"] == go.nnz
        comp, nc = oracle.components(go)
        assert g.info()["n_comp"] == nc
        assert np.array_equal(cpu(g.components()), comp)
    g.free()


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16", "fp8"])
def test_dense_stored_values_bit_exact(dtype):
    w = synth.read_small(9, n_snp=300, n_reads=200, span=(20, 60))
    g = gpu_graph(w, "read_signed", dtype)
    J = oracle_graph(w).dense()
    S = cpu(g.export_rows(0, g.info()["n"], stored=True))
    assert np.array_equal(S, stored_J(J, dtype))
    tiles = g.info()["dense_tiles"]
    assert 0 < tiles <= 4 * 4


@pytest.fixture(scope="module")
def mhc():
    w = synth.read_mhc()
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    W, _ = oracle.read_graph_dense(w.n_snp, w.frag_ptr, w.snp, M, "signed")
    return w, W


def test_read_graph_mhc_scale_sampled_rows(mhc):
    """Full MHC-scale read graph (8,000 reads): sampled rows, master and FP16 copy."""
    w, W = mhc
    g = gpu_graph(w, "read_signed", "f16")
    n = g.info()["n"]
    assert n == W.shape[0]
    rows = sorted(set([0, 1, 63, 64, 65, n // 2, n - 65, n - 64, n - 2, n - 1] +
                      list(np.random.default_rng(0).integers(0, n, 40))))
    for r in rows:
        assert np.array_equal(cpu(g.export_rows(r, r + 1))[0], W[r].astype(np.float64)), r
        assert np.array_equal(cpu(g.export_rows(r, r + 1, stored=True))[0],
                              quant.round_to("f16", W[r].astype(np.float64))), r
    assert g.info()["nnz"] == int(np.count_nonzero(W))


SNP_CASES = {
    "snp2000": dict(make=lambda: synth.snp_small(3, n_snp=2000), k=10, band=0),
    "snp2000_k5": dict(make=lambda: synth.snp_small(4, n_snp=2000), k=5, band=0),
    "snp_q_low": dict(make=lambda: synth.snp_small(12, n_snp=800, q=(2, 12)), k=10, band=0),
    "porec3000": dict(make=lambda: synth.snp_porec(41, n_snp=3000, n_edges=3000, zipf_s=1.0), k=10,
                      band=100),
    # eight fragments of 500-1,336 SNPs: longer than the builder's per-wave LDS staging
    "snp_long_reads": dict(make=lambda: synth.snp_small(13, n_snp=1500, coverage=4.0, read_mean=80000.0,
                                                        gap_mean=100.0), k=2, band=0),
    "snp_long_reads_band": dict(make=lambda: synth.snp_small(13, n_snp=1500, coverage=4.0, read_mean=80000.0,
                                                             gap_mean=100.0), k=2, band=50),
}


@pytest.mark.parametrize("case", list(SNP_CASES))
def test_snp_graph_normwise(case):
    c = SNP_CASES[case]
    w = c["make"]()
    g = gpu_graph(w, "snp_llr", "f32", linkage_k=c["k"], band_limit=c["band"])
    go = oracle_graph(w, "snp_llr", c["k"])
    D = cpu(g.export_rows(0, go.n))
    T = snp_abs_terms(w, c["k"])
    assert np.all(np.abs(D - go.dense()) <= 1e-12 * T)
    comp, nc = oracle.components(go)
    assert g.info()["n_comp"] == nc
    assert np.array_equal(cpu(g.components()), comp)
    if c["band"]:
        assert g.info()["longrange_nnz"] > 0


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_skyline_stored_values_bit_exact(dtype):
    w = synth.snp_porec(42, n_snp=1500, n_edges=1500, zipf_s=1.0)
    g = gpu_graph(w, "snp_llr", dtype, band_limit=100)
    S = cpu(g.export_rows(0, g.info()["n"], stored=True))
    J = oracle_graph(w, "snp_llr").dense()
    tol = 1e-12 * snp_abs_terms(w)
    lo, hi = quant.round_to(dtype, J - tol), quant.round_to(dtype, J + tol)
    if dtype == "bf16":
        # BF16 storage flushes magnitudes below 2^(E - 31), E = exponent of the largest weight
        thr = 2.0 ** (np.floor(np.log2(np.abs(J).max())) - 31)
        lo = np.where(np.abs(J) + tol < thr, 0.0, lo)
        hi = np.where(np.abs(J) - tol < thr, np.where(np.abs(J) + tol < thr, 0.0, hi), hi)
        maybe = (np.abs(J) - tol < thr) & (np.abs(J) + tol >= thr)
        assert np.all(np.where(maybe, (S == 0) | (S == lo) | (S == hi), True))
        lo = np.where(maybe, S, lo)
        hi = np.where(maybe, S, hi)
    sure = lo == hi          # the master's last-bit freedom cannot move the rounding
    assert sure.mean() > 0.999
    assert np.array_equal(S[sure], lo[sure])
    assert np.all((S[~sure] == lo[~sure]) | (S[~sure] == hi[~sure]))


# ----------------------------------------------------------------------------- one step

def _one_step_case(g, J, dtype, R, rng_seed, product_format, steps=100, k=37, plan=0, discrete=False,
                   field=False, lr_band=None):
    n = J.shape[0]
    rng = np.random.default_rng(rng_seed)
    x0 = f32(rng.uniform(-1.0, 1.0, (n, R)))
    y0 = f32(rng.uniform(-0.6, 0.6, (n, R)))
    # deformation field: a few units of the typical coupling sum, zero on some rows
    h = f32(rng.normal(0.0, 1.0, n) * max(1.0, float(np.abs(J).sum(axis=1).mean()))) if field else None
    if field:
        h[::7] = 0.0
    pump = np.linspace(0.0, 1.0, steps).astype(np.float32)
    c0 = 0.4 / max(1.0, float(np.sqrt((J ** 2).sum() / max(n - 1, 1))))
    c0 = float(np.float32(c0))
    p = float(pump[k])
    dt = 0.5
    x = torch.tensor(x0, dtype=torch.float32, device="cuda").contiguous()
    y = torch.tensor(y0, dtype=torch.float32, device="cuda").contiguous()
    qh.bsb_solve(g, R, steps, dt=dt, c0=c0, pump=torch.tensor(pump, device="cuda"), init=False,
                 x=x, y=y, step_begin=k, step_end=k + 1, readout=False, plan=plan, discrete=discrete,
                 field=None if h is None else torch.tensor(h, dtype=torch.float32, device="cuda"))
    xg, yg = cpu(x).astype(np.float64), cpu(y).astype(np.float64)
    xu, yu = step_with_rounded_copy(J, x0, y0, p, dt, c0, 1.0, product_format, walls=False, discrete=discrete,
                                    field=h, lr_band=lr_band)
    xo, yo = step_with_rounded_copy(J, x0, y0, p, dt, c0, 1.0, product_format, walls=True, discrete=discrete,
                                    field=h, lr_band=lr_band)
    if discrete:
        xq = np.ones_like(x0)
    else:
        xq = x0 if product_format is None else quant.round_to(product_format, x0)
    mag = np.abs(J) @ np.abs(xq)
    if h is not None:
        mag = mag + np.abs(h)[:, None]
    tol_x, tol_y = step_bounds(mag, x0, y0, p, dt, c0)
    ambiguous = np.abs(np.abs(xu) - 1.0) <= tol_x
    ok = ~ambiguous
    assert ok.mean() > 0.9
    assert np.all(np.abs(xg - xo)[ok] <= tol_x[ok])
    assert np.all(np.abs(yg - yo)[ok] <= tol_y[ok])
    assert np.all(np.abs(xg) <= 1.0)
    assert np.all(yg[np.abs(xg) == 1.0][~ambiguous[np.abs(xg) == 1.0]] == 0.0)


@pytest.mark.parametrize("plan", [1, 2, 0])       # per-step kernel; persistent kernel; autotuned
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16", "fp8"])
@pytest.mark.parametrize("R", [16, 32, 64, 128])
def test_dense_one_step(dtype, R, plan):
    if plan == 2 and dtype == "f32":
        pytest.skip("the persistent plan is offered for 16- and 8-bit dense storage")
    w = synth.read_small(13, n_snp=300, n_reads=150, span=(20, 60))     # 3 row tiles, ragged tail
    g = gpu_graph(w, "read_signed", dtype)
    J = stored_J(oracle_graph(w).dense(), dtype)
    _one_step_case(g, J, dtype, R, 100 + R, FMT[dtype], plan=plan)


@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("dtype", ["f16", "bf16", "fp8"])
def test_dense_one_step_against_unrounded_oracle(dtype, plan):
    """The 16-bit copy of x that the 16/8-bit dense products multiply, bounded against the
    oracle's unrounded step (stored J, FP64, x itself in the product): rounding x_j to the
    copy's format moves it by at most u |x_j| + a (u = 2^-11 for binary16, used by F16 and FP8
    tiles; 2^-8 for bfloat16; a = 2^-25 below binary16's normal range), so the coupling sum
    moves by at most sum_j |J_ij| (u |x_j| + a), y by c0 dt times that and x by a0 dt times
    y's bound, on top of the FP32 step tolerance."""
    w = synth.read_small(13, n_snp=300, n_reads=150, span=(20, 60))
    g = gpu_graph(w, "read_signed", dtype)
    J = stored_J(oracle_graph(w).dense(), dtype)
    n, R, k, steps, dt = J.shape[0], 64, 37, 100, 0.5
    fmt = FMT[dtype]
    rng = np.random.default_rng(321)
    x0 = f32(rng.uniform(-1.0, 1.0, (n, R)))
    y0 = f32(rng.uniform(-0.6, 0.6, (n, R)))
    pump = np.linspace(0.0, 1.0, steps).astype(np.float32)
    c0 = float(np.float32(0.4 / max(1.0, float(np.sqrt((J ** 2).sum() / (n - 1))))))
    p = float(pump[k])
    x = torch.tensor(x0, dtype=torch.float32, device="cuda").contiguous()
    y = torch.tensor(y0, dtype=torch.float32, device="cuda").contiguous()
    qh.bsb_solve(g, R, steps, dt=dt, c0=c0, pump=torch.tensor(pump, device="cuda"), init=False, x=x, y=y,
                 step_begin=k, step_end=k + 1, readout=False, plan=plan)
    xg, yg = cpu(x).astype(np.float64), cpu(y).astype(np.float64)
    xu, yu = oracle.bsb_step_dense(J, x0, y0, p, dt, c0, 1.0, walls=False)
    xo, yo = oracle.bsb_step_dense(J, x0, y0, p, dt, c0, 1.0, walls=True)
    tol_x, tol_y = step_bounds(np.abs(J) @ np.abs(x0), x0, y0, p, dt, c0)
    copy = c0 * dt * (np.abs(J) @ (COPY_UNIT[fmt] * np.abs(x0) + COPY_ABS[fmt]))
    tol_y = tol_y + copy
    tol_x = tol_x + dt * copy
    ok = np.abs(np.abs(xu) - 1.0) > tol_x        # entries not within the tolerance of a wall
    assert ok.mean() > 0.9
    assert np.all(np.abs(yg - yo)[ok] <= tol_y[ok])
    assert np.all(np.abs(xg - xo)[ok] <= tol_x[ok])
    # the bound is not vacuous: the copy's effect is visible and of the size it predicts
    dev = np.abs(yg - yo)[ok]
    assert dev.max() > 1e-3 * copy[ok].max()


@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("dtype", ["f32", "f16", "fp8"])
@pytest.mark.parametrize("R", [32, 64])
def test_dense_one_step_discrete(dtype, R, plan):
    """Discrete variant: the coupling takes sgn(x_j) (sgn(0) = +1), on every dense path."""
    if plan == 2 and dtype == "f32":
        pytest.skip("the persistent plan is offered for 16- and 8-bit dense storage")
    w = synth.read_small(13, n_snp=300, n_reads=150, span=(20, 60))
    g = gpu_graph(w, "read_signed", dtype)
    J = stored_J(oracle_graph(w).dense(), dtype)
    _one_step_case(g, J, dtype, R, 700 + R, None, plan=plan, discrete=True)


@pytest.mark.parametrize("plan", [3, 4, 5])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_skyline_one_step_discrete(dtype, plan):
    w = synth.snp_porec(43, n_snp=2500, n_edges=4000, zipf_s=1.0)
    g = gpu_graph(w, "snp_llr", dtype, band_limit=100)
    assert g.info()["longrange_nnz"] > 0
    J = stored_J(oracle_graph(w, "snp_llr").dense(), dtype)
    _one_step_case(g, J, dtype, 64, 800, None, plan=plan, discrete=True)


@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16", "fp8"])
def test_dense_one_step_field(dtype, plan):
    """Deformation field h on the dense paths: y' = y + (-(a0 - p) x + c0 (J x + h)) dt."""
    if plan == 2 and dtype == "f32":
        pytest.skip("the persistent plan is offered for 16- and 8-bit dense storage")
    w = synth.read_small(13, n_snp=300, n_reads=150, span=(20, 60))
    g = gpu_graph(w, "read_signed", dtype)
    J = stored_J(oracle_graph(w).dense(), dtype)
    _one_step_case(g, J, dtype, 64, 900, FMT[dtype], plan=plan, field=True)
    _one_step_case(g, J, dtype, 32, 901, None, plan=plan, discrete=True, field=True)


@pytest.mark.parametrize("plan", [3, 4, 5])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_skyline_one_step_field(dtype, plan):
    """The field on the SNP step kernels, with long-range rows (chunk partials) present (16-bit
    storage: the long-range entries multiply the binary16 copy of x)."""
    w = synth.snp_porec(43, n_snp=2500, n_edges=4000, zipf_s=1.0)
    g = gpu_graph(w, "snp_llr", dtype, band_limit=100)
    assert g.info()["longrange_nnz"] > 0
    J = stored_J(oracle_graph(w, "snp_llr").dense(), dtype)
    _one_step_case(g, J, dtype, 64, 902, None, plan=plan, field=True, lr_band=None if dtype == "f32" else 100)


def test_field_solves_match_oracle_plans_and_batches():
    """Whole solves under a field: the oracle's cut within 0.1 %; h = 0 is the plain solve
    bit for bit; every dense plan, the band kernels and the batched plans agree bit for
    bit with the per-step solve of each graph."""
    rng = np.random.default_rng(5)
    w = synth.read_tiny()
    g = gpu_graph(w, "read_signed", "f16")
    go = oracle_graph(w)
    n = g.info()["n"]
    h = f32(rng.normal(0.0, 2.0, n))
    ht = torch.tensor(h, dtype=torch.float32, device="cuda")
    ro = oracle.solve(go, 16, 1000, 0.5, seed=11, integer=True, field=h)
    rg = qh.bsb_solve(g, 16, 1000, seed=11, field=ht)
    assert _gap(ro["best_cut"], float(cpu(rg["best_cut"])[0])) <= 1e-3
    # h = 0 is no field
    for gg, plan in ((g, 1), (gpu_graph(synth.snp_small(61, n_snp=400), "snp_llr", "bf16"), 4)):
        m = gg.info()["n"]
        xa = torch.empty((m, 32), dtype=torch.float32, device="cuda")
        xb = torch.empty_like(xa)
        qh.bsb_solve(gg, 32, 200, seed=3, x=xa, readout=False, plan=plan)
        qh.bsb_solve(gg, 32, 200, seed=3, x=xb, readout=False, plan=plan,
                     field=torch.zeros(m, dtype=torch.float32, device="cuda"))
        assert torch.equal(xa, xb)
    # dense plans: per-step, persistent (both synchronisations), captured graph
    wm = synth.read_mhc(seed=78, n_snp=1500, n_reads=1000, region=500_000)
    gm = gpu_graph(wm, "read_signed", "f16")
    nm = gm.info()["n"]
    hm = torch.tensor(f32(rng.normal(0.0, 3.0, nm)), dtype=torch.float32, device="cuda")
    outs = []
    for plan, sync, ug in ((1, 0, False), (2, 1, False), (2, 2, False), (1, 0, True)):
        x = torch.empty((nm, 64), dtype=torch.float32, device="cuda")
        y = torch.empty((nm, 64), dtype=torch.float32, device="cuda")
        r = qh.bsb_solve(gm, 64, 300, seed=31, x=x, y=y, plan=plan, persistent_sync=sync, use_graph=ug, field=hm)
        outs.append((x, y, r))
    x0 = torch.empty((nm, 64), dtype=torch.float32, device="cuda")
    qh.bsb_solve(gm, 64, 300, seed=31, x=x0, plan=1)
    assert not torch.equal(x0, outs[0][0])            # the field changes the run
    for o in outs[1:]:
        assert torch.equal(outs[0][0], o[0]) and torch.equal(outs[0][1], o[1])
        assert torch.equal(outs[0][2]["best_cut"], o[2]["best_cut"])
    # SNP band kernels: rows = band FMA bit for bit, band MFMA to rounding
    wp = synth.snp_porec(43, n_snp=2500, n_edges=4000, zipf_s=1.0)
    gp = gpu_graph(wp, "snp_llr", "f32", band_limit=100)
    npv = gp.info()["n"]
    hp = torch.tensor(f32(rng.normal(0.0, 1.0, npv)), dtype=torch.float32, device="cuda")
    xs = {}
    for plan in (3, 4, 5):
        xs[plan] = torch.empty((npv, 64), dtype=torch.float32, device="cuda")
        qh.bsb_solve(gp, 64, 200, seed=4, x=xs[plan], readout=False, plan=plan, field=hp)
    assert torch.equal(xs[3], xs[4])
    assert float((xs[3] - xs[5]).abs().max()) <= 1e-2
    # batched: packed field, each block equal to its single solve
    blocks = [synth.read_small(50, n_snp=200, n_reads=40), synth.snp_small(60, n_snp=350), w]
    kinds = ["read_signed", "snp_llr", "read_signed"]
    gs = [gpu_graph(b, k, d) for b, k, d in zip(blocks, kinds, ["fp8", "bf16", "f16"])]
    ns = [gg.info()["n"] for gg in gs]
    hb = torch.tensor(f32(rng.normal(0.0, 2.0, sum(ns))), dtype=torch.float32, device="cuda")
    for plan in (1, 2):
        rb = qh.bsb_solve_batched(gs, 32, 300, seed=9, return_state=True, plan=plan, field=hb)
        off = rb["vertex_offset"]
        for b, gg in enumerate(gs):
            lo, hi = int(off[b]), int(off[b + 1])
            xs1 = torch.empty(ns[b], 32, dtype=torch.float32, device="cuda")
            rs = qh.bsb_solve(gg, 32, 300, seed=9, plan=1, x=xs1, field=hb[lo:hi].contiguous())
            assert torch.equal(rb["x"][lo * 32:hi * 32], xs1.reshape(-1)), (plan, b)
            assert torch.equal(rb["best_cut"][b:b + 1], rs["best_cut"]), (plan, b)
    with pytest.raises(ValueError):
        qh.bsb_solve(g, 16, 10, field=ht[:-1])
    with pytest.raises(TypeError):
        qh.bsb_solve(g, 16, 10, field=ht.double())


def test_refine_deformation_matches_oracle():
    """Adaptive deformation in the library's refinement equals the oracle's: on weights
    gauge-flipped around a good partition, rough two-step rounds (no greedy pass) cut
    negatively, so deformed re-solves run; the number run, the rounds, the applied cuts
    and the flip counters agree, and the weights are restored."""
    w = synth.snp_small(24, n_snp=800)
    go = oracle_graph(w, "snp_llr")
    s0 = oracle.solve(go, 16, 600, 0.5, seed=1)["best"]
    g = gpu_graph(w, "snp_llr", "f32")
    n = g.info()["n"]
    qh.flip_crossing(g, torch.tensor(s0, dtype=torch.int8, device="cuda"))
    g2 = oracle.flip_crossing(go, s0)
    master = cpu(g.export_rows(0, n))
    ro = oracle.refine(g2, w.init_h1, 16, 2, 0.5, seed=3, max_rounds=3, greedy_pass=False, deform=0.5,
                       deform_tries=4)
    rr = qh.refine(g, 16, 2, seed=3, max_rounds=3, greedy=False, deform=0.5, deform_tries=4)
    assert np.array_equal(cpu(g.export_rows(0, n)), master)
    assert ro["deformed"] >= 1
    assert rr["deformed"] == ro["deformed"] and rr["rounds"] == ro["rounds"]
    assert np.allclose(rr["round_cuts"], ro["round_cuts"], rtol=1e-9, atol=1e-9)
    assert np.array_equal(cpu(rr["flips"]), ro["flips"])
    # full-length rounds: the flip counters carry exactly the applied cuts
    rr = qh.refine(g, 16, 300, seed=3, max_rounds=4, deform=0.5, deform_tries=2)
    assert np.array_equal(cpu(g.export_rows(0, n)), master)
    comp, nc = oracle.components(g2)
    S = np.where(cpu(rr["flips"]) % 2 == 1, -1, 1).astype(np.int8)
    assert oracle.cuts(g2, comp, nc, S).sum() == pytest.approx(sum(rr["round_cuts"]), rel=1e-9, abs=1e-9)
    with pytest.raises(qh.QhapError) as e:
        qh.refine(g, 16, 10, deform=-1.0, deform_tries=1)
    assert e.value.status == qh.Status.EINVAL


def test_discrete_whole_solves_match_oracle_and_plans():
    """Discrete variant end to end: cut gap to the oracle's discrete solve, persistent =
    per-step bit for bit, batched = single bit for bit."""
    w = synth.read_tiny()
    g = gpu_graph(w, "read_signed", "f16")
    ro = oracle.solve(oracle_graph(w), 16, 1000, 0.5, seed=11, integer=True, discrete=True)
    rs = qh.bsb_solve(g, 16, 1000, seed=11, discrete=True)
    assert _gap(ro["best_cut"], float(cpu(rs["best_cut"])[0])) <= 1e-3
    wm = synth.read_mhc(seed=78, n_snp=1500, n_reads=1000, region=500_000)
    gm = gpu_graph(wm, "read_signed", "f16")
    n = gm.info()["n"]
    outs = []
    for plan, sync in ((1, 0), (2, 1), (2, 2)):
        x = torch.empty((n, 64), dtype=torch.float32, device="cuda")
        y = torch.empty((n, 64), dtype=torch.float32, device="cuda")
        r = qh.bsb_solve(gm, 64, 300, seed=31, x=x, y=y, plan=plan, discrete=True, persistent_sync=sync)
        outs.append((x, y, r))
    for o in outs[1:]:
        assert torch.equal(outs[0][0], o[0]) and torch.equal(outs[0][1], o[1])
        assert torch.equal(outs[0][2]["best_cut"], o[2]["best_cut"])
    ws = synth.snp_small(61, n_snp=400)
    gs_ = gpu_graph(ws, "snp_llr", "bf16")
    rb = qh.bsb_solve_batched([g, gs_], 32, 300, seed=9, discrete=True)
    for b, gg in enumerate((g, gs_)):
        r1 = qh.bsb_solve(gg, 32, 300, seed=9, discrete=True, plan=1)
        assert torch.equal(rb["best_cut"][b:b + 1], r1["best_cut"])
        lo, hi = int(rb["vertex_offset"][b]), int(rb["vertex_offset"][b + 1])
        assert torch.equal(rb["best_spins"][lo:hi], r1["best_spins"])


@pytest.mark.parametrize("dtype", ["f16", "bf16", "fp8"])
@pytest.mark.parametrize("R", [16, 64, 256])
def test_persistent_equals_per_step_bit_exact(dtype, R):
    """The persistent plan runs the same MFMA sequence and update as the per-step kernel,
    so 300 steps of both must agree bit for bit (state and readout), with either way of
    passing x between workgroups (cache-wide fences, device-coherent accesses)."""
    w = synth.read_mhc(seed=78, n_snp=1500, n_reads=1000, region=500_000)
    g = gpu_graph(w, "read_signed", dtype)
    n = g.info()["n"]
    out = []
    # one fused kernel per step; persistent with fences; persistent with coherent accesses
    for plan, sync in ((1, 0), (2, 1), (2, 2)):
        x = torch.empty((n, R), dtype=torch.float32, device="cuda")
        y = torch.empty((n, R), dtype=torch.float32, device="cuda")
        r = qh.bsb_solve(g, R, 300, seed=31, x=x, y=y, plan=plan, persistent_sync=sync)
        if plan == 2:
            info = g.plan_info(R)
            assert info["plan_used"] == 2 and info["persistent_sync"] == sync
        out.append((x, y, r))
    xa, ya, ra = out[0]
    for xb, yb, rb in out[1:]:
        assert torch.equal(xa, xb) and torch.equal(ya, yb)
        assert torch.equal(ra["best_spins"], rb["best_spins"]) and torch.equal(ra["best_cut"], rb["best_cut"])


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16", "fp8"])
def test_replica_tiles_bit_exact(dtype):
    """The per-step dense kernel with 64, 32 or 16 replicas per workgroup computes every
    replica's product and update identically; the autotuned plan equals them too."""
    w = synth.read_mhc(seed=79, n_snp=1500, n_reads=900, region=500_000)
    g = gpu_graph(w, "read_signed", dtype)
    n, R = g.info()["n"], 128
    out = []
    for tile, depth in ((64, 2), (64, 4), (32, 0), (16, 0)):
        x = torch.empty((n, R), dtype=torch.float32, device="cuda")
        y = torch.empty((n, R), dtype=torch.float32, device="cuda")
        r = qh.bsb_solve(g, R, 200, seed=5, x=x, y=y, plan=1, replica_tile=tile, tiles_in_flight=depth)
        out.append((x, y, r))
    x = torch.empty((n, R), dtype=torch.float32, device="cuda")
    y = torch.empty((n, R), dtype=torch.float32, device="cuda")
    out.append((x, y, qh.bsb_solve(g, R, 200, seed=5, x=x, y=y, plan=0)))
    info = g.plan_info(R)
    assert info["replica_tile"] in (16, 32, 64) and info["us_per_step"][0] > 0
    assert info["tiles_in_flight"] in (2, 4)
    xa, ya, ra = out[0]
    for xb, yb, rb in out[1:]:
        assert torch.equal(xa, xb) and torch.equal(ya, yb)
        assert torch.equal(ra["cuts"], rb["cuts"]) and torch.equal(ra["best_spins"], rb["best_spins"])
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve(g, 32, 10, replica_tile=16)
    assert e.value.status == qh.Status.EINVAL
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve(g, 64, 10, tiles_in_flight=3)
    assert e.value.status == qh.Status.EINVAL
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve(g, 64, 10, persistent_sync=3)
    assert e.value.status == qh.Status.EINVAL


@pytest.mark.parametrize("plan", [0, 3, 4, 5])   # autotuned; per row; band FMA (R % 64 == 0); band MFMA
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("R", [16, 32, 64, 128])
def test_skyline_one_step(dtype, R, plan):
    w = synth.snp_small(14, n_snp=1500)
    g = gpu_graph(w, "snp_llr", dtype)
    J = stored_J(oracle_graph(w, "snp_llr").dense(), dtype)
    _one_step_case(g, J, dtype, R, 200 + R, None, plan=plan)


@pytest.mark.parametrize("case", ["snp", "porec", "snp_large", "porec_wide", "snp_tiny"])
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_band_kernel_equals_row_kernel_bit_exact(dtype, case):
    """Band blocks add exact zeros around each row's range in the same ascending column
    order as the per-row kernel, so 200 steps of both agree bit for bit.  BF16 band values
    are stored as binary16 of value x 2^s when one power of two makes all of them exact
    there (the kernels multiply the band sums by 2^-s; BF16 storage flushes magnitudes 2^31
    below the largest, so this always holds unless the scale leaves the float range), else
    as BF16: "snp_large" scales every fragment weight by 1e5 (past the binary16 range),
    "porec_wide" shrinks the Pore-C contacts in the band by 1e-12 (flushed), "snp_tiny"
    scales every weight by 1e-35 (the scale would be 2^128: the band stays BF16)."""
    if case in ("snp", "snp_large", "snp_tiny"):
        w, band = synth.snp_small(26, n_snp=1700), 0
        if case == "snp_large":
            if dtype == "f16":
                pytest.skip("weights past the binary16 range")
            w.alpha = w.alpha * 1e5
        if case == "snp_tiny":
            if dtype == "f16":
                pytest.skip("weights below the binary16 range")
            w.alpha = w.alpha * 1e-35
    elif case == "porec_wide":
        w, band = synth.snp_porec(45, n_snp=2000, n_edges=2500, zipf_s=1.0), 0
        w.alpha = np.where(w.alpha < 1.0, w.alpha * 1e-12, w.alpha)
    else:
        w, band = synth.snp_porec(45, n_snp=2000, n_edges=2500, zipf_s=1.0), 100
    g = gpu_graph(w, "snp_llr", dtype, band_limit=band)
    want_band = {"f32": 0, "f16": 1, "bf16": 2 if case == "snp_tiny" else 1}[dtype]
    assert g.info()["band_dtype"] == want_band
    n, R = g.info()["n"], 128
    out = []
    for plan in (4, 3):          # band blocks on FMAs; per-row kernel
        x = torch.empty((n, R), dtype=torch.float32, device="cuda")
        y = torch.empty((n, R), dtype=torch.float32, device="cuda")
        r = qh.bsb_solve(g, R, 200, seed=33, x=x, y=y, plan=plan)
        out.append((x, y, r))
    (xa, ya, ra), (xb, yb, rb) = out
    assert torch.equal(xa, xb) and torch.equal(ya, yb)
    assert torch.equal(ra["best_spins"], rb["best_spins"]) and torch.equal(ra["best_cut"], rb["best_cut"])


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_band_mfma_whole_solve_and_tuner(dtype):
    """Band blocks on MFMAs over a whole solve: the final cut tracks the oracle's, the
    autotuner reports both band kernels, and plans 4 and 5 agree to FP32 rounding."""
    w = synth.snp_small(27, n_snp=1800)
    g = gpu_graph(w, "snp_llr", dtype)
    go = oracle_graph(w, "snp_llr")
    ro = oracle.solve(go, 64, 600, 0.5, seed=3)
    r5 = qh.bsb_solve(g, 64, 600, seed=3, plan=5)
    assert g.plan_info(64)["skyline_kernel"] == 5
    assert _gap(ro["best_cut"], float(cpu(r5["best_cut"])[0])) <= 1e-3
    n = g.info()["n"]
    xs = []
    for plan in (4, 5):
        x = torch.empty((n, 64), dtype=torch.float32, device="cuda")
        y = torch.empty((n, 64), dtype=torch.float32, device="cuda")
        qh.bsb_solve(g, 64, 3, seed=3, x=x, y=y, plan=plan, readout=False)
        xs.append(cpu(x))
    assert np.allclose(xs[0], xs[1], rtol=0, atol=1e-5)
    g2 = gpu_graph(w, "snp_llr", dtype)
    qh.bsb_solve(g2, 64, 100, seed=3, plan=0, readout=False)
    info = g2.plan_info(64)
    assert info["skyline_kernel"] in (4, 5) and min(info["skyline_us"]) > 0
    gd = gpu_graph(synth.read_tiny())
    with pytest.raises(qh.QhapError) as e:      # skyline plans on a dense graph
        qh.bsb_solve(gd, 16, 10, plan=5)
    assert e.value.status == qh.Status.EINVAL


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("R", [32, 64])
def test_longrange_hub_one_step(dtype, R):
    """Long-range rows, hub rows among them (chunk partials from the packet kernel for R = 64,
    per chunk for R = 32); 16-bit storage gathers the binary16 copy of x."""
    w = synth.snp_porec(43, n_snp=2500, n_edges=4000, zipf_s=1.0)
    g = gpu_graph(w, "snp_llr", dtype, band_limit=100)
    assert g.info()["longrange_nnz"] > 0
    J = stored_J(oracle_graph(w, "snp_llr").dense(), dtype)
    _one_step_case(g, J, dtype, R, 300 + R, None, lr_band=None if dtype == "f32" else 100)


@pytest.mark.parametrize("plan", [3, 4, 5])
@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_longrange_copy_against_unrounded_oracle(dtype, plan):
    """The binary16 copy of x that 16-bit SNP graphs gather for their long-range entries,
    bounded against the oracle's unrounded step (stored J, FP64): rounding x_j to binary16
    moves it by at most 2^-11 |x_j| + 2^-25, so row i's coupling sum moves by at most
    sum over its long-range j of |J_ij| (2^-11 |x_j| + 2^-25), y by c0 dt times that and x by
    a0 dt times y's bound, on top of the FP32 step tolerance; band entries take x itself."""
    w = synth.snp_porec(43, n_snp=2500, n_edges=4000, zipf_s=1.0)
    g = gpu_graph(w, "snp_llr", dtype, band_limit=100)
    J = stored_J(oracle_graph(w, "snp_llr").dense(), dtype)
    n, R, k, steps, dt = J.shape[0], 64, 37, 100, 0.5
    rng = np.random.default_rng(654)
    x0 = f32(rng.uniform(-1.0, 1.0, (n, R)))
    y0 = f32(rng.uniform(-0.6, 0.6, (n, R)))
    pump = np.linspace(0.0, 1.0, steps).astype(np.float32)
    c0 = float(np.float32(0.4 / max(1.0, float(np.sqrt((J ** 2).sum() / (n - 1))))))
    p = float(pump[k])
    x = torch.tensor(x0, dtype=torch.float32, device="cuda").contiguous()
    y = torch.tensor(y0, dtype=torch.float32, device="cuda").contiguous()
    qh.bsb_solve(g, R, steps, dt=dt, c0=c0, pump=torch.tensor(pump, device="cuda"), init=False, x=x, y=y,
                 step_begin=k, step_end=k + 1, readout=False, plan=plan)
    xg, yg = cpu(x).astype(np.float64), cpu(y).astype(np.float64)
    xu, yu = oracle.bsb_step_dense(J, x0, y0, p, dt, c0, 1.0, walls=False)
    xo, yo = oracle.bsb_step_dense(J, x0, y0, p, dt, c0, 1.0, walls=True)
    tol_x, tol_y = step_bounds(np.abs(J) @ np.abs(x0), x0, y0, p, dt, c0)
    Jfar = np.where(far_mask(n, 100), np.abs(J), 0.0)
    assert Jfar.sum() > 0
    copy = c0 * dt * (Jfar @ (COPY_UNIT["f16"] * np.abs(x0) + COPY_ABS["f16"]))
    tol_y = tol_y + copy
    tol_x = tol_x + dt * copy
    ok = np.abs(np.abs(xu) - 1.0) > tol_x        # entries not within the tolerance of a wall
    assert ok.mean() > 0.9
    assert np.all(np.abs(yg - yo)[ok] <= tol_y[ok])
    assert np.all(np.abs(xg - xo)[ok] <= tol_x[ok])


@pytest.mark.parametrize("plan", [2, 1])
def test_mhc_scale_one_step_f16(mhc, plan):
    """One step at the full MHC-scale shape and the benchmark's launch (R = 256, FP16):
    plan 2 requires the persistent kernel the benchmark uses, plan 1 the per-step kernel."""
    w, W = mhc
    g = gpu_graph(w, "read_signed", "f16")
    _one_step_case(g, W.astype(np.float64), "f16", 256, 7, "f16", steps=2000, k=999, plan=plan)


# ----------------------------------------------------------------------------- init, resume, graphs

def test_init_bit_exact():
    w = synth.read_small(15, n_snp=200, n_reads=70)
    g = gpu_graph(w)
    n = g.info()["n"]
    for R in (16, 64):
        x = torch.empty((n, R), dtype=torch.float32, device="cuda")
        y = torch.empty((n, R), dtype=torch.float32, device="cuda")
        qh.bsb_solve(g, R, 1, seed=12345, init=True, x=x, y=y, step_begin=1, step_end=1, readout=False)
        xo, yo = oracle.init_state(12345, n, R)
        assert np.array_equal(cpu(x), xo.astype(np.float32))
        assert np.array_equal(cpu(y), yo.astype(np.float32))


RESUME_CASES = [("read_signed", "f32"), ("read_signed", "f16"), ("read_signed", "fp8"), ("snp_llr", "f32"),
                ("snp_llr", "bf16")]


@pytest.mark.parametrize("kind,dtype", RESUME_CASES)
def test_resume_and_graph_replay_bit_identical(kind, dtype):
    w = synth.read_small(16, n_snp=300, n_reads=140) if kind != "snp_llr" else synth.snp_small(16, n_snp=900)
    g = gpu_graph(w, kind, dtype)
    n, R, steps = g.info()["n"], 64, 200
    def run(**kw):
        x = torch.empty((n, R), dtype=torch.float32, device="cuda")
        y = torch.empty((n, R), dtype=torch.float32, device="cuda")
        r = qh.bsb_solve(g, R, steps, seed=5, x=x, y=y, **kw)
        return x, y, r
    xa, ya, ra = run()
    xb, yb, _ = run(step_end=120, readout=False)
    xb2 = xb.clone(); yb2 = yb.clone()
    qh.bsb_solve(g, R, steps, init=False, x=xb2, y=yb2, step_begin=120, step_end=200, readout=False)
    assert torch.equal(xa, xb2) and torch.equal(ya, yb2)
    # captured step loop, replayed several times with eager work in between
    for rep in range(3):
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        xc, yc, rc = run(use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(xa, xc) and torch.equal(ya, yc), rep
        assert torch.equal(ra["best_spins"], rc["best_spins"]) and torch.equal(ra["best_cut"], rc["best_cut"])
        del junk


# ----------------------------------------------------------------------------- readout

def _readout_case(w, kind, R, seed, exact):
    g = gpu_graph(w, kind, "f32")
    go = oracle_graph(w, kind)
    n = go.n
    rng = np.random.default_rng(seed)
    x0 = f32(np.where(rng.random((n, R)) < 0.5, -0.5, 0.5))
    x0[rng.random((n, R)) < 0.05] = 0.0          # sgn(0) = +1
    y0 = np.zeros((n, R))
    x = torch.tensor(x0, dtype=torch.float32, device="cuda")
    y = torch.tensor(y0, dtype=torch.float32, device="cuda")
    res = qh.bsb_solve(g, R, 1, init=False, x=x, y=y, step_begin=1, step_end=1, readout=True, greedy=True,
                       all_spins=True, per_component=True)
    s = oracle.signs(x0)
    comp, nc = oracle.components(go)
    cut = oracle.cuts(go, comp, nc, s)
    best, br = oracle.select(comp, nc, s, cut)
    sel = float(sum(cut[br[c], c] for c in range(nc)))
    gbest, rounds = oracle.greedy(go, best, oracle.greedy_eps(go, exact))
    final = float(oracle.cuts(go, comp, nc, gbest).sum())
    assert np.array_equal(cpu(res["all_spins"]), s)
    if exact:
        assert np.array_equal(cpu(res["cut_rc"])[:, :nc], cut)
        assert np.array_equal(cpu(res["cuts"]), cut.sum(axis=1))
        assert np.array_equal(cpu(res["best_replica"])[:nc], br)
        assert cpu(res["selected_cut"])[0] == sel
        assert np.array_equal(cpu(res["best_spins"]), gbest)
        assert cpu(res["best_cut"])[0] == final
        assert int(cpu(res["greedy_rounds"])[0]) == rounds
    else:
        scale = np.abs(go.val).sum()
        assert np.allclose(cpu(res["cut_rc"])[:, :nc], cut, rtol=0, atol=1e-12 * scale)
        assert cpu(res["selected_cut"])[0] == pytest.approx(sel, abs=1e-12 * scale)
        assert cpu(res["best_cut"])[0] == pytest.approx(final, abs=1e-9 * scale)


@pytest.mark.parametrize("R", [16, 64, 256])
def test_readout_integer_exact(R):
    _readout_case(synth.read_small(17, n_snp=600, n_reads=250, span=(5, 40)), "read_signed", R, R, True)


def test_readout_conflict_many_components():
    _readout_case(synth.read_small(18, n_snp=3000, n_reads=200, span=(3, 15)), "read_conflict", 32, 3, True)


def test_readout_float_weights():
    _readout_case(synth.snp_small(19, n_snp=1200), "snp_llr", 64, 4, False)


# ----------------------------------------------------------------------------- phasing

def test_phase_vote_exact():
    w = synth.read_small(20, n_snp=500, n_reads=260, span=(5, 50), error=0.08)
    g = gpu_graph(w)
    go = oracle_graph(w)
    comp, nc = oracle.components(go)
    rng = np.random.default_rng(1)
    s = np.where(w.origin == 0, 1, -1).astype(np.int8)
    s[rng.random(s.shape[0]) < 0.2] *= -1
    h1, blk = qh.phase(g, torch.tensor(s, device="cuda"))
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    ho, bo = oracle.phase_vote(w.n_snp, w.frag_ptr, w.snp, M, s, comp, w.init_h1)
    assert np.array_equal(cpu(h1), ho) and np.array_equal(cpu(blk), bo)


def test_phase_parity_exact():
    w = synth.snp_small(21, n_snp=1500)
    g = gpu_graph(w, "snp_llr")
    go = oracle_graph(w, "snp_llr")
    comp, nc = oracle.components(go)
    s = np.where(np.random.default_rng(2).random(go.n) < 0.4, 1, -1).astype(np.int8)
    h1, blk = qh.phase(g, torch.tensor(s, device="cuda"))
    ho, bo = oracle.phase_parity(comp, nc, s, w.init_h1)
    assert np.array_equal(cpu(h1), ho) and np.array_equal(cpu(blk), bo)


def test_phase_batched_equals_per_graph_phase():
    """qh_phase_batched over a list of read and SNP graphs (one and zero fragments, long-range
    rows, many components among them), with random spins packed as a batched solve packs
    them: every graph's slice of h1 and block equals qh_phase on that graph, bit for bit; and
    on the spins of a batched solve, every block's haplotype equals its qh_phase."""
    batch = synth.batched_blocks(93, n_blocks=40, n_lo=20, n_hi=600)
    gs = [gpu_graph(w, "read_signed" if i % 2 == 0 else "snp_llr", w.solve["dtype"])
          for i, w in enumerate(batch.blocks)]
    gs.append(gpu_graph(synth.read_tiny(), "read_conflict"))
    gs.append(gpu_graph(synth.snp_porec(45, n_snp=2000, n_edges=2500, zipf_s=1.0), "snp_llr", "bf16",
                        band_limit=64))
    for nf in (1, 0):
        w = synth.read_small(25, n_snp=50, n_reads=1, span=(5, 10))
        fp = w.frag_ptr[: nf + 1].copy()
        gs.append(qh.build_graph(qh.to_device(fp), qh.to_device(w.snp[: fp[-1]].copy()),
                                 qh.to_device(w.allele[: fp[-1]].copy()), qh.to_device(w.phred[: fp[-1]].copy()),
                                 qh.to_device(w.init_h1)))
    ns = [g.info()["n"] for g in gs]
    vo = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    rng = np.random.default_rng(17)
    spins = torch.tensor(rng.choice(np.array([-1, 1], dtype=np.int8), size=max(int(vo[-1]), 1)), device="cuda")
    h1, blk, so = qh.phase_batched(gs, spins)
    assert len(so) == len(gs) + 1 and int(so[-1]) == sum(g.n_snp for g in gs)
    for b, g in enumerate(gs):
        sb = spins[int(vo[b]):int(vo[b + 1])] if ns[b] else torch.ones(1, dtype=torch.int8, device="cuda")
        h1b, blkb = qh.phase(g, sb)
        assert torch.equal(h1[int(so[b]):int(so[b + 1])], h1b), b
        assert torch.equal(blk[int(so[b]):int(so[b + 1])], blkb), b
    # the spins of a batched solve
    r = qh.bsb_solve_batched(gs[:40], 32, 200, seed=4)
    h1, blk, so = qh.phase_batched(gs[:40], r["best_spins"])
    off = r["vertex_offset"]
    for b, g in enumerate(gs[:40]):
        h1b, blkb = qh.phase(g, r["best_spins"][int(off[b]):int(off[b + 1])])
        assert torch.equal(h1[int(so[b]):int(so[b + 1])], h1b) and torch.equal(blk[int(so[b]):int(so[b + 1])], blkb)
    arr = (ctypes.c_void_p * 2)(gs[0].handle.value, None)       # a null graph in the list
    rc = qh.load().qh_phase_batched(arr, 2, spins.data_ptr(), h1.data_ptr(), blk.data_ptr(), None)
    assert rc == qh.Status.EINVAL


def test_flip_crossing_matches_oracle():
    w = synth.snp_small(22, n_snp=1000)
    g = gpu_graph(w, "snp_llr", "f32")
    go = oracle_graph(w, "snp_llr")
    s = np.where(np.random.default_rng(3).random(go.n) < 0.5, 1, -1).astype(np.int8)
    qh.flip_crossing(g, torch.tensor(s, device="cuda"))
    D = cpu(g.export_rows(0, go.n))
    Do = oracle.flip_crossing(go, s).dense()
    assert np.all(np.abs(D - Do) <= 1e-12 * snp_abs_terms(w))
    S = cpu(g.export_rows(0, go.n, stored=True))
    assert np.array_equal(S, quant.round_to("f32", D))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_refine_gauge_identity_restore_and_single_round(dtype):
    """Eqs. (15)-(17) in the library: the flip counters' partition has, on the original
    weights (cut by the oracle), exactly the sum of the per-round cuts; the graph is
    restored bit for bit; one round equals the parity phasing of one solve."""
    w = synth.snp_small(24, n_snp=1500)
    g = gpu_graph(w, "snp_llr", dtype)
    go = oracle_graph(w, "snp_llr")
    n = go.n
    master, stored = cpu(g.export_rows(0, n)), cpu(g.export_rows(0, n, stored=True))
    rr = qh.refine(g, 32, 600, seed=1, max_rounds=15)
    assert np.array_equal(cpu(g.export_rows(0, n)), master)
    assert np.array_equal(cpu(g.export_rows(0, n, stored=True)), stored)
    assert rr["rounds"] >= 1 and all(c > 0 for c in rr["round_cuts"])
    comp, nc = oracle.components(go)
    S = np.where(cpu(rr["flips"]) % 2 == 1, -1, 1).astype(np.int8)
    total = oracle.cuts(go, comp, nc, S).sum()
    assert total == pytest.approx(sum(rr["round_cuts"]), rel=1e-9)
    # the oracle's refinement at the same schedule reaches the same total within 0.1 %
    ro = oracle.refine(go, w.init_h1, 32, 600, 0.5, seed=1, max_rounds=15)
    assert _gap(sum(ro["round_cuts"]), total) <= 1e-3
    # one round is the single-round parity phasing of the round-0 solve
    r1 = qh.refine(g, 32, 600, seed=1, max_rounds=1)
    rs = qh.bsb_solve(g, 32, 600, seed=1)
    h1, blk = qh.phase(g, rs["best_spins"])
    assert torch.equal(r1["h1"], h1) and torch.equal(r1["block"], blk)
    assert r1["round_cuts"][0] == pytest.approx(float(cpu(rs["best_cut"])[0]), rel=1e-12)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_refine_adaptive_schedule_planted_twin(dtype):
    """The size-adaptive settings end to end on an error-free planted twin (500 steps below
    5,000 vertices, 128 replicas, at most 15 rounds, deformation on) against the oracle's
    refinement with the same settings, seed and deformation: the applied round cuts agree in
    total within 0.1 % and the switch errors are equal."""
    w = synth.snp_small(8, n_snp=900, error=0.0)
    g = gpu_graph(w, "snp_llr", dtype)
    rr = qh.refine_adaptive(g, seed=2, deform=0.5, deform_tries=2)
    sc = rr["schedule"]
    assert sc["steps"] == 500 and sc["replicas"] == 128 and sc["max_rounds"] == 15
    assert sc["size"] == g.info()["largest_component"]
    assert 1 <= rr["rounds"] <= 15
    ro = oracle.refine(oracle_graph(w, "snp_llr"), w.init_h1, sc["replicas"], sc["steps"], seed=2,
                       max_rounds=sc["max_rounds"], deform=0.5, deform_tries=2)
    assert _gap(sum(ro["round_cuts"]), sum(rr["round_cuts"])) <= 1e-3
    assert metrics.switch_error(cpu(rr["h1"]), w.truth, cpu(rr["block"])) == \
        metrics.switch_error(ro["h1"], w.truth, ro["block"])


def test_refine_planted_twin_and_errors():
    w = synth.snp_small(8, n_snp=600, error=0.0)
    g = gpu_graph(w, "snp_llr", "f32")
    rr = qh.refine(g, 32, 600, seed=5)
    assert metrics.switch_error(cpu(rr["h1"]), w.truth, cpu(rr["block"])) == 0.0
    gr = gpu_graph(synth.read_tiny())
    with pytest.raises(qh.QhapError) as e:
        qh.refine(gr, 16, 10)
    assert e.value.status == qh.Status.EUNSUPPORTED
    with pytest.raises(qh.QhapError) as e:
        qh.refine(g, 32, 10, max_rounds=0)
    assert e.value.status == qh.Status.EINVAL


# ----------------------------------------------------------------------------- whole solves

def _gap(oracle_cut, gpu_cut):
    return (oracle_cut - gpu_cut) / abs(oracle_cut)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16", "fp8"])
def test_read_tiny_final_cut_and_switch_error(dtype):
    """Read-based tiny workload: R = 16, 1,000 steps, dt = 0.5, linear pump."""
    w = synth.read_tiny()
    g = gpu_graph(w, "read_signed", dtype)
    go = oracle_graph(w)
    ro = oracle.solve(go, 16, 1000, 0.5, seed=11, integer=True)
    rg = qh.bsb_solve(g, 16, 1000, dt=0.5, seed=11)
    assert _gap(ro["best_cut"], float(cpu(rg["best_cut"])[0])) <= 1e-3
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    ho, bo = oracle.phase_vote(w.n_snp, w.frag_ptr, w.snp, M, ro["best"], ro["comp"], w.init_h1)
    hg, bg = qh.phase(g, rg["best_spins"])
    assert metrics.switch_error(cpu(hg), w.truth, cpu(bg)) == metrics.switch_error(ho, w.truth, bo)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16", "fp8"])
def test_read_midsize_final_cut(dtype):
    w = synth.read_mhc(seed=77, n_snp=2400, n_reads=1600, region=800_000)
    g = gpu_graph(w, "read_signed", dtype)
    go = oracle_graph(w)
    ro = oracle.solve(go, 64, 1000, 0.5, seed=3, integer=True)
    rg = qh.bsb_solve(g, 64, 1000, dt=0.5, seed=3, use_graph=True)
    assert _gap(ro["best_cut"], float(cpu(rg["best_cut"])[0])) <= 1e-3
    M = oracle.encode(w.snp, w.allele, w.init_h1)
    ho, bo = oracle.phase_vote(w.n_snp, w.frag_ptr, w.snp, M, ro["best"], ro["comp"], w.init_h1)
    hg, bg = qh.phase(g, rg["best_spins"])
    assert metrics.switch_error(cpu(hg), w.truth, cpu(bg)) <= metrics.switch_error(ho, w.truth, bo)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_snp_final_cut(dtype):
    w = synth.snp_small(23, n_snp=2000)
    g = gpu_graph(w, "snp_llr", dtype)
    go = oracle_graph(w, "snp_llr")
    ro = oracle.solve(go, 64, 1000, 0.5, seed=4)
    rg = qh.bsb_solve(g, 64, 1000, dt=0.5, seed=4, use_graph=True)
    assert _gap(ro["best_cut"], float(cpu(rg["best_cut"])[0])) <= 1e-3
    comp, nc = oracle.components(go)
    ho, bo = oracle.phase_parity(comp, nc, ro["best"], w.init_h1)
    hg, bg = qh.phase(g, rg["best_spins"])
    assert metrics.switch_error(cpu(hg), w.truth, cpu(bg)) <= metrics.switch_error(ho, w.truth, bo)


@pytest.mark.parametrize("n_snp,dtype", [(600, "f16"), (1500, "f32"), (1500, "f16")])
def test_snp_planted_twin_switch_error_equals_oracle(n_snp, dtype):
    """Error-free reads: the GPU's switch error equals the FP64 oracle's at the same
    schedule (on long SNP chains bSB can keep domain walls; both sides then agree)."""
    w = synth.snp_small(24, n_snp=n_snp, error=0.0)
    g = gpu_graph(w, "snp_llr", dtype)
    go = oracle_graph(w, "snp_llr")
    rg = qh.bsb_solve(g, 32, 600, dt=0.5, seed=1)
    ro = oracle.solve(go, 32, 600, 0.5, seed=1)
    comp, nc = oracle.components(go)
    ho, bo = oracle.phase_parity(comp, nc, ro["best"], w.init_h1)
    hg, bg = qh.phase(g, rg["best_spins"])
    se_o = metrics.switch_error(ho, w.truth, bo)
    assert metrics.switch_error(cpu(hg), w.truth, cpu(bg)) == se_o
    assert _gap(ro["best_cut"], float(cpu(rg["best_cut"])[0])) <= 1e-3


def test_porec_final_cut():
    w = synth.snp_porec(44, n_snp=2500, n_edges=3000, zipf_s=1.0)
    g = gpu_graph(w, "snp_llr", "bf16", band_limit=100)
    go = oracle_graph(w, "snp_llr")
    ro = oracle.solve(go, 64, 800, 0.5, seed=6)
    rg = qh.bsb_solve(g, 64, 800, dt=0.5, seed=6)
    assert _gap(ro["best_cut"], float(cpu(rg["best_cut"])[0])) <= 1e-3


@pytest.mark.parametrize("threads", [0, 1, 5])
def test_build_graphs_equals_single_builds(threads):
    """qh_build_graphs (host threads, a stream each) returns the graphs that qh_build_graph
    builds one by one: equal info, FP64 master and stored rows bit for bit, equal components
    (deterministic builds: the default SNP build sums Eq. 14 terms with atomics, whose order,
    and so the last bit, may change from one build to the next).  A malformed block fails
    the whole call with its index, and no graph is returned."""
    blocks = [synth.read_small(70 + b, n_snp=200, n_reads=30 + 25 * b) for b in range(6)] + \
             [synth.snp_small(80 + b, n_snp=120 + 150 * b) for b in range(6)] + [synth.read_tiny()] + \
             [synth.snp_porec(45, n_snp=2000, n_edges=2500, zipf_s=1.0)]
    kinds = ["read_signed"] * 6 + ["snp_llr"] * 6 + ["read_conflict", "snp_llr"]
    dtypes = ["fp8", "f16", "bf16", "f32", "fp8", "f16", "bf16", "f16", "f32", "bf16", "f16", "f32", "f32", "bf16"]
    specs = []
    for b, (w, k, dt) in enumerate(zip(blocks, kinds, dtypes)):
        d = device_reads(w)
        specs.append(dict(frag_ptr=d["frag_ptr"], snp=d["snp"], allele=d["allele"], phred=d["phred"],
                          init_h1=d["init_h1"], kind=k, dtype=dt, alpha=d["alpha"], deterministic=True,
                          band_limit=64 if b == 13 else 0))
    # degenerate graphs among them: one fragment, and none
    for nf in (1, 0):
        w = synth.read_small(25, n_snp=50, n_reads=1, span=(5, 10))
        fp = w.frag_ptr[: nf + 1].copy()
        specs.append(dict(frag_ptr=qh.to_device(fp), snp=qh.to_device(w.snp[: fp[-1]].copy()),
                          allele=qh.to_device(w.allele[: fp[-1]].copy()),
                          phred=qh.to_device(w.phred[: fp[-1]].copy()), init_h1=qh.to_device(w.init_h1)))
    many = qh.build_graphs(specs, threads=threads)
    assert len(many) == len(specs)
    assert many[13].info()["longrange_nnz"] > 0 and many[-1].info()["n"] == 0 and many[-2].info()["n"] == 1
    for b, (sp, gm) in enumerate(zip(specs, many)):
        g1 = qh.build_graph(**sp)
        assert g1.info() == gm.info(), b
        n = g1.info()["n"]
        if n:
            assert torch.equal(g1.export_rows(0, n), gm.export_rows(0, n)), b
            assert torch.equal(g1.export_rows(0, n, stored=True), gm.export_rows(0, n, stored=True)), b
            assert torch.equal(g1.components(), gm.components()), b
        g1.free()
    for g in many:
        g.free()
    # many small blocks: every worker recycles its temporaries many times over
    batch = synth.batched_blocks(91, n_blocks=240, n_lo=20, n_hi=300)
    specs2 = []
    for i, w in enumerate(batch.blocks):
        d = device_reads(w)
        k = "read_signed" if i % 2 == 0 else "snp_llr"
        specs2.append(dict(frag_ptr=d["frag_ptr"], snp=d["snp"], allele=d["allele"], phred=d["phred"],
                           init_h1=d["init_h1"], kind=k, dtype=w.solve["dtype"], alpha=d["alpha"],
                           deterministic=True))
    many = qh.build_graphs(specs2, threads=threads)
    for b, (sp, gm) in enumerate(zip(specs2, many)):
        g1 = qh.build_graph(**sp)
        assert g1.info() == gm.info(), b
        n = g1.info()["n"]
        assert torch.equal(g1.export_rows(0, n, stored=True), gm.export_rows(0, n, stored=True)), b
        assert torch.equal(g1.components(), gm.components()), b
        g1.free()
        gm.free()
    bad = dict(specs[7])
    snp = bad["snp"].clone()
    snp[0] = bad["init_h1"].numel()           # a SNP index past the last SNP
    bad["snp"] = snp
    with pytest.raises(qh.QhapError) as e:
        qh.build_graphs(specs[:7] + [bad] + specs[8:], threads=threads)
    assert e.value.status == qh.Status.EINVAL and "graph 7" in str(e.value)


@pytest.mark.parametrize("R,plan", [(16, 1), (32, 1), (64, 1), (16, 2), (32, 2), (64, 2), (32, 0)])
def test_batched_matches_single_solves(R, plan):
    """Uneven blocks of every storage and dtype, per-step (1), whole-block (2) or autotuned
    (0) plan: each block's state, replica cuts, selection and greedy result equal its
    single-graph solve bit for bit."""
    blocks = [synth.read_small(50 + b, n_snp=200, n_reads=40 + 30 * b) for b in range(4)] + \
             [synth.snp_small(60 + b, n_snp=150 + 200 * b) for b in range(3)] + [synth.read_tiny()]
    kinds = ["read_signed"] * 4 + ["snp_llr"] * 3 + ["read_signed"]
    dtypes = ["fp8", "f16", "bf16", "f32", "bf16", "f16", "f32", "f16"]
    gs = [gpu_graph(w, k, d) for w, k, d in zip(blocks, kinds, dtypes)]     # reads dense, SNPs skyline
    steps = 300
    rb = qh.bsb_solve_batched(gs, R, steps, seed=9, return_state=True, plan=plan)
    assert rb["plan_used"] == plan or (plan == 0 and rb["plan_used"] in (1, 2))
    off = rb["vertex_offset"]
    for b, (w, k, g) in enumerate(zip(blocks, kinds, gs)):
        n = g.info()["n"]
        xs = torch.empty(n, R, dtype=torch.float32, device="cuda")
        ys = torch.empty(n, R, dtype=torch.float32, device="cuda")
        rs = qh.bsb_solve(g, R, steps, seed=9, plan=1, x=xs, y=ys)
        lo, hi = int(off[b]), int(off[b + 1])
        assert hi - lo == n
        assert torch.equal(rb["x"][lo * R:hi * R], xs.reshape(-1)), b
        assert torch.equal(rb["y"][lo * R:hi * R], ys.reshape(-1)), b
        assert torch.equal(rb["cuts"][b * R:(b + 1) * R], rs["cuts"]), b
        assert torch.equal(rb["selected_cut"][b:b + 1], rs["selected_cut"]), b
        assert torch.equal(rb["best_spins"][lo:hi], rs["best_spins"]), b
        assert torch.equal(rb["best_cut"][b:b + 1], rs["best_cut"]), b
    # and the single solves track the oracle
    for b in (0, 4):
        go = oracle_graph(blocks[b], kinds[b])
        ro = oracle.solve(go, R, steps, 0.5, seed=9, integer=(kinds[b] != "snp_llr"))
        rs = qh.bsb_solve(gs[b], R, steps, seed=9)
        assert _gap(ro["best_cut"], float(cpu(rs["best_cut"])[0])) <= 1e-3, b


def test_batched_graph_replay_equals_per_step_plan():
    """use_graph = 1: the per-step plan's launches captured once and replayed.  Every replay
    (with eager solves and syncs in between, and a recapture for another seed) gives the
    per-step plan's results bit for bit; the whole-block plan refuses it."""
    blocks = [synth.read_small(50 + b, n_snp=200, n_reads=40 + 30 * b) for b in range(3)] + \
             [synth.snp_small(60 + b, n_snp=150 + 200 * b) for b in range(2)]
    kinds = ["read_signed"] * 3 + ["snp_llr"] * 2
    dtypes = ["fp8", "f16", "f32", "bf16", "f16"]
    gs = [gpu_graph(w, k, d) for w, k, d in zip(blocks, kinds, dtypes)]
    for seed in (9, 9, 10, 9):
        ref = qh.bsb_solve_batched(gs, 32, 200, seed=seed, plan=1, return_state=True)
        torch.cuda.synchronize()
        rg = qh.bsb_solve_batched(gs, 32, 200, seed=seed, use_graph=True, return_state=True)
        assert rg["plan_used"] == 1
        for k in ("x", "y", "cuts", "best_spins", "best_cut", "selected_cut"):
            assert torch.equal(rg[k], ref[k]), (seed, k)
        qh.bsb_solve(gs[0], 32, 50, seed=1)      # eager work between replays
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve_batched(gs, 32, 20, plan=2, use_graph=True)
    assert e.value.status == qh.Status.EUNSUPPORTED


def test_batched_errors_and_empty_batch():
    w = synth.snp_porec(43, n_snp=2500, n_edges=4000, zipf_s=1.0)
    g_lr = gpu_graph(w, "snp_llr", "f32", band_limit=100)
    assert g_lr.info()["longrange_nnz"] > 0
    g_ok = gpu_graph(synth.read_tiny())
    with pytest.raises(qh.QhapError) as e:      # long-range couplings need the single-graph path
        qh.bsb_solve_batched([g_ok, g_lr], 32, 10)
    assert e.value.status == qh.Status.EUNSUPPORTED
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve_batched([g_ok], 128, 10)
    assert e.value.status == qh.Status.EUNSUPPORTED
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve_batched([g_ok, g_ok], 32, 10)
    assert e.value.status == qh.Status.EINVAL
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve_batched([g_ok], 32, 10, plan=3)
    assert e.value.status == qh.Status.EINVAL
    r = qh.bsb_solve_batched([], 32, 10)
    assert r["vertex_offset"].tolist() == [0]


# ----------------------------------------------------------------------------- errors, edges

def test_error_paths():
    w = synth.read_tiny()
    g = gpu_graph(w)
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve(g, 48, 10)
    assert e.value.status == qh.Status.EINVAL
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve(g, 16, 10, step_begin=5, step_end=20)
    assert e.value.status == qh.Status.EINVAL
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    with pytest.raises(qh.QhapError) as e:     # SNP index beyond n_snp
        qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"][:100])
    assert e.value.status == qh.Status.EINVAL
    with pytest.raises(qh.QhapError) as e:
        qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="read_signed",
                       storage="skyline")
    assert e.value.status == qh.Status.EUNSUPPORTED
    with pytest.raises(qh.QhapError) as e:
        qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="snp_llr",
                       dtype="fp8")
    assert e.value.status == qh.Status.EUNSUPPORTED
    bad = d["snp"].clone()
    bad[5], bad[6] = bad[6].item(), bad[5].item()        # not ascending inside fragment 0
    for kind in ("read_signed", "snp_llr"):
        with pytest.raises(qh.QhapError) as e:
            qh.build_graph(d["frag_ptr"], bad, d["allele"], d["phred"], d["init_h1"], kind=kind)
        assert e.value.status == qh.Status.EINVAL
    al = d["allele"].clone()
    al[17] = 2                                           # allele outside {0, 1}
    with pytest.raises(qh.QhapError) as e:
        qh.build_graph(d["frag_ptr"], d["snp"], al, d["phred"], d["init_h1"])
    assert e.value.status == qh.Status.EINVAL
    fp = d["frag_ptr"].clone()
    fp[3] = fp[4] + 1                                    # frag_ptr decreases at fragment 3
    with pytest.raises(qh.QhapError) as e:
        qh.build_graph(fp, d["snp"], d["allele"], d["phred"], d["init_h1"])
    assert e.value.status == qh.Status.EINVAL
    for i, v in ((0, 1), (-1, -1)):                      # frag_ptr[0] != 0; a negative count
        fp = d["frag_ptr"].clone()
        fp[i] = v
        with pytest.raises(qh.QhapError) as e:
            qh.build_graph(fp, d["snp"], d["allele"], d["phred"], d["init_h1"])
        assert e.value.status == qh.Status.EINVAL
    n = g.info()["n"]
    x = torch.zeros((n, 16), device="cuda")
    x[3, 2] = float("nan")
    y = torch.zeros((n, 16), device="cuda")
    with pytest.raises(qh.QhapError) as e:
        qh.bsb_solve(g, 16, 1, init=False, x=x, y=y, step_begin=1, step_end=1)
    assert e.value.status == qh.Status.ENUMERIC


@pytest.mark.parametrize("kind,dtype", [("read_signed", "fp8"), ("snp_llr", "bf16")])
def test_device_memory_cap(kind, dtype):
    """max_device_bytes: a graph that fits is built unchanged at exactly its footprint; one
    byte less, or a tiny cap, fails with ENOMEM and keeps nothing; a negative cap is EINVAL."""
    w = synth.snp_porec(43, n_snp=600, n_edges=500, zipf_s=1.0) if kind == "snp_llr" else synth.read_tiny()
    d = device_reads(w)
    # (deterministic SNP weights: with FP64 atomics a cancelling entry may come out as an
    # exact zero in one build and as residue in the next, which changes nnz and the footprint)
    kw = dict(kind=kind, dtype=dtype, alpha=d["alpha"], band_limit=100 if kind == "snp_llr" else 0,
              deterministic=kind == "snp_llr")
    g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], **kw)
    need = g.info()["device_bytes"]
    assert need > 0
    g2 = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], max_device_bytes=need, **kw)
    assert g2.info()["device_bytes"] == need
    assert torch.equal(g2.export_rows(0, g.info()["n"]), g.export_rows(0, g.info()["n"]))
    for cap, status in ((need - 1, qh.Status.ENOMEM), (4096, qh.Status.ENOMEM), (-1, qh.Status.EINVAL)):
        with pytest.raises(qh.QhapError) as e:
            qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], max_device_bytes=cap,
                           **kw)
        assert e.value.status == status, cap
    # the library still works after the refusals
    r = qh.bsb_solve(g, 16 if kind != "snp_llr" else 64, 50, seed=1)
    assert np.isfinite(float(cpu(r["best_cut"])[0]))


@pytest.mark.parametrize("kind,dtype", [("read_signed", "f16"), ("snp_llr", "f32")])
def test_best_energy_matches_eq5(kind, dtype):
    """best_energy is the Ising energy E(s) = -1/2 s'Js of the returned spins (Eq. 5), here
    evaluated by the oracle's dense J in FP64; total_weight is -1/2 sum J."""
    w = synth.read_small(13, n_snp=300, n_reads=150, span=(20, 60)) if kind == "read_signed" else \
        synth.snp_small(14, n_snp=800)
    g = gpu_graph(w, kind, dtype)
    J = oracle_graph(w, kind).dense()
    assert g.info()["total_weight"] == pytest.approx(-0.5 * J.sum(), rel=1e-12)
    r = qh.bsb_solve(g, 32, 300, seed=4)
    s = cpu(r["best_spins"]).astype(np.float64)
    e = -0.5 * s @ J @ s
    assert float(cpu(r["best_energy"])[0]) == pytest.approx(e, rel=1e-10, abs=1e-9)
    assert float(cpu(r["best_energy"])[0]) == pytest.approx(g.info()["total_weight"] - 2 * float(cpu(r["best_cut"])[0]),
                                                            rel=1e-14, abs=1e-12)


def test_energy_trace_resumes_one_schedule():
    """energy_trace is one solve read out every 100 steps: its last row is the energy (Eq. 5)
    of every replica after a straight solve of the same schedule, bit for bit, and its first
    rows match the oracle's energies of the same steps' signs."""
    w = synth.read_tiny()
    g = gpu_graph(w, "read_signed", "f32")
    tr = qh.energy_trace(g, 16, 300, 100, seed=7)
    assert tr["steps"] == [100, 200, 300] and tr["energy"].shape == (3, 16)
    r = qh.bsb_solve(g, 16, 300, seed=7, greedy=False, plan=1)
    W = g.info()["total_weight"]
    assert np.array_equal(tr["energy"][-1], W - 2.0 * cpu(r["cuts"]))
    go = oracle_graph(w)
    J = go.dense()
    x, y = oracle.init_state(7, go.n, 16)
    oracle.bsb_run(go, x, y, oracle.pump_linear(300), 0.5, oracle.c0(go), 1.0, 0, 100)
    s = np.where(x >= 0, 1.0, -1.0)
    e = -0.5 * np.einsum("ir,ij,jr->r", s, J, s)
    assert np.allclose(tr["energy"][0], e, rtol=0, atol=1e-9)
    assert tr["best"][-1] <= tr["best"][0]


EVAL_CASES = {
    # (workload, kind, dtype, R, steps, m, plan)
    "read_f32": (lambda: synth.read_tiny(), "read_signed", "f32", 16, 300, 70, 1),
    "read_f16_persistent": (lambda: synth.read_mhc(seed=78, n_snp=1500, n_reads=1000, region=500_000),
                            "read_signed", "f16", 64, 200, 45, 2),
    "read_fp8_step": (lambda: synth.read_small(16, n_snp=300, n_reads=140), "read_signed", "fp8", 32, 150, 40, 1),
    "snp_f16_band": (lambda: synth.snp_small(19, n_snp=1200), "snp_llr", "f16", 64, 200, 60, 4),
    "porec_bf16": (lambda: synth.snp_porec(45, n_snp=2000, n_edges=2500, zipf_s=1.0), "snp_llr", "bf16", 64, 120,
                   50, 0),
}


@pytest.mark.parametrize("case", list(EVAL_CASES))
def test_eval_every_matches_the_readout_definition(case):
    """Readouts every m steps (eval_every): the trajectory is the straight solve's (final
    state bit-identical); the energy row of readout e is -1/2 s'Js (Eq. 5, oracle's FP64
    dense J) of the signs after that readout's step, which a straight solve ending there
    returns; best_spins (no greedy) and selected_cut are the oracle's best-so-far merge of
    those readouts' signs (merge_best), exactly."""
    make, kind, dtype, R, steps, m, plan = EVAL_CASES[case]
    w = make()
    g = gpu_graph(w, kind, dtype, band_limit=64 if case.startswith("porec") else 0)
    n = g.info()["n"]
    go = oracle_graph(w, kind)
    J = go.dense()
    comp, nc = oracle.components(go)
    xe = torch.empty((n, R), dtype=torch.float32, device="cuda")
    r = qh.bsb_solve(g, R, steps, seed=9, greedy=False, plan=plan, eval_every=m, energy=True, x=xe,
                     per_component=True)
    marks = list(range(m, steps, m)) + [steps]
    E = cpu(r["energy"])
    assert E.shape == (len(marks), R)
    sets = []
    for e, k1 in enumerate(marks):
        xs = torch.empty((n, R), dtype=torch.float32, device="cuda")
        rs = qh.bsb_solve(g, R, steps, seed=9, greedy=False, plan=plan, step_end=k1, all_spins=True, x=xs)
        sp = cpu(rs["all_spins"])
        sets.append(sp)
        sd = sp.astype(np.float64)
        ref = -0.5 * np.einsum("ir,ij,jr->r", sd, J, sd)
        scale = max(1.0, float(np.abs(J).sum()))
        assert np.allclose(E[e], ref, rtol=0, atol=1e-12 * scale), e
        if k1 == steps:
            assert torch.equal(xs, xe)          # readouts do not disturb the trajectory
    best, best_c, best_r = oracle.merge_best(go, comp, nc, sets)
    assert np.array_equal(cpu(r["best_spins"]), best)
    assert np.array_equal(cpu(r["best_replica"]), best_r)
    assert float(cpu(r["selected_cut"])[0]) == pytest.approx(float(best_c.sum()), rel=1e-12, abs=1e-9)
    W = g.info()["total_weight"]
    assert np.array_equal(E[-1], W - 2.0 * cpu(r["cuts"]))


def test_eval_every_rejects_bad_combinations():
    g = gpu_graph(synth.read_tiny(), "read_signed", "f32")
    for kw in (dict(eval_every=-1), dict(eval_every=10, use_graph=True), dict(eval_every=10, readout=False)):
        with pytest.raises(qh.QhapError) as e:
            qh.bsb_solve(g, 16, 50, **kw)
        assert e.value.status == qh.Status.EINVAL, kw


def test_eval_every_whole_solve_tracks_the_oracle():
    """A whole solve with readouts every 100 steps against the oracle's at the same schedule
    (FP32 read graph): best cut within 0.1 %, and never below the plain solve's selected cut."""
    w = synth.read_small(13, n_snp=300, n_reads=150, span=(20, 60))
    g = gpu_graph(w, "read_signed", "f32")
    go = oracle_graph(w)
    r = qh.bsb_solve(g, 32, 500, seed=4, eval_every=100)
    ro = oracle.solve(go, 32, 500, 0.5, seed=4, integer=True, eval_every=100)
    cut = float(cpu(r["best_cut"])[0])
    assert (ro["best_cut"] - cut) / abs(ro["best_cut"]) <= 1e-3
    rp = qh.bsb_solve(g, 32, 500, seed=4)
    assert float(cpu(r["selected_cut"])[0]) >= float(cpu(rp["selected_cut"])[0])


def test_flip_crossing_refreshes_total_weight():
    """Eq. (15) flips the sign of every crossing edge: total_weight (-1/2 sum J) follows, and
    best_energy of a solve on the flipped graph is -1/2 s'Js with the flipped J (the
    oracle's flip_crossing)."""
    w = synth.snp_small(22, n_snp=1000)
    g = gpu_graph(w, "snp_llr", "f32")
    go = oracle_graph(w, "snp_llr")
    rng = np.random.default_rng(3)
    s = np.where(rng.random(go.n) < 0.5, 1, -1).astype(np.int8)
    qh.flip_crossing(g, qh.to_device(s))
    Jf = oracle.flip_crossing(go, s).dense()
    assert g.info()["total_weight"] == pytest.approx(-0.5 * Jf.sum(), rel=1e-12, abs=1e-9)
    r = qh.bsb_solve(g, 64, 200, seed=6)
    b = cpu(r["best_spins"]).astype(np.float64)
    assert float(cpu(r["best_energy"])[0]) == pytest.approx(-0.5 * b @ Jf @ b, rel=1e-10, abs=1e-8)


def test_deterministic_snp_build():
    """deterministic = 1: fixed-point sums give the same SNP weights bit for bit on every
    build (and so the same solve), within 2^-40 per Eq. (14) term of the oracle's FP64 sum."""
    w = synth.snp_porec(43, n_snp=1200, n_edges=1500, zipf_s=1.0)
    d = device_reads(w)
    kw = dict(kind="snp_llr", dtype="bf16", alpha=d["alpha"], band_limit=100, deterministic=True)
    g1 = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], **kw)
    g2 = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], **kw)
    n = g1.info()["n"]
    assert g1.info()["longrange_nnz"] > 0
    m1, m2 = g1.export_rows(0, n), g2.export_rows(0, n)
    assert torch.equal(m1, m2)
    assert torch.equal(g1.export_rows(0, n, stored=True), g2.export_rows(0, n, stored=True))
    J = oracle_graph(w, "snp_llr").dense()
    diff = np.abs(cpu(m1) - J)
    # each entry sums at most a few hundred terms, each rounded by at most 2^-41; entries
    # that are not FP64 cancellation residue keep their place
    assert diff.max() <= 1e3 * 2.0 ** -41
    assert np.all(cpu(m1)[np.abs(J) > 1e-9] != 0)
    r1 = qh.bsb_solve(g1, 64, 200, seed=2)
    r2 = qh.bsb_solve(g2, 64, 200, seed=2)
    assert torch.equal(r1["best_spins"], r2["best_spins"]) and torch.equal(r1["best_cut"], r2["best_cut"])


def test_autotune_cache_and_explicit_options(tmp_path):
    """qh_autotune on its own: the chosen options, passed explicitly, run the tuned kernels
    with the plan-0 solve's results bit for bit; the cache file holds one JSON line per
    tuning and load_tuned finds the options again by graph shape and replica count."""
    path = str(tmp_path / "tune.jsonl")
    wm = synth.read_mhc(seed=78, n_snp=1500, n_reads=1000, region=500_000)
    cases = [(gpu_graph(wm, "read_signed", "f16"), 64, (1, 2)),
             (gpu_graph(synth.snp_small(14, n_snp=1500), "snp_llr", "f16"), 64, (3, 4, 5))]
    for g, R, plans in cases:
        ch = qh.autotune(g, R, 200, cache_path=path)
        assert ch["plan"] in plans and ch["us_per_step"][0] > 0.0
        opts = {k: ch[k] for k in ("plan", "replica_tile", "tiles_in_flight", "persistent_sync")}
        n = g.info()["n"]
        xa = torch.empty((n, R), dtype=torch.float32, device="cuda")
        xb = torch.empty_like(xa)
        ra = qh.bsb_solve(g, R, 200, seed=3, x=xa)
        rb = qh.bsb_solve(g, R, 200, seed=3, x=xb, **opts)
        assert torch.equal(xa, xb) and torch.equal(ra["best_cut"], rb["best_cut"])
        info = g.plan_info(R)
        if ch["plan"] == 2:
            assert info["plan_used"] == 2 and info["persistent_sync"] == ch["persistent_sync"]
        elif ch["plan"] == 1:
            assert info["plan_used"] == 1 and info["replica_tile"] == ch["replica_tile"]
        else:
            assert info["skyline_kernel"] == ch["plan"]
        assert qh.load_tuned(path, g, R) == opts
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and all(json.loads(line)["replicas"] == 64 for line in lines)
    assert qh.load_tuned(path, cases[0][0], 128) is None


def test_degenerate_graphs():
    # one fragment: no edges, no components; zero fragments
    for nf in (1, 0):
        w = synth.read_small(25, n_snp=50, n_reads=max(nf, 1), span=(5, 10))
        fp = w.frag_ptr[: nf + 1].copy()
        snp = w.snp[: fp[-1]].copy()
        d = dict(frag_ptr=qh.to_device(fp), snp=qh.to_device(snp), allele=qh.to_device(w.allele[: fp[-1]].copy()),
                 phred=qh.to_device(w.phred[: fp[-1]].copy()), init_h1=qh.to_device(w.init_h1))
        g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"])
        inf = g.info()
        assert inf["n"] == nf and inf["n_comp"] == 0 and inf["nnz"] == 0
        r = qh.bsb_solve(g, 16, 20)
        assert float(cpu(r["best_cut"])[0]) == 0.0
        h1, blk = qh.phase(g, r["best_spins"] if nf else torch.ones(1, dtype=torch.int8, device="cuda"))
        assert np.all(cpu(h1) == -1)


def test_release_cached_memory():
    """A freed graph's device blocks stay cached (a rebuild reuses them) until
    qh_release_cached_memory hands them back; a second release finds nothing, and the
    library allocates afresh afterwards."""
    w = synth.read_tiny()
    d = device_reads(w)
    torch.cuda.synchronize()
    qh.release_cached_memory()

    def build():
        return qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="read_signed",
                              dtype="fp8")

    g = build()
    need = g.info()["device_bytes"]
    ref = qh.bsb_solve(g, 16, 50, seed=3)["best_cut"].cpu()
    g.free()
    assert qh.release_cached_memory() >= need
    assert qh.release_cached_memory() == 0
    g = build()
    assert torch.equal(qh.bsb_solve(g, 16, 50, seed=3)["best_cut"].cpu(), ref)
    # blocks in use stay: a live graph solves the same after another one's blocks are released
    g2 = build()
    g2.free()
    assert qh.release_cached_memory() >= need
    assert torch.equal(qh.bsb_solve(g, 16, 50, seed=3)["best_cut"].cpu(), ref)
    g.free()

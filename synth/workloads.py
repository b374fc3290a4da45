"""Seeded synthetic stand-ins for the paper's sequencing workloads.

The paper measures on GIAB HG002 reads (CycloneSEQ / HiFi / ONT / Pore-C) in the
MHC region and on chromosome 22 (Results, "Performance" and "Chromosome-scale
phasing").  Those data are not available, so every workload here is drawn from
a common model with the shapes of those inputs:

* a planted haplotype ``truth`` ~ Bernoulli(1/2) per SNP (haplotype 2 is its
  complement);
* each read comes from either planted haplotype with probability 1/2;
* every SNP inside a read's genomic span is observed;
* observed alleles flip i.i.d. at the stated error rate;
* Phred qualities are independent uniform integers in the stated range;
* reads with fewer than 2 SNPs are dropped;
* the initial haplotype assignment ``init_h1`` is a random draw per SNP
  (Methods, "Haplotype initialization").

Alleles are 0 (reference) / 1 (alternative).  Fragments are stored as CSR:
``frag_ptr[F+1]`` (int64), ``snp`` (int32, strictly ascending inside a
fragment), ``allele`` (uint8), ``phred`` (uint8); ``alpha`` (float64 per
fragment) is the Pore-C down-weighting factor (1.0 for ordinary reads).
Fragments are sorted by their first SNP, which is the vertex order of the
read-based graph.

Every generator has an error-free twin (``error=0``) whose Max-Cut optimum is
known in closed form.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    n_snp: int
    pos: np.ndarray          # int64 [n_snp], genomic coordinate (bp)
    truth: np.ndarray        # uint8 [n_snp], allele carried by planted haplotype 1
    init_h1: np.ndarray      # uint8 [n_snp], allele assigned to H1 by the random init
    frag_ptr: np.ndarray     # int64 [F+1]
    snp: np.ndarray          # int32 [nobs]
    allele: np.ndarray       # uint8 [nobs]
    phred: np.ndarray        # uint8 [nobs]
    alpha: np.ndarray        # float64 [F]
    origin: np.ndarray       # uint8 [F], planted haplotype each fragment came from
    solve: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def n_frag(self) -> int:
        return int(self.frag_ptr.shape[0] - 1)

    @property
    def n_obs(self) -> int:
        return int(self.snp.shape[0])

    def arrays(self) -> Dict[str, np.ndarray]:
        return dict(frag_ptr=self.frag_ptr, snp=self.snp, allele=self.allele,
                    phred=self.phred, alpha=self.alpha, init_h1=self.init_h1)


@dataclasses.dataclass
class Batch:
    name: str
    blocks: List[Workload]
    solve: Dict[str, object] = dataclasses.field(default_factory=dict)


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def _snps(rng: np.random.Generator, n_snp: int, gap_mean: float):
    gaps = rng.exponential(gap_mean, size=n_snp)
    pos = np.floor(np.cumsum(gaps)).astype(np.int64)
    # strictly increasing coordinates
    pos = pos + np.arange(n_snp, dtype=np.int64)
    truth = rng.integers(0, 2, size=n_snp, dtype=np.uint8)
    init_h1 = rng.integers(0, 2, size=n_snp, dtype=np.uint8)
    return pos, truth, init_h1


def _csr_from_runs(first: np.ndarray, count: np.ndarray):
    """Fragments observing the consecutive SNP runs [first, first+count)."""
    count = count.astype(np.int64)
    frag_ptr = np.zeros(first.shape[0] + 1, dtype=np.int64)
    np.cumsum(count, out=frag_ptr[1:])
    total = int(frag_ptr[-1])
    base = np.repeat(first.astype(np.int64) - frag_ptr[:-1], count)
    snp = (base + np.arange(total, dtype=np.int64)).astype(np.int32)
    return frag_ptr, snp


def _observe(rng, frag_ptr, snp, truth, err_per_frag, q_lo, q_hi):
    nfrag = frag_ptr.shape[0] - 1
    counts = np.diff(frag_ptr)
    origin = rng.integers(0, 2, size=nfrag, dtype=np.uint8)
    true_allele = truth[snp] ^ np.repeat(origin, counts)
    err = np.repeat(np.asarray(err_per_frag, dtype=np.float64), counts)
    flip = (rng.random(snp.shape[0]) < err).astype(np.uint8)
    allele = (true_allele ^ flip).astype(np.uint8)
    phred = rng.integers(q_lo, q_hi + 1, size=snp.shape[0], dtype=np.int64).astype(np.uint8)
    return allele, phred, origin


def _reads_by_span(rng, pos, n_reads, length_sampler: Callable, region: int,
                   max_tries: int = 50):
    """Reads with a genomic span; keep those with >= 2 SNPs until n_reads."""
    firsts, counts, starts = [], [], []
    kept = 0
    for _ in range(max_tries):
        need = n_reads - kept
        if need <= 0:
            break
        m = int(need * 1.2) + 16
        ln = np.minimum(length_sampler(m), region - 1).astype(np.int64)
        st = (rng.random(m) * (region - ln)).astype(np.int64)
        a = np.searchsorted(pos, st, side="left")
        b = np.searchsorted(pos, st + ln, side="left")
        c = b - a
        ok = c >= 2
        a, c, st = a[ok], c[ok], st[ok]
        take = min(need, a.shape[0])
        firsts.append(a[:take]); counts.append(c[:take]); starts.append(st[:take])
        kept += take
    first = np.concatenate(firsts)
    count = np.concatenate(counts)
    start = np.concatenate(starts)
    order = np.lexsort((count, start, first))
    return first[order], count[order]


def _assemble(name, pos, truth, init_h1, frag_ptr, snp, allele, phred, alpha, origin, solve):
    return Workload(name=name, n_snp=int(pos.shape[0]), pos=pos, truth=truth, init_h1=init_h1,
                    frag_ptr=frag_ptr, snp=snp, allele=allele, phred=phred,
                    alpha=alpha, origin=origin, solve=dict(solve))


# ----------------------------------------------------------------------------
# read-based workloads (vertices = reads)
# ----------------------------------------------------------------------------

def read_small(seed: int, n_snp: int = 200, n_reads: int = 60, span=(20, 60),
               error: float = 0.05, q=(10, 40), name: str = "read_small") -> Workload:
    """Reads covering U{span} consecutive SNPs from a uniform start."""
    rng = np.random.default_rng(seed)
    pos, truth, init_h1 = _snps(rng, n_snp, 330.0)
    lo, hi = span
    hi = min(hi, n_snp)
    lo = min(lo, hi)
    count = rng.integers(lo, hi + 1, size=n_reads)
    first = (rng.random(n_reads) * (n_snp - count + 1)).astype(np.int64)
    order = np.lexsort((count, first))
    first, count = first[order], count[order]
    frag_ptr, snp = _csr_from_runs(first, count)
    allele, phred, origin = _observe(rng, frag_ptr, snp, truth, np.full(n_reads, error), q[0], q[1])
    alpha = np.ones(n_reads, dtype=np.float64)
    solve = dict(kind="read_signed", storage="dense", dtype="f32", replicas=16, steps=1000,
                 dt=0.5)
    return _assemble(name, pos, truth, init_h1, frag_ptr, snp, allele, phred, alpha, origin, solve)


def read_tiny(seed: int = 1000, error: float = 0.05) -> Workload:
    """200 het SNPs, 60 reads of 20-60 consecutive SNPs, 5% flips, Phred 10-40."""
    return read_small(seed, 200, 60, (20, 60), error, (10, 40), name="read_tiny")


def read_mhc(seed: int = 2000, n_snp: int = 12000, n_reads: int = 8000,
             region: int = 4_000_000, read_mean: float = 15000.0, sigma_log: float = 0.5,
             error_range=(0.01, 0.08), error: Optional[float] = None,
             name: str = "read_mhc") -> Workload:
    """MHC-scale read graph: exponential SNP gaps (mean region/n_snp), lognormal reads.

    ``error`` overrides the per-read error draw (0.0 gives the error-free twin).
    """
    rng = np.random.default_rng(seed)
    pos, truth, init_h1 = _snps(rng, n_snp, region / n_snp)
    region = max(region, int(pos[-1]) + 1)
    mu = np.log(read_mean) - 0.5 * sigma_log ** 2
    first, count = _reads_by_span(rng, pos, n_reads,
                                  lambda m: rng.lognormal(mu, sigma_log, size=m), region)
    frag_ptr, snp = _csr_from_runs(first, count)
    nfrag = first.shape[0]
    if error is None:
        err = rng.uniform(error_range[0], error_range[1], size=nfrag)
    else:
        err = np.full(nfrag, float(error))
    allele, phred, origin = _observe(rng, frag_ptr, snp, truth, err, 10, 40)
    alpha = np.ones(nfrag, dtype=np.float64)
    solve = dict(kind="read_signed", storage="dense", dtype="f16", replicas=256, steps=2000,
                 dt=0.5)
    return _assemble(name, pos, truth, init_h1, frag_ptr, snp, allele, phred, alpha, origin, solve)


# ----------------------------------------------------------------------------
# SNP-based workloads (vertices = SNPs)
# ----------------------------------------------------------------------------

# Mean SNP spacing of the chromosome-scale model: 1,430 bp gives 40 linked SNPs per SNP on
# average (10.0 M couplings over 250,000 SNPs) with 30x of 20 kb reads at linkage depth 10/10.
CHROM_GAP_BP = 1430.0


def snp_small(seed: int, n_snp: int = 2000, coverage: float = 30.0, read_mean: float = 20000.0,
              sigma_log: float = 0.3, gap_mean: float = 1000.0, error: float = 0.06,
              q=(7, 40), name: str = "snp_small") -> Workload:
    """Chromosome-style SNP workload scaled to n_snp SNPs."""
    rng = np.random.default_rng(seed)
    pos, truth, init_h1 = _snps(rng, n_snp, gap_mean)
    region = int(pos[-1]) + 1
    n_reads = max(2, int(round(coverage * region / read_mean)))
    mu = np.log(read_mean) - 0.5 * sigma_log ** 2
    first, count = _reads_by_span(rng, pos, n_reads,
                                  lambda m: rng.lognormal(mu, sigma_log, size=m), region)
    frag_ptr, snp = _csr_from_runs(first, count)
    nfrag = first.shape[0]
    allele, phred, origin = _observe(rng, frag_ptr, snp, truth, np.full(nfrag, error), q[0], q[1])
    alpha = np.ones(nfrag, dtype=np.float64)
    solve = dict(kind="snp_llr", storage="skyline", dtype="f32", replicas=64, steps=3000,
                 dt=0.5, linkage_k=10)
    return _assemble(name, pos, truth, init_h1, frag_ptr, snp, allele, phred, alpha, origin, solve)


def snp_chrom(seed: int = 3000, n_snp: int = 250_000, error: float = 0.06) -> Workload:
    """250,000 SNPs, 1.43 kb mean gaps (40 couplings per SNP), 30x of lognormal 20 kb reads,
    Phred 7-40."""
    w = snp_small(seed, n_snp=n_snp, gap_mean=CHROM_GAP_BP, error=error, name="snp_chrom")
    return w


def _add_porec(rng, w: Workload, n_edges: int, zipf_s: float, d_range, alpha_range,
               error: float, q) -> Workload:
    """Append pairwise Pore-C fragments until ``n_edges`` distinct SNP pairs exist.

    Contact distance has density proportional to d^-1.1 on d_range; the anchor SNP is
    drawn with a Zipf-like propensity (rank^-zipf_s over a random ranking) so that a
    few hub SNPs collect thousands of contacts.
    """
    n = w.n_snp
    pos = w.pos
    region = int(pos[-1]) + 1
    rank = np.empty(n, dtype=np.float64)
    rank[rng.permutation(n)] = np.arange(1, n + 1, dtype=np.float64)
    prop = rank ** (-zipf_s)
    cdf = np.cumsum(prop)
    cdf /= cdf[-1]
    a, b = float(d_range[0]), float(d_range[1])
    ea, eb = a ** -0.1, b ** -0.1
    keys_all, us, vs = [], [], []
    n_distinct = 0
    seen = None
    while n_distinct < n_edges:
        m = max(200_000, int((n_edges - n_distinct) * 1.5))
        u = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1)
        d = (ea + rng.random(m) * (eb - ea)) ** -10.0
        sgn = np.where(rng.random(m) < 0.5, -1.0, 1.0)
        tgt = pos[u] + sgn * d
        ok = (tgt >= 0) & (tgt < region)
        u, tgt = u[ok], tgt[ok].astype(np.int64)
        v = np.searchsorted(pos, tgt, side="left")
        v = np.minimum(v, n - 1)
        ok = v != u
        u, v = u[ok], v[ok]
        lo = np.minimum(u, v).astype(np.int64)
        hi = np.maximum(u, v).astype(np.int64)
        keys = lo * n + hi
        keys_all.append(keys); us.append(lo); vs.append(hi)
        allk = np.concatenate(keys_all)
        uniq, first_idx = np.unique(allk, return_index=True)
        n_distinct = uniq.shape[0]
        seen = (uniq, first_idx)
    allk = np.concatenate(keys_all)
    lo = np.concatenate(us)
    hi = np.concatenate(vs)
    uniq, first_idx = seen
    # keep every sampled fragment up to the first occurrence of the n_edges-th distinct pair
    cut = int(np.sort(first_idx)[n_edges - 1]) + 1
    lo, hi = lo[:cut], hi[:cut]
    m = lo.shape[0]
    pf_ptr = np.arange(0, 2 * m + 1, 2, dtype=np.int64)
    psnp = np.stack([lo, hi], axis=1).reshape(-1).astype(np.int32)
    allele, phred, origin = _observe(rng, pf_ptr, psnp, w.truth, np.full(m, error), q[0], q[1])
    palpha = rng.uniform(alpha_range[0], alpha_range[1], size=m)
    frag_ptr = np.concatenate([w.frag_ptr, w.frag_ptr[-1] + pf_ptr[1:]])
    return _assemble(w.name, w.pos, w.truth, w.init_h1, frag_ptr,
                     np.concatenate([w.snp, psnp]), np.concatenate([w.allele, allele]),
                     np.concatenate([w.phred, phred]), np.concatenate([w.alpha, palpha]),
                     np.concatenate([w.origin, origin]), w.solve)


def snp_porec(seed: int = 4000, n_snp: int = 250_000, n_edges: int = 600_000,
              error: float = 0.06, zipf_s: float = 0.6) -> Workload:
    """Chromosome workload plus pairwise Pore-C contacts (100 kb - 100 Mb)."""
    base = snp_small(seed, n_snp=n_snp, gap_mean=CHROM_GAP_BP, error=error, name="snp_porec")
    rng = np.random.default_rng(seed + 7)
    w = _add_porec(rng, base, n_edges, zipf_s, (1e5, 1e8), (0.1, 0.5), error, (7, 40))
    w.solve.update(dict(storage="skyline_long", dtype="bf16", replicas=64, steps=4000))
    return w


# ----------------------------------------------------------------------------
# batched blocks
# ----------------------------------------------------------------------------

def batched_blocks(seed: int = 5000, n_blocks: int = 3000, n_lo: int = 50, n_hi: int = 5000,
                   error_read: float = 0.05, error_snp: float = 0.06) -> Batch:
    """Independent phasing blocks with log-uniform node counts.

    Even blocks are dense read graphs (reads of 20-60 consecutive SNPs over 200 SNPs),
    odd blocks are SNP graphs of the chromosome model scaled to the block's node count.
    """
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    sizes = np.round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=n_blocks))).astype(int)
    child = ss.spawn(n_blocks)
    blocks = []
    for b in range(n_blocks):
        bseed = int(child[b].generate_state(1)[0])
        nb = int(sizes[b])
        if b % 2 == 0:
            blk = read_small(bseed, n_snp=200, n_reads=nb, span=(20, 60), error=error_read,
                             name=f"block{b}_read")
            blk.solve.update(dict(dtype="fp8", replicas=32, steps=500))
        else:
            blk = snp_small(bseed, n_snp=nb, gap_mean=CHROM_GAP_BP, error=error_snp, name=f"block{b}_snp")
            blk.solve.update(dict(dtype="bf16", replicas=32, steps=500))
        blocks.append(blk)
    return Batch(name="batched", blocks=blocks,
                 solve=dict(replicas=32, steps=500, dt=0.5))


def workload_hash(w: Workload) -> str:
    """SHA-256 of a workload's input arrays (fragments, qualities, factors, initial and
    planted haplotypes): stored next to reference results so that a change of the generator
    is noticed."""
    import hashlib
    h = hashlib.sha256()
    for a in (w.frag_ptr, w.snp, w.allele, w.phred, w.alpha, w.init_h1, w.truth):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def batch_hash(batch: Batch) -> str:
    """SHA-256 over the workload hashes of a batch's blocks, in order."""
    import hashlib
    h = hashlib.sha256()
    for w in batch.blocks:
        h.update(workload_hash(w).encode())
    return h.hexdigest()


def stratified_subset(batch: Batch, stride: int = 20) -> List[int]:
    """Block indices of a stratified sample of a batched workload: within each block kind
    (even blocks dense read graphs, odd blocks SNP graphs) the blocks are ranked by vertex
    count (reads for read blocks, SNPs for SNP blocks) and every stride-th is taken from rank
    stride // 2 on, so the sample spans the whole size range of both kinds."""
    out: List[int] = []
    for parity in (0, 1):
        idx = [b for b in range(len(batch.blocks)) if b % 2 == parity]
        idx.sort(key=lambda b: (batch.blocks[b].n_frag if parity == 0 else batch.blocks[b].n_snp, b))
        out += idx[stride // 2::stride]
    return sorted(out)


CONFIGS = {
    "read_tiny": read_tiny,
    "read_mhc": read_mhc,
    "snp_chrom": snp_chrom,
    "snp_porec": snp_porec,
    "batched": batched_blocks,
}


def by_name(name: str, **kw):
    return CONFIGS[name](**kw)

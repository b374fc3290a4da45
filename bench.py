"""Benchmark: bSB edge-updates/s of the phasing hot path on one MI355X.

Default workload (the line of record): ``batched`` -- 3,000 independent phasing blocks with
log-uniform sizes of 50-5,000 vertices, even blocks dense read graphs stored as FP8 with
per-row scales, odd blocks SNP graphs stored as BF16 (skyline band), R = 32 replicas, 500
bSB steps (the paper's count for graphs below 5,000 nodes), dt = 0.5, linear pump, c0 auto
per block.  One benchmark step = one batched solve of all blocks: seeded initial state,
500 fused bSB steps of every block (the per-step plan replayed from a captured hipGraph),
FP64 cuts of every replica and component, per-component selection and the greedy pass.
The graphs are built before the timed region (the metric counts solver work; graph
construction and time-to-phase are reported beside it).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|read_mhc|snp_chrom|snp_porec]
                    [--no-cpu-baseline] [--no-extras]

Prints one JSON line.  ``--workload read_mhc | snp_chrom | snp_porec`` measure the other
configurations (the MHC-scale dense read graph, the chromosome SNP graph, the SNP graph with
Pore-C contacts) with the same fields.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bSB edge-updates/s (nnz×replicas×steps) at ≤0.1% cut gap vs FP64 oracle"
PEAK_HBM_GBS = 8000.0
# dense MFMA peaks (TFLOP/s); FP8 tiles are expanded to binary16 and multiplied on the f16 MFMA
PEAK_TFLOPS = {"f16": 2500.0, "bf16": 2500.0, "fp8": 2500.0, "f32": 157.3}
GOLDEN = os.path.join(ROOT, "tests", "golden")
COPY_BYTES = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=["batched", "read_mhc", "snp_chrom", "snp_porec"])
    ap.add_argument("--dtype", default=None, choices=["f32", "f16", "bf16", "fp8"],
                    help="read_mhc / snp_*: storage of J (default f16, f16, bf16); batched blocks carry their own")
    ap.add_argument("--graph", type=int, default=None,
                    help="1: replay the step loop from a captured hipGraph (default for batched, whose graphs "
                         "are built once); 0: direct launches (default for the others, which build a fresh "
                         "graph per job)")
    ap.add_argument("--plan", type=int, default=0,
                    help="0 auto; batched: 1 per-step, 2 whole-block; read_mhc: 1 per-step, 2 persistent")
    ap.add_argument("--persistent-sync", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--build-threads", type=int, default=0,
                    help="host threads of the batch's graph build (qh_build_graphs; 0 = the library's 8)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the time-to-phase and plain-FP32 measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 1 GiB (3 times): the reference kernel that scales "
                         "the FETCH_SIZE / WRITE_SIZE counters to HBM bytes")
    return ap.parse_args()


def calibrate_copy():
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes_read=COPY_BYTES, copy_bytes_written=COPY_BYTES, launches=3)), flush=True)


# ----------------------------------------------------------------------------- helpers

def _section(src, begin, end):
    a = src.index(begin)
    return src[a:src.index(end, a + len(begin))]


def kernel_source_hash(kernel):
    """Hash of the source a step kernel is compiled from (its section of bsb.hip, the shared
    update helpers, formats.h), so that counter summaries taken on older code are not used."""
    csrc = os.path.join(ROOT, "paper_2603_25762_amd", "csrc")
    h = hashlib.sha256()
    if kernel.startswith("k_dense_persistent"):
        h.update(open(os.path.join(csrc, "persistent_kernel.h"), "rb").read())
    else:
        src = open(os.path.join(csrc, "bsb.hip")).read()
        h.update(_section(src, "struct StepArgs", "// skyline band + long-range CSR").encode())
        if kernel.startswith("k_band_step") or kernel.startswith("k_lr_packets") or "band" in kernel:
            h.update(_section(src, "// skyline band + long-range CSR", "// batched blocks:").encode())
        if kernel.startswith("k_batched_rowtile"):
            # the whole-row-tile product and its kernel (the launch code around them is not part)
            h.update(_section(src, "// Product of S 16-row strips", "__global__ __launch_bounds__(256) void "
                                                                      "k_batched_init").encode())
        elif kernel.startswith("k_batched"):
            h.update(_section(src, "// batched blocks:", "// host orchestration").encode())
    h.update(open(os.path.join(csrc, "formats.h"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries (the `traffic:`
    lines of profiles/*.md), or None when none covers it or its source changed since."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        vals = {}
        for line in open(path):
            if line.startswith("traffic:"):
                k, _, v = line[len("traffic:"):].strip().partition("=")
                vals[k.strip()] = v.strip()
        if vals.get("kernel") == kernel and vals.get("source_sha") == kernel_source_hash(kernel):
            return int(float(vals["hbm_bytes_per_launch"]))
    return None


def roofline(bound, bytes_, flops, launch_us, dtype, kernel, **extra):
    """achieved / peak for the dominant kernel: algorithmic bytes (hbm) or flops (mfma) of one
    launch over its measured average duration."""
    gbs = bytes_ / (launch_us * 1e-6) / 1e9
    tfs = flops / (launch_us * 1e-6) / 1e12
    hbm_frac, mfma_frac = gbs / PEAK_HBM_GBS, tfs / PEAK_TFLOPS[dtype]
    if bound == "hbm":
        r = dict(bound="hbm", achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s", frac=round(hbm_frac, 4))
    else:
        r = dict(bound="mfma", achieved=round(tfs, 2), peak=PEAK_TFLOPS[dtype], unit="TFLOP/s",
                 frac=round(mfma_frac, 4))
    r["traffic"] = measured_traffic(kernel)
    r.update(kernel=kernel, launch_us=round(launch_us, 3), bytes_per_launch=int(bytes_), flop_per_launch=flops,
             hbm_frac=round(hbm_frac, 4), mfma_frac=round(mfma_frac, 4), source_sha=kernel_source_hash(kernel))
    r.update(extra)
    return r


def golden(name, hash_):
    """Oracle reference results for a workload, when the stored input hash matches."""
    path = os.path.join(GOLDEN, f"{name}_reference.json")
    if not os.path.exists(path):
        return None
    ref = json.load(open(path))
    return ref if ref.get("hash") == hash_ else None


def event_ms(fn):
    """HIP-event time (ms) of fn() on torch's current stream, which the library launches on."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def phasing_errors(h1, block, truth, pos=None):
    """Switch error and orientation-free Hamming error against the planted haplotype
    (consecutive phased SNPs of each block; unphased SNPs skipped), the phased fraction
    (phasing completeness: every input SNP is a true heterozygous site here, so SNP
    completeness is the same number) and, given positions, the haplotype N50 in bp (block
    span = last - first phased position + 1; the span where the descending running sum
    first reaches half the total)."""
    import numpy as np
    sw = pairs = mis = tot = 0
    ok = (h1 >= 0) & (block >= 0)
    spans = []
    for b in np.unique(block[ok]):
        idx = np.nonzero(ok & (block == b))[0]
        rel = h1[idx] == truth[idx]
        sw += int(np.count_nonzero(rel[1:] != rel[:-1]))
        pairs += max(idx.shape[0] - 1, 0)
        m = int(np.count_nonzero(~rel))
        mis += min(m, idx.shape[0] - m)
        tot += idx.shape[0]
        if pos is not None:
            spans.append(int(pos[idx[-1]]) - int(pos[idx[0]]) + 1)
    out = dict(switch_error=sw / pairs if pairs else 0.0, hamming_error_min=mis / tot if tot else 0.0,
               phased_fraction=float(ok.mean()) if ok.size else 0.0)
    if pos is not None:
        sp = np.sort(np.array(spans, dtype=np.int64))[::-1]
        cs = np.cumsum(sp)
        out["haplotype_n50_bp"] = int(sp[np.searchsorted(2 * cs, cs[-1] if cs.size else 0)]) if sp.size else 0
    return out


def _timed_jobs(job, steps, warmup):
    """Run warmup untimed jobs, then time exactly `steps` jobs between device
    synchronisations; returns (ms per job, last job's result)."""
    import torch
    res = None
    for _ in range(warmup):
        res = job(res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = job(res)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / max(steps, 1), res


# ----------------------------------------------------------------------------- batched (default)

BATCH_R, BATCH_STEPS, BATCH_DT, BATCH_SEED = 32, 500, 0.5, 11
BATCH_CPU_SAMPLE = (0, 5)       # oracle sample: the stratified subset's blocks 0, 5, 10, ...


def batch_inputs(qh, batch):
    """Every block's fragment arrays on the device from one host-to-device copy per array
    kind: the blocks' arrays are views into the concatenation."""
    import numpy as np
    import torch
    names = ("frag_ptr", "snp", "allele", "phred", "alpha", "init_h1")
    arrs = [w.arrays() for w in batch.blocks]
    views = [dict() for _ in arrs]
    for k in names:
        parts = [np.ascontiguousarray(a[k]) for a in arrs]
        off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
        # the blocks' arrays are packed straight into pinned host memory (one pass over the
        # host bytes), from which the copy to the device runs at DMA speed
        host = torch.empty(int(off[-1]), dtype=torch.from_numpy(parts[0][:0]).dtype, pin_memory=True)
        np.concatenate(parts, out=host.numpy())
        dev = host.to("cuda", non_blocking=True)
        for b in range(len(arrs)):
            views[b][k] = dev[int(off[b]):int(off[b + 1])]
    return views


BUILD_THREADS = 0


def build_batch(qh, batch, dtype=None, inputs=None):
    """The batch's graphs (even blocks read graphs, odd blocks SNP graphs), built together by
    qh_build_graphs (BUILD_THREADS host threads; 0 = the library's default) from `inputs`
    (batch_inputs), which are made here when not given."""
    specs = []
    inputs = batch_inputs(qh, batch) if inputs is None else inputs
    for i, (w, d) in enumerate(zip(batch.blocks, inputs)):
        kind = "read_signed" if i % 2 == 0 else "snp_llr"
        specs.append(dict(frag_ptr=d["frag_ptr"], snp=d["snp"], allele=d["allele"], phred=d["phred"],
                          init_h1=d["init_h1"], kind=kind, dtype=dtype or w.solve["dtype"],
                          alpha=d["alpha"] if kind == "snp_llr" else None))
    return qh.build_graphs(specs, threads=BUILD_THREADS)


def batch_gaps(qh, gs, r, batch, ref):
    """Cut gap of every block of the oracle's subset, and whether its switch error equals the
    oracle's (the block's h1 from qh_phase on the block's selected spins)."""
    import numpy as np
    bc = r["best_cut"].cpu().numpy()
    off = r["vertex_offset"]
    gaps, se_eq, ses = [], 0, []
    for blk in ref["blocks"]:
        b = blk["block"]
        gaps.append((blk["best_cut"] - float(bc[b])) / abs(blk["best_cut"]))
        h1, bl = qh.phase(gs[b], r["best_spins"][int(off[b]):int(off[b + 1])])
        se = phasing_errors(h1.cpu().numpy(), bl.cpu().numpy(), batch.blocks[b].truth)["switch_error"]
        se_eq += int(se == blk["switch_error"])
        ses.append(se)
    gaps = np.array(gaps)
    tot_ref = sum(b["best_cut"] for b in ref["blocks"])
    tot = sum(float(bc[b["block"]]) for b in ref["blocks"])
    return dict(cut_gap=float(gaps.max()), cut_gap_mean=float(gaps.mean()), cut_gap_total=(tot_ref - tot) / abs(tot_ref),
                blocks_over_0p1pct=int((gaps > 1e-3).sum()), blocks_compared=len(gaps),
                switch_error_equal=se_eq, switch_error_mean=float(np.mean(ses)),
                oracle_switch_error_mean=float(np.mean([b["switch_error"] for b in ref["blocks"]])))


def cpu_baseline_batched(batch, ref):
    """The FP64 oracle on the host cores: a bounded sample of the batch's blocks (graph built
    untimed, then the whole solve: bSB steps, cuts, selection, greedy), in edge-updates/s."""
    import oracle
    first, stride = BATCH_CPU_SAMPLE
    sample = [b["block"] for b in ref["blocks"]][first::stride]
    eu = 0.0
    t = 0.0
    for b in sample:
        kind = "read_signed" if b % 2 == 0 else "snp_llr"
        g = oracle.build_graph(batch.blocks[b], kind)
        t0 = time.perf_counter()
        oracle.solve(g, BATCH_R, BATCH_STEPS, BATCH_DT, seed=BATCH_SEED, integer=kind != "snp_llr")
        t += time.perf_counter() - t0
        eu += g.nnz * BATCH_R * BATCH_STEPS
    return dict(value=eu / t, unit="edge-updates/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{len(sample)} of the 3,000 blocks (every {stride}th block of the oracle's stratified 5% "
                       f"subset from its {first}th, all sizes and both kinds; {eu:.3e} edge-updates, "
                       f"{eu / 3.0e13 * 100:.2f}% of the job): whole oracle solves (R = {BATCH_R}, {BATCH_STEPS} "
                       f"steps, cuts, selection, greedy), graph builds untimed; {t:.1f} s")


def bench_batched(a):
    import numpy as np
    import torch

    import paper_2603_25762_amd as qh
    import synth

    R, STEPS, DT, SEED = BATCH_R, BATCH_STEPS, BATCH_DT, BATCH_SEED
    use_graph = True if a.graph is None else bool(a.graph)
    torch.cuda.set_device(0)
    batch = synth.batched_blocks()
    ref = golden("batched", synth.batch_hash(batch))
    t0 = time.perf_counter()
    gs = build_batch(qh, batch)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    infos = [g.info() for g in gs]
    nnz = sum(i["nnz"] for i in infos)
    dense = [i for i, inf in enumerate(infos) if inf["storage"] == 0]
    sparse = [i for i, inf in enumerate(infos) if inf["storage"] != 0]
    plan = 1 if use_graph else a.plan
    kw = dict(dt=DT, seed=SEED, use_graph=use_graph, plan=plan)

    def job(_):
        return qh.bsb_solve_batched(gs, R, STEPS, **kw)

    ms, r = _timed_jobs(job, a.steps, a.warmup)
    value = nnz * R * STEPS / (ms * 1e-3)

    # dominant kernel: the dense FP8 class (one launch per step over every dense block's row
    # tiles), timed with HIP events on the library's stream: the dense blocks solved as a
    # batch of their own, dynamics only, so the 500 launches of that class are all it runs
    sub_d = [gs[i] for i in dense]
    sub_s = [gs[i] for i in sparse]
    qh.bsb_solve_batched(sub_d, R, STEPS, readout=False, **kw)              # capture / warm
    dense_us = event_ms(lambda: qh.bsb_solve_batched(sub_d, R, STEPS, readout=False, **kw)) * 1e3 / STEPS
    qh.bsb_solve_batched(sub_s, R, STEPS, readout=False, **kw)
    band_us = event_ms(lambda: qh.bsb_solve_batched(sub_s, R, STEPS, readout=False, **kw)) * 1e3 / STEPS
    n_d = np.array([infos[i]["n"] for i in dense], dtype=np.float64)
    t_d = np.array([infos[i]["dense_tiles"] for i in dense], dtype=np.float64)
    # per dense block and step: its stored 64 x 64 FP8 tiles (all-zero tiles are not stored),
    # N row scales, and per (row, replica) x and y read and written (16 B) plus the 16-bit
    # copy of x written and read (4 B); 2 flop per stored entry and replica
    dense_bytes = float(4096 * t_d.sum() + 4 * n_d.sum() + 20 * n_d.sum() * R)
    dense_flops = float(2 * 4096 * t_d.sum() * R)
    n_s = np.array([infos[i]["n"] for i in sparse], dtype=np.float64)
    band_bytes = float(sum(infos[i]["stored_bytes"] - 16 * infos[i]["n"] for i in sparse) + 16 * n_s.sum() * R)
    roof = roofline("hbm", dense_bytes, dense_flops, dense_us, "fp8", "k_batched_rowtile<fp8>",
                    steps_per_launch=1, per_step_us={"dense_fp8_class": round(dense_us, 2),
                                                     "band_class": round(band_us, 2)},
                    band_class_hbm_frac=round(band_bytes / (band_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                    band_class_bytes_per_launch=int(band_bytes),
                    stored_tiles=int(t_d.sum()), nnz_flop_per_launch=float(2 * sum(infos[i]["nnz"] for i in dense) * R),
                    note="dense FP8 class per step: sum_b (4096 T_b + 4 N_b + 20 N_b R) bytes, 2 * 4096 T_b R flop "
                         "(T_b stored tiles of block b)")

    out = dict(metric=METRIC, value=value, unit="edge-updates/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="fp8+bf16 storage, fp32 accumulate", data="synthetic",
               config=dict(workload="batched: 3,000 independent phasing blocks, vertex counts log-uniform 50-5,000; "
                                    "even blocks dense read graphs (FP8 + row scales), odd blocks SNP graphs "
                                    "(BF16 band); R = 32, 500 bSB steps, dt = 0.5, linear pump, c0 auto per block",
                           blocks=len(gs), dense_blocks=len(dense), snp_blocks=len(sparse), nnz=int(nnz),
                           dense_entries=int((n_d ** 2).sum()), vertices=int(sum(i["n"] for i in infos)),
                           replicas=R, bsb_steps=STEPS, dt=DT, seed=SEED,
                           plan="per-step, hipGraph replay" if use_graph else f"plan {r['plan_used']}",
                           parallelism="single GPU"),
               plan_used=r["plan_used"], build_s=round(build_s, 3), roofline=roof)
    if ref is not None:
        out.update(batch_gaps(qh, gs, r, batch, ref))
        out["oracle_reference"] = "tests/golden/batched_reference.json (stratified 5% subset: 150 blocks)"
    out["graph_device_bytes"] = int(sum(i["device_bytes"] for i in infos))
    # the batch is done: its device blocks go back to the library's cache, from which the
    # next batch's graphs are built, as in a loop over batches
    for g in gs:
        g.free()
    if not a.no_extras:
        ttp, parts = time_to_phase_batched(qh, batch, R, STEPS, kw)
        out["time_to_phase_ms"] = round(ttp, 1)
        out["time_to_phase_parts_ms"] = parts
        out["fp32_form"] = fp32_form_batched(qh, batch, R, STEPS, DT, SEED, ref, a)
    if not a.no_cpu_baseline and ref is not None:
        out["cpu_baseline"] = cpu_baseline_batched(batch, ref)
    print(json.dumps(out), flush=True)


def time_to_phase_batched(qh, batch, R, STEPS, kw):
    """Host fragments in -> haplotypes out for the whole batch: H2D of every block's
    fragments (one copy per array kind), the graph builds (qh_build_graphs), the batched
    solve with the benchmark's options `kw`, the phasing of every block (qh_phase_batched),
    D2H."""
    import torch
    torch.cuda.synchronize()
    t = [time.perf_counter()]
    inputs = batch_inputs(qh, batch)
    torch.cuda.synchronize()
    t.append(time.perf_counter())
    gs = build_batch(qh, batch, inputs=inputs)
    t.append(time.perf_counter())
    r = qh.bsb_solve_batched(gs, R, STEPS, **kw)
    torch.cuda.synchronize()
    t.append(time.perf_counter())
    # every block phased in one call (qh_phase_batched), outputs packed by SNP
    h1, blk, _ = qh.phase_batched(gs, r["best_spins"])
    torch.cuda.synchronize()
    t.append(time.perf_counter())
    h1 = h1.cpu()
    blk = blk.cpu()
    t.append(time.perf_counter())
    del h1, blk
    for g in gs:
        g.free()
    parts = {k: round((t[i + 1] - t[i]) * 1e3, 1) for i, k in enumerate(("h2d", "build", "solve", "phase", "d2h"))}
    return (t[-1] - t[0]) * 1e3, parts


def fp32_form_batched(qh, batch, R, STEPS, DT, SEED, ref, a):
    """The plain FP32 form on the same batch: every block's J stored in FP32."""
    import torch
    gs = build_batch(qh, batch, dtype="f32")
    nnz = sum(g.info()["nnz"] for g in gs)
    kw = dict(dt=DT, seed=SEED, use_graph=True, plan=1)
    r = qh.bsb_solve_batched(gs, R, STEPS, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = qh.bsb_solve_batched(gs, R, STEPS, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out = dict(value=nnz * R * STEPS / (ms * 1e-3), ms_per_step=round(ms, 3))
    if ref is not None:
        g = batch_gaps(qh, gs, r, batch, ref)
        out.update(cut_gap=g["cut_gap"], switch_error_equal=g["switch_error_equal"])
    for g in gs:
        g.free()
    return out


# ----------------------------------------------------------------------------- read_mhc

def bench_read_mhc(a):
    import torch

    import paper_2603_25762_amd as qh
    import synth

    dtype = a.dtype or "bf16"     # one of the workload's named forms (FP32, BF16, FP8 with row scales)
    R, STEPS, DT = 256, 2000, 0.5
    torch.cuda.set_device(0)
    w = synth.read_mhc()
    ref = golden("read_mhc", synth.workload_hash(w))
    seed = ref["seed"] if ref else 2026
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    torch.cuda.synchronize()

    def build():
        return qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="read_signed",
                              dtype=dtype)

    plan, kw = a.plan, {}
    if plan == 0:   # the autotuner picks the plan once (untimed); every job then runs it
        g = build()
        qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, plan=0, readout=False)
        tune = g.plan_info(R)
        g.free()
        plan = tune["plan_used"]
        kw = dict(replica_tile=tune["replica_tile"], tiles_in_flight=tune["tiles_in_flight"]) if plan == 1 else \
            dict(persistent_sync=tune["persistent_sync"])
    elif plan == 2:
        kw = dict(persistent_sync=a.persistent_sync)
    use_graph = bool(a.graph) if a.graph is not None else False

    def job(prev):
        if prev is not None:
            prev[0].free()
        g = build()
        r = qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=use_graph, plan=plan, **kw)
        h1, blk = qh.phase(g, r["best_spins"])
        return g, r, h1, blk

    ms, (g, r, h1, blk) = _timed_jobs(job, a.steps, a.warmup)
    info = g.info()
    nnz, n, tiles = info["nnz"], info["n"], info["dense_tiles"]
    value = nnz * R * STEPS / (ms * 1e-3)
    best_cut = float(r["best_cut"].cpu()[0])
    solve_ms = event_ms(lambda: qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=use_graph, plan=plan, **kw))
    loop_ms = event_ms(lambda: qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=use_graph, readout=False,
                                            plan=plan, **kw))
    eb = {"f32": 4, "f16": 2, "bf16": 2, "fp8": 1}[dtype]
    # algorithmic work (§ measurement): 2 nnz R flop per step on the true nonzeros
    if plan == 2:
        kernel = f"k_dense_persistent<{dtype}, {'coherent' if kw.get('persistent_sync') == 2 else 'fences'}>"
        launch_us, steps_per_launch = loop_ms * 1e3, STEPS
    else:
        kernel, launch_us, steps_per_launch = f"k_dense_step<{dtype}>", loop_ms * 1e3 / STEPS, 1
    flops = 2.0 * nnz * R * steps_per_launch
    copy = 0 if dtype == "f32" else 4
    bytes_ = (tiles * 4096 * eb + n * R * 16 + steps_per_launch * n * R * copy) if plan == 2 else \
        (tiles * 4096 * eb + n * R * (16 + copy))
    roof = roofline("mfma", bytes_, flops, launch_us, dtype, kernel, steps_per_launch=steps_per_launch,
                    us_per_bsb_step=round(loop_ms * 1e3 / STEPS, 3),
                    executed_flop_per_launch=2.0 * tiles * 4096 * R * steps_per_launch,
                    executed_mfma_frac=round(2.0 * tiles * 4096 * R * steps_per_launch / (launch_us * 1e-6) / 1e12
                                             / PEAK_TFLOPS[dtype], 4))
    out = dict(metric=METRIC, value=value, unit="edge-updates/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype=f"{dtype} storage, fp32 accumulate", data="synthetic",
               config=dict(workload="read_mhc: 4 Mb region, 12,000 het SNPs, 8,000 lognormal 15 kb reads, 1-8% "
                                    "allele errors; dense 8000x8000 signed read graph; R = 256, 2,000 steps",
                           n=n, nnz=nnz, dense_tiles=tiles, replicas=R, bsb_steps=STEPS, dt=DT, precision=dtype,
                           plan="persistent" if plan == 2 else "per-step", parallelism="single GPU"),
               solve_ms=round(solve_ms, 3), solve_edge_updates_per_s=nnz * R * STEPS / (solve_ms * 1e-3),
               best_cut=best_cut, roofline=roof, plan_options=kw)
    if ref is not None:
        out.update(oracle_best_cut=ref["best_cut"], cut_gap=(ref["best_cut"] - best_cut) / abs(ref["best_cut"]),
                   oracle_switch_error=ref["switch_error"])
    out.update(phasing_errors(h1.cpu().numpy(), blk.cpu().numpy(), w.truth, w.pos))
    if ref is not None:
        out["switch_error_equal"] = out["switch_error"] == ref["switch_error"]
    if not a.no_extras:
        out["time_to_phase_ms"] = round(time_to_phase_single(qh, w, "read_signed", dtype, R, STEPS, DT, seed,
                                                             plan=plan, **kw), 2)
        # the plain form: J stored in FP32 (the autotuner's plan for it), one whole solve
        g32 = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="read_signed",
                             dtype="f32")
        qh.bsb_solve(g32, R, STEPS, dt=DT, seed=seed, plan=0, readout=False)
        r32 = qh.bsb_solve(g32, R, STEPS, dt=DT, seed=seed)
        ms32 = event_ms(lambda: qh.bsb_solve(g32, R, STEPS, dt=DT, seed=seed))
        cut32 = float(r32["best_cut"].cpu()[0])
        out["fp32_form"] = dict(value=nnz * R * STEPS / (ms32 * 1e-3), ms_per_solve=round(ms32, 3),
                                cut_gap=(ref["best_cut"] - cut32) / abs(ref["best_cut"]) if ref else None)
        g32.free()
    g.free()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_single(w, "read_signed", R, STEPS, DT, seed, STEPS)
    print(json.dumps(out), flush=True)


def time_to_phase_single(qh, w, kind, dtype, R, STEPS, DT, seed, band_limit=0, **kw):
    """Host fragments in -> haplotypes out: H2D, graph build, solve, phase, D2H."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind=kind, dtype=dtype,
                       alpha=d["alpha"] if kind == "snp_llr" else None, band_limit=band_limit)
    r = qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, **kw)
    h1, blk = qh.phase(g, r["best_spins"])
    h1, blk = h1.cpu(), blk.cpu()
    ms = (time.perf_counter() - t0) * 1e3
    g.free()
    return ms


def cpu_baseline_single(w, kind, R, STEPS, DT, seed, sample_steps):
    """The FP64 oracle on the host cores: full graph build + the first `sample_steps` bSB
    steps, extrapolated linearly to the whole solve, in edge-updates/s."""
    import oracle
    t0 = time.perf_counter()
    g = oracle.build_graph(w, kind)
    t_build = time.perf_counter() - t0
    x, y = oracle.init_state(seed, g.n, R)
    t0 = time.perf_counter()
    oracle.bsb_run(g, x, y, oracle.pump_linear(STEPS), DT, oracle.c0(g), 1.0, 0, sample_steps)
    t_steps = time.perf_counter() - t0
    t_job = t_build + t_steps * STEPS / sample_steps
    return dict(value=g.nnz * R * STEPS / t_job, unit="edge-updates/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"oracle graph build (full) + bSB steps 0..{sample_steps} of {STEPS} (R={R}), extrapolated "
                       f"linearly to the whole job; build {t_build:.2f} s, {sample_steps} steps {t_steps:.2f} s")


# ----------------------------------------------------------------------------- SNP graphs

def bench_snp(a):
    import torch

    import paper_2603_25762_amd as qh
    import synth

    porec = a.workload == "snp_porec"
    name = a.workload
    dtype = a.dtype or ("bf16" if porec else "f16")
    R, STEPS, DT, SEED = 64, (4000 if porec else 3000), 0.5, 7
    band = 64 if porec else 0     # every read pair stays in the band, every Pore-C contact goes long-range
    torch.cuda.set_device(0)
    w = synth.snp_porec() if porec else synth.snp_chrom()
    ref = golden(name, synth.workload_hash(w))
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    torch.cuda.synchronize()

    def build():
        return qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="snp_llr",
                              dtype=dtype, alpha=d["alpha"], band_limit=band)

    g = build()     # the autotuner times the band kernels once (untimed); every job then runs its choice
    qh.bsb_solve(g, R, STEPS, dt=DT, seed=SEED, plan=0, readout=False)
    tune = g.plan_info(R)
    plan = tune["skyline_kernel"]     # 3 per-row, 4 band FMA, 5 band MFMA: the plan that runs it
    g.free()
    use_graph = bool(a.graph) if a.graph is not None else False

    def job(prev):
        if prev is not None:
            prev[0].free()
        g = build()
        r = qh.bsb_solve(g, R, STEPS, dt=DT, seed=SEED, use_graph=use_graph, plan=plan)
        h1, blk = qh.phase(g, r["best_spins"])
        return g, r, h1, blk

    ms, (g, r, h1, blk) = _timed_jobs(job, a.steps, a.warmup)
    info = g.info()
    nnz, n, lr = info["nnz"], info["n"], info["longrange_nnz"]
    loop_ms = event_ms(lambda: qh.bsb_solve(g, R, STEPS, dt=DT, seed=SEED, use_graph=use_graph, readout=False,
                                            plan=plan))
    step_us = loop_ms * 1e3 / STEPS
    # one step: the stored band (no column indices) and the long-range CSR once, x and y read
    # and written once (gathers of x rows by long-range entries are cache traffic)
    bytes_ = info["stored_bytes"] - 16 * n + n * R * 16
    kernel = {4: "k_band_step", 5: "k_band_step_mfma", 3: "k_sky_step"}[plan] + ("+k_lr_packets" if lr else "")
    roof = roofline("hbm", bytes_, 2.0 * nnz * R, step_us, "f32", kernel + f"<{dtype}>",
                    note="one launch = one bSB step (all kernels of the step)")
    best_cut = float(r["best_cut"].cpu()[0])
    out = dict(metric=METRIC, value=nnz * R * STEPS / (ms * 1e-3), unit="edge-updates/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype=f"{dtype} storage, fp32 accumulate", data="synthetic",
               config=dict(workload=("snp_porec: snp_chrom plus 600,000 Pore-C contacts (distance ~ d^-1.1, "
                                     "100 kb-100 Mb, Zipf anchors), band limit 64" if porec else
                                     "snp_chrom: 250,000 het SNPs, 30x of 20 kb reads, 6% errors, Phred 7-40") +
                           f"; R = {R}, {STEPS} steps",
                           n=n, nnz=nnz, longrange_nnz=lr, replicas=R, bsb_steps=STEPS, dt=DT,
                           storage="skyline band blocks" + (" + long-range packets" if lr else ""),
                           parallelism="single GPU"),
               best_cut=best_cut, roofline=roof, autotune=tune)
    if ref is not None:
        out.update(oracle_best_cut=ref["best_cut"], cut_gap=(ref["best_cut"] - best_cut) / abs(ref["best_cut"]),
                   oracle_switch_error=ref["switch_error"])
    out.update(phasing_errors(h1.cpu().numpy(), blk.cpu().numpy(), w.truth, w.pos))
    if ref is not None:
        out["switch_error_equal"] = out["switch_error"] == ref["switch_error"]
    if not a.no_extras:
        out["time_to_phase_ms"] = round(time_to_phase_single(qh, w, "snp_llr", dtype, R, STEPS, DT, SEED,
                                                             band_limit=band, plan=plan), 2)
    g.free()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_single(w, "snp_llr", R, STEPS, DT, SEED, 60)
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.gpus != 1:
        print(f"bench.py drives one GPU; --gpus {a.gpus} is not offered (how the path would shard across GPUs "
              "is described in the design notes only)", file=sys.stderr)
        sys.exit(2)
    global BUILD_THREADS
    BUILD_THREADS = a.build_threads
    {"batched": bench_batched, "read_mhc": bench_read_mhc, "snp_chrom": bench_snp,
     "snp_porec": bench_snp}[a.workload](a)


if __name__ == "__main__":
    main()

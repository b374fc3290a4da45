"""Benchmark: bSB edge-updates/s of the whole phasing job on one MI355X.

One benchmark step = one pass of the whole hot path over one synthetic batch:
build_graph (encode + read-graph weights + components + tiles + quantize) ->
bsb_solve (init, 2,000 fused bSB steps over 256 replicas, FP64 cuts, per-component
selection, greedy pass) -> phase.  Inputs (fragments) are resident in HBM before
the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f16] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bSB edge-updates/s (nnz×replicas×steps) at ≤0.1% cut gap vs FP64 oracle"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f16": 2500.0, "bf16": 2500.0, "fp8": 2500.0, "f32": 157.3}  # fp8 codes run on f16 MFMA


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="read_mhc", choices=["read_mhc", "snp_chrom", "snp_porec", "batched"],
                    help="read_mhc (default) is the benchmark line; the others profile the SNP and batched paths")
    ap.add_argument("--dtype", default=None, choices=["f32", "f16", "bf16", "fp8"],
                    help="default: f16 (read_mhc, snp_chrom), bf16 (snp_porec); batched blocks carry their own")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: capture the step loop in a hipGraph (pays off only when a graph is solved again; "
                         "every job here builds a fresh graph, so the default launches the steps directly)")
    ap.add_argument("--plan", type=int, default=0,
                    help="0 auto (persistent when it applies), 1 one kernel per step, 2 persistent")
    ap.add_argument("--persistent-sync", type=int, default=0, choices=[0, 1, 2],
                    help="persistent plan: 0 tuned, 1 cache-wide fences, 2 device-coherent accesses")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 1 GiB (3 times): the reference kernel that scales "
                         "the FETCH_SIZE / WRITE_SIZE counters to HBM bytes")
    return ap.parse_args()


COPY_BYTES = 1 << 30


def calibrate_copy():
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes_read=COPY_BYTES, copy_bytes_written=COPY_BYTES, launches=3)), flush=True)


def kernel_source_hash(kernel="k_dense_step"):
    """Hash of a step kernel's source.  k_dense_step: the dense-tile section of bsb.hip
    (from StepArgs to the skyline banner, the update helpers included); k_dense_persistent:
    persistent_kernel.h; k_band_step: the update helpers and the skyline section of bsb.hip.
    formats.h (the number formats) is part of every hash."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_25762_amd", "csrc")
    if kernel.startswith("k_dense_persistent"):
        h.update(open(os.path.join(csrc, "persistent_kernel.h"), "rb").read())
    elif kernel.startswith("k_band_step"):
        src = open(os.path.join(csrc, "bsb.hip")).read()
        a = src.index("struct StepArgs")
        b = src.index("struct StepArgs") + src[a:].index("// ------", 1)
        h.update(src[a:b].encode())                      # StepArgs and the update helpers
        a = src.index("// skyline band + long-range CSR")
        b = src.index("// batched blocks:")
        h.update(src[a:b].encode())                      # the skyline / band kernels
    else:
        src = open(os.path.join(csrc, "bsb.hip")).read()
        a = src.index("struct StepArgs")
        b = src.index("// skyline band + long-range CSR")
        h.update(src[a:b].encode())
    h.update(open(os.path.join(csrc, "formats.h"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, replica_tile=None, depth=None):
    """HBM bytes per launch of `kernel` from the committed counter summaries (the
    `traffic:` lines of profiles/*.md), or None when none covers this kernel and
    configuration or the kernel's source changed since the counters were taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        vals = {}
        for line in open(path):
            if line.startswith("traffic:"):
                k, _, v = line[len("traffic:"):].strip().partition("=")
                vals[k.strip()] = v.strip()
        if vals.get("kernel") != kernel or vals.get("source_sha") != kernel_source_hash(kernel):
            continue
        if replica_tile is not None and int(vals.get("replica_tile", 0)) != replica_tile:
            continue
        if depth is not None and int(vals.get("tiles_in_flight", 2)) != depth:
            continue
        return int(float(vals["hbm_bytes_per_launch"]))
    return None


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.gpus != 1:
        print(f"bench.py drives one GPU; --gpus {a.gpus} is not offered (sharding replicas across GPUs "
              "is described in the design notes only)", file=sys.stderr)
        sys.exit(2)
    if a.workload in ("snp_chrom", "snp_porec"):
        return bench_snp(a)
    if a.workload == "batched":
        return bench_batched(a)
    if a.dtype is None:
        a.dtype = "f16"
    import numpy as np
    import torch

    import paper_2603_25762_amd as qh
    import synth

    R, STEPS, DT = 256, 2000, 0.5
    ref_path = os.path.join(ROOT, "tests", "golden", "read_mhc_reference.json")
    ref = json.load(open(ref_path)) if os.path.exists(ref_path) else None
    seed = ref["seed"] if ref else 2026

    torch.cuda.set_device(0)
    w = synth.read_mhc()
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    torch.cuda.synchronize()

    plan = a.plan
    tune = None
    if plan == 0:
        # let the library's autotuner pick the step-loop plan for this graph and replica count,
        # then run every timed job with that plan (the tuner itself stays out of the timed region)
        g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"],
                           kind="read_signed", dtype=a.dtype)
        qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, plan=0, readout=False)
        tune = g.plan_info(R)
        plan = tune["plan_used"]
        g.free()
    # the tuned per-step tile and depth, or the tuned persistent variant, passed explicitly to
    # every job's fresh graph
    kw = {}
    if tune is not None and plan == 1:
        kw = dict(replica_tile=tune["replica_tile"], tiles_in_flight=tune["tiles_in_flight"])
    elif tune is not None and plan == 2:
        kw = dict(persistent_sync=tune["persistent_sync"])
    elif plan == 2:
        kw = dict(persistent_sync=a.persistent_sync)

    def job():
        g = qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"],
                           kind="read_signed", dtype=a.dtype)
        r = qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=bool(a.graph), plan=plan, **kw)
        h1, blk = qh.phase(g, r["best_spins"])
        return g, r, h1, blk

    for _ in range(a.warmup):
        g, r, h1, blk = job()
        g.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(a.steps):
        g, r, h1, blk = job()
        results.append((g, r, h1, blk))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    g, r, h1, blk = results[-1]
    info = g.info()
    nnz = info["nnz"]
    value = nnz * R * STEPS / (ms_per_step * 1e-3)
    best_cut = float(r["best_cut"].cpu()[0])
    for gg, *_ in results[:-1]:
        gg.free()

    # solve-only rate and the dominant kernel (the fused dense step) timed with HIP events on
    # the stream the library launches on (torch's current stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=bool(a.graph), plan=plan, **kw)
    torch.cuda.synchronize()
    ev0.record()
    qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=bool(a.graph), plan=plan, **kw)
    ev1.record()
    torch.cuda.synchronize()
    solve_ms = ev0.elapsed_time(ev1)
    qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=bool(a.graph), readout=False, plan=plan, **kw)
    torch.cuda.synchronize()
    ev0.record()
    qh.bsb_solve(g, R, STEPS, dt=DT, seed=seed, use_graph=bool(a.graph), readout=False, plan=plan, **kw)
    ev1.record()
    torch.cuda.synchronize()
    loop_ms = ev0.elapsed_time(ev1)
    step_us = loop_ms * 1e3 / STEPS

    tiles = info["dense_tiles"]
    n = info["n"]
    eb = {"f32": 4, "f16": 2, "bf16": 2, "fp8": 1}[a.dtype]
    copy = 0 if a.dtype == "f32" else 2 + 2          # 16-bit product copy of x: written once, read once
    if plan == 2:
        # one launch runs every step: J and the fp32 state cross HBM once; the 16-bit copy of x
        # is exchanged every step
        launches_steps = STEPS
        launch_us = loop_ms * 1e3
        flops = 2.0 * tiles * 4096 * R * STEPS
        bytes_ = tiles * 4096 * eb + n * R * 16 + STEPS * n * R * copy
        sync_name = {1: "fences", 2: "coherent"}.get(kw.get("persistent_sync"), "fences")
        kernel = f"k_dense_persistent<{a.dtype}, {sync_name}>"
    else:
        # one launch = one step: the stored tiles once, x and y read and written once, the
        # 16-bit copy written and read once (re-reads of x columns by other row tiles are
        # cache traffic, not algorithmic)
        launches_steps = 1
        launch_us = step_us
        flops = 2.0 * tiles * 4096 * R               # executed MFMA work of one launch (one step)
        bytes_ = tiles * 4096 * eb + n * R * 16 + n * R * copy
        kernel = f"k_dense_step<{a.dtype}>"
    ach_tf = flops / (launch_us * 1e-6) / 1e12
    ach_gbs = bytes_ / (launch_us * 1e-6) / 1e9
    frac_m = ach_tf / PEAK_TFLOPS[a.dtype]
    frac_h = ach_gbs / PEAK_HBM_GBS
    rtile = (tune or {}).get("replica_tile") or 64
    depth = (tune or {}).get("tiles_in_flight") or 2
    traffic = measured_traffic(kernel, rtile, depth) if plan != 2 else measured_traffic(kernel)
    if frac_m >= frac_h:
        roof = dict(bound="mfma", achieved=round(ach_tf, 2), peak=PEAK_TFLOPS[a.dtype], unit="TFLOP/s",
                    frac=round(frac_m, 4), traffic=traffic)
    else:
        roof = dict(bound="hbm", achieved=round(ach_gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(frac_h, 4), traffic=traffic)
    roof.update(kernel=kernel, replica_tile=rtile if plan != 2 else None,
                tiles_in_flight=depth if plan != 2 else None, launch_us=round(launch_us, 3),
                steps_per_launch=launches_steps,
                us_per_bsb_step=round(step_us, 3), flop_per_launch=flops, bytes_per_launch=bytes_,
                mfma_frac=round(frac_m, 4), hbm_frac=round(frac_h, 4), source_sha=kernel_source_hash(kernel))

    out = dict(metric=METRIC, value=value, unit="edge-updates/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=round(ms_per_step, 3), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype=a.dtype, data="synthetic",
               config=dict(workload="read_mhc: 4 Mb region, 12,000 het SNPs, 8,000 lognormal 15 kb reads, "
                                    "1-8% allele errors; dense 8000x8000 signed read graph",
                           n=n, nnz=nnz, dense_tiles=tiles, replicas=R, bsb_steps=STEPS, dt=DT,
                           storage="dense 64x64 tiles (zero tiles skipped)", precision=a.dtype,
                           plan="persistent" if plan == 2 else "per-step",
                           parallelism="single GPU"),
               solve_ms=round(solve_ms, 3), solve_edge_updates_per_s=nnz * R * STEPS / (solve_ms * 1e-3),
               best_cut=best_cut, roofline=roof)
    if tune is not None:
        out["autotune"] = tune
    if ref is not None and ref.get("nnz") == nnz:
        out["oracle_best_cut"] = ref["best_cut"]
        out["cut_gap"] = (ref["best_cut"] - best_cut) / abs(ref["best_cut"])
    out.update(phasing_errors(h1.cpu().numpy(), blk.cpu().numpy(), w.truth, w.pos))

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, R, STEPS, DT, seed, a.cpu_sample_steps)
    print(json.dumps(out), flush=True)


def _time_loop(fn, reps=1):
    """HIP-event time (ms) of fn() on torch's current stream, which the library launches on."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_snp(a):
    """SNP-based chromosome-scale workloads: skyline band (+ long-range CSR for Pore-C)."""
    import torch
    import paper_2603_25762_amd as qh
    import synth
    porec = a.workload == "snp_porec"
    dtype = a.dtype or ("bf16" if porec else "f16")
    R, STEPS, DT, SEED = 64, (4000 if porec else 3000), 0.5, 7
    band = 64 if porec else 0     # every read pair stays in the band, every Pore-C contact goes long-range
    torch.cuda.set_device(0)
    w = synth.snp_porec() if porec else synth.snp_chrom()
    d = {k: qh.to_device(v) for k, v in w.arrays().items()}
    torch.cuda.synchronize()

    def build():
        return qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind="snp_llr",
                              dtype=dtype, alpha=d["alpha"], band_limit=band)

    # the autotuner times the two band kernels once (untimed); every job then runs its choice
    g = build()
    qh.bsb_solve(g, R, STEPS, dt=DT, seed=SEED, plan=0, readout=False)
    tune = g.plan_info(R)
    plan = tune["skyline_kernel"]
    g.free()

    def job():
        g = build()
        r = qh.bsb_solve(g, R, STEPS, dt=DT, seed=SEED, use_graph=bool(a.graph), plan=plan)
        h1, blk = qh.phase(g, r["best_spins"])
        return g, r, h1, blk

    for _ in range(a.warmup):
        job()[0].free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [job() for _ in range(a.steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.steps
    g, r, h1, blk = res[-1]
    for gg, *_ in res[:-1]:
        gg.free()
    info = g.info()
    nnz, n = info["nnz"], info["n"]
    loop_ms = _time_loop(lambda: qh.bsb_solve(g, R, STEPS, dt=DT, seed=SEED, use_graph=bool(a.graph),
                                              readout=False, plan=plan))
    step_us = loop_ms * 1e3 / STEPS
    # one step: the stored band (no column indices) and the long-range CSR once, x and y read
    # and written once (gathers of x rows by long-range entries are cache traffic)
    lr = info["longrange_nnz"]
    bytes_ = info["stored_bytes"] + n * R * 16
    ach = bytes_ / (step_us * 1e-6) / 1e9
    kernel = ("k_band_step_mfma" if plan == 5 else "k_band_step" if plan == 4 else "k_sky_step") + \
        ("+k_lr_packets" if lr else "") + f"<{dtype}>"
    out = dict(metric=METRIC, value=nnz * R * STEPS / (ms * 1e-3), unit="edge-updates/s", n_gpus=1,
               steps=a.steps, warmup=a.warmup, ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=dtype, data="synthetic",
               config=dict(workload=("snp_porec: snp_chrom plus 600,000 Pore-C contacts (distance ~ d^-1.1, "
                                     "100 kb-100 Mb, Zipf anchors), band limit 64" if porec else
                                     "snp_chrom: 250,000 het SNPs, 30x of 20 kb reads, 6% errors, Phred 7-40"),
                           n=n, nnz=nnz, longrange_nnz=lr, replicas=R, bsb_steps=STEPS, dt=DT,
                           storage="skyline band blocks" + (" + long-range packets" if lr else ""),
                           parallelism="single GPU"),
               roofline=dict(bound="hbm", achieved=round(ach, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                             frac=round(ach / PEAK_HBM_GBS, 4),
                             traffic=None if lr else measured_traffic(kernel), kernel=kernel,
                             source_sha=kernel_source_hash(kernel),
                             launch_us=round(step_us, 3), bytes_per_launch=bytes_,
                             note="per bSB step (all kernels of one step)"),
               autotune=tune)
    out.update(phasing_errors(h1.cpu().numpy(), blk.cpu().numpy(), w.truth, w.pos))
    print(json.dumps(out), flush=True)


def bench_batched(a):
    """3,000 uneven blocks (dense FP8 read blocks, BF16 SNP blocks), R = 32, 500 steps.
    Graphs are built before the timed region; one step = one batched solve."""
    import torch
    import paper_2603_25762_amd as qh
    import synth
    R, STEPS, DT, SEED = 32, 500, 0.5, 11
    torch.cuda.set_device(0)
    batch = synth.batched_blocks()
    gs = []
    for i, w in enumerate(batch.blocks):
        d = {k: qh.to_device(v) for k, v in w.arrays().items()}
        kind = "read_signed" if i % 2 == 0 else "snp_llr"
        gs.append(qh.build_graph(d["frag_ptr"], d["snp"], d["allele"], d["phred"], d["init_h1"], kind=kind,
                                 dtype=w.solve["dtype"], alpha=d["alpha"] if kind == "snp_llr" else None))
    torch.cuda.synchronize()
    nnz = sum(g.info()["nnz"] for g in gs)
    r = None
    for _ in range(a.warmup):
        r = qh.bsb_solve_batched(gs, R, STEPS, dt=DT, seed=SEED, plan=a.plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        r = qh.bsb_solve_batched(gs, R, STEPS, dt=DT, seed=SEED, plan=a.plan)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.steps
    out = dict(metric=METRIC, value=nnz * R * STEPS / (ms * 1e-3), unit="edge-updates/s", n_gpus=1,
               steps=a.steps, warmup=a.warmup, ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="fp8+bf16", data="synthetic",
               config=dict(workload="batched: 3,000 blocks, log-uniform 50-5,000 vertices, even blocks dense "
                                    "FP8 read graphs, odd blocks BF16 SNP graphs",
                           blocks=len(gs), nnz=nnz, replicas=R, bsb_steps=STEPS, dt=DT,
                           plan_used=r["plan_used"], parallelism="single GPU"))
    print(json.dumps(out), flush=True)


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


def cpu_baseline(w, R, STEPS, DT, seed, sample_steps):
    """The FP64 oracle on the host cores: full graph build + a bounded sample of bSB steps,
    extrapolated linearly to the whole job in edge-updates/s."""
    import oracle
    t0 = time.perf_counter()
    g = oracle.build_graph(w, "read_signed")
    t_build = time.perf_counter() - t0
    x, y = oracle.init_state(seed, g.n, R)
    pump = oracle.pump_linear(STEPS)
    t0 = time.perf_counter()
    oracle.bsb_run(g, x, y, pump, DT, oracle.c0(g), 1.0, 0, sample_steps)
    t_steps = time.perf_counter() - t0
    t_job = t_build + t_steps * STEPS / sample_steps
    return dict(value=g.nnz * R * STEPS / t_job, unit="edge-updates/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"oracle graph build (full) + bSB steps 0..{sample_steps} of {STEPS} (R={R}), "
                       f"extrapolated linearly to the whole job; build {t_build:.2f} s, "
                       f"{sample_steps} steps {t_steps:.2f} s")


if __name__ == "__main__":
    main()

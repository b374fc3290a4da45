/*
 * qhap.h -- C ABI of the MI355X (gfx950) haplotype-phasing hot path.
 *
 * The paper (QHap) phases diploid haplotypes by posing them as weighted
 * Max-Cut and solving the Ising form with ballistic simulated bifurcation
 * (bSB).  This library implements that path on one GPU:
 *
 *   qh_build_graph  reads + SNPs  -> coupling matrix J      (Methods, graph construction;
 *                                                              qh_build_graphs: many at once)
 *   qh_bsb_solve    J             -> spins, FP64 cuts        (Methods, SB algorithm solution)
 *   qh_phase        J, spins      -> haplotype 1 per SNP     (Methods, consistency processing /
 *                                                              SNP-based parity reconstruction)
 *
 * Conventions shared by every entry point
 *  - Every function returns qh_status.  On failure a thread-local message is
 *    available from qh_last_error(); output buffers are left untouched.
 *    No C++ exception crosses the ABI.
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary CPU memory.  The caller owns every buffer it passes;
 *    the library owns everything inside a qh_graph.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is stream-ordered; device outputs are valid once the stream has
 *    synchronised.  Calls that must read back a count (graph build, the greedy
 *    pass) synchronise the stream themselves and say so.
 *  - The library recycles its device temporaries in stream order: make its calls from
 *    one host thread at a time (qh_build_graphs runs host threads of its own inside).
 *    Device memory it releases (temporaries, freed graphs) stays cached for its later
 *    requests, up to a quarter of the device's memory (at most 64 GiB per device);
 *    qh_release_cached_memory hands it back to the device.
 *  - Spin / momentum state is laid out [n][R] (replica index fastest), FP32.
 *  - Ising convention (Eqs. 4-6): E(s) = -1/2 s^T J s, A = -J, and
 *    cut(s) = 1/4 sum_{a,b} A_ab (1 - s_a s_b).
 */
#ifndef QHAP_H
#define QHAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QH_OK = 0,
    QH_EINVAL = 1,        /* bad argument: null pointer, size, index out of range, bad enum */
    QH_ENOMEM = 2,        /* device or host allocation failed */
    QH_EHIP = 3,          /* a HIP runtime call failed (message names it) */
    QH_EUNSUPPORTED = 4,  /* valid but not implemented combination (e.g. FP8 on a skyline) */
    QH_ENUMERIC = 5       /* NaN / Inf detected in couplings or final state */
} qh_status;

/* Graph kinds.
 *  READ_CONFLICT  vertices = fragments, A_ab = number of shared SNPs whose ternary
 *                 codes disagree (Eqs. 2-3), J = -A (Eq. 4).
 *  READ_SIGNED    vertices = fragments, J_ab = sum_j M_aj M_bj (agree minus disagree).
 *  SNP_LLR        vertices = SNPs, A_uv = w_uv of Eq. 14 (Phred-weighted log-likelihood
 *                 ratios, Eqs. 9-13, scaled by the per-fragment Pore-C factor alpha),
 *                 J = -A. Linkage depth k/10: each SNP links to its floor(k(|S_i|-1)/10)
 *                 nearest downstream SNPs of fragment i.  Observations with Phred <= 3
 *                 are dropped (the likelihood ratio is undefined or sign-flipped there). */
typedef enum { QH_READ_CONFLICT = 0, QH_READ_SIGNED = 1, QH_SNP_LLR = 2 } qh_graph_kind;

/* Storage of J for the step kernels.
 *  DENSE    64x64 tiles; all-zero tiles are not stored.  Read graphs only.
 *  SKYLINE  per row the contiguous column range [lo_u, hi_u] of linked SNPs (no column
 *           indices); pairs farther apart than band_limit columns go to a long-range
 *           CSR (the Pore-C contacts).  SNP graphs only. */
typedef enum { QH_STORE_DENSE = 0, QH_STORE_SKYLINE = 1 } qh_storage;

/* Stored value type of J for the step kernels (accumulation is always FP32).
 *  FP8_ROWSCALE: OCP E4M3 codes with one FP32 scale per row, s_i = RNE_f32(max_j|J_ij|/448),
 *  code = RNE_e4m3(J_ij / s_i) (quotient in FP64, saturating).  Dense storage only. */
typedef enum { QH_F32 = 0, QH_F16 = 1, QH_BF16 = 2, QH_FP8_ROWSCALE = 3 } qh_dtype;

/* Fragments (reads) in CSR form.  All pointers are device pointers.
 *  frag_ptr  int64 [n_frag + 1], frag_ptr[0] = 0, non-decreasing.
 *  snp       int32 [frag_ptr[n_frag]], SNP index in [0, n_snp), strictly ascending
 *            inside each fragment (index order = genomic order).
 *  allele    uint8, 0 = reference allele, 1 = alternative allele.
 *  phred     uint8 base quality (used by SNP_LLR only).
 *  alpha     float64 [n_frag] per-fragment weight factor (Pore-C down-weighting), or
 *            NULL for all ones (used by SNP_LLR only).
 * For read graphs fragment f is vertex f; pass fragments sorted by first SNP so that
 * J is band-shaped and the dense tiles skip most of the matrix. */
typedef struct {
    int64_t n_frag;
    const int64_t *frag_ptr;
    const int32_t *snp;
    const uint8_t *allele;
    const uint8_t *phred;
    const double *alpha;
} qh_reads;

/* SNP set.  init_h1 (device, uint8 [n_snp]) is the allele placed on the initial
 * haplotype H1 at each SNP (Methods, haplotype initialization); H2 carries the other. */
typedef struct {
    int32_t n_snp;
    const uint8_t *init_h1;
} qh_snps;

typedef struct {
    int32_t kind;        /* qh_graph_kind */
    int32_t storage;     /* qh_storage */
    int32_t dtype;       /* qh_dtype */
    int32_t linkage_k;   /* SNP_LLR: 1..10 (10 = every pair inside a fragment) */
    int32_t band_limit;  /* SKYLINE: max column distance kept in the band; 0 = no limit */
    int64_t max_device_bytes; /* cap on the device memory the graph may own (qh_graph_info
                            .device_bytes); 0 = no cap.  Checked before the master weights and
                            each storage copy are allocated, and on the finished graph:
                            ENOMEM (nothing kept) when the graph would exceed it. */
    int32_t deterministic; /* SNP_LLR: 1 = each Eq. (14) term is rounded to a multiple of
                            2^-40 and the terms are summed in 64-bit integers, so the weights
                            are bit-identical from build to build (the FP64 sum of atomics, 0,
                            depends on the order of the additions in its last bits).  This
                            trades the relative error bound of the FP64 sum (<= 1e-12 of the
                            summed |terms|) for an absolute one: at most 2^-41 per term, which
                            for very small weights is larger in relative terms.  A term of
                            magnitude 2^20 or more fails the build with ENUMERIC.  Read graphs
                            are integer sums: exact either way. */
} qh_graph_opts;

typedef struct qh_graph qh_graph;

typedef struct {
    int64_t n;               /* vertices */
    int64_t n_snp;           /* SNPs of the input (haplotype length for qh_phase) */
    int64_t nnz;             /* nonzero off-diagonal entries of J (both directions) */
    int64_t n_comp;          /* connected components with >= 2 vertices */
    int64_t stored_entries;  /* entries the step kernel reads per step and replica */
    int64_t stored_bytes;    /* bytes of J the step kernel reads per step */
    int64_t longrange_nnz;   /* entries in the long-range CSR (SKYLINE) */
    int64_t dense_tiles;     /* stored 64x64 tiles (DENSE) */
    int64_t device_bytes;    /* device memory owned by the graph */
    int32_t kind, storage, dtype;
    int32_t integer_weights; /* 1 when every J_ij is an integer (read graphs) */
    double c0_auto;          /* 0.5 / sqrt(sum_{i!=j} J_ij^2 / (n - 1)) */
    int32_t band_dtype;      /* SKYLINE: encoding of the band blocks the step kernel reads: the
                                graph's dtype, or QH_F16 for a BF16 graph whose band values are
                                all exactly representable in binary16 (same values) */
    double total_weight;     /* W = -1/2 sum_ab J_ab (the edge weights of A = -J summed once):
                                the Ising energy of Eq. (5) is E(s) = W - 2 cut(s).  Kept current
                                by qh_flip_crossing. */
    int64_t largest_component; /* vertices of the largest connected component (0 when every
                                component is a single vertex) */
} qh_graph_info;

/* Builds J from fragments (Methods: read-based Eqs. 1-3, SNP-based Eqs. 9-14).
 * Computes the FP64 master values, the connected components (single-vertex
 * components get label -1), the storage copy in `dtype`, and what qh_phase needs.
 * Synchronises `stream`.  Errors: EINVAL for malformed fragments (index out of range,
 * non-ascending SNPs, bad enum, max_device_bytes < 0), EUNSUPPORTED for
 * kind/storage/dtype combinations not offered, ENOMEM (also when the graph would
 * exceed opts->max_device_bytes), EHIP. */
qh_status qh_build_graph(const qh_reads *reads, const qh_snps *snps, const qh_graph_opts *opts,
                         qh_graph **out, void *stream);

/* Builds `count` graphs (Methods, as qh_build_graph for each): reads[i], snps[i] and
 * opts[i] describe graph i, out[i] receives it.  Host threads (`threads`, 0 = 8, at
 * most 64) take the graphs in index order, each building on a stream of its own, so
 * that the synchronisations inside one build overlap the work of the others; the
 * result is the same as count calls of qh_build_graph.  The device is synchronised first
 * (the fragment arrays may be written on `stream`); every graph is complete on return.
 * No other call of the library may run on another host thread meanwhile.
 * On failure no graph is returned (out is left untouched, graphs already built are
 * freed), the status is that of a graph that failed and qh_last_error names its index;
 * building stops early.  The caller owns the graphs (qh_graph_free each).  Errors as for qh_build_graph, and
 * EINVAL for count < 0 or threads outside 0..64. */
qh_status qh_build_graphs(int64_t count, const qh_reads *reads, const qh_snps *snps,
                          const qh_graph_opts *opts, qh_graph **out, int32_t threads,
                          void *stream);

qh_status qh_graph_free(qh_graph *g);
qh_status qh_graph_get_info(const qh_graph *g, qh_graph_info *out);

/* FP64 master values of rows [row0, row1) as dense rows: out is device
 * double [(row1 - row0) * n], fully overwritten (zeros where no edge). */
qh_status qh_graph_export_rows(const qh_graph *g, int64_t row0, int64_t row1, double *out,
                               void *stream);

/* The values the step kernel multiplies with, dequantized to FP64 (scale * code for
 * FP8_ROWSCALE), rows [row0, row1) as dense rows; device double [(row1-row0) * n]. */
qh_status qh_graph_export_stored_rows(const qh_graph *g, int64_t row0, int64_t row1,
                                      double *out, void *stream);

/* Component label per vertex (device int32 [n]); labels are numbered in the
 * order of each component's lowest vertex, -1 for single-vertex components. */
qh_status qh_graph_components(const qh_graph *g, int32_t *comp, void *stream);

/* ---------------------------------------------------------------------------
 * Ballistic simulated bifurcation (Methods, SB algorithm solution; the update
 * is the published bSB: symplectic Euler, y first):
 *   y_i <- y_i + [-(a0 - p_k) x_i + c0 (J x)_i] dt
 *   x_i <- x_i + a0 y_i dt
 *   |x_i| > 1  =>  x_i <- sgn(x_i), y_i <- 0        (inelastic walls)
 * for k = step_begin .. step_end-1, all R replicas at once; then s = sgn(x) with
 * sgn(0) = +1, FP64 cuts per replica and per component from the master values,
 * the best replica per component (ties -> lowest replica), oriented so that the
 * component's lowest vertex reads +1, and an optional greedy single-flip pass.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t replicas;    /* R: 16, 32, or a multiple of 64 */
    int32_t steps;       /* length of the pump schedule (>= 1) */
    int32_t step_begin;  /* run steps [step_begin, step_end) of the schedule; */
    int32_t step_end;    /*   step_end = 0 means `steps` (checkpoint / resume) */
    double dt;           /* time step */
    double c0;           /* coupling scale; <= 0 selects qh_graph_info.c0_auto */
    double a0;           /* detuning / mass term; 0 selects 1.0 */
    const float *pump;   /* device float [steps] schedule p_k, or NULL = p_k = k/(steps-1) */
    uint64_t seed;       /* SplitMix64 seed for x0, y0 when init = 1 */
    int32_t init;        /* 1: x0, y0 ~ U(-0.1, 0.1) from the seed (draw k = 2(r n + i) + {0,1});
                            0: start from the state passed in qh_result.x / .y */
    int32_t readout;     /* 1: signs, cuts, selection (+ greedy); 0: dynamics only */
    int32_t greedy;      /* 1: greedy single-flip rounds on the selected spins */
    int32_t use_graph;   /* 1: replay the step loop from a captured hipGraph (cached per
                            graph and option set); 0: plain stream launches */
    int32_t plan;        /* step-loop plan: 0 = autotuned; 1 = one fused kernel per step
                            (the tuned kernel when there is one); 2 = persistent (dense
                            16/8-bit graphs only).  SNP (skyline) graphs only: 3 = per-row
                            kernel; 4 = band blocks on FMAs (bit-identical to 3); 5 = band
                            blocks on MFMAs (four columns summed per MFMA: equal to 3-4 up
                            to FP32 rounding).  Plan 0 on SNP graphs times 4 and 5 once. */
    int32_t replica_tile; /* dense graphs, per-step plan, R >= 64: replicas per workgroup
                            (16, 32 or 64); 0 = the autotuner's choice (plan 0) or 64.
                            Every tile gives bit-identical results. */
    int32_t variant;     /* 0: ballistic SB (the coupling takes x_j); 1: discrete SB, the
                            same update with sgn(x_j) (sgn(0) = +1) in the coupling term */
    int32_t tiles_in_flight; /* dense per-step plan with 64 replicas per workgroup: stored
                            tiles whose loads are issued together (2 or 4); 0 = the
                            autotuner's choice or 2.  Bit-identical either way. */
    int32_t persistent_sync; /* persistent plan: how the 16-bit copy of x crosses workgroups
                            each step.  1 = plain accesses with agent-scope release/acquire
                            fences (L2 write-back / invalidate); 2 = every access of the copy
                            is device-coherent, no cache-wide fences; 0 = the autotuner's
                            choice or 1.  Bit-identical either way. */
    const float *field;  /* deformation term h of the adaptive strategy (Methods, SNP-based
                            solution): device float [n], the same for every replica, added
                            to the coupling sum of every step, y += (-(a0 - p_k) x_i +
                            c0 (sum_j J_ij x_j + h_i)) dt, the field of an Ising energy
                            -x'Jx/2 - h'x.  NULL = no field (the plain bSB step).  Batched
                            solves take it packed like the results (block b's vertices from
                            its vertex offset).  Caller-owned; read during the call only. */
    int32_t eval_every;  /* readout cadence m (Methods, SB algorithm solution: the best of many
                            samples; the solver comparison follows the energy over the run).
                            0: the spins are read out after the last step only.  m > 0: they
                            are also read out after steps step_begin + m, step_begin + 2m, ...
                            (and always after the last step); every evaluation computes the FP64
                            cut of every replica and component, and each component keeps the
                            best (evaluation, replica) seen so far -- largest cut, ties to the
                            earlier evaluation, then the lower replica -- whose spins become
                            best_spins (before the greedy pass).  The trajectory is the same as
                            with m = 0.  Needs readout = 1 and use_graph = 0 (EINVAL otherwise);
                            batched solves take 0 only. */
} qh_bsb_opts;

/* Result buffers (all device, caller-owned; optional ones may be NULL).
 *  x, y          float [n][R] state.  With init = 0 they supply the starting state.
 *                On return they hold the state after step_end-1 (if non-NULL).
 *  best_spins    int8 [n]      selected spins (after greedy when enabled)
 *  cuts          double [R]    FP64 cut of every replica (sum over components)
 *  cut_rc        double [R][n_comp] FP64 cut per replica and component (optional)
 *  best_replica  int32 [n_comp] selected replica per component (optional)
 *  selected_cut  double [1]    cut of the selected spins before greedy (optional)
 *  best_cut      double [1]    cut of best_spins
 *  all_spins     int8 [n][R]   every replica's signs (optional)
 *  greedy_rounds int32 [1]     rounds that flipped something (optional, host or device: device)
 *  best_energy   double [1]    Ising energy of best_spins, E = -1/2 s'Js (Eq. 5) = W - 2 best_cut
 *                              (optional; readout = 1)
 *  energy        double [n_eval][R]  Ising energy (Eq. 5) of every replica's signs at each
 *                              evaluation (optional; readout = 1), n_eval = 1 when eval_every = 0,
 *                              else max(1, ceil((step_end - step_begin) / eval_every)); row e is
 *                              the state after step min(step_begin + (e + 1) m, step_end).
 *  With eval_every > 0: cuts and cut_rc are those of the last evaluation; best_replica[c] and
 *  selected_cut refer to the best-so-far pick of each component. */
typedef struct {
    float *x;
    float *y;
    int8_t *best_spins;
    double *cuts;
    double *cut_rc;
    int32_t *best_replica;
    double *selected_cut;
    double *best_cut;
    int8_t *all_spins;
    int32_t *greedy_rounds;
    double *best_energy;
    double *energy;
} qh_result;

/* Runs bSB on one graph.  Synchronises the stream only when greedy = 1.
 * Errors: EINVAL (replicas not 16/32/64k, steps < 1, range outside the schedule,
 * init = 0 without x/y, readout without best_spins/cuts/best_cut, eval_every < 0 or
 * eval_every > 0 with readout = 0 or use_graph = 1), ENUMERIC when the state read out holds
 * NaN/Inf (checked when readout = 1), ENOMEM, EHIP. */
qh_status qh_bsb_solve(const qh_graph *g, const qh_bsb_opts *opts, qh_result *res, void *stream);

/* Step-loop plan chosen for (graph, replicas) by earlier solves.  plan_used: 0 = no solve
 * yet, 1 = one fused kernel per step, 2 = persistent (all steps in one cooperative
 * launch, state in registers, J in LDS).  With opts.plan = 0 the first solve of a
 * (graph, replicas) pair times the candidates on scratch state (64 steps each) and keeps
 * the fastest: the per-step kernel with 64 (two or four tiles in flight), 32 and 16
 * replicas per workgroup (dense graphs, R >= 64) and the persistent plan where it fits
 * (every candidate gives bit-identical results); us_per_step holds those
 * measurements (0 when not measured).  Host output.
 * The persistent plan synchronises neighbouring workgroups with agent-scope
 * release / acquire on per-workgroup step counters. */
typedef struct {
    int32_t plan_used;
    int32_t persistent_ok;      /* 1 when the persistent plan fits this graph */
    int32_t replicas_per_group; /* persistent plan: replicas per independent group */
    int32_t groups;             /* persistent plan: replica groups */
    int32_t workgroups_per_group;
    int32_t lds_bytes;          /* persistent plan: LDS per workgroup */
    float us_per_step[2];       /* autotuner: [per-step plan (best tile), persistent plan] */
    int32_t replica_tile;       /* per-step dense plan: replicas per workgroup in use */
    int32_t tiles_in_flight;    /* per-step dense plan: stored tiles whose loads are issued together */
    int32_t skyline_kernel;     /* SNP graphs: step kernel of the last solve: 3 rows, 4 band FMA, 5 band MFMA */
    float skyline_us[2];        /* SNP autotuner: [band FMA, band MFMA] microseconds per step (0 = not timed) */
    int32_t persistent_sync;    /* persistent plan of the last solve: 1 fences, 2 coherent accesses */
    float us_persistent_coherent; /* autotuner: persistent plan with coherent accesses (0 = not timed) */
} qh_plan_info;

qh_status qh_solve_plan_info(const qh_graph *g, int32_t replicas, qh_plan_info *out);

/* Runs the plan-0 autotuner for (graph, opts->replicas) on its own: the timing runs on
 * scratch state that qh_bsb_solve makes on its first plan-0 call, with opts' schedule.
 * *chosen receives *opts with plan, replica_tile, tiles_in_flight and persistent_sync
 * set to the choice: a qh_bsb_solve with them runs the same kernels without tuning (and
 * gives the same results, every candidate being bit-identical).  us_per_step (host float
 * [2], optional): the chosen plan's measured microseconds per step; SNP graphs: [band
 * FMA, band MFMA].  cache_path (optional): one JSON line is appended to this file with
 * the graph's shape (n, nnz, kind, storage, dtype, dense_tiles), the replica count, the
 * chosen options and the timings, for a later process to reuse.  Synchronises the stream.
 * Errors: EINVAL (options as for qh_bsb_solve; the cache file cannot be opened), EHIP. */
qh_status qh_autotune(const qh_graph *g, const qh_bsb_opts *opts, qh_bsb_opts *chosen, float *us_per_step,
                      const char *cache_path, void *stream);

/* Many independent graphs (phasing blocks) solved together: every block runs the same
 * schedule (steps, dt, a0, pump, seed) with its own c0 (opts->c0 <= 0: each block's
 * c0_auto), and block b's results equal qh_bsb_solve on graph b with the same options,
 * bit for bit.  R must be 16, 32 or 64; init = 1; the whole schedule; no long-range
 * couplings; each graph at most once per batch.  opts->plan: 1 = one launch per step over
 * work items of every block (a dense row tile, or four band blocks); 2 = one persistent
 * launch with whole blocks per workgroup (longest-processing-time placement); 0 = time
 * both on this batch (8 steps each) and cache the faster for this list of graphs and R.
 * Results are packed: block b's vertices start at vertex_offset[b] (= sum of the
 * previous blocks' n) in best_spins / x / y, and its replicas at b * R in cuts.
 *  best_spins int8 [sum n]; cuts double [n_blocks * R]; best_cut double [n_blocks];
 *  selected_cut double [n_blocks] (optional); x, y optional float [sum n * R];
 *  plan_used (host output) the plan that ran.  Greedy is applied per block when
 *  requested.  opts->use_graph = 1 runs the per-step plan from a captured hipGraph: the step
 *  launches are captured once per list of graphs, R and schedule (steps, dt, a0, pump, seed)
 *  and replayed by later calls with the same ones (the library keeps the last few batches);
 *  results are those of plan 1, bit for bit.  use_graph with plan 2 is EUNSUPPORTED, and
 *  plan 0 with use_graph runs plan 1 without tuning.  eval_every must be 0.  readout = 0
 *  runs the dynamics only (the result arrays other than x and y may then be NULL).
 *  Synchronises the stream. */
typedef struct {
    int8_t *best_spins;
    double *cuts;
    double *best_cut;
    double *selected_cut;
    float *x;
    float *y;
    int32_t plan_used;
} qh_batched_result;

qh_status qh_bsb_solve_batched(const qh_graph *const *graphs, int32_t n_graphs,
                               const qh_bsb_opts *opts, qh_batched_result *res, void *stream);

/* Haplotype reconstruction from spins (device int8 [n], +1 = subset S1).
 * Read graphs: per SNP the vote counts of Eqs. 7-8 and the hierarchical rule of the
 * paper; h1[j] is the allele of output haplotype 1 (= subset S1), -1 where the SNP is
 * filtered (no decisive support) or covered only by single-fragment components.
 * SNP graphs: one parity round (Eqs. 16-17): in each component the smaller subset
 * S_min (equal sizes: the s = -1 subset) swaps H1/H2; single-vertex components -> -1.
 * block[j] = component label of the SNP's phase block, -1 when unphased by structure.
 * h1 device int8 [n_snp], block device int32 [n_snp]. */
qh_status qh_phase(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block,
                   void *stream);

/* qh_phase for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same outputs as qh_phase, bit
 * for bit, with the per-component counters of the SNP parity round held in a static device
 * array of the library (4 MiB per device, kept until the process ends) instead of memory
 * allocated per call.  It allocates nothing, does not synchronise the stream, and clears the
 * counters with a kernel (no memset node when captured).  Limit: SNP graphs of at most 2^19
 * connected components (EINVAL beyond; read graphs have no limit, their vote needs no
 * scratch).  Every call on one device shares that array: calls that overlap on one device
 * (two streams, or two threads) race and may return wrong haplotypes; serialise them.
 * Errors: EINVAL (null argument, too many components, graph on another device), EHIP. */
qh_status qh_phase_noalloc(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block,
                           void *stream);

/* qh_phase of many graphs in one call (Methods, as qh_phase for each), for the blocks of a
 * batched solve: spins device int8 packed as qh_bsb_solve_batched's best_spins (graph b's
 * n_b vertices from sum_{c<b} n_c); h1 device int8 and block device int32 packed by SNP
 * (graph b's n_snp_b SNPs from sum_{c<b} n_snp_c).  Graph b's slices equal qh_phase on graph
 * b with its slice of spins, bit for bit (labels are each graph's own).  A few launches for
 * the whole list instead of a few per graph; allocates its tables and counters and
 * synchronises the stream.  Errors: EINVAL (null argument or graph, n_graphs < 0, a graph
 * on another device), ENOMEM, EHIP. */
qh_status qh_phase_batched(const qh_graph *const *graphs, int32_t n_graphs, const int8_t *spins,
                           int8_t *h1, int32_t *block, void *stream);

/* Eq. 15: J_uv <- -J_uv for every edge whose endpoints disagree in `spins` (device
 * int8 [n]); updates the master and the stored copy in place and recomputes
 * qh_graph_info.total_weight (c0_auto depends on J^2 only and does not change).
 * Synchronises the stream. */
qh_status qh_flip_crossing(qh_graph *g, const int8_t *spins, void *stream);

/* Iterative refinement of the SNP-based method (Eqs. 15-17), SNP graphs only.  Round t
 * (t = 0 .. max_rounds-1) runs qh_bsb_solve with opts (seed + t, readout on, whole
 * schedule) on the current weights.  Adaptive deformation (Methods, SNP-based solution;
 * deform > 0 and deform_tries > 0): while a component still being refined has a negative
 * cut, round t is solved again, at most deform_tries times, under the deformation field
 * h_i = (deform / c0) (2 u_i - 1) (opts.field replaced; u_i from SplitMix64 with the
 * round's seed at draw 2 n R + (a - 1) n + i for attempt a = 1, 2, ...), and each such
 * component takes the attempt's spins when their cut is higher.  deform = 0 or
 * deform_tries = 0: no deformation.  A component is finished for good when the cut of
 * its selected spins is not positive or they put all its vertices on one side.  In each
 * other component the vertices of the smaller subset S_min (the s = -1 subset on a tie)
 * add one to their flip counter C, and every edge crossing the partition changes sign
 * (Eq. 15).  The loop ends when every component is finished or after max_rounds.  The
 * graph's weights are restored exactly before return (also on error).  Outputs:
 *  h1         device int8 [n_snp]  H1 where C is even, H2 where C is odd; -1 unphased
 *  block      device int32 [n_snp] component label, -1 for single-vertex components
 *  flips      device int32 [n]     flip counters C (optional)
 *  round_cuts host double [max_rounds] cut applied in each round, summed over the
 *             components that flipped (optional)
 *  rounds     host int32           rounds that flipped something (optional)
 *  deformed   host int32           deformed solves run, over all rounds (optional)
 * Synchronises the stream.  Errors: EUNSUPPORTED (read graph), EINVAL (max_rounds < 1,
 * deform or deform_tries negative, init = 0, options as for qh_bsb_solve), ENUMERIC,
 * ENOMEM, EHIP. */
qh_status qh_refine(qh_graph *g, const qh_bsb_opts *opts, int32_t max_rounds, float deform, int32_t deform_tries,
                    int8_t *h1, int32_t *block, int32_t *flips, double *round_cuts, int32_t *rounds,
                    int32_t *deformed, void *stream);

/* Size-adaptive bSB settings of the SNP-based method (Tables 1 and 2, footnotes): 500
 * iterations for graphs below 5,000 nodes and 1,000 otherwise, 100 samples, at most 15
 * refinement rounds.  `size` is the vertex count the rule is applied to.  The paper solves
 * components independently; here the components of one graph share one schedule, so pass
 * the largest component's size (qh_graph_info.largest_component): every component then gets
 * at least the paper's count for its own size.  The solvers take 16, 32 or a multiple of 64
 * replicas, so the 100 samples run as replicas = 128 (more samples never lower the best cut
 * of a component).  Host output; no device work.  Errors: EINVAL (null out, size < 0). */
typedef struct {
    int32_t steps;
    int32_t samples;     /* the paper's sample count */
    int32_t replicas;    /* replicas the solvers run for those samples */
    int32_t max_rounds;  /* refinement rounds (qh_refine's max_rounds) */
    int64_t size;        /* the vertex count the rule was applied to */
} qh_schedule;

qh_status qh_adaptive_schedule(int64_t size, qh_schedule *out);

/* Hands every cached idle block of device memory (see Conventions) back to the devices
 * with hipFree, for callers that need the memory elsewhere (PyTorch's allocator, other
 * libraries).  Blocks in use are untouched.  released (optional host int64): the bytes
 * handed back.  Must not run concurrently with another library call.  Errors: none beyond
 * EHIP. */
qh_status qh_release_cached_memory(int64_t *released);

const char *qh_last_error(void);
const char *qh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QHAP_H */

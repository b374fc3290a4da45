// Internal declarations of the gfx950 phasing library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "qhap.h"

namespace qh {

// Internal failure carried to the ABI boundary, where it becomes a qh_status.
struct Failure {
    qh_status st;
};

void set_error(const char *fmt, ...);
[[noreturn]] void fail(qh_status st, const char *fmt, ...);
[[noreturn]] void fail_hip(hipError_t e, const char *what, const char *file, int line);

#define QH_HIP(call)                                                        \
    do {                                                                    \
        hipError_t qh_e_ = (call);                                          \
        if (qh_e_ != hipSuccess) ::qh::fail_hip(qh_e_, #call, __FILE__, __LINE__); \
    } while (0)

#define QH_CHECK_LAUNCH() QH_HIP(hipGetLastError())

// Library device memory (memory.hip): size-classed blocks cached per device.
void *device_alloc(size_t bytes);   // nullptr when the device is out of memory
void device_free(void *p);
// Pools of the block cache: the calling thread takes and returns blocks in pool `tag`
// (0 = the shared pool); merge_pool moves pool `tag` of a device into the shared pool
// (only once no queued work can still use its blocks).
void set_pool(uintptr_t tag);
void merge_pool(int device, uintptr_t tag);
// hands every cached idle block of every device back with hipFree; returns the bytes released
size_t release_cached();

// Owning device buffer.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        if (p) {   // the old block may still be read by queued work on any stream
            QH_HIP(hipDeviceSynchronize());
            release();
        }
        if (count == 0) count = 1;
        p = (T *)device_alloc(count * sizeof(T));
        if (!p) fail(QH_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
        n = count;
    }
    void release() {
        device_free(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    void upload(const T *host, size_t count, hipStream_t st) {
        if (count) QH_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, st));
    }
    void zero(hipStream_t st) { if (p) QH_HIP(hipMemsetAsync(p, 0, n * sizeof(T), st)); }
};

template <class T>
std::vector<T> download(const T *dev, size_t count, hipStream_t st) {
    std::vector<T> h(count);
    if (count) {
        QH_HIP(hipMemcpyAsync(h.data(), dev, count * sizeof(T), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
    }
    return h;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kTile = 64;            // dense tile edge
constexpr int kTileElems = kTile * kTile;

// Bytes per stored element of each dtype.
inline int dtype_bytes(int dt) {
    switch (dt) {
        case QH_F32: return 4;
        case QH_F16: case QH_BF16: return 2;
        case QH_FP8_ROWSCALE: return 1;
    }
    return 0;
}

struct PersistPlan;

// Cached state of one solve configuration (scratch buffers + captured graph).
struct SolvePlan {
    std::shared_ptr<PersistPlan> pp;   // persistent dense plan (null until tried)
    bool pp_tried = false;
    int tuned_plan = 0;                // autotuner's choice for plan 0: 1 per-step, 2 persistent
    int last_plan = 0;                 // plan the last solve ran
    int sky_kernel = 0;                // SNP graphs: kSkyBandFma, kSkyBandMfma or kSkyRows
    bool sky_tuned = false;            // the band kernels have been timed on this graph
    int sky_best = 0;                  // the faster band kernel
    float sky_us[3] = {0, 0, 0};       // measured microseconds per step of each kernel
    float tuned_us[2] = {0, 0};        // measured microseconds per step: per-step, persistent (fences)
    float tuned_us_coh = 0;            // persistent with device-coherent accesses
    bool tuned_coh = false;            // the autotuner's persistent variant is the coherent one
    int last_coh = 0;                  // variant of the last persistent run
    int tuned_rt = 0;                  // autotuner's replica tile for the per-step dense kernel
    int tuned_depth = 2;               // autotuner's tiles in flight for 64-replica tiles (2 or 4)
    int run_rt = 64;                   // replica tile of the dense step launches (R >= 64)
    int run_depth = 2;                 // tiles in flight of those launches
    int R = 0;
    int64_t n_pad = 0;
    DevBuf<float> xa, xb, y;        // fp32 state, [n_pad][R]
    DevBuf<uint16_t> ha, hb;        // 16-bit product copies of x (dense f16/bf16/fp8 paths)
    DevBuf<uint16_t> la, lb;        // binary16 copies of x [n][R] (paired with xa / xb) that the
                                    // long-range gathers read (16-bit SNP graphs with long-range rows)
    DevBuf<float> pump_lin;         // linear schedule for `steps`
    int pump_steps = 0;
    DevBuf<int8_t> spins;           // [n][R]
    DevBuf<double> part;            // [n_chunks][R] cut partials
    DevBuf<double> rowcut;          // [n_ord][R] cut row sums (vertices in component order)
    DevBuf<double> cut_rc;          // [R][n_comp]
    DevBuf<int32_t> best_r;         // [n_comp]
    DevBuf<double> gain;            // [n]
    DevBuf<int8_t> flag;            // [n]
    DevBuf<int32_t> counter;        // small scalars
    DevBuf<double> part1;           // [n_chunks] partials for one vector
    DevBuf<double> cut1;            // [n_comp]
    DevBuf<float> hub_part;         // [n_hub_chunks][R] long-range partial sums of hub rows
    // readout every eval_every steps: best (evaluation, replica) so far per component
    DevBuf<double> ev_cut;          // [n_comp] its cut
    DevBuf<int32_t> ev_r;           // [n_comp] its replica
    DevBuf<int8_t> ev_take;         // [n_comp] 1 when the current evaluation replaced it
    // captured step loop
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::tuple<int, int, int, double, double, double, const float *, int, int, const float *> graph_key{};
    ~SolvePlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

}  // namespace qh

struct qh_graph {
    uint64_t serial = 0;   // unique per graph in the process (keys cached batch plans)
    int64_t max_bytes = 0; // cap on the device memory the graph owns (0: none)
    int deterministic = 0; // SNP weights summed in fixed point (order-independent)
    int device = 0;
    int kind = 0, storage = 0, dtype = 0;
    int64_t n = 0;         // vertices
    int32_t n_snp = 0;
    bool integer = false;

    // FP64 master: CSR of the nonzero off-diagonal couplings, columns ascending.
    qh::DevBuf<int64_t> m_ptr;
    qh::DevBuf<int32_t> m_col;
    qh::DevBuf<double> m_val;
    int64_t nnz = 0;

    // Components (labels in order of lowest vertex, -1 = singleton).
    qh::DevBuf<int32_t> comp;        // [n]
    int64_t n_comp = 0;
    int64_t largest_comp = 0;        // vertices of the largest component
    qh::DevBuf<int32_t> comp_first;  // [n_comp] lowest vertex
    qh::DevBuf<int32_t> comp_order;  // vertices of non-singleton components sorted by (comp, vertex)
    int64_t n_ord = 0;               // length of comp_order
    // reduction chunks over comp_order: (comp, begin, end) per chunk; chunks of a
    // component are consecutive and in vertex order
    qh::DevBuf<int32_t> chunk_comp, chunk_begin, chunk_end;
    int64_t n_chunks = 0;
    qh::DevBuf<int32_t> comp_chunk_ptr;  // [n_comp + 1]

    // Dense tiles (read graphs).
    int64_t n_rt = 0;                   // row tiles
    int64_t n_tiles = 0;
    qh::DevBuf<int32_t> t_ptr;          // [n_rt + 1]
    qh::DevBuf<int32_t> t_col;          // [n_tiles] column-tile index
    qh::DevBuf<uint8_t> t_val;          // [n_tiles][4096] elements in MFMA fragment order
    qh::DevBuf<float> row_scale;        // FP8: per-row scale (x 256 for the code decode)

    // Skyline band (SNP graphs).
    qh::DevBuf<int64_t> s_off;          // [n]
    qh::DevBuf<int32_t> s_lo, s_len;    // [n]
    qh::DevBuf<uint8_t> s_val;          // slots in dtype
    int64_t s_slots = 0;
    int32_t band_limit = 0;
    // Band blocks of kBandRows consecutive rows: the union column range [bb_lo, bb_lo + bb_w)
    // of the block's skyline rows, stored column by column with kBandRows row values each
    // (zero outside a row's own range), in dtype.
    qh::DevBuf<int64_t> bb_off;         // [n_bblk] element offset of the block
    qh::DevBuf<int32_t> bb_lo, bb_w;    // [n_bblk]
    qh::DevBuf<uint8_t> bb_val;
    int64_t n_bblk = 0, bb_elems = 0;
    // Encoding of bb_val: the graph's dtype, except that the BF16 band values of a graph are
    // stored as binary16 holding value * 2^s when one power of two brings all of them into
    // binary16 exactly (cheaper to expand); the band kernels multiply their sums by
    // bb_scale = 2^-s, which restores the BF16 products bit for bit.
    int bb_dtype = 0;
    float bb_scale = 1.0f;
    double snp_flush = 0.0;             // BF16 SNP storage: magnitudes below this are stored as 0
    // Long-range CSR (pairs farther apart than band_limit).
    qh::DevBuf<int64_t> l_ptr;          // [n + 1]
    qh::DevBuf<int32_t> l_col;
    qh::DevBuf<uint8_t> l_val;          // dtype
    int64_t l_nnz = 0;
    // Long-range rows are summed by chunks of at most kHubChunk entries in a separate
    // kernel (full parallelism for the gathers, long rows split); the step kernel adds the
    // chunk partials of its row in order.  Chunks tile the long-range entries in row order.
    qh::DevBuf<int32_t> row_chunk_ptr;  // [n + 1] chunks of row u: [ptr[u], ptr[u + 1])
    qh::DevBuf<int64_t> hub_chunk_beg, hub_chunk_end;
    qh::DevBuf<int32_t> lr_pk_ptr;      // [n_lr_pk + 1] first chunk of each packet (<= 64 entries)
    int64_t n_hub_chunks = 0, n_lr_pk = 0;

    // Phasing support.
    qh::DevBuf<uint8_t> init_h1;        // [n_snp]
    qh::DevBuf<int64_t> cov_ptr;        // read graphs: per-SNP coverage lists
    qh::DevBuf<int32_t> cov_frag;
    qh::DevBuf<int8_t> cov_M;

    double c0_auto = 0.0;
    double total_weight = 0.0;   // -1/2 sum of the master J (fixed-order sum)
    double greedy_eps = 0.0;
    int64_t device_bytes = 0;

    std::map<int, std::unique_ptr<qh::SolvePlan>> plans;  // keyed by replicas
};

namespace qh {

constexpr int kBandRows = 16;       // rows per band block (one wave's accumulators)
constexpr int kSkyBandFma = 0, kSkyBandMfma = 1, kSkyRows = 2;   // SNP step kernels
constexpr int kHubChunk = 64;       // entries per hub partial

// graph_build.hip
void build_read_graph(qh_graph *g, const qh_reads *r, const qh_snps *s, hipStream_t st);
void build_snp_graph(qh_graph *g, const qh_reads *r, const qh_snps *s, int linkage_k,
                     int band_limit, hipStream_t st);
void finalize_graph(qh_graph *g, hipStream_t st);
void export_master_rows(const qh_graph *g, int64_t r0, int64_t r1, double *out, hipStream_t st);
void export_stored_rows(const qh_graph *g, int64_t r0, int64_t r1, double *out, hipStream_t st);
void flip_crossing(qh_graph *g, const int8_t *spins, hipStream_t st);

// bsb.hip
void bsb_solve(const qh_graph *g, const qh_bsb_opts *o, qh_result *res, hipStream_t st);
void autotune(const qh_graph *g, const qh_bsb_opts *o, qh_bsb_opts *chosen, float *us, hipStream_t st);

// What the readout needs of a graph (a single graph, or the block-diagonal union of a batch).
struct ReadoutView {
    int64_t n = 0, n_comp = 0, n_chunks = 0, n_ord = 0;
    const int64_t *m_ptr = nullptr;
    const int32_t *m_col = nullptr;
    const double *m_val = nullptr;
    const int32_t *comp = nullptr, *comp_first = nullptr, *comp_order = nullptr;
    const int32_t *chunk_begin = nullptr, *chunk_end = nullptr, *comp_chunk_ptr = nullptr;
    double eps = 0.0;                  // greedy tolerance
    const double *eps_v = nullptr;     // per-vertex tolerance (overrides eps when set)
};
ReadoutView view_of(const qh_graph *g);
// One evaluation of a solve read out every eval_every steps: its index, whether it is the
// last, and the energy row it fills (nullptr: none); W = -1/2 sum J.
struct EvalArgs {
    int index = 0;
    bool last = true;
    double W = 0.0;
    double *energy_row = nullptr;
};
// finish = false leaves the non-finite check to the caller (p.counter[1] != 0 after a sync).
// ev != nullptr: one evaluation of a solve read out every eval_every steps; only the last one
// runs the greedy pass and the final cut (and the check, with finish).
void readout(const ReadoutView &g, SolvePlan &p, int R, const float *xfin, const float *yfin, qh_result *res,
             bool greedy, hipStream_t st, bool finish = true, const EvalArgs *ev = nullptr);
void alloc_readout_scratch(SolvePlan &p, int64_t n, int64_t n_comp, int64_t n_chunks, int R);

// One block of a batched readout: its graph view, final state, plan scratch and result slots.
struct ReadoutDesc {
    int64_t n, n_comp, n_chunks, n_ord;
    const int64_t *m_ptr;
    const int32_t *m_col;
    const double *m_val;
    const int32_t *comp, *comp_first, *comp_order, *chunk_begin, *chunk_end, *comp_chunk_ptr;
    double eps;
    const float *x, *y;
    int8_t *spins;
    double *rowcut, *part, *cut_rc;
    int32_t *best_r;
    double *gain;
    int8_t *flag;
    double *part1, *cut1;
    int8_t *best_spins;
    double *cuts, *best_cut, *selected_cut;
    int32_t integer;            // 1: integer weights (any summation order is exact)
    double *gain_acc;           // integer blocks: sum of the greedy pass's applied gains (set by the readout)
};
void readout_batched(const std::vector<ReadoutDesc> &descs, int R, bool greedy, hipStream_t st);
void plan_info(const qh_graph *g, int R, qh_plan_info *out);

// phase.hip
void phase(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block, hipStream_t st);
void phase_noalloc(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block, hipStream_t st);
void phase_batched(const qh_graph *const *gs, int nb, const int8_t *spins, int8_t *h1, int32_t *block,
                   hipStream_t st);
void refine(qh_graph *g, const qh_bsb_opts *o, int max_rounds, float deform, int deform_tries, int8_t *h1,
            int32_t *block, int32_t *flips, double *round_cuts, int32_t *rounds_out, int32_t *deformed_out,
            hipStream_t st);

// Device-side descriptor of one block of a batched solve.
struct BlockDesc {
    int32_t kind;               // 0 dense tiles, 1 band blocks
    int32_t dtype;
    int64_t n;
    float *x, *y;               // fp32 state [n_pad][R]; x holds the final spins' amplitudes
    int64_t n_rt;
    const int32_t *t_ptr, *t_col;
    const uint8_t *t_val;
    const float *row_scale;
    int64_t n_bblk;
    const int64_t *bb_off;
    const int32_t *bb_lo, *bb_w;
    const uint8_t *bb_val;
    float c0;
    float bscale;               // band blocks: scale undoing their binary16 encoding (1: none)
    int32_t discrete;           // 1: the coupling takes sgn(x_j)
    uint16_t *h0, *h1;          // dense 16/8-bit: product copies [n_pad/8][R][8]
    float *xs;                  // dense f32 / band: second x buffer [n_pad][R]
    const float *field;         // deformation field of the block's vertices [n] (nullptr: none)
};
void launch_batched(int R, int workers, const BlockDesc *blocks, const int32_t *sched_ptr, const int32_t *sched,
                    int steps, float dt, float a0, const float *pump, uint64_t seed, hipStream_t st);
int batched_workers_per_cu(int R);
// per-step plan: init of every block, then per step one launch per class over that class's
// work items (x = block, y = row tile of a dense block or group of four band blocks);
// class c's items are items[class_ptr[c] .. class_ptr[c + 1])
constexpr int kBatchClasses = 7;   // dense F32/F16/BF16/FP8, band F32/F16/BF16
// The items of one class split into one list per XCD: XCD x (the XCD that runs workgroup
// blockIdx.x when blockIdx.x % 8 == x) works through items [off[x], off[x + 1]) of the
// class, in order.  Whole blocks go to one XCD (their x copy stays in that XCD's L2).
constexpr int kXcds = 8;
struct XcdSplit {
    int64_t off[kXcds + 1];
};
void launch_batched_steps(int R, int nb, const BlockDesc *blocks, const int2 *items, const int64_t *class_ptr,
                          const XcdSplit *splits, int steps, float dt, float a0, const float *pump, uint64_t seed,
                          hipStream_t st);
// SplitMix64 (Steele, Lea & Flood 2014): the k-th output of the generator seeded with seed
__device__ inline uint64_t sm64_draw(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

SolvePlan &solve_plan(const qh_graph *g, int R, hipStream_t st);
// Between these two calls on one thread, new plans' state buffers are collected instead of
// cleared one by one; the end clears them all with one kernel (and synchronises st).
void begin_plan_zeroing(std::vector<std::pair<void *, size_t>> &list);
void end_plan_zeroing(std::vector<std::pair<void *, size_t>> &list, DevBuf<uint64_t> &table, hipStream_t st);
const float *linear_pump(SolvePlan &p, int steps, hipStream_t st);   // p_k = k / (steps - 1)

// batched.hip
void bsb_solve_batched(const qh_graph *const *gs, int n, const qh_bsb_opts *o,
                       qh_batched_result *res, hipStream_t st);

// host-side components from unions
int64_t label_components(int64_t n, std::vector<int32_t> &parent, std::vector<int32_t> &comp_out);
void upload_components(qh_graph *g, const std::vector<int32_t> &comp, int64_t n_comp,
                       hipStream_t st);

}  // namespace qh

// Many independent phasing blocks (connected components / regions) solved together.
// Every block keeps its own couplings, c0, state and readout; the blocks share the
// schedule (steps, dt, a0, pump) and the seed.  Two plans:
//
//  per-step (plan 1): one launch per step over work items of every block (a dense row
//    tile, or four band blocks), so a large block is spread over many workgroups and the
//    chip sees tens of thousands of independent items per step;
//  whole-block (plan 2): one persistent launch, whole blocks per workgroup, placed by the
//    longest-processing-time rule on estimated bytes per step; the steps of a block are
//    separated by workgroup barriers only.  Best when every block is small.
//
// Plan 0 times both on the batch (a few steps each) and caches the faster for that list of
// graphs and replica count.  Either way the arithmetic and its order are those of the
// single-graph kernels, so block b's result equals qh_bsb_solve on graph b, bit for bit.
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <queue>
#include <vector>

#include "internal.h"

namespace qh {

static std::mutex g_plan_mu;
static std::map<std::vector<uint64_t>, int> g_plan_cache;   // (graph serials..., R) -> plan

static int cached_batch_plan(const std::vector<uint64_t> &key) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plan_cache.find(key);
    return it == g_plan_cache.end() ? 0 : it->second;
}

static void store_batch_plan(const std::vector<uint64_t> &key, int plan) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plan_cache.size() > 256) g_plan_cache.clear();
    g_plan_cache[key] = plan;
}

// The per-step plan's launches captured once for a batch (graph serials + R) and one set of
// launch arguments (block table, work items, steps, dt, a0, pump, seed): replayed while the
// key matches.  The block table and item list it points to live here too, so a replay never
// reads a freed buffer; the few most recent batches are kept.  An entry is destroyed when a
// newer batch pushes it out; those still listed at process exit are left to the process's
// end (no static destructor touches the runtime while it tears itself down).
struct CapturedBatch {
    std::vector<uint64_t> key;           // graph serials..., R, device
    DevBuf<BlockDesc> desc;
    DevBuf<int2> items;
    int64_t class_ptr[kBatchClasses + 1] = {0};
    std::vector<XcdSplit> splits;
    std::tuple<int, float, float, const float *, uint64_t> args{};
    hipGraphExec_t exec = nullptr;
};
static std::vector<CapturedBatch *> g_captured;   // most recent last; at most kCapturedBatches
constexpr size_t kCapturedBatches = 4;

static double block_cost(const qh_graph *g, int R) {
    const double eb = dtype_bytes(g->dtype);
    const double state = (double)g->n * R * 12.0;
    if (g->storage == QH_STORE_DENSE) return (double)g->n_tiles * kTile * kTile * eb + state;
    return (double)g->bb_elems * eb + state;
}

void bsb_solve_batched(const qh_graph *const *gs, int nb, const qh_bsb_opts *o, qh_batched_result *res,
                       hipStream_t st) {
    const int R = o->replicas;
    if (R != 16 && R != 32 && R != 64) fail(QH_EUNSUPPORTED, "batched solves take 16, 32 or 64 replicas");
    if (!o->init) fail(QH_EINVAL, "batched solves start from the seeded initial state (init = 1)");
    if (o->step_begin != 0 || (o->step_end != 0 && o->step_end != o->steps))
        fail(QH_EINVAL, "batched solves run the whole schedule");
    if (o->plan < 0 || o->plan > 2) fail(QH_EINVAL, "batched plan must be 0, 1 or 2, got %d", o->plan);
    res->plan_used = 0;
    if (nb == 0) return;
    int dev = 0;
    QH_HIP(hipGetDevice(&dev));
    for (int b = 0; b < nb; ++b) {
        if (!gs[b]) fail(QH_EINVAL, "graph %d is null", b);
        if (gs[b]->device != dev) fail(QH_EINVAL, "graph %d lives on device %d, current device is %d", b,
                                       gs[b]->device, dev);
        if (gs[b]->storage != QH_STORE_DENSE && gs[b]->l_nnz > 0)
            fail(QH_EUNSUPPORTED, "graph %d has long-range couplings; solve it on its own", b);
        if (gs[b]->storage != QH_STORE_DENSE && gs[b]->dtype == QH_FP8_ROWSCALE)
            fail(QH_EUNSUPPORTED, "graph %d: FP8 applies to dense storage only", b);
    }
    {   // every block owns its state buffers: a graph may appear once per batch
        std::vector<const qh_graph *> seen(gs, gs + nb);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            fail(QH_EINVAL, "a graph appears twice in one batch");
    }
    const double a0 = o->a0 > 0.0 ? o->a0 : 1.0;

    // per-block plans: state buffers and readout scratch of the single-graph solve
    std::vector<SolvePlan *> plans(nb);
    {   // new plans' buffers cleared together, with one kernel
        std::vector<std::pair<void *, size_t>> zl;
        DevBuf<uint64_t> zt;
        begin_plan_zeroing(zl);
        try {
            for (int b = 0; b < nb; ++b) plans[b] = &solve_plan(gs[b], R, st);
        } catch (...) {
            // the plans made so far stay with their graphs: clear them before failing
            try {
                end_plan_zeroing(zl, zt, st);
            } catch (...) {
            }
            throw;
        }
        end_plan_zeroing(zl, zt, st);
    }
    const float *pump = o->pump ? o->pump : linear_pump(*plans[0], o->steps, st);

    std::vector<BlockDesc> desc(nb);
    int64_t foff = 0;   // the field is packed like the results: block b from its vertex offset
    for (int b = 0; b < nb; ++b) {
        const qh_graph *g = gs[b];
        SolvePlan &p = *plans[b];
        BlockDesc &d = desc[b];
        d = BlockDesc{};
        d.kind = g->storage == QH_STORE_DENSE ? 0 : 1;
        d.dtype = g->storage == QH_STORE_DENSE ? g->dtype : g->bb_dtype;
        d.bscale = g->storage == QH_STORE_DENSE ? 1.0f : g->bb_scale;
        d.n = g->n;
        d.x = p.xa.p;
        d.y = p.y.p;
        d.c0 = (float)(o->c0 > 0.0 ? o->c0 : g->c0_auto);
        d.discrete = o->variant == 1;
        d.field = o->field ? o->field + foff : nullptr;
        foff += g->n;
        if (d.kind == 0) {
            d.n_rt = g->n_rt;
            d.t_ptr = g->t_ptr.p;
            d.t_col = g->t_col.p;
            d.t_val = g->t_val.p;
            d.row_scale = g->row_scale.p;
            if (g->dtype == QH_F32) d.xs = p.xb.p;
            else { d.h0 = p.ha.p; d.h1 = p.hb.p; }
        } else {
            d.n_bblk = g->n_bblk;
            d.bb_off = g->bb_off.p;
            d.bb_lo = g->bb_lo.p;
            d.bb_w = g->bb_w.p;
            d.bb_val = g->bb_val.p;
            d.xs = p.xb.p;
        }
    }

    std::vector<double> cost(nb);
    for (int b = 0; b < nb; ++b) cost[b] = block_cost(gs[b], R);
    std::vector<int> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    DevBuf<BlockDesc> d_desc(nb);
    QH_HIP(hipMemcpyAsync(d_desc.p, desc.data(), nb * sizeof(BlockDesc), hipMemcpyHostToDevice, st));

    // per-step plan: work items grouped by class (storage x dtype); within a class the blocks
    // are spread over the XCDs by the longest-processing-time rule on their bytes per step
    // (a block's items stay on one XCD, whose L2 then holds its x copy), and each XCD's list
    // runs its largest blocks first, items of a block adjacent.  Sorted blocks split into
    // contiguous ranges per XCD would give one XCD all the longest row tiles.
    std::vector<int2> items;
    int64_t class_ptr[kBatchClasses + 1] = {0};
    std::vector<XcdSplit> splits(kBatchClasses);
    auto class_of = [](const qh_graph *g) {
        if (g->storage == QH_STORE_DENSE)
            return g->dtype == QH_F32 ? 0 : g->dtype == QH_F16 ? 1 : g->dtype == QH_BF16 ? 2 : 3;
        return g->bb_dtype == QH_F32 ? 4 : g->bb_dtype == QH_F16 ? 5 : 6;
    };
    for (int c = 0; c < kBatchClasses; ++c) {
        std::vector<std::vector<int32_t>> lists(kXcds);
        double load[kXcds] = {0};
        for (int b : order) {
            if (class_of(gs[b]) != c) continue;
            const int x = (int)(std::min_element(load, load + kXcds) - load);
            load[x] += cost[b];
            lists[x].push_back(b);
        }
        XcdSplit &xs = splits[c];
        xs.off[0] = 0;
        for (int x = 0; x < kXcds; ++x) {
            for (int b : lists[x]) {
                const qh_graph *g = gs[b];
                const int64_t m = g->storage == QH_STORE_DENSE ? g->n_rt : ceil_div(g->n_bblk, 4);
                for (int64_t i = 0; i < m; ++i) items.push_back(make_int2(b, (int)i));
            }
            xs.off[x + 1] = (int64_t)items.size() - class_ptr[c];
        }
        class_ptr[c + 1] = (int64_t)items.size();
    }
    const int64_t n_items = (int64_t)items.size();
    DevBuf<int2> d_items(std::max<int64_t>(n_items, 1));
    if (n_items)
        QH_HIP(hipMemcpyAsync(d_items.p, items.data(), n_items * sizeof(int2), hipMemcpyHostToDevice, st));

    // whole-block plan: longest-processing-time placement of blocks on workers
    int cus = 0;
    QH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int workers = (int)std::min<int64_t>(nb, (int64_t)std::max(cus, 1) * batched_workers_per_cu(R));
    using Load = std::pair<double, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int w = 0; w < workers; ++w) heap.push({0.0, w});
    std::vector<std::vector<int32_t>> lists(workers);
    for (int b : order) {
        Load l = heap.top();
        heap.pop();
        lists[l.second].push_back(b);
        heap.push({l.first + cost[b], l.second});
    }
    std::vector<int32_t> sptr(workers + 1, 0), sched;
    sched.reserve(nb);
    for (int w = 0; w < workers; ++w) {
        sched.insert(sched.end(), lists[w].begin(), lists[w].end());
        sptr[w + 1] = (int32_t)sched.size();
    }
    DevBuf<int32_t> d_sptr(workers + 1), d_sched(nb);
    QH_HIP(hipMemcpyAsync(d_sptr.p, sptr.data(), (workers + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    QH_HIP(hipMemcpyAsync(d_sched.p, sched.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));

    auto run = [&](int plan, int steps, uint64_t seed) {
        if (plan == 2) launch_batched(R, workers, d_desc.p, d_sptr.p, d_sched.p, steps, (float)o->dt, (float)a0, pump,
                                      seed, st);
        else launch_batched_steps(R, nb, d_desc.p, d_items.p, class_ptr, splits.data(), steps, (float)o->dt,
                                  (float)a0, pump, seed, st);
    };
    // use_graph: the per-step plan replayed from a captured hipGraph.  The capture reads the
    // block table and items from buffers owned by the cache entry; the table is uploaded into
    // it on every call (same graphs and R: same layout), so a replay sees this call's c0,
    // variant and field.
    auto run_captured = [&](int steps, uint64_t seed) {
        std::vector<uint64_t> key(nb + 2);
        for (int b = 0; b < nb; ++b) key[b] = gs[b]->serial;
        key[nb] = (uint64_t)R;
        key[nb + 1] = (uint64_t)dev;
        std::lock_guard<std::mutex> lk(g_plan_mu);
        CapturedBatch *cb = nullptr;
        for (size_t i = 0; i < g_captured.size(); ++i)
            if (g_captured[i]->key == key) {
                cb = g_captured[i];
                g_captured.erase(g_captured.begin() + i);
                break;
            }
        if (!cb) {
            cb = new CapturedBatch();
            cb->key = key;
            cb->desc.alloc(nb);
            cb->items.alloc(std::max<int64_t>(n_items, 1));
            if (n_items)
                QH_HIP(hipMemcpyAsync(cb->items.p, items.data(), n_items * sizeof(int2), hipMemcpyHostToDevice, st));
            std::copy(class_ptr, class_ptr + kBatchClasses + 1, cb->class_ptr);
            cb->splits = splits;
        }
        g_captured.push_back(cb);   // most recent last
        if (g_captured.size() > kCapturedBatches) {
            // drop the least recent entry once no queued replay can still read its buffers
            CapturedBatch *old = g_captured.front();
            g_captured.erase(g_captured.begin());
            QH_HIP(hipDeviceSynchronize());
            if (old->exec) (void)hipGraphExecDestroy(old->exec);
            delete old;
        }
        QH_HIP(hipMemcpyAsync(cb->desc.p, desc.data(), nb * sizeof(BlockDesc), hipMemcpyHostToDevice, st));
        const auto args = std::make_tuple(steps, (float)o->dt, (float)a0, pump, seed);
        if (!cb->exec || cb->args != args) {
            if (cb->exec) { (void)hipGraphExecDestroy(cb->exec); cb->exec = nullptr; }
            hipStream_t cs;
            QH_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            QH_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            try {
                launch_batched_steps(R, nb, cb->desc.p, cb->items.p, cb->class_ptr, cb->splits.data(), steps,
                                     (float)o->dt, (float)a0, pump, seed, cs);
            } catch (...) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(cs, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                (void)hipStreamDestroy(cs);
                throw;
            }
            QH_HIP(hipStreamEndCapture(cs, &graph));
            QH_HIP(hipStreamDestroy(cs));
            const hipError_t e = hipGraphInstantiate(&cb->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) { cb->exec = nullptr; fail_hip(e, "hipGraphInstantiate", __FILE__, __LINE__); }
            cb->args = args;
        }
        QH_HIP(hipGraphLaunch(cb->exec, st));
    };
    if (o->use_graph && o->plan == 2)
        fail(QH_EUNSUPPORTED, "the whole-block plan is one launch already; use_graph applies to the per-step plan");
    int plan = o->plan == 2 ? 2 : 1;
    if (o->plan == 0 && o->steps > 0 && !o->use_graph) {
        std::vector<uint64_t> key(nb + 1);
        for (int b = 0; b < nb; ++b) key[b] = gs[b]->serial;
        key[nb] = (uint64_t)R;
        plan = cached_batch_plan(key);
        if (!plan) {
            // time both plans on the real buffers (a few steps each; the state is re-seeded below)
            const int nt = std::min(o->steps, 8);
            hipEvent_t e0, e1;
            QH_HIP(hipEventCreate(&e0));
            QH_HIP(hipEventCreate(&e1));
            float ms[2] = {0, 0};
            for (int c = 0; c < 2; ++c) {
                run(c + 1, nt, 0x5eed);                         // warm
                QH_HIP(hipEventRecord(e0, st));
                run(c + 1, nt, 0x5eed);
                QH_HIP(hipEventRecord(e1, st));
                QH_HIP(hipEventSynchronize(e1));
                QH_HIP(hipEventElapsedTime(&ms[c], e0, e1));
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            plan = ms[1] < ms[0] ? 2 : 1;
            store_batch_plan(key, plan);
        }
    }
    if (o->steps > 0) {
        if (o->use_graph) run_captured(o->steps, o->seed);
        else run(plan, o->steps, o->seed);
    }
    res->plan_used = plan;
    // the per-step plan ping-pongs x like the single-graph solve; the whole-block plan
    // leaves the final x in the first half
    const int final_half = plan == 1 ? (o->steps & 1) : 0;

    if (!o->readout) {   // dynamics only: the final state of every block, when asked for
        int64_t off = 0;
        for (int b = 0; b < nb; ++b) {
            const qh_graph *g = gs[b];
            SolvePlan &p = *plans[b];
            const int64_t nR = g->n * R;
            const bool pingpong = !(g->storage == QH_STORE_DENSE && g->dtype != QH_F32);
            const float *xfin = (pingpong && final_half) ? p.xb.p : p.xa.p;
            if (res->x && nR)
                QH_HIP(hipMemcpyAsync(res->x + off * R, xfin, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
            if (res->y && nR)
                QH_HIP(hipMemcpyAsync(res->y + off * R, p.y.p, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
            off += g->n;
        }
        QH_HIP(hipStreamSynchronize(st));
        return;
    }

    // readout of every block in one launch per kernel: FP64 cuts, component selection,
    // optional greedy, cut of the result
    std::vector<ReadoutDesc> rd(nb);
    int64_t voff = 0;
    for (int b = 0; b < nb; ++b) {
        const qh_graph *g = gs[b];
        SolvePlan &p = *plans[b];
        const int64_t nR = g->n * R;
        const bool pingpong = !(g->storage == QH_STORE_DENSE && g->dtype != QH_F32);
        const float *xfin = (pingpong && final_half) ? p.xb.p : p.xa.p;
        if (res->x && nR)
            QH_HIP(hipMemcpyAsync(res->x + voff * R, xfin, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (res->y && nR)
            QH_HIP(hipMemcpyAsync(res->y + voff * R, p.y.p, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
        const ReadoutView v = view_of(g);
        ReadoutDesc &d = rd[b];
        d.n = v.n;
        d.n_comp = v.n_comp;
        d.n_chunks = v.n_chunks;
        d.n_ord = v.n_ord;
        d.m_ptr = v.m_ptr;
        d.m_col = v.m_col;
        d.m_val = v.m_val;
        d.comp = v.comp;
        d.comp_first = v.comp_first;
        d.comp_order = v.comp_order;
        d.chunk_begin = v.chunk_begin;
        d.chunk_end = v.chunk_end;
        d.comp_chunk_ptr = v.comp_chunk_ptr;
        d.eps = v.eps;
        d.integer = g->integer ? 1 : 0;
        d.x = xfin;
        d.y = p.y.p;
        d.spins = p.spins.p;
        d.rowcut = p.rowcut.p;
        d.part = p.part.p;
        d.cut_rc = p.cut_rc.p;
        d.best_r = p.best_r.p;
        d.gain = p.gain.p;
        d.flag = p.flag.p;
        d.part1 = p.part1.p;
        d.cut1 = p.cut1.p;
        d.best_spins = res->best_spins + voff;
        d.cuts = res->cuts + (int64_t)b * R;
        d.best_cut = res->best_cut + b;
        d.selected_cut = res->selected_cut ? res->selected_cut + b : nullptr;
        voff += g->n;
    }
    readout_batched(rd, R, o->greedy != 0, st);
}

}  // namespace qh

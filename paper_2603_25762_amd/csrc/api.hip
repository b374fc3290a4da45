// C ABI entry points: argument validation, error capture, ownership.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace qh {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void fail(qh_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    throw Failure{st};
}

void fail_hip(hipError_t e, const char *what, const char *file, int line) {
    (void)hipGetLastError();
    qh_status st = (e == hipErrorOutOfMemory) ? QH_ENOMEM : QH_EHIP;
    snprintf(g_err, sizeof(g_err), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    throw Failure{st};
}

template <class F>
static qh_status guarded(F &&f) {
    try {
        f();
        return QH_OK;
    } catch (const Failure &e) {
        return e.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return QH_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return QH_EHIP;
    }
}

}  // namespace qh

using namespace qh;

extern "C" {

const char *qh_last_error(void) { return g_err; }
const char *qh_version(void) { return "qhap-gfx950 0.1.0"; }

}  // extern "C"

namespace qh {

// Validation and build of one graph on stream st (synchronised on return).
static qh_graph *build_one(const qh_reads *reads, const qh_snps *snps, const qh_graph_opts *opts, hipStream_t st) {
    if (reads->n_frag < 0) fail(QH_EINVAL, "n_frag < 0");
    if (snps->n_snp < 0) fail(QH_EINVAL, "n_snp < 0");
    if (reads->n_frag > 0 && (!reads->frag_ptr || !reads->snp || !reads->allele))
        fail(QH_EINVAL, "null fragment array");
    if (snps->n_snp > 0 && !snps->init_h1) fail(QH_EINVAL, "null init_h1");
    if (opts->kind < QH_READ_CONFLICT || opts->kind > QH_SNP_LLR) fail(QH_EINVAL, "bad kind");
    if (opts->storage < QH_STORE_DENSE || opts->storage > QH_STORE_SKYLINE)
        fail(QH_EINVAL, "bad storage");
    if (opts->dtype < QH_F32 || opts->dtype > QH_FP8_ROWSCALE) fail(QH_EINVAL, "bad dtype");
    bool read_kind = opts->kind != QH_SNP_LLR;
    if (read_kind && opts->storage != QH_STORE_DENSE)
        fail(QH_EUNSUPPORTED, "read graphs use DENSE storage");
    if (!read_kind && opts->storage != QH_STORE_SKYLINE)
        fail(QH_EUNSUPPORTED, "SNP graphs use SKYLINE storage");
    if (!read_kind && opts->dtype == QH_FP8_ROWSCALE)
        fail(QH_EUNSUPPORTED, "FP8 row scales are offered on dense storage only");
    if (!read_kind && opts->kind == QH_SNP_LLR && reads->n_frag > 0 && !reads->phred)
        fail(QH_EINVAL, "SNP graphs need phred");
    if (!read_kind && (opts->linkage_k < 1 || opts->linkage_k > 10))
        fail(QH_EINVAL, "linkage_k must be in 1..10");
    if (opts->band_limit < 0) fail(QH_EINVAL, "band_limit < 0");
    if (opts->max_device_bytes < 0) fail(QH_EINVAL, "max_device_bytes < 0");
    std::unique_ptr<qh_graph> g(new qh_graph());
    static std::atomic<uint64_t> next_serial{1};
    g->serial = next_serial.fetch_add(1);
    QH_HIP(hipGetDevice(&g->device));
    g->kind = opts->kind;
    g->storage = opts->storage;
    g->dtype = opts->dtype;
    g->n_snp = snps->n_snp;
    g->max_bytes = opts->max_device_bytes;
    if (opts->deterministic != 0 && opts->deterministic != 1) fail(QH_EINVAL, "deterministic must be 0 or 1");
    g->deterministic = opts->deterministic;
    if (read_kind) build_read_graph(g.get(), reads, snps, st);
    else build_snp_graph(g.get(), reads, snps, opts->linkage_k, opts->band_limit, st);
    finalize_graph(g.get(), st);
    QH_HIP(hipStreamSynchronize(st));
    return g.release();
}

}  // namespace qh

extern "C" {

qh_status qh_build_graph(const qh_reads *reads, const qh_snps *snps, const qh_graph_opts *opts,
                         qh_graph **out, void *stream) {
    return guarded([&] {
        if (!reads || !snps || !opts || !out) fail(QH_EINVAL, "null argument");
        *out = build_one(reads, snps, opts, (hipStream_t)stream);
    });
}

qh_status qh_build_graphs(int64_t count, const qh_reads *reads, const qh_snps *snps, const qh_graph_opts *opts,
                          qh_graph **out, int32_t threads, void *stream) {
    return guarded([&] {
        if (count < 0) fail(QH_EINVAL, "count < 0");
        if (threads < 0 || threads > 64) fail(QH_EINVAL, "threads must be in 0..64");
        if (count == 0) return;
        if (!reads || !snps || !opts || !out) fail(QH_EINVAL, "null argument");
        std::vector<qh_graph *> built((size_t)count, nullptr);   // out is written on success only
        const int nt = (int)std::min<int64_t>(threads ? threads : 8, count);
        int dev = 0;
        QH_HIP(hipGetDevice(&dev));
        // inputs may come from the caller's stream; and with all queued work done, every block
        // of the shared device-memory pool may serve any worker's stream
        (void)stream;
        QH_HIP(hipDeviceSynchronize());
        std::atomic<int64_t> next{0};
        std::atomic<bool> stop{false};
        std::mutex mu;
        qh_status first = QH_OK;
        std::string msg;
        auto record = [&](qh_status st, int64_t i) {
            std::lock_guard<std::mutex> lk(mu);
            if (first == QH_OK) {
                first = st;
                msg = i >= 0 ? "graph " + std::to_string(i) + ": " + qh_last_error() : std::string(qh_last_error());
            }
            stop = true;
        };
        // Each worker builds on a stream of its own, so that one build's synchronisations
        // overlap the others' work; the graphs are picked in index order.  A worker's
        // temporaries are recycled through a device-memory pool of its own (stream-ordered
        // reuse), which joins the shared pool once its stream is idle.
        auto worker = [&]() {
            hipStream_t ws = nullptr;
            const qh_status st = guarded([&] {
                QH_HIP(hipSetDevice(dev));
                QH_HIP(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));
                set_pool((uintptr_t)ws);
                for (;;) {
                    if (stop) break;
                    const int64_t i = next.fetch_add(1);
                    if (i >= count) break;
                    const qh_status si = guarded([&] { built[i] = build_one(reads + i, snps + i, opts + i, ws); });
                    if (si != QH_OK) {
                        record(si, i);
                        break;
                    }
                }
            });
            if (st != QH_OK) record(st, -1);
            if (ws) {
                (void)hipStreamSynchronize(ws);
                set_pool(0);
                merge_pool(dev, (uintptr_t)ws);
                (void)hipStreamDestroy(ws);
            }
        };
        std::vector<std::thread> pool;
        try {
            for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
        } catch (...) {
            stop = true;
            for (auto &th : pool) th.join();
            throw;
        }
        for (auto &th : pool) th.join();
        if (first != QH_OK) {
            for (qh_graph *g : built) delete g;
            fail(first, "%s", msg.c_str());
        }
        for (int64_t i = 0; i < count; ++i) out[i] = built[i];
    });
}

qh_status qh_release_cached_memory(int64_t *released) {
    return guarded([&] {
        const size_t b = release_cached();
        if (released) *released = (int64_t)b;
    });
}

qh_status qh_graph_free(qh_graph *g) {
    return guarded([&] {
        if (!g) return;
        int cur = 0;
        const int dev = g->device;
        QH_HIP(hipGetDevice(&cur));
        if (cur != dev) QH_HIP(hipSetDevice(dev));
        QH_HIP(hipDeviceSynchronize());
        delete g;
        if (cur != dev) QH_HIP(hipSetDevice(cur));
    });
}

qh_status qh_graph_get_info(const qh_graph *g, qh_graph_info *out) {
    return guarded([&] {
        if (!g || !out) fail(QH_EINVAL, "null argument");
        qh_graph_info i{};
        i.n = g->n;
        i.n_snp = g->n_snp;
        i.nnz = g->nnz;
        i.n_comp = g->n_comp;
        i.longrange_nnz = g->l_nnz;
        i.dense_tiles = g->n_tiles;
        if (g->storage == QH_STORE_DENSE) {
            i.stored_entries = g->n_tiles * kTileElems;
            i.stored_bytes = i.stored_entries * dtype_bytes(g->dtype) +
                             (g->dtype == QH_FP8_ROWSCALE ? g->n * 4 : 0);
        } else {
            i.stored_entries = g->s_slots + g->l_nnz;
            i.stored_bytes = i.stored_entries * dtype_bytes(g->dtype) + g->l_nnz * 4 + g->n * 16;
        }
        i.device_bytes = g->device_bytes;
        i.kind = g->kind;
        i.storage = g->storage;
        i.dtype = g->dtype;
        i.integer_weights = g->integer ? 1 : 0;
        i.c0_auto = g->c0_auto;
        i.total_weight = g->total_weight;
        i.band_dtype = g->storage == QH_STORE_SKYLINE ? g->bb_dtype : g->dtype;
        i.largest_component = g->largest_comp;
        *out = i;
    });
}

qh_status qh_graph_export_rows(const qh_graph *g, int64_t row0, int64_t row1, double *out,
                               void *stream) {
    return guarded([&] {
        if (!g || !out) fail(QH_EINVAL, "null argument");
        if (row0 < 0 || row1 < row0 || row1 > g->n) fail(QH_EINVAL, "row range out of bounds");
        export_master_rows(g, row0, row1, out, (hipStream_t)stream);
    });
}

qh_status qh_graph_export_stored_rows(const qh_graph *g, int64_t row0, int64_t row1,
                                      double *out, void *stream) {
    return guarded([&] {
        if (!g || !out) fail(QH_EINVAL, "null argument");
        if (row0 < 0 || row1 < row0 || row1 > g->n) fail(QH_EINVAL, "row range out of bounds");
        export_stored_rows(g, row0, row1, out, (hipStream_t)stream);
    });
}

qh_status qh_graph_components(const qh_graph *g, int32_t *comp, void *stream) {
    return guarded([&] {
        if (!g || !comp) fail(QH_EINVAL, "null argument");
        if (g->n)
            QH_HIP(hipMemcpyAsync(comp, g->comp.p, g->n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream));
    });
}

static void validate_opts(const qh_bsb_opts *o) {
    if (!o) fail(QH_EINVAL, "null options");
    int R = o->replicas;
    if (!(R == 16 || R == 32 || (R >= 64 && R % 64 == 0)) || R > 4096)
        fail(QH_EINVAL, "replicas must be 16, 32 or a multiple of 64 (<= 4096), got %d", R);
    if (o->steps < 1) fail(QH_EINVAL, "steps must be >= 1");
    int end = o->step_end == 0 ? o->steps : o->step_end;
    if (o->step_begin < 0 || end < o->step_begin || end > o->steps)
        fail(QH_EINVAL, "step range [%d, %d) outside the schedule of %d steps", o->step_begin, end,
             o->steps);
    if (!(o->dt > 0.0)) fail(QH_EINVAL, "dt must be > 0");
    if (o->plan < 0 || o->plan > 5) fail(QH_EINVAL, "plan must be 0-5, got %d", o->plan);
    if (o->variant != 0 && o->variant != 1) fail(QH_EINVAL, "variant must be 0 (ballistic) or 1 (discrete)");
    if (o->persistent_sync < 0 || o->persistent_sync > 2)
        fail(QH_EINVAL, "persistent_sync must be 0, 1 or 2, got %d", o->persistent_sync);
    if (o->tiles_in_flight != 0 && o->tiles_in_flight != 2 && o->tiles_in_flight != 4)
        fail(QH_EINVAL, "tiles_in_flight must be 0, 2 or 4, got %d", o->tiles_in_flight);
    if (o->eval_every < 0) fail(QH_EINVAL, "eval_every must be >= 0, got %d", o->eval_every);
    const int t = o->replica_tile;
    if (t != 0 && (!(t == 16 || t == 32 || t == 64) || R < 64))
        fail(QH_EINVAL, "replica_tile must be 0, or 16, 32 or 64 with R >= 64, got %d", t);
}

qh_status qh_bsb_solve(const qh_graph *g, const qh_bsb_opts *opts, qh_result *res, void *stream) {
    return guarded([&] {
        if (!g || !res) fail(QH_EINVAL, "null argument");
        validate_opts(opts);
        if (!opts->init && (!res->x || !res->y)) fail(QH_EINVAL, "init = 0 needs x and y");
        if (opts->readout && (!res->best_spins || !res->cuts || !res->best_cut))
            fail(QH_EINVAL, "readout needs best_spins, cuts and best_cut");
        if (opts->eval_every > 0 && !opts->readout) fail(QH_EINVAL, "eval_every > 0 needs readout = 1");
        if (opts->eval_every > 0 && opts->use_graph)
            fail(QH_EINVAL, "eval_every > 0 reads out between steps: it needs use_graph = 0");
        bsb_solve(g, opts, res, (hipStream_t)stream);
    });
}

qh_status qh_solve_plan_info(const qh_graph *g, int32_t replicas, qh_plan_info *out) {
    return guarded([&] {
        if (!g || !out) fail(QH_EINVAL, "null argument");
        plan_info(g, replicas, out);
    });
}

qh_status qh_autotune(const qh_graph *g, const qh_bsb_opts *opts, qh_bsb_opts *chosen, float *us_per_step,
                      const char *cache_path, void *stream) {
    return guarded([&] {
        if (!g || !chosen) fail(QH_EINVAL, "null argument");
        validate_opts(opts);
        float us[2] = {0.0f, 0.0f};
        qh_bsb_opts c{};
        autotune(g, opts, &c, us, (hipStream_t)stream);
        QH_HIP(hipStreamSynchronize((hipStream_t)stream));
        if (cache_path) {
            FILE *f = std::fopen(cache_path, "a");
            if (!f) fail(QH_EINVAL, "cannot open the cache file %s", cache_path);
            std::fprintf(f,
                         "{\"n\": %lld, \"nnz\": %lld, \"kind\": %d, \"storage\": %d, \"dtype\": %d, "
                         "\"dense_tiles\": %lld, \"replicas\": %d, \"plan\": %d, \"replica_tile\": %d, "
                         "\"tiles_in_flight\": %d, \"persistent_sync\": %d, \"us_per_step\": [%.4f, %.4f]}\n",
                         (long long)g->n, (long long)g->nnz, g->kind, g->storage, g->dtype, (long long)g->n_tiles,
                         opts->replicas, c.plan, c.replica_tile, c.tiles_in_flight, c.persistent_sync, us[0], us[1]);
            const bool bad = std::ferror(f) != 0;
            if (std::fclose(f) != 0 || bad) fail(QH_EINVAL, "cannot write the cache file %s", cache_path);
        }
        *chosen = c;
        if (us_per_step) {
            us_per_step[0] = us[0];
            us_per_step[1] = us[1];
        }
    });
}

qh_status qh_bsb_solve_batched(const qh_graph *const *graphs, int32_t n_graphs,
                               const qh_bsb_opts *opts, qh_batched_result *res, void *stream) {
    return guarded([&] {
        if (!graphs || !res || n_graphs < 0) fail(QH_EINVAL, "null argument");
        validate_opts(opts);
        for (int b = 0; b < n_graphs; ++b)
            if (!graphs[b]) fail(QH_EINVAL, "null graph %d", b);
        if (opts->readout && (!res->best_spins || !res->cuts || !res->best_cut))
            fail(QH_EINVAL, "batched readout needs best_spins, cuts and best_cut");
        if (opts->eval_every != 0) fail(QH_EINVAL, "batched solves read out after the last step only (eval_every = 0)");
        bsb_solve_batched(graphs, n_graphs, opts, res, (hipStream_t)stream);
    });
}

qh_status qh_phase(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block,
                   void *stream) {
    return guarded([&] {
        if (!g || !spins || !h1 || !block) fail(QH_EINVAL, "null argument");
        phase(g, spins, h1, block, (hipStream_t)stream);
    });
}

qh_status qh_phase_noalloc(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block, void *stream) {
    return guarded([&] {
        if (!g || !spins || !h1 || !block) fail(QH_EINVAL, "null argument");
        phase_noalloc(g, spins, h1, block, (hipStream_t)stream);
    });
}

qh_status qh_phase_batched(const qh_graph *const *graphs, int32_t n_graphs, const int8_t *spins, int8_t *h1,
                           int32_t *block, void *stream) {
    return guarded([&] {
        if (n_graphs < 0) fail(QH_EINVAL, "n_graphs < 0");
        if (n_graphs == 0) return;
        if (!graphs || !spins || !h1 || !block) fail(QH_EINVAL, "null argument");
        phase_batched(graphs, n_graphs, spins, h1, block, (hipStream_t)stream);
    });
}

qh_status qh_flip_crossing(qh_graph *g, const int8_t *spins, void *stream) {
    return guarded([&] {
        if (!g || !spins) fail(QH_EINVAL, "null argument");
        flip_crossing(g, spins, (hipStream_t)stream);
    });
}

qh_status qh_refine(qh_graph *g, const qh_bsb_opts *opts, int32_t max_rounds, float deform, int32_t deform_tries,
                    int8_t *h1, int32_t *block, int32_t *flips, double *round_cuts, int32_t *rounds,
                    int32_t *deformed, void *stream) {
    return guarded([&] {
        if (!g || !h1 || !block) fail(QH_EINVAL, "null argument");
        validate_opts(opts);
        refine(g, opts, max_rounds, deform, deform_tries, h1, block, flips, round_cuts, rounds, deformed,
               (hipStream_t)stream);
    });
}

qh_status qh_adaptive_schedule(int64_t size, qh_schedule *out) {
    return guarded([&] {
        if (!out) fail(QH_EINVAL, "null argument");
        if (size < 0) fail(QH_EINVAL, "size must be >= 0, got %lld", (long long)size);
        qh_schedule s{};
        s.size = size;
        s.steps = s.size < 5000 ? 500 : 1000;
        s.samples = 100;
        s.replicas = 128;
        s.max_rounds = 15;
        *out = s;
    });
}

}  // extern "C"

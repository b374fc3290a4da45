// Readout after the step loop (Eqs. 4-6 and the precision form): signs with a watchdog
// for non-finite state, FP64 cuts per replica and component from the master weights,
// per-component selection (ties -> lowest replica, lowest vertex reads +1), optional
// greedy single-flip rounds with FP64 gains, and the cut of the final spins.
//
// Every kernel body is a grid-stride loop over its own index space with the workgroup
// index and count passed in, and every output element is computed by one thread in a
// fixed order.  The single-graph kernels run a body with (blockIdx.x, gridDim.x); the
// batched kernels give each block of a batch a slice of one launch (found by binary
// search in a per-kernel prefix of workgroup counts) and run the same body on it, so a
// batched readout equals the single-graph readout of every block bit for bit.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace qh {

static int grid_for(int64_t n, int block = 256, int64_t cap = 65536) {
    int64_t g = ceil_div(n, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

#define QH_FOR(i, count)                                                                  \
    for (int64_t i = bx * (int64_t)blockDim.x + threadIdx.x; i < (count); i += gx * (int64_t)blockDim.x)

// ----------------------------------------------------------------------------- bodies

__device__ inline void signs_body(int64_t bx, int64_t gx, int64_t n, int R, const float *__restrict__ x,
                                  const float *__restrict__ y, int8_t *__restrict__ s, int32_t *__restrict__ bad,
                                  int32_t bad_value) {
    int local_bad = 0;
    QH_FOR(t, n * R) {
        const float v = x[t];
        if (!isfinite(v) || !isfinite(y[t])) local_bad = 1;
        s[t] = v >= 0.0f ? 1 : -1;
    }
    if (local_bad) atomicMax(bad, bad_value);
}

// rowcut[v][r] = sum_j A_aj (1 - s_a s_j), a = order[v], A = -J, entries in CSR order
__device__ inline void cut_rows_body(int64_t bx, int64_t gx, int64_t n_ord, int R, const int32_t *__restrict__ order,
                                     const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                     const double *__restrict__ val, const int8_t *__restrict__ s,
                                     double *__restrict__ rowcut) {
    if (R % 8 == 0) {
        // eight replicas per thread: one 8-byte spin gather per entry serves all eight, and
        // each replica's sum takes the entries in CSR order as below
        const int G = R / 8;
        QH_FOR(t, n_ord * G) {
            const int64_t v = t / G;
            const int g8 = (int)(t - v * G);
            const int64_t a = order[v];
            int8_t sa[8];
            __builtin_memcpy(sa, s + a * R + 8 * g8, 8);
            double racc[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) racc[q] = 0.0;
            int64_t e = ptr[a];
            const int64_t e1 = ptr[a + 1];
            for (; e + 8 <= e1; e += 8) {
                int32_t c[8];
                double w[8];
                uint2 sb[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) { c[k] = col[e + k]; w[k] = val[e + k]; }
#pragma unroll
                for (int k = 0; k < 8; ++k) sb[k] = *(const uint2 *)(s + (int64_t)c[k] * R + 8 * g8);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    int8_t b8[8];
                    __builtin_memcpy(b8, &sb[k], 8);
#pragma unroll
                    for (int q = 0; q < 8; ++q) racc[q] += -w[k] * (1.0 - (double)(sa[q] * b8[q]));
                }
            }
            for (; e < e1; ++e) {
                int8_t b8[8];
                __builtin_memcpy(b8, s + (int64_t)col[e] * R + 8 * g8, 8);
                const double w = val[e];
#pragma unroll
                for (int q = 0; q < 8; ++q) racc[q] += -w * (1.0 - (double)(sa[q] * b8[q]));
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) rowcut[v * R + 8 * g8 + q] = racc[q];
        }
        return;
    }
    QH_FOR(t, n_ord * R) {
        const int64_t v = t / R;
        const int r = (int)(t - v * R);
        const int64_t a = order[v];
        const int sa = s[a * R + r];
        double racc = 0.0;
        int64_t e = ptr[a];
        const int64_t e1 = ptr[a + 1];
        // eight entries per round: column and value loads, then the spin gathers, then the
        // adds in entry order (the same sum as the plain loop)
        for (; e + 8 <= e1; e += 8) {
            int32_t c[8];
            double w[8];
            int sb[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) { c[k] = col[e + k]; w[k] = val[e + k]; }
#pragma unroll
            for (int k = 0; k < 8; ++k) sb[k] = s[(int64_t)c[k] * R + r];
#pragma unroll
            for (int k = 0; k < 8; ++k) racc += -w[k] * (1.0 - (double)(sa * sb[k]));
        }
        for (; e < e1; ++e) {
            const int sb = s[(int64_t)col[e] * R + r];
            racc += -val[e] * (1.0 - (double)(sa * sb));
        }
        rowcut[t] = racc;
    }
}

// part[ch][r] = 1/4 sum_{v in chunk} rowcut[v][r], vertices in chunk order
__device__ inline void cut_chunks_body(int64_t bx, int64_t gx, int64_t n_chunks, int R,
                                       const int32_t *__restrict__ chunk_begin, const int32_t *__restrict__ chunk_end,
                                       const double *__restrict__ rowcut, double *__restrict__ part) {
    QH_FOR(t, n_chunks * R) {
        const int64_t ch = t / R;
        const int r = (int)(t - ch * R);
        double acc = 0.0;
        for (int v = chunk_begin[ch]; v < chunk_end[ch]; ++v) acc += 0.25 * rowcut[(int64_t)v * R + r];
        part[t] = acc;
    }
}

// cut_rc[r][c] = sum of the component's chunk partials, chunks in order
__device__ inline void cut_reduce_body(int64_t bx, int64_t gx, int64_t n_comp, int R,
                                       const int32_t *__restrict__ comp_chunk_ptr, const double *__restrict__ part,
                                       double *__restrict__ cut_rc) {
    for (int64_t c = bx; c < n_comp; c += gx)
        for (int r = threadIdx.x; r < R; r += blockDim.x) {
            double acc = 0.0;
            for (int ch = comp_chunk_ptr[c]; ch < comp_chunk_ptr[c + 1]; ++ch) acc += part[(int64_t)ch * R + r];
            cut_rc[(int64_t)r * n_comp + c] = acc;
        }
}

__device__ inline void select_body(int64_t bx, int64_t gx, int64_t n_comp, int R, const double *__restrict__ cut_rc,
                                   int32_t *__restrict__ best_r) {
    QH_FOR(c, n_comp) {
        int br = 0;
        double bv = cut_rc[c];
        for (int r = 1; r < R; ++r) {
            const double v = cut_rc[(int64_t)r * n_comp + c];
            if (v > bv) { bv = v; br = r; }
        }
        best_r[c] = br;
    }
}

__device__ inline void replica_totals_body(int64_t bx, int64_t gx, int64_t n_comp, int R,
                                           const double *__restrict__ cut_rc, double *__restrict__ cuts) {
    QH_FOR(r, (int64_t)R) {
        double acc = 0.0;
        for (int64_t c = 0; c < n_comp; ++c) acc += cut_rc[r * n_comp + c];
        cuts[r] = acc;
    }
}

// Deterministic sum of cut_rc[best_r[c]][c] over components: one workgroup of 256
// threads, a fixed tree.
__device__ inline void selected_total_body(int64_t n_comp, const double *__restrict__ cut_rc,
                                           const int32_t *__restrict__ best_r, double *__restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < n_comp; c += blockDim.x)
        acc += best_r ? cut_rc[(int64_t)best_r[c] * n_comp + c] : cut_rc[c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__device__ inline void best_spins_body(int64_t bx, int64_t gx, int64_t n, int R, const int32_t *__restrict__ comp,
                                       const int32_t *__restrict__ comp_first, const int32_t *__restrict__ best_r,
                                       const int8_t *__restrict__ s, int8_t *__restrict__ best) {
    QH_FOR(a, n) {
        const int c = comp[a];
        if (c < 0) { best[a] = 1; continue; }
        const int rb = best_r[c];
        const int v = s[a * R + rb];
        const int o = s[(int64_t)comp_first[c] * R + rb];
        best[a] = (int8_t)(v * o);
    }
}

// g_a = s_a sum_j A_aj s_j, A = -J
__device__ inline void gain_body(int64_t bx, int64_t gx, int64_t n, const int64_t *__restrict__ ptr,
                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                 const int8_t *__restrict__ s, double *__restrict__ g) {
    QH_FOR(a, n) {
        double acc = 0.0;
        int64_t e = ptr[a];
        const int64_t e1 = ptr[a + 1];
        for (; e + 8 <= e1; e += 8) {      // loads of eight entries in flight, adds in order
            int32_t c[8];
            double w[8];
            int sb[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) { c[k] = col[e + k]; w[k] = val[e + k]; }
#pragma unroll
            for (int k = 0; k < 8; ++k) sb[k] = s[c[k]];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += -w[k] * (double)sb[k];
        }
        for (; e < e1; ++e) acc += -val[e] * (double)s[col[e]];
        g[a] = (double)s[a] * acc;
    }
}

// Flip a when g_a > eps and a beats every neighbour j with g_j > eps (larger gain, or
// equal gain and lower index): the flipped set is independent.
__device__ inline void pick_body(int64_t bx, int64_t gx, int64_t n, const int64_t *__restrict__ ptr,
                                 const int32_t *__restrict__ col, const double *__restrict__ g, double eps_all,
                                 const double *__restrict__ eps_v, int8_t *__restrict__ flag,
                                 int32_t *__restrict__ count) {
    int local = 0;
    QH_FOR(a, n) {
        int8_t f = 0;
        const double ga = g[a];
        const double eps = eps_v ? eps_v[a] : eps_all;
        if (ga > eps) {
            f = 1;
            for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) {
                const int64_t j = col[e];
                const double gj = g[j];
                if (gj > eps && (gj > ga || (gj == ga && j < a))) { f = 0; break; }
            }
        }
        flag[a] = f;
        local += f;
    }
    if (local) atomicAdd(count, local);
}

__device__ inline void apply_flips_body(int64_t bx, int64_t gx, int64_t n, const int8_t *__restrict__ flag,
                                        int8_t *__restrict__ s) {
    QH_FOR(a, n) if (flag[a]) s[a] = (int8_t)-s[a];
}

#undef QH_FOR

// threads per vertex of cut_rows_body: one per eight replicas when R is a multiple of 8
static inline int64_t rows_threads(int R) { return R % 8 == 0 ? R / 8 : R; }

// ----------------------------------------------------------------------------- single graph

#define QH_G blockIdx.x, gridDim.x
__global__ void k_signs(int64_t n, int R, const float *x, const float *y, int8_t *s, int32_t *bad) {
    signs_body(QH_G, n, R, x, y, s, bad, 1);
}
__global__ void k_cut_rows(int64_t n_ord, int R, const int32_t *order, const int64_t *ptr, const int32_t *col,
                           const double *val, const int8_t *s, double *rowcut) {
    cut_rows_body(QH_G, n_ord, R, order, ptr, col, val, s, rowcut);
}
__global__ void k_cut_chunks(int64_t n_chunks, int R, const int32_t *cb, const int32_t *ce, const double *rowcut,
                             double *part) {
    cut_chunks_body(QH_G, n_chunks, R, cb, ce, rowcut, part);
}
__global__ void k_cut_reduce(int64_t n_comp, int R, const int32_t *ccp, const double *part, double *cut_rc) {
    cut_reduce_body(QH_G, n_comp, R, ccp, part, cut_rc);
}
__global__ void k_select(int64_t n_comp, int R, const double *cut_rc, int32_t *best_r) {
    select_body(QH_G, n_comp, R, cut_rc, best_r);
}
__global__ void k_replica_totals(int64_t n_comp, int R, const double *cut_rc, double *cuts) {
    replica_totals_body(QH_G, n_comp, R, cut_rc, cuts);
}
__global__ void k_selected_total(int64_t n_comp, const double *cut_rc, const int32_t *best_r, double *out) {
    selected_total_body(n_comp, cut_rc, best_r, out);
}
__global__ void k_best_spins(int64_t n, int R, const int32_t *comp, const int32_t *comp_first,
                             const int32_t *best_r, const int8_t *s, int8_t *best) {
    best_spins_body(QH_G, n, R, comp, comp_first, best_r, s, best);
}
__global__ void k_gain(int64_t n, const int64_t *ptr, const int32_t *col, const double *val, const int8_t *s,
                       double *g) {
    gain_body(QH_G, n, ptr, col, val, s, g);
}
__global__ void k_pick(int64_t n, const int64_t *ptr, const int32_t *col, const double *g, double eps_all,
                       const double *eps_v, int8_t *flag, int32_t *count) {
    pick_body(QH_G, n, ptr, col, g, eps_all, eps_v, flag, count);
}
__global__ void k_apply_flips(int64_t n, const int8_t *flag, int8_t *s) { apply_flips_body(QH_G, n, flag, s); }

// Readout every eval_every steps: component c's pick of this evaluation (replica best_r[c])
// replaces the best so far when its cut is larger (the first evaluation always replaces).
__global__ void k_eval_merge(int64_t n_comp, const double *__restrict__ cut_rc, const int32_t *__restrict__ best_r,
                             int first, double *__restrict__ best_cut, int32_t *__restrict__ best_rr,
                             int8_t *__restrict__ take) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_comp; c += gridDim.x * (int64_t)blockDim.x) {
        const double v = cut_rc[(int64_t)best_r[c] * n_comp + c];
        const bool t = first || v > best_cut[c];
        if (t) {
            best_cut[c] = v;
            best_rr[c] = best_r[c];
        }
        take[c] = t ? 1 : 0;
    }
}

// Spins of the components whose pick was replaced, oriented so that the component's lowest
// vertex reads +1; single-vertex components read +1.
__global__ void k_eval_take(int64_t n, int R, const int32_t *__restrict__ comp, const int32_t *__restrict__ comp_first,
                            const int32_t *__restrict__ best_r, const int8_t *__restrict__ take,
                            const int8_t *__restrict__ s, int8_t *__restrict__ best) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += gridDim.x * (int64_t)blockDim.x) {
        const int c = comp[a];
        if (c < 0) { best[a] = 1; continue; }
        if (!take[c]) continue;
        const int rb = best_r[c];
        best[a] = (int8_t)(s[a * R + rb] * s[(int64_t)comp_first[c] * R + rb]);
    }
}

// Eq. (5): E_r = W - 2 cut_r for every replica
__global__ void k_energy_row(int R, double W, const double *__restrict__ cuts, double *__restrict__ e) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) e[r] = W - 2.0 * cuts[r];
}
#undef QH_G

void alloc_readout_scratch(SolvePlan &p, int64_t n, int64_t n_comp, int64_t n_chunks, int R) {
    p.spins.alloc((size_t)std::max<int64_t>(n, 1) * R);
    p.part.alloc((size_t)std::max<int64_t>(n_chunks, 1) * R);
    p.rowcut.alloc((size_t)std::max<int64_t>(n, 1) * R);
    p.cut_rc.alloc((size_t)std::max<int64_t>(n_comp, 1) * R);
    p.best_r.alloc(std::max<int64_t>(n_comp, 1));
    p.gain.alloc(std::max<int64_t>(n, 1));
    p.flag.alloc(std::max<int64_t>(n, 1));
    p.counter.alloc(4);
    p.part1.alloc(std::max<int64_t>(n_chunks, 1));
    p.cut1.alloc(std::max<int64_t>(n_comp, 1));
}

ReadoutView view_of(const qh_graph *g) {
    ReadoutView v;
    v.n = g->n;
    v.n_comp = g->n_comp;
    v.n_chunks = g->n_chunks;
    v.n_ord = g->n_ord;
    v.m_ptr = g->m_ptr.p;
    v.m_col = g->m_col.p;
    v.m_val = g->m_val.p;
    v.comp = g->comp.p;
    v.comp_first = g->comp_first.p;
    v.comp_order = g->comp_order.p;
    v.chunk_begin = g->chunk_begin.p;
    v.chunk_end = g->chunk_end.p;
    v.comp_chunk_ptr = g->comp_chunk_ptr.p;
    v.eps = g->greedy_eps;
    return v;
}

void readout(const ReadoutView &g, SolvePlan &p, int R, const float *xfin, const float *yfin, qh_result *res,
             bool greedy, hipStream_t st, bool finish, const EvalArgs *ev) {
    const int64_t n = g.n;
    const int64_t nR = n * R;

    // signs + non-finite watchdog (kept over the evaluations of one solve)
    if (!ev || ev->index == 0) QH_HIP(hipMemsetAsync(p.counter.p, 0, 4 * sizeof(int32_t), st));
    if (nR) {
        hipLaunchKernelGGL(k_signs, dim3(grid_for(nR)), dim3(256), 0, st, n, R, xfin, yfin, p.spins.p,
                           p.counter.p + 1);
        QH_CHECK_LAUNCH();
    }
    if (res->all_spins && nR)
        QH_HIP(hipMemcpyAsync(res->all_spins, p.spins.p, nR, hipMemcpyDeviceToDevice, st));
    // FP64 cuts per replica and component
    const int64_t nc = g.n_comp;
    if (nc) {
        hipLaunchKernelGGL(k_cut_rows, dim3(grid_for(g.n_ord * rows_threads(R))), dim3(256), 0, st, g.n_ord, R,
                           g.comp_order,
                           g.m_ptr, g.m_col, g.m_val, p.spins.p, p.rowcut.p);
        hipLaunchKernelGGL(k_cut_chunks, dim3(grid_for(g.n_chunks * R)), dim3(256), 0, st, g.n_chunks, R,
                           g.chunk_begin, g.chunk_end, p.rowcut.p, p.part.p);
        hipLaunchKernelGGL(k_cut_reduce, dim3((unsigned)std::min<int64_t>(nc, 1 << 20)), dim3(256), 0, st, nc, R,
                           g.comp_chunk_ptr, p.part.p, p.cut_rc.p);
        hipLaunchKernelGGL(k_select, dim3(grid_for(nc)), dim3(256), 0, st, nc, R, p.cut_rc.p, p.best_r.p);
        hipLaunchKernelGGL(k_replica_totals, dim3(grid_for(R)), dim3(256), 0, st, nc, R, p.cut_rc.p, res->cuts);
        if (!ev)
            hipLaunchKernelGGL(k_selected_total, dim3(1), dim3(256), 0, st, nc, p.cut_rc.p, p.best_r.p,
                               res->selected_cut ? res->selected_cut : res->best_cut);
        QH_CHECK_LAUNCH();
    } else {
        QH_HIP(hipMemsetAsync(res->cuts, 0, R * sizeof(double), st));
        QH_HIP(hipMemsetAsync(res->selected_cut ? res->selected_cut : res->best_cut, 0, sizeof(double), st));
    }
    if (ev && ev->energy_row) {
        hipLaunchKernelGGL(k_energy_row, dim3(grid_for(R)), dim3(256), 0, st, R, ev->W, res->cuts, ev->energy_row);
        QH_CHECK_LAUNCH();
    }
    if (res->cut_rc && nc && (!ev || ev->last))
        QH_HIP(hipMemcpyAsync(res->cut_rc, p.cut_rc.p, nc * R * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (ev) {
        // best (evaluation, replica) so far per component, its spins into best_spins
        if (ev->index == 0 && p.ev_cut.n < (size_t)std::max<int64_t>(nc, 1)) {
            p.ev_cut.alloc(std::max<int64_t>(nc, 1));
            p.ev_r.alloc(std::max<int64_t>(nc, 1));
            p.ev_take.alloc(std::max<int64_t>(nc, 1));
        }
        if (nc) {
            hipLaunchKernelGGL(k_eval_merge, dim3(grid_for(nc)), dim3(256), 0, st, nc, p.cut_rc.p, p.best_r.p,
                               ev->index == 0 ? 1 : 0, p.ev_cut.p, p.ev_r.p, p.ev_take.p);
            QH_CHECK_LAUNCH();
        }
        if (n) {
            hipLaunchKernelGGL(k_eval_take, dim3(grid_for(n)), dim3(256), 0, st, n, R, g.comp, g.comp_first,
                               p.best_r.p, p.ev_take.p, p.spins.p, res->best_spins);
            QH_CHECK_LAUNCH();
        }
        if (!ev->last) return;
        if (nc) {
            hipLaunchKernelGGL(k_selected_total, dim3(1), dim3(256), 0, st, nc, p.ev_cut.p, (const int32_t *)nullptr,
                               res->selected_cut ? res->selected_cut : res->best_cut);
            QH_CHECK_LAUNCH();
            if (res->best_replica)
                QH_HIP(hipMemcpyAsync(res->best_replica, p.ev_r.p, nc * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                      st));
        }
    } else {
        if (res->best_replica && nc)
            QH_HIP(hipMemcpyAsync(res->best_replica, p.best_r.p, nc * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                  st));
        if (n) {
            hipLaunchKernelGGL(k_best_spins, dim3(grid_for(n)), dim3(256), 0, st, n, R, g.comp, g.comp_first,
                               p.best_r.p, p.spins.p, res->best_spins);
            QH_CHECK_LAUNCH();
        }
    }
    int32_t rounds = 0;
    if (greedy && n && nc) {
        for (int it = 0; it < 100000; ++it) {
            hipLaunchKernelGGL(k_gain, dim3(grid_for(n)), dim3(256), 0, st, n, g.m_ptr, g.m_col, g.m_val,
                               res->best_spins, p.gain.p);
            QH_HIP(hipMemsetAsync(p.counter.p, 0, sizeof(int32_t), st));
            hipLaunchKernelGGL(k_pick, dim3(grid_for(n)), dim3(256), 0, st, n, g.m_ptr, g.m_col, p.gain.p,
                               g.eps, g.eps_v, p.flag.p, p.counter.p);
            QH_CHECK_LAUNCH();
            int32_t cnt = 0;
            QH_HIP(hipMemcpyAsync(&cnt, p.counter.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            QH_HIP(hipStreamSynchronize(st));
            if (cnt == 0) break;
            hipLaunchKernelGGL(k_apply_flips, dim3(grid_for(n)), dim3(256), 0, st, n, p.flag.p, res->best_spins);
            QH_CHECK_LAUNCH();
            ++rounds;
        }
    }
    // cut of the final spins
    if (nc) {
        hipLaunchKernelGGL(k_cut_rows, dim3(grid_for(g.n_ord)), dim3(256), 0, st, g.n_ord, 1, g.comp_order,
                           g.m_ptr, g.m_col, g.m_val, res->best_spins, p.rowcut.p);
        hipLaunchKernelGGL(k_cut_chunks, dim3(grid_for(g.n_chunks)), dim3(256), 0, st, g.n_chunks, 1,
                           g.chunk_begin, g.chunk_end, p.rowcut.p, p.part1.p);
        hipLaunchKernelGGL(k_cut_reduce, dim3((unsigned)std::min<int64_t>(nc, 1 << 20)), dim3(64), 0, st, nc, 1,
                           g.comp_chunk_ptr, p.part1.p, p.cut1.p);
        hipLaunchKernelGGL(k_selected_total, dim3(1), dim3(256), 0, st, nc, p.cut1.p, (const int32_t *)nullptr,
                           res->best_cut);
        QH_CHECK_LAUNCH();
    } else {
        QH_HIP(hipMemsetAsync(res->best_cut, 0, sizeof(double), st));
    }
    if (res->greedy_rounds)
        QH_HIP(hipMemcpyAsync(res->greedy_rounds, &rounds, sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!finish) return;
    int32_t bad = 0;
    QH_HIP(hipMemcpyAsync(&bad, p.counter.p + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    QH_HIP(hipStreamSynchronize(st));
    if (bad) fail(QH_ENUMERIC, "non-finite spin or momentum in the final state");
}

// ----------------------------------------------------------------------------- batched

// Launch slice of one block: the workgroups [wg[b], wg[b + 1]) of a launch serve block b.
__device__ inline int slice_of(const int32_t *__restrict__ wg, int nb, int64_t &bx, int64_t &gx) {
    int lo = 0, hi = nb;   // largest b with wg[b] <= blockIdx.x
    const int32_t g = (int32_t)blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wg[mid] <= g) lo = mid;
        else hi = mid;
    }
    bx = g - wg[lo];
    gx = wg[lo + 1] - wg[lo];
    return lo;
}

// Integer weights: FP64 sums of integers (all below 2^53) are exact in any order, so one
// wave takes one row and its lanes take the entries, with coalesced loads and a tree sum at
// the end; the result equals the one-thread-per-row loop of gain_body bit for bit (no term
// of a gain is -0).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// gains of vertices [0, n) of a slice, one per wave: out[a] = s_a * sum_j -w_j s_j
__device__ inline void gain_wave_body(int64_t bx, int64_t gx, int64_t n, const int64_t *__restrict__ ptr,
                                      const int32_t *__restrict__ col, const double *__restrict__ val,
                                      const int8_t *__restrict__ s, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t a = bx * 4 + wave; a < n; a += gx * 4) {
        const int sa = s[a];
        const int64_t e1 = ptr[a + 1];
        double acc = 0.0;
        for (int64_t e = ptr[a] + lane; e < e1; e += 4 * 64) {   // four entries per lane in flight
            int32_t c[4];
            double w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t ek = e + 64 * k;
                c[k] = ek < e1 ? col[ek] : 0;
                w[k] = ek < e1 ? val[ek] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (e + 64 * k >= e1) break;
                acc += -w[k] * (double)s[c[k]];
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) out[a] = (double)sa * acc;
    }
}

enum : int { kSigns, kRowsR, kChunksR, kReduce, kComp, kOne, kVert, kRows1, kChunks1, kGain, kSlices };

#define QH_B(slice)                                     \
    int64_t bx, gx;                                     \
    const int b = slice_of(wg + (slice) * (nb + 1), nb, bx, gx); \
    const ReadoutDesc &D = tbl[b];

__global__ void kb_signs(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R, int32_t *bad) {
    QH_B(kSigns);
    signs_body(bx, gx, D.n, R, D.x, D.y, D.spins, bad, b + 1);
}
__global__ void kb_cut_rows(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R, int final_cut) {
    QH_B(final_cut ? kRows1 : kRowsR);
    if (D.n_comp == 0) return;
    if (final_cut && D.integer) return;   // (no workgroups are given to it: see kb_totals)
    cut_rows_body(bx, gx, D.n_ord, final_cut ? 1 : R, D.comp_order, D.m_ptr, D.m_col, D.m_val,
                  final_cut ? D.best_spins : D.spins, D.rowcut);
}
__global__ void kb_cut_chunks(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R, int final_cut) {
    QH_B(final_cut ? kChunks1 : kChunksR);
    if (D.n_comp == 0 || (final_cut && D.integer)) return;
    cut_chunks_body(bx, gx, D.n_chunks, final_cut ? 1 : R, D.chunk_begin, D.chunk_end, D.rowcut,
                    final_cut ? D.part1 : D.part);
}
__global__ void kb_cut_reduce(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R, int final_cut) {
    QH_B(kReduce);
    if (final_cut && D.integer) return;
    cut_reduce_body(bx, gx, D.n_comp, final_cut ? 1 : R, D.comp_chunk_ptr, final_cut ? D.part1 : D.part,
                    final_cut ? D.cut1 : D.cut_rc);
}
__global__ void kb_select(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R) {
    QH_B(kComp);
    select_body(bx, gx, D.n_comp, R, D.cut_rc, D.best_r);
}
// one workgroup per block: replica totals, then the selected (or final) total
__global__ void kb_totals(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R, int final_cut) {
    QH_B(kOne);
    if (final_cut) {
        if (D.n_comp && D.integer) {   // the selected cut plus the applied gains (kb_apply_flips)
            if (threadIdx.x == 0) *D.best_cut = *(D.selected_cut ? D.selected_cut : D.best_cut) + *D.gain_acc;
        } else if (D.n_comp) {
            selected_total_body(D.n_comp, D.cut1, nullptr, D.best_cut);
        } else if (threadIdx.x == 0) {
            *D.best_cut = 0.0;
        }
        return;
    }
    double *sel = D.selected_cut ? D.selected_cut : D.best_cut;
    if (D.n_comp == 0) {
        for (int r = threadIdx.x; r < R; r += blockDim.x) D.cuts[r] = 0.0;
        if (threadIdx.x == 0) *sel = 0.0;
        return;
    }
    replica_totals_body(0, 1, D.n_comp, R, D.cut_rc, D.cuts);
    selected_total_body(D.n_comp, D.cut_rc, D.best_r, sel);
}
__global__ void kb_best_spins(const ReadoutDesc *tbl, const int32_t *wg, int nb, int R) {
    QH_B(kVert);
    best_spins_body(bx, gx, D.n, R, D.comp, D.comp_first, D.best_r, D.spins, D.best_spins);
}
__global__ void kb_gain(const ReadoutDesc *tbl, const int32_t *wg, int nb) {
    QH_B(kGain);
    if (D.n_comp == 0) return;
    if (D.integer) {
        gain_wave_body(bx, gx, D.n, D.m_ptr, D.m_col, D.m_val, D.best_spins, D.gain);
        return;
    }
    gain_body(bx, gx, D.n, D.m_ptr, D.m_col, D.m_val, D.best_spins, D.gain);
}
__global__ void kb_pick(const ReadoutDesc *tbl, const int32_t *wg, int nb, int32_t *count) {
    QH_B(kVert);
    if (D.n_comp == 0) return;
    pick_body(bx, gx, D.n, D.m_ptr, D.m_col, D.gain, D.eps, nullptr, D.flag, count);
}
// Integer blocks also add up the gains they apply: a round flips an independent set, which
// raises the cut by exactly the sum of its gains, integers that FP64 adds exactly in any
// order, so the final cut is the selected one plus that sum, as a recount would give it.
__global__ void kb_apply_flips(const ReadoutDesc *tbl, const int32_t *wg, int nb) {
    QH_B(kVert);
    if (D.n_comp == 0) return;
    if (D.integer) {
        __shared__ double part[4];
        double s = 0.0;
        for (int64_t a = bx * (int64_t)blockDim.x + threadIdx.x; a < D.n; a += gx * (int64_t)blockDim.x)
            if (D.flag[a]) s += D.gain[a];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double t = part[0] + part[1] + part[2] + part[3];
            if (t != 0.0) atomicAdd(D.gain_acc, t);
        }
    }
    apply_flips_body(bx, gx, D.n, D.flag, D.best_spins);
}
#undef QH_B

// Readout of every block of a batch with one launch per kernel (plus one synchronisation
// per greedy round for the whole batch).
void readout_batched(const std::vector<ReadoutDesc> &descs_in, int R, bool greedy, hipStream_t st) {
    const int nb = (int)descs_in.size();
    if (nb == 0) return;
    DevBuf<double> acc(nb);   // applied greedy gains per block (integer blocks)
    acc.zero(st);
    std::vector<ReadoutDesc> descs(descs_in);
    for (int b = 0; b < nb; ++b) descs[b].gain_acc = acc.p + b;
    // workgroups per block for every index space, as the single-graph launches size them
    std::vector<int32_t> wg((size_t)kSlices * (nb + 1), 0);
    auto fill = [&](int slice, auto work) {
        int32_t *w = wg.data() + (size_t)slice * (nb + 1);
        for (int b = 0; b < nb; ++b) w[b + 1] = w[b] + work(descs[b]);
    };
    fill(kSigns, [&](const ReadoutDesc &d) { return grid_for(d.n * R); });
    fill(kRowsR, [&](const ReadoutDesc &d) { return grid_for(d.n_ord * rows_threads(R)); });
    fill(kChunksR, [&](const ReadoutDesc &d) { return grid_for(d.n_chunks * R); });
    fill(kReduce, [&](const ReadoutDesc &d) { return (int)std::max<int64_t>(1, std::min<int64_t>(d.n_comp, 1 << 20)); });
    fill(kComp, [&](const ReadoutDesc &d) { return grid_for(d.n_comp); });
    fill(kOne, [&](const ReadoutDesc &) { return 1; });
    fill(kVert, [&](const ReadoutDesc &d) { return grid_for(d.n); });
    // the integer blocks' greedy gains take one wave per row (four rows per workgroup), and
    // their final cut comes from the applied gains, with no pass over their rows
    fill(kRows1, [&](const ReadoutDesc &d) { return d.integer ? 0 : grid_for(d.n_ord); });
    fill(kGain, [&](const ReadoutDesc &d) { return d.integer ? grid_for(d.n, 4) : grid_for(d.n); });
    fill(kChunks1, [&](const ReadoutDesc &d) { return d.integer ? 0 : grid_for(d.n_chunks); });
    auto total = [&](int slice) { return (unsigned)wg[(size_t)slice * (nb + 1) + nb]; };
    DevBuf<ReadoutDesc> d_tbl(nb);
    DevBuf<int32_t> d_wg(wg.size()), d_cnt(2);
    QH_HIP(hipMemcpyAsync(d_tbl.p, descs.data(), nb * sizeof(ReadoutDesc), hipMemcpyHostToDevice, st));
    QH_HIP(hipMemcpyAsync(d_wg.p, wg.data(), wg.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    d_cnt.zero(st);
    const ReadoutDesc *T = d_tbl.p;
    const int32_t *W = d_wg.p;
    int32_t *bad = d_cnt.p + 1;

    hipLaunchKernelGGL(kb_signs, dim3(total(kSigns)), dim3(256), 0, st, T, W, nb, R, bad);
    hipLaunchKernelGGL(kb_cut_rows, dim3(total(kRowsR)), dim3(256), 0, st, T, W, nb, R, 0);
    hipLaunchKernelGGL(kb_cut_chunks, dim3(total(kChunksR)), dim3(256), 0, st, T, W, nb, R, 0);
    hipLaunchKernelGGL(kb_cut_reduce, dim3(total(kReduce)), dim3(256), 0, st, T, W, nb, R, 0);
    hipLaunchKernelGGL(kb_select, dim3(total(kComp)), dim3(256), 0, st, T, W, nb, R);
    hipLaunchKernelGGL(kb_totals, dim3(total(kOne)), dim3(256), 0, st, T, W, nb, R, 0);
    hipLaunchKernelGGL(kb_best_spins, dim3(total(kVert)), dim3(256), 0, st, T, W, nb, R);
    QH_CHECK_LAUNCH();
    if (greedy) {
        for (int it = 0; it < 100000; ++it) {
            hipLaunchKernelGGL(kb_gain, dim3(total(kGain)), dim3(256), 0, st, T, W, nb);
            QH_HIP(hipMemsetAsync(d_cnt.p, 0, sizeof(int32_t), st));
            hipLaunchKernelGGL(kb_pick, dim3(total(kVert)), dim3(256), 0, st, T, W, nb, d_cnt.p);
            QH_CHECK_LAUNCH();
            int32_t cnt = 0;
            QH_HIP(hipMemcpyAsync(&cnt, d_cnt.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            QH_HIP(hipStreamSynchronize(st));
            if (cnt == 0) break;
            hipLaunchKernelGGL(kb_apply_flips, dim3(total(kVert)), dim3(256), 0, st, T, W, nb);
            QH_CHECK_LAUNCH();
        }
    }
    if (total(kRows1)) hipLaunchKernelGGL(kb_cut_rows, dim3(total(kRows1)), dim3(256), 0, st, T, W, nb, R, 1);
    if (total(kChunks1)) hipLaunchKernelGGL(kb_cut_chunks, dim3(total(kChunks1)), dim3(256), 0, st, T, W, nb, R, 1);
    hipLaunchKernelGGL(kb_cut_reduce, dim3(total(kReduce)), dim3(64), 0, st, T, W, nb, R, 1);
    hipLaunchKernelGGL(kb_totals, dim3(total(kOne)), dim3(256), 0, st, T, W, nb, R, 1);
    QH_CHECK_LAUNCH();
    int32_t badb = 0;
    QH_HIP(hipMemcpyAsync(&badb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    QH_HIP(hipStreamSynchronize(st));
    if (badb) fail(QH_ENUMERIC, "non-finite spin or momentum in the final state of block %d", badb - 1);
}

}  // namespace qh

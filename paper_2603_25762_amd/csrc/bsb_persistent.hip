// Persistent dense bSB: every step of a solve inside one cooperative launch.
//
// The replicas split into `ng` independent groups of RT replicas; each group's
// workgroups cover all row tiles.  A workgroup owns a contiguous range of up to
// MAXT row tiles: their stored J tiles sit in LDS for the whole solve and their
// x / y state sits in VGPRs (wave w holds rows 16w..16w+15 of every row tile).
// Per step a workgroup only exchanges the 16-bit copy of x: it waits until every
// workgroup owning one of its column tiles has published the previous step,
// stages those column tiles into LDS, runs the MFMA product + bSB update, writes
// its own rows of the copy into the other half of a double buffer and publishes
// the step count.  J is symmetric, so "reads from" and "is read by" are the same
// neighbour relation, which makes the double buffer safe.
//
// Waits are bounded: a workgroup that polls longer than `max_polls` sets the
// error word and stops waiting, every later wait returns at once, and the grid
// always drains; the host then reports the failure.
#include <algorithm>
#include <cstring>
#include <vector>

#include "formats.h"
#include "internal.h"
#include "persistent.h"

namespace qh {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ inline void pbsb_update(float z, float &x, float &y, float coef, float c0, float dt, float a0) {
    float yn = y + (-coef * x + c0 * z) * dt;
    float xn = x + a0 * yn * dt;
    if (fabsf(xn) > 1.0f) {
        xn = xn > 0.0f ? 1.0f : -1.0f;
        yn = 0.0f;
    }
    x = xn;
    y = yn;
}

// COH selects how the 16-bit copy of x crosses workgroups between steps:
//  COH = 0: plain loads and stores, made visible by an agent-scope release fence before the
//           step flag (L2 write-back) and an agent-scope acquire fence after the wait (L2
//           invalidate);
//  COH = 1: every load and store of the copy is itself an agent-scope (device-coherent)
//           access, so no cache-wide write-back or invalidate is needed: a workgroup waits
//           for its own copy stores to complete before it raises its flag, and reads its
//           neighbours' copies only after seeing their flags.
template <int DT, int NB, int MAXT, int COH>
__global__ __launch_bounds__(256, 1) void k_dense_persistent(PersistArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int RT = NB * 16;
    constexpr int EB = (DT == QH_FP8_ROWSCALE) ? 1 : 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g4 = lane >> 4;
    const int grp = blockIdx.x % a.ng, w = blockIdx.x / a.ng;
    const int64_t R = a.R;
    const int64_t r0 = (int64_t)grp * RT;
    const int rt_b = a.wg_rt[w], rt_e = a.wg_rt[w + 1];
    const int T = rt_e - rt_b;
    const int jt0 = a.t_ptr[rt_b], jt1 = a.t_ptr[rt_e];
    const int n_ct = a.wg_ct_ptr[w + 1] - a.wg_ct_ptr[w];
    const int *ct_list = a.wg_ct + a.wg_ct_ptr[w];
    uint8_t *lds_j = smem;
    uint16_t *lds_h = (uint16_t *)(smem + a.lds_j_bytes);
    const int ct_elems = 64 * RT;   // 16-bit elements per staged column tile

    // J tiles of this workgroup's rows -> LDS (once)
    {
        const int64_t bytes = (int64_t)(jt1 - jt0) * kTileElems * EB;
        const uint4 *src = (const uint4 *)(a.t_val + (int64_t)jt0 * kTileElems * EB);
        uint4 *dst = (uint4 *)lds_j;
        for (int64_t o = tid; o < bytes / 16; o += 256) dst[o] = src[o];
    }
    // state -> registers
    float xs[MAXT][NB][4], ys[MAXT][NB][4], sc[MAXT][4];
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = (int64_t)(rt_b + ti) * kTile + wave * 16 + 4 * g4 + q;
            const bool live = ti < T && i < a.n;
            sc[ti][q] = (DT == QH_FP8_ROWSCALE && live) ? a.row_scale[i] : 1.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int64_t idx = i * R + r0 + b * 16 + l16;
                xs[ti][b][q] = live ? a.x[idx] : 0.0f;
                ys[ti][b][q] = live ? a.y[idx] : 0.0f;
            }
        }
    }
    __syncthreads();

    const int *flags = a.flags + (int64_t)grp * a.wpg;
    const int nbr_b = a.nbr_ptr[w], n_nbr = a.nbr_ptr[w + 1] - nbr_b;
    const int steps = a.ke - a.kb;
    for (int s = 0; s < steps; ++s) {
        // 1. wait for the neighbours' previous step
        if (s > 0) {
            if (tid < n_nbr) {
                const int *f = flags + a.nbr[nbr_b + tid];
                int64_t polls = 0;
                while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < s) {
                    if ((++polls & 1023) == 0 &&
                        (polls > a.max_polls ||
                         __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                        __hip_atomic_fetch_or(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if constexpr (!COH) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        // 2. stage the column tiles of x (16-bit copy, half s % 2) into LDS
        const uint16_t *hin = (s & 1) ? a.h1 : a.h0;
        uint16_t *hout = (s & 1) ? a.h0 : a.h1;
        {
            // a column tile is 8 row groups of 8 rows; each group holds RT replicas x 8 values
            // contiguously.  Issue a batch of 16-byte loads before any LDS store so that one
            // round trip to memory covers the whole batch.
            constexpr int kBatch = 8;
            const int total = n_ct * 8 * RT;
            for (int base = 0; base < total; base += 256 * kBatch) {
                uint4 v[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int e = base + u * 256 + tid;
                    if (e < total) {
                        const int c = e / (8 * RT), rem = e - c * 8 * RT;
                        const int jgl = rem / RT, rl = rem - jgl * RT;
                        const uint16_t *src = hin + (((int64_t)ct_list[c] * 8 + jgl) * R + r0 + rl) * 8;
                        if constexpr (COH) {
                            uint64_t *q = (uint64_t *)src;
                            const uint64_t lo = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            const uint64_t hi = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            v[u] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
                        } else {
                            v[u] = *(const uint4 *)src;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int e = base + u * 256 + tid;
                    if (e < total) *(uint4 *)(lds_h + (int64_t)e * 8) = v[u];
                }
            }
        }
        __syncthreads();

        // 3. product and update, row tile by row tile
        const float coef = a.a0 - a.pump[a.kb + s];
#pragma unroll
        for (int ti = 0; ti < MAXT; ++ti) {
            if (ti >= T) break;
            const int rt = rt_b + ti;
            float4_t acc[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] = float4_t{0.f, 0.f, 0.f, 0.f};
            for (int t = a.t_ptr[rt]; t < a.t_ptr[rt + 1]; ++t) {
                const int slot = a.tile_slot[t];
                const uint8_t *jt = lds_j + (int64_t)(t - jt0) * kTileElems * EB;
                const uint16_t *ht = lds_h + (int64_t)slot * ct_elems;
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const int frag = wave * 2 + kb;
                    half8_t av;
                    if constexpr (DT == QH_FP8_ROWSCALE) {
                        uint2 c = *(const uint2 *)(jt + ((frag * 64 + lane) << 3));
                        uint16_t hb[8];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            hb[e] = e4m3_to_f16_bits_scaled((uint8_t)(c.x >> (8 * e)));
                            hb[4 + e] = e4m3_to_f16_bits_scaled((uint8_t)(c.y >> (8 * e)));
                        }
                        __builtin_memcpy(&av, hb, 16);
                    } else {
                        av = *(const half8_t *)((const uint16_t *)jt + ((frag * 64 + lane) << 3));
                    }
                    const int jgl = kb * 4 + g4;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const uint16_t *hp = ht + (jgl * RT + b * 16 + l16) * 8;
                        if constexpr (DT == QH_BF16) {
                            bf16x8_t bv = *(const bf16x8_t *)hp;
                            bf16x8_t aw;
                            __builtin_memcpy(&aw, &av, 16);
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bv, acc[b], 0, 0, 0);
                        } else {
                            half8_t bv = *(const half8_t *)hp;
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc[b], 0, 0, 0);
                        }
                    }
                }
            }
            const int64_t rowbase = (int64_t)rt * kTile + wave * 16 + 4 * g4;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                uint16_t hv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float z = acc[b][q];
                    if constexpr (DT == QH_FP8_ROWSCALE) z *= sc[ti][q];
                    pbsb_update(z, xs[ti][b][q], ys[ti][b][q], coef, a.c0, a.dt, a.a0);
                    const bool live = rowbase + q < a.n;
                    const float cv = a.discrete ? (xs[ti][b][q] >= 0.f ? 1.f : -1.f) : xs[ti][b][q];
                    if constexpr (DT == QH_BF16) hv[q] = live ? f32_to_bf16_rne(cv) : 0;
                    else hv[q] = live ? f32_to_f16_rne(cv) : 0;
                }
                uint2 pk;
                pk.x = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
                pk.y = (uint32_t)hv[2] | ((uint32_t)hv[3] << 16);
                uint16_t *dst = hout + ((rowbase >> 3) * R + r0 + b * 16 + l16) * 8 + (rowbase & 7);
                if constexpr (COH)
                    __hip_atomic_store((uint64_t *)dst, (uint64_t)pk.x | ((uint64_t)pk.y << 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                else
                    *(uint2 *)dst = pk;
            }
        }
        // 4. publish: own stores done, then one agent-scope release per workgroup
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            if constexpr (!COH) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(a.flags + (int64_t)grp * a.wpg + w, s + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // final state -> memory
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = (int64_t)(rt_b + ti) * kTile + wave * 16 + 4 * g4 + q;
            if (ti >= T || i >= a.n) continue;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int64_t idx = i * R + r0 + b * 16 + l16;
                a.x[idx] = xs[ti][b][q];
                a.y[idx] = ys[ti][b][q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static constexpr int kMaxT = 8;
static constexpr int64_t kLdsLimit = 160 * 1024;

// Replica-group widths to try, most groups first (more workgroups, fewer row tiles each).
static std::vector<int> group_widths(int R) {
    std::vector<int> out;
    for (int div : {8, 4, 2, 1}) {
        if (R % div) continue;
        int rt = R / div;
        if ((rt == 16 || rt == 32 || rt == 64) && std::find(out.begin(), out.end(), rt) == out.end())
            out.push_back(rt);
    }
    if (out.empty() && R % 64 == 0) out.push_back(64);
    return out;
}

// Decide whether the persistent plan applies and build its tables.  Returns false
// (and leaves `pp.ok` false) when the state or J would not fit on chip.
bool build_persistent_plan(const qh_graph *g, int R, PersistPlan &pp, hipStream_t st) {
    pp.ok = false;
    if (g->storage != QH_STORE_DENSE || g->dtype == QH_F32 || g->n_rt == 0) return false;
    int dev = 0, n_cu = 0, coop = 0;
    QH_HIP(hipGetDevice(&dev));
    QH_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    QH_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return false;
    const int64_t n_rt = g->n_rt;
    auto tptr = download(g->t_ptr.p, n_rt + 1, st);
    auto tcol = download(g->t_col.p, g->n_tiles, st);
    const int eb = dtype_bytes(g->dtype);
    for (int RT : group_widths(R)) {
    const int ng = R / RT;
    if (ng > n_cu) continue;
    const int64_t ct_bytes = 64 * (int64_t)RT * 2;
    // try workgroup counts from the most to the fewest per group
    int max_wpg = (int)std::min<int64_t>(n_rt, n_cu / ng);
    for (int wpg = max_wpg; wpg >= 1; --wpg) {
        if (ceil_div(n_rt, wpg) > kMaxT) break;   // fewer workgroups only makes T larger
        // contiguous partition balanced by stored tiles (+1 per row tile for the update)
        std::vector<int64_t> work(n_rt + 1, 0);
        for (int64_t rt = 0; rt < n_rt; ++rt) work[rt + 1] = work[rt] + (tptr[rt + 1] - tptr[rt]) + 1;
        std::vector<int32_t> wg_rt(wpg + 1, 0);
        int64_t cur = 0;
        bool ok = true;
        for (int w = 0; w < wpg; ++w) {
            wg_rt[w] = (int32_t)cur;
            int64_t e;
            if (w == wpg - 1) {
                e = n_rt;
            } else {
                const int64_t target = work[n_rt] * (w + 1) / wpg;
                e = cur + 1;
                while (e < n_rt && work[e] < target) ++e;
                const int64_t max_e = n_rt - (wpg - w - 1);
                if (e > max_e) e = max_e;
            }
            if (e <= cur || e - cur > kMaxT) { ok = false; break; }
            cur = e;
        }
        wg_rt[wpg] = (int32_t)n_rt;
        if (!ok || cur != n_rt) continue;
        std::vector<int32_t> owner(n_rt);
        for (int w = 0; w < wpg; ++w)
            for (int32_t rt = wg_rt[w]; rt < wg_rt[w + 1]; ++rt) owner[rt] = w;
        std::vector<int32_t> ct_ptr(wpg + 1, 0), cts, slot(g->n_tiles), nbr_ptr(wpg + 1, 0), nbrs;
        int64_t lds_max_j = 0, lds_max_h = 0;
        for (int w = 0; w < wpg && ok; ++w) {
            std::vector<int32_t> u;
            for (int32_t t = tptr[wg_rt[w]]; t < tptr[wg_rt[w + 1]]; ++t) u.push_back(tcol[t]);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            ct_ptr[w] = (int32_t)cts.size();
            for (int32_t t = tptr[wg_rt[w]]; t < tptr[wg_rt[w + 1]]; ++t)
                slot[t] = (int32_t)(std::lower_bound(u.begin(), u.end(), tcol[t]) - u.begin());
            cts.insert(cts.end(), u.begin(), u.end());
            std::vector<int32_t> nb;
            for (int32_t c : u)
                if (owner[c] != w) nb.push_back(owner[c]);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            if (nb.size() > 256) ok = false;
            nbr_ptr[w] = (int32_t)nbrs.size();
            nbrs.insert(nbrs.end(), nb.begin(), nb.end());
            int64_t jb = (int64_t)(tptr[wg_rt[w + 1]] - tptr[wg_rt[w]]) * kTileElems * eb;
            lds_max_j = std::max(lds_max_j, jb);
            lds_max_h = std::max(lds_max_h, (int64_t)u.size() * ct_bytes);
        }
        ct_ptr[wpg] = (int32_t)cts.size();
        nbr_ptr[wpg] = (int32_t)nbrs.size();
        lds_max_j = ceil_div(lds_max_j, 16) * 16;
        if (!ok || lds_max_j + lds_max_h > kLdsLimit) continue;
        // upload
        pp.RT = RT;
        pp.ng = ng;
        pp.wpg = wpg;
        pp.lds_j_bytes = lds_max_j;
        pp.lds_bytes = lds_max_j + lds_max_h;
        pp.wg_rt.alloc(wpg + 1);
        pp.wg_rt.upload(wg_rt.data(), wpg + 1, st);
        pp.wg_ct_ptr.alloc(wpg + 1);
        pp.wg_ct_ptr.upload(ct_ptr.data(), wpg + 1, st);
        pp.wg_ct.alloc(cts.size());
        pp.wg_ct.upload(cts.data(), cts.size(), st);
        pp.tile_slot.alloc(slot.size());
        pp.tile_slot.upload(slot.data(), slot.size(), st);
        pp.nbr_ptr.alloc(wpg + 1);
        pp.nbr_ptr.upload(nbr_ptr.data(), wpg + 1, st);
        pp.nbr.alloc(std::max<size_t>(nbrs.size(), 1));
        pp.nbr.upload(nbrs.data(), nbrs.size(), st);
        pp.flags.alloc((size_t)ng * wpg + 64);
        QH_HIP(hipStreamSynchronize(st));
        pp.ok = true;
        return true;
    }
    }
    return false;
}

template <int DT, int NB, int COH>
static void launch_t(const PersistArgs &args, int grid, int lds, hipStream_t st) {
    auto fn = k_dense_persistent<DT, NB, kMaxT, COH>;
    if (hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
        (void)hipGetLastError();
    int per_cu = 0;
    QH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, 256, lds));
    int dev = 0, n_cu = 0;
    QH_HIP(hipGetDevice(&dev));
    QH_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (per_cu * n_cu < grid)
        fail(QH_EUNSUPPORTED, "persistent plan needs %d co-resident workgroups, device holds %d", grid,
             per_cu * n_cu);
    PersistArgs a = args;
    void *kargs[] = {&a};
    QH_HIP(hipLaunchCooperativeKernel((const void *)fn, dim3(grid), dim3(256), kargs, (unsigned)lds, st));
}

void launch_persistent(const qh_graph *g, const PersistPlan &pp, const PersistArgs &args, int coherent,
                       hipStream_t st) {
    const int grid = pp.ng * pp.wpg;
    const int lds = (int)pp.lds_bytes;
#define QH_PC(DTV, NBV)                                                  \
    do {                                                                 \
        if (coherent) launch_t<DTV, NBV, 1>(args, grid, lds, st);        \
        else launch_t<DTV, NBV, 0>(args, grid, lds, st);                 \
    } while (0)
#define QH_P(DTV)                                                     \
    do {                                                              \
        if (pp.RT == 16) QH_PC(DTV, 1);                               \
        else if (pp.RT == 32) QH_PC(DTV, 2);                          \
        else QH_PC(DTV, 4);                                           \
    } while (0)
    switch (g->dtype) {
        case QH_F16: QH_P(QH_F16); break;
        case QH_BF16: QH_P(QH_BF16); break;
        case QH_FP8_ROWSCALE: QH_P(QH_FP8_ROWSCALE); break;
        default: fail(QH_EUNSUPPORTED, "persistent plan needs a 16- or 8-bit dense graph");
    }
#undef QH_P
#undef QH_PC
}

}  // namespace qh

namespace qh {

void plan_info(const qh_graph *g, int R, qh_plan_info *out) {
    qh_plan_info i{};
    auto it = g->plans.find(R);
    if (it != g->plans.end()) {
        const SolvePlan &p = *it->second;
        i.plan_used = p.last_plan;
        if (p.pp && p.pp->ok) {
            i.persistent_ok = 1;
            i.replicas_per_group = p.pp->RT;
            i.groups = p.pp->ng;
            i.workgroups_per_group = p.pp->wpg;
            i.lds_bytes = (int32_t)p.pp->lds_bytes;
        }
        i.us_per_step[0] = p.tuned_us[0];
        i.us_per_step[1] = p.tuned_us[1];
        i.replica_tile = g->storage == QH_STORE_DENSE ? (R >= 64 ? p.run_rt : R) : 0;
        i.tiles_in_flight = g->storage == QH_STORE_DENSE ? (R >= 64 && p.run_rt == 64 ? p.run_depth : 4) : 0;
        i.persistent_sync = p.last_plan == 2 ? 1 + p.last_coh : 0;
        i.us_persistent_coherent = p.tuned_us_coh;
        if (g->storage != QH_STORE_DENSE) {
            int sk = p.sky_kernel;
            if (sk == kSkyBandFma && !(R >= 64 && g->n_bblk > 0)) sk = kSkyRows;
            if (sk == kSkyBandMfma && g->n_bblk == 0) sk = kSkyRows;
            i.skyline_kernel = sk == kSkyRows ? 3 : sk == kSkyBandFma ? 4 : 5;
            i.skyline_us[0] = p.sky_us[kSkyBandFma];
            i.skyline_us[1] = p.sky_us[kSkyBandMfma];
        }
    }
    *out = i;
}

}  // namespace qh

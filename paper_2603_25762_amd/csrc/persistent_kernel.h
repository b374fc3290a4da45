// The persistent dense bSB kernel and its launch dispatch, shared by the translation
// units that instantiate it without (bsb_persistent.hip) and with (bsb_persistent_field.hip)
// a deformation field, so that the two halves compile in parallel.
#pragma once

#include "formats.h"
#include "internal.h"
#include "persistent.h"

namespace qh {

static constexpr int kMaxT = 8;     // row tiles per workgroup (kernels for 2, 4 and 8)

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ inline void pbsb_update(float z, float &x, float &y, float coef, float c0, float dt, float a0) {
    const float yn = y + (-coef * x + c0 * z) * dt;
    const float xn = x + a0 * yn * dt;
    // walls: past |x| = 1, x = sgn(x) (the median of -1, xn, 1) and y = 0
    y = fabsf(xn) > 1.0f ? 0.0f : yn;
    x = __builtin_amdgcn_fmed3f(xn, -1.0f, 1.0f);
}

// COH selects how the 16-bit copy of x crosses workgroups between steps:
//  COH = 0: plain loads and stores, made visible by an agent-scope release fence before the
//           step flag (L2 write-back) and an agent-scope acquire fence after the wait (L2
//           invalidate);
//  COH = 1: every load and store of the copy is itself an agent-scope (device-coherent)
//           access, so no cache-wide write-back or invalidate is needed: a workgroup waits
//           for its own copy stores to complete before it raises its flag, and reads its
//           neighbours' copies only after seeing their flags.
// FLD = 1 adds the deformation field h of the row to its coupling sum before the update
// (a separate instantiation, so that the plain kernel carries no trace of it).
template <int DT, int NB, int MAXT, int COH, int FLD>
__global__ __launch_bounds__(256, 1) void k_dense_persistent(PersistArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    constexpr int RT = NB * 16;
    constexpr int EB = (DT == QH_FP8_ROWSCALE) ? 1 : 2;
    // 16-byte staging loads per thread in flight together (fewer where the state of more
    // row tiles occupies the registers)
    constexpr int kStageBatch = MAXT <= 2 ? 16 : (MAXT <= 4 ? 12 : 4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, g4 = lane >> 4;
    const int grp = blockIdx.x % a.ng, w = blockIdx.x / a.ng;
    const int64_t R = a.R;
    const int64_t r0 = (int64_t)grp * RT;
    const int rt_b = a.wg_rt[w], rt_e = a.wg_rt[w + 1];
    const int T = rt_e - rt_b;
    const int jt0 = a.t_ptr[rt_b], jt1 = a.t_ptr[rt_e];
    // stored-tile range of each own row tile, read once (wave-uniform, kept in SGPRs)
    int tile_b[MAXT + 1];
#pragma unroll
    for (int ti = 0; ti <= MAXT; ++ti)
        tile_b[ti] = __builtin_amdgcn_readfirstlane(ti <= T ? a.t_ptr[rt_b + ti] : jt1);
    const int n_ct = a.wg_ct_ptr[w + 1] - a.wg_ct_ptr[w];
    const int *ct_list = a.wg_ct + a.wg_ct_ptr[w];
    uint8_t *lds_j = smem;
    uint16_t *lds_h = (uint16_t *)(smem + a.lds_j_bytes);
    int32_t *lds_slot = (int32_t *)(smem + a.lds_tab_off);   // staging slot of each own stored tile
    int32_t *lds_xct = lds_slot + a.max_wg_tiles;             // column tiles staged from memory ...
    int32_t *lds_xslot = lds_xct + a.max_ct;                  // ... and their staging slots
    const int ct_elems = 64 * RT;   // 16-bit elements per staged column tile
    for (int i = tid; i < jt1 - jt0; i += 256) lds_slot[i] = a.tile_slot[jt0 + i];
    // Column tiles that are this workgroup's own row tiles reach LDS straight from the
    // registers that hold their x; the others (the neighbours' rows) are staged from memory.
    int own_slot[MAXT];
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) own_slot[ti] = -1;
    int n_ext = 0;
    for (int c = 0; c < n_ct; ++c) {          // wave-uniform walk over a short list
        const int ct = ct_list[c];
        if (ct >= rt_b && ct < rt_e) {
#pragma unroll
            for (int ti = 0; ti < MAXT; ++ti)
                if (ct == rt_b + ti) own_slot[ti] = c;
        } else {
            if (tid == 0) {
                lds_xct[n_ext] = ct;
                lds_xslot[n_ext] = c;
            }
            ++n_ext;
        }
    }

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
    // 16-bit copy of the lane's four rows of (row tile ti, replica block b), as the other
    // workgroups receive it (rows past n hold 0)
    auto pack_copy = [&](int ti, int b) -> uint2 {
        const int64_t rowbase = (int64_t)(rt_b + ti) * kTile + wave * 16 + 4 * g4;
        uint16_t hv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool live = rowbase + q < a.n;
            const float cv = a.discrete ? (xs[ti][b][q] >= 0.f ? 1.f : -1.f) : xs[ti][b][q];
            if constexpr (DT == QH_BF16) hv[q] = live ? f32_to_bf16_rne(cv) : 0;
            else hv[q] = live ? f32_to_f16_rne(cv) : 0;
        }
        return make_uint2((uint32_t)hv[0] | ((uint32_t)hv[1] << 16), (uint32_t)hv[2] | ((uint32_t)hv[3] << 16));
    };
    // the packed copy of the own rows is kept for the LDS write where registers allow (up to
    // four row tiles) and packed again from x otherwise
    constexpr bool kKeepPk = MAXT <= 4;
    uint2 pkw[kKeepPk ? MAXT : 1][NB];
    // own rows -> their staging slots (rows 4 g4 .. 4 g4 + 3 of the wave's 16)
    auto write_own = [&]() {
        const int lr = wave * 16 + 4 * g4;
#pragma unroll
        for (int ti = 0; ti < MAXT; ++ti) {
            if (ti >= T || own_slot[ti] < 0) continue;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                *(uint2 *)(lds_h + (int64_t)own_slot[ti] * ct_elems + ((lr >> 3) * RT + b * 16 + l16) * 8 + (lr & 7)) =
                    kKeepPk ? pkw[kKeepPk ? ti : 0][b] : pack_copy(ti, b);
        }
    };
    if constexpr (kKeepPk) {
#pragma unroll
        for (int ti = 0; ti < MAXT; ++ti)
#pragma unroll
            for (int b = 0; b < NB; ++b) pkw[ti][b] = ti < T ? pack_copy(ti, b) : make_uint2(0, 0);
    }
    write_own();
    __syncthreads();
    // The staging pattern is the same every step.  A column tile is 8 row groups of 8 rows;
    // each group holds RT replicas x 8 values contiguously (one 16-byte piece).  The pieces of
    // the first batch keep their source offsets and LDS destinations (in pieces) in registers.
    const int total = n_ext * 8 * RT;
    uint32_t soff[kStageBatch], doff[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
        const int e = u * 256 + tid;
        soff[u] = doff[u] = 0;
        if (e < total) {
            const int k = e / (8 * RT), rem = e - k * 8 * RT;
            const int jgl = rem / RT, rl = rem - jgl * RT;
            soff[u] = (uint32_t)(((int64_t)lds_xct[k] * 8 + jgl) * R + r0 + rl);
            doff[u] = (uint32_t)(lds_xslot[k] * 8 * RT + rem);
        }
    }

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
            // Every 16-byte load of a batch is issued before the first LDS store, so that one
            // round trip to memory covers the batch (kStageBatch x 4 KB; later batches, for
            // longer column-tile lists, take their sources from the LDS copy of the list).
            for (int base = 0; base < total; base += 256 * kStageBatch) {
                uint4 v[kStageBatch];
#pragma unroll
                for (int u = 0; u < kStageBatch; ++u) {
                    const int e = base + u * 256 + tid;
                    if (e < total) {
                        uint32_t off;
                        if (base == 0) {
                            off = soff[u];
                        } else {
                            const int k = e / (8 * RT), rem = e - k * 8 * RT;
                            const int jgl = rem / RT, rl = rem - jgl * RT;
                            off = (uint32_t)(((int64_t)lds_xct[k] * 8 + jgl) * R + r0 + rl);
                        }
                        const uint16_t *src = hin + (int64_t)off * 8;
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
                for (int u = 0; u < kStageBatch; ++u) {
                    const int e = base + u * 256 + tid;
                    if (e < total) {
                        const int k = e / (8 * RT);
                        const uint32_t d = base == 0 ? doff[u] : (uint32_t)(lds_xslot[k] * 8 * RT + e - k * 8 * RT);
                        *(uint4 *)(lds_h + (int64_t)d * 8) = v[u];
                    }
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
            const int tb = tile_b[ti], te = tile_b[ti + 1];
            // A fragments (J) and B fragments (x copy) of one stored tile, for both K halves
            half8_t af[2][2], bf[2][2][NB];
            // staging slot of tile t (clamped into the row tile's range): read two tiles
            // ahead, so that waiting for it never waits for the fragment loads issued since
            auto slot_of = [&](int t) { return lds_slot[min(t, te - 1) - jt0]; };
            // fragments of tile t; a slot past the row tile's last tile reloads that tile with
            // A = 0, which adds exactly zero, so that the loop below has no branches (the
            // accumulators then stay in place across iterations)
            auto load_frags = [&](int t, int slot, half8_t (&A)[2], half8_t (&Bv)[2][NB]) {
                t = min(t, te - 1);
                const uint8_t *jt = lds_j + (int64_t)(t - jt0) * kTileElems * EB;
                const uint16_t *ht = lds_h + (int64_t)slot * ct_elems;
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const int frag = wave * 2 + kb;
                    if constexpr (DT == QH_FP8_ROWSCALE) {
                        uint2 c = *(const uint2 *)(jt + ((frag * 64 + lane) << 3));
                        A[kb] = e4m3x8_to_f16_scaled(c);
                    } else {
                        A[kb] = *(const half8_t *)((const uint16_t *)jt + ((frag * 64 + lane) << 3));
                    }
                    const int jgl = kb * 4 + g4;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        Bv[kb][b] = *(const half8_t *)(ht + (jgl * RT + b * 16 + l16) * 8);
                }
            };
            // (pad: the slot is past the row tile's last tile, A = 0; applied here, where the
            // MFMAs wait for the fragments anyway)
            auto mfmas = [&](const half8_t (&A)[2], const half8_t (&Bv)[2][NB], bool pad) {
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const half8_t ak = pad ? half8_t{} : A[kb];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if constexpr (DT == QH_BF16) {
                            bf16x8_t aw, bw;
                            __builtin_memcpy(&aw, &ak, 16);
                            __builtin_memcpy(&bw, &Bv[kb][b], 16);
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bw, acc[b], 0, 0, 0);
                        } else {
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ak, Bv[kb][b], acc[b], 0, 0, 0);
                        }
                    }
                }
            };
            // two tiles per iteration, each one's fragments loaded before the other's MFMAs
            if (tb < te) {
                int sl_next = slot_of(tb + 1);
                load_frags(tb, slot_of(tb), af[0], bf[0]);
                for (int t = tb; t < te; t += 2) {
                    const int sl2 = slot_of(t + 2), sl3 = slot_of(t + 3);
                    load_frags(t + 1, sl_next, af[1], bf[1]);
                    __builtin_amdgcn_sched_barrier(0);   // keep the next tile's loads ahead of these MFMAs
                    mfmas(af[0], bf[0], false);
                    __builtin_amdgcn_sched_barrier(0);
                    load_frags(t + 2, sl2, af[0], bf[0]);
                    __builtin_amdgcn_sched_barrier(0);
                    mfmas(af[1], bf[1], t + 1 >= te);
                    __builtin_amdgcn_sched_barrier(0);
                    sl_next = sl3;
                }
            }
            const int64_t rowbase = (int64_t)rt * kTile + wave * 16 + 4 * g4;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float z = acc[b][q];
                    if constexpr (DT == QH_FP8_ROWSCALE) z *= sc[ti][q];
                    if constexpr (FLD) {
                        if (rowbase + q < a.n) z += a.field[rowbase + q];
                    }
                    pbsb_update(z, xs[ti][b][q], ys[ti][b][q], coef, a.c0, a.dt, a.a0);
                }
                const uint2 pk = pack_copy(ti, b);
                if constexpr (kKeepPk) pkw[kKeepPk ? ti : 0][b] = pk;
                uint16_t *dst = hout + ((rowbase >> 3) * R + r0 + b * 16 + l16) * 8 + (rowbase & 7);
                if constexpr (COH)
                    __hip_atomic_store((uint64_t *)dst, (uint64_t)pk.x | ((uint64_t)pk.y << 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                else
                    *(uint2 *)dst = pk;
            }
        }
        // 4. publish: own stores done, then one agent-scope release per workgroup.  Every wave
        // is past this step's product here, so the own column tiles can take the new x.
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        write_own();
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

template <int DT, int NB, int MAXT, int COH, int FLD>
static void launch_t(const PersistArgs &args, int grid, int lds, hipStream_t st) {
    auto fn = k_dense_persistent<DT, NB, MAXT, COH, FLD>;
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

template <int FLD>
static void launch_persistent_fld(const qh_graph *g, const PersistPlan &pp, const PersistArgs &args, int coherent,
                                  hipStream_t st) {
    const int grid = pp.ng * pp.wpg;
    const int lds = (int)pp.lds_bytes;
#define QH_PM(DTV, NBV, COHV)                                                   \
    do {                                                                        \
        if (pp.max_t <= 2) launch_t<DTV, NBV, 2, COHV, FLD>(args, grid, lds, st);    \
        else if (pp.max_t <= 4) launch_t<DTV, NBV, 4, COHV, FLD>(args, grid, lds, st); \
        else launch_t<DTV, NBV, kMaxT, COHV, FLD>(args, grid, lds, st);              \
    } while (0)
#define QH_PC(DTV, NBV)                                                  \
    do {                                                                 \
        if (coherent) QH_PM(DTV, NBV, 1);                                \
        else QH_PM(DTV, NBV, 0);                                         \
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
#undef QH_PM
}

}  // namespace qh

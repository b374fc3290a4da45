// Ballistic simulated bifurcation on gfx950 (Methods, SB algorithm solution).
//
// One step, for all R replicas at once:
//   z = J x                                   (coupling product)
//   y <- y + [-(a0 - p_k) x + c0 z] dt        (symplectic Euler, y first)
//   x <- x + a0 y dt
//   |x| > 1  =>  x <- sgn x, y <- 0           (inelastic walls)
// The product and the update are fused in one kernel per step; z never
// reaches memory.  After the last step: s = sgn(x) (sgn 0 = +1), FP64 cuts
// per replica and component from the master couplings (Eqs. 4-6), the best
// replica per component, and the greedy single-flip rounds.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "formats.h"
#include "internal.h"
#include "persistent.h"

namespace qh {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// initial state: SplitMix64 (Steele, Lea & Flood 2014), draw k = 2 (r n + i) + {0, 1}
// ---------------------------------------------------------------------------

__global__ void k_init(uint64_t seed, int64_t n, int R, float *__restrict__ x, float *__restrict__ y) {
    int64_t total = n * R;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / R, r = t - i * R;
        uint64_t c = 2ull * ((uint64_t)r * (uint64_t)n + (uint64_t)i);
        double ux = (double)(sm64_draw(seed, c) >> 11) * 0x1.0p-53;
        double uy = (double)(sm64_draw(seed, c + 1) >> 11) * 0x1.0p-53;
        x[t] = (float)(0.2 * ux - 0.1);
        y[t] = (float)(0.2 * uy - 0.1);
    }
}

__global__ void k_pump_linear(int steps, float *__restrict__ p) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < steps; k += gridDim.x * blockDim.x)
        p[k] = steps > 1 ? (float)((double)k / (double)(steps - 1)) : 0.0f;
}

// 16-bit product copy of x in the layout [n_pad / 8][R][8]: eight consecutive
// rows of one replica are contiguous, which is the B-operand register order of
// v_mfma_f32_16x16x32_{f16,bf16}.
// value of x_j that enters the coupling product: x_j, or sgn(x_j) (sgn(0) = +1) in the
// discrete variant; +-1 is exact in every storage format
__device__ inline float coupling_value(float x, int discrete) { return discrete ? (x >= 0.f ? 1.f : -1.f) : x; }

template <bool BF16>
__global__ void k_x_to_h(int64_t n, int R, const float *__restrict__ x, uint16_t *__restrict__ h, int discrete) {
    int64_t total = n * R;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / R, r = t - i * R;
        const float v = coupling_value(x[t], discrete);
        h[((i >> 3) * R + r) * 8 + (i & 7)] = BF16 ? f32_to_bf16_rne(v) : f32_to_f16_rne(v);
    }
}

// binary16 copy of x in the state layout [n][R] for the long-range gathers: a gather then
// moves 2R bytes instead of 4R (|x| <= 1: binary16 keeps 11 significant bits down to 2^-14)
__device__ inline uint16_t lr_copy_value(float x, int discrete) { return f32_to_f16_rne(coupling_value(x, discrete)); }

__global__ void k_x_to_lh(int64_t total, const float *__restrict__ x, uint16_t *__restrict__ h, int discrete) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x)
        h[t] = lr_copy_value(x[t], discrete);
}

// x_j as a long-range gather sees it: from the binary16 copy (H16) or from x itself
template <bool H16>
__device__ inline float lr_x(const float *x_in, const uint16_t *h_in, int64_t idx, int discrete) {
    if constexpr (H16) return f16_bits_to_f32(h_in[idx]);
    else return coupling_value(x_in[idx], discrete);
}

struct StepArgs {
    float c0, dt, a0;
    const float *pump;
    int k;
    int discrete;   // 1: the coupling takes sgn(x_j) (discrete variant), 0: x_j
    float bscale;   // band blocks: power of two undoing the scale of their binary16 encoding (1: none)
    const float *field;   // deformation field h [n] joining the coupling sum (nullptr: none)
    uint16_t *lr_out = nullptr;   // SNP kernels: binary16 copy of the new x for the long-range gathers
};

// the new x of state element idx into the long-range copy, when the step keeps one
__device__ inline void store_lr_copy(const StepArgs &sa, int64_t idx, float x) {
    if (sa.lr_out) sa.lr_out[idx] = lr_copy_value(x, sa.discrete);
}

// The coupling sum of row i with the deformation field added: the field enters after the
// whole sum J x, so every step kernel rounds it identically.
__device__ inline float with_field(float z, int64_t i, const StepArgs &s) {
    return s.field ? z + s.field[i] : z;
}


__device__ inline void bsb_update(float z, float &x, float &y, float coef, const StepArgs &s) {
    const float yn = y + (-coef * x + s.c0 * z) * s.dt;
    const float xn = x + s.a0 * yn * s.dt;
    // walls: past |x| = 1, x = sgn(x) (the median of -1, xn, 1) and y = 0
    y = fabsf(xn) > 1.0f ? 0.0f : yn;
    x = __builtin_amdgcn_fmed3f(xn, -1.0f, 1.0f);
}

// XCD-aware block index: hardware dispatches workgroup b to XCD b % 8; give each
// XCD a contiguous range of logical tiles so that neighbouring row tiles (which
// share columns of x) meet in the same L2.
__device__ inline int64_t xcd_remap(int64_t bid, int64_t G) {
    int64_t xcd = bid & 7, q = bid >> 3;
    int64_t per = G >> 3, rem = G & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + q;
}

// ---------------------------------------------------------------------------
// dense tiles, MFMA product (read graphs)
// ---------------------------------------------------------------------------
// Workgroup = 4 waves = one 64-row tile x RT replicas.  Wave w owns rows
// 16w..16w+15 of the tile and NB = RT/16 replica blocks of 16.
//  DT = QH_F16 / QH_BF16: v_mfma_f32_16x16x32_{f16,bf16}, A = stored tile fragment,
//       B = 16-bit copy of x.
//  DT = QH_FP8_ROWSCALE: E4M3 codes expanded exactly to f16 (value * 2^-8) in
//       registers; the row scale (x 256) multiplies z in the epilogue.
//  DT = QH_F32: v_mfma_f32_16x16x4f32 on the FP32 tile and FP32 x.
// Product of stored tiles [t_beg, t_end) of one row tile with x, for the 16 rows of this
// wave and RT = 16 NB replicas starting at r0.  Shared by the per-step and batched kernels.
// U = stored tiles whose loads are in flight together (16/8-bit paths).
template <int DT, int NB, int U = (NB >= 4 ? 2 : 4)>
__device__ inline void dense_product(float4_t (&acc)[NB], int t_beg, int t_end, const int32_t *__restrict__ t_col,
                                     const uint8_t *__restrict__ t_val, const float *x_in,
                                     const uint16_t *__restrict__ h_in, int64_t R, int64_t r0, int wave, int lane,
                                     int discrete) {
    const int l16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = float4_t{0.f, 0.f, 0.f, 0.f};
    if constexpr (DT == QH_F32) {
        for (int t = t_beg; t < t_end; ++t) {
            const int64_t j0 = (int64_t)t_col[t] * kTile;
            const float *tile = (const float *)t_val + (int64_t)t * kTileElems;
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) {
                float4_t a4 = *(const float4_t *)(tile + (((wave * 4 + kq) * 64 + lane) << 2));
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    const int64_t j = j0 + (kq * 4 + e4) * 4 + g4;
                    const float *xr = x_in + j * R + r0 + l16;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[e4], coupling_value(xr[b * 16], discrete),
                                                                      acc[b], 0, 0, 0);
                }
            }
        }
    } else {
        // U tiles per round: all their loads are issued before the first MFMA of the round
        // (the scheduling barrier keeps them there), so the latency of the column-index,
        // tile and x-copy loads is paid once per round.  Slots past t_end reload the last
        // tile with A = 0, which adds exactly zero; the MFMA order is the tile order, as in
        // the persistent kernel.
        for (int t = t_beg; t < t_end; t += U) {
            half8_t a[U][2], bv[U][2][NB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int tt = t + u < t_end ? t + u : t_end - 1;
                const int64_t j0 = (int64_t)t_col[tt] * kTile;
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const int frag = wave * 2 + kb;
                    if constexpr (DT == QH_FP8_ROWSCALE) {
                        const uint8_t *tile = t_val + (int64_t)tt * kTileElems;
                        uint2 c = *(const uint2 *)(tile + ((frag * 64 + lane) << 3));
                        a[u][kb] = e4m3x8_to_f16_scaled(c);
                    } else {
                        const uint16_t *tile = (const uint16_t *)t_val + (int64_t)tt * kTileElems;
                        a[u][kb] = *(const half8_t *)(tile + ((frag * 64 + lane) << 3));
                    }
                    if (t + u >= t_end) a[u][kb] = half8_t{};
                    const int64_t jg = (j0 + kb * 32) / 8 + g4;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        bv[u][kb][b] = *(const half8_t *)(h_in + (jg * R + r0 + b * 16 + l16) * 8);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if constexpr (DT == QH_BF16) {
                            bf16x8_t av, bb;
                            __builtin_memcpy(&av, &a[u][kb], 16);
                            __builtin_memcpy(&bb, &bv[u][kb][b], 16);
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bb, acc[b], 0, 0, 0);
                        } else {
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[u][kb], bv[u][kb][b], acc[b], 0, 0,
                                                                            0);
                        }
                    }
            }
        }
    }
}

// Own state of the lane (rows rowbase..rowbase+3, replicas r0 + 16b + l16).
template <int NB>
__device__ inline void dense_load_state(float (&xo)[NB][4], float (&yo)[NB][4], int64_t rowbase, int64_t n,
                                        const float *x_in, const float *y, int64_t R, int64_t r0, int lane) {
    const int l16 = lane & 15;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = rowbase + q;
            const int64_t idx = i * R + r0 + b * 16 + l16;
            xo[b][q] = i < n ? x_in[idx] : 0.f;
            yo[b][q] = i < n ? y[idx] : 0.f;
        }
}

// Fused update of the lane's rows and the 16-bit copy of the new x.
template <int DT, int NB>
__device__ inline void dense_update(const float4_t (&acc)[NB], const float (&xo)[NB][4], const float (&yo)[NB][4],
                                    int64_t rowbase, int64_t n, int64_t R, int64_t r0, int lane,
                                    const float *__restrict__ row_scale, float *x_out, float *y,
                                    uint16_t *__restrict__ h_out, float coef, const StepArgs &sa) {
    const int l16 = lane & 15;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int64_t r = r0 + b * 16 + l16;
        uint16_t hv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = rowbase + q;
            hv[q] = 0;
            if (i < n) {
                float z = acc[b][q];
                if constexpr (DT == QH_FP8_ROWSCALE) z *= row_scale[i];
                z = with_field(z, i, sa);
                const int64_t idx = i * R + r;
                float xv = xo[b][q], yv = yo[b][q];
                bsb_update(z, xv, yv, coef, sa);
                y[idx] = yv;
                x_out[idx] = xv;
                if constexpr (DT == QH_BF16) hv[q] = f32_to_bf16_rne(coupling_value(xv, sa.discrete));
                else if constexpr (DT != QH_F32) hv[q] = f32_to_f16_rne(coupling_value(xv, sa.discrete));
            }
        }
        if constexpr (DT != QH_F32) {
            // rows rowbase..rowbase+3 share one 8-row group: one 8-byte store
            uint2 pk;
            pk.x = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
            pk.y = (uint32_t)hv[2] | ((uint32_t)hv[3] << 16);
            *(uint2 *)(h_out + ((rowbase >> 3) * R + r) * 8 + (rowbase & 7)) = pk;
        }
    }
}

template <int DT, int NB, int U>
__global__ __launch_bounds__(256) void k_dense_step(
    int64_t n, int R, int64_t n_rt, int64_t G, const int32_t *__restrict__ t_ptr,
    const int32_t *__restrict__ t_col, const uint8_t *__restrict__ t_val, const float *__restrict__ row_scale,
    const float *x_in, float *x_out, float *__restrict__ y,
    const uint16_t *__restrict__ h_in, uint16_t *__restrict__ h_out, StepArgs sa) {
    constexpr int RT = NB * 16;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t logical = xcd_remap(blockIdx.x, G);
    const int64_t rt = logical % n_rt;
    const int64_t r0 = (logical / n_rt) * RT;
    const int64_t rowbase = rt * kTile + wave * 16 + 4 * (lane >> 4);
    float xo[NB][4], yo[NB][4];
    dense_load_state<NB>(xo, yo, rowbase, n, x_in, y, R, r0, lane);   // latency hides under the product
    float4_t acc[NB];
    dense_product<DT, NB, U>(acc, t_ptr[rt], t_ptr[rt + 1], t_col, t_val, x_in, h_in, R, r0, wave, lane, sa.discrete);
    dense_update<DT, NB>(acc, xo, yo, rowbase, n, R, r0, lane, row_scale, x_out, y, h_out,
                         sa.a0 - sa.pump[sa.k], sa);
}

// ---------------------------------------------------------------------------
// skyline band + long-range CSR (SNP graphs)
// ---------------------------------------------------------------------------

template <int DT>
__device__ inline float ld_val(const uint8_t *__restrict__ p, int64_t e) {
    if constexpr (DT == QH_F32) return ((const float *)p)[e];
    else if constexpr (DT == QH_F16) return f16_bits_to_f32(((const uint16_t *)p)[e]);
    else return bf16_bits_to_f32(((const uint16_t *)p)[e]);
}

// Partial sums of the long-range lists, one per chunk of at most kHubChunk entries
// (replica tiles of 16 or 32: several chunks per wave).
template <int DT, int RT, bool H16>
__global__ __launch_bounds__(256) void k_hub_partials(
    int64_t n_chunks, int R, const int64_t *__restrict__ cbeg,
    const int64_t *__restrict__ cend, const int32_t *__restrict__ l_col, const uint8_t *__restrict__ l_val,
    const float *__restrict__ x_in, const uint16_t *__restrict__ h_in, float *__restrict__ part, int discrete) {
    constexpr int RPW = 64 / RT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / RT, rr = lane % RT;
    const int64_t r = (int64_t)blockIdx.y * RT + rr;
    for (int64_t c = (int64_t)blockIdx.x * 4 * RPW + wave * RPW + sub; c < n_chunks;
         c += (int64_t)gridDim.x * 4 * RPW) {
        float z = 0.f;
#pragma unroll 4
        for (int64_t e = cbeg[c]; e < cend[c]; ++e)
            z += ld_val<DT>(l_val, e) * lr_x<H16>(x_in, h_in, (int64_t)l_col[e] * R + r, discrete);
        part[c * R + r] = z;
    }
}

// The same partials for replica tiles of 64, one packet (<= 64 entries, whole chunks) per
// wave: lane j loads entry j's column and value once, then every entry's x row is
// gathered with the column broadcast from its lane, so the gathers of a packet are
// independent of one another and of any further index load.  Each chunk is summed in
// entry order, as in k_hub_partials.
constexpr int kLrInFlight = 32;    // x-row gathers a wave keeps in flight (a packet has at most 64)
template <int DT, bool H16>
__global__ __launch_bounds__(256) void k_lr_packets(
    int64_t n_pk, int R, const int32_t *__restrict__ pk_ptr, const int64_t *__restrict__ cbeg,
    const int64_t *__restrict__ cend, const int32_t *__restrict__ l_col, const uint8_t *__restrict__ l_val,
    const float *__restrict__ x_in, const uint16_t *__restrict__ h_in, float *__restrict__ part, int discrete) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t r = (int64_t)blockIdx.y * 64 + lane;
    for (int64_t p = (int64_t)blockIdx.x * 4 + wave; p < n_pk; p += (int64_t)gridDim.x * 4) {
        const int32_t c0 = pk_ptr[p], c1 = pk_ptr[p + 1];
        const int64_t e0 = cbeg[c0];
        const int32_t cnt = (int32_t)(cend[c1 - 1] - e0);      // <= 64 by construction
        int32_t my_col = 0, my_end = 0;
        float my_val = 0.f;
        if (lane < cnt) {
            my_col = l_col[e0 + lane];
            my_val = ld_val<DT>(l_val, e0 + lane);
        }
        if (lane < c1 - c0) my_end = (int32_t)(cend[c0 + lane] - e0);   // <= 64 chunks per packet
        // kLrInFlight gathers in flight across chunk boundaries; a chunk's sum is flushed when
        // its last entry has been added
        int32_t c = c0, ce = __builtin_amdgcn_readlane(my_end, 0);
        float z = 0.f;
        for (int32_t j = 0; j < cnt; j += kLrInFlight) {
            float xv[kLrInFlight], vv[kLrInFlight];
#pragma unroll
            for (int k = 0; k < kLrInFlight; ++k) {
                const int32_t jj = j + k < 63 ? j + k : 63;      // lanes past cnt hold column 0
                vv[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_val), jj));
                xv[k] = lr_x<H16>(x_in, h_in, (int64_t)__builtin_amdgcn_readlane(my_col, jj) * R + r, discrete);
            }
#pragma unroll
            for (int k = 0; k < kLrInFlight; ++k) {
                if (j + k < cnt) {
                    if (j + k == ce) {
                        part[(int64_t)c * R + r] = z;
                        ++c;
                        ce = __builtin_amdgcn_readlane(my_end, c - c0);
                        z = 0.f;
                    }
                    z += vv[k] * xv[k];
                }
            }
        }
        part[(int64_t)c * R + r] = z;
    }
}

// One wave handles RPW = 64/RT rows x RT replicas; lane = (row slot, replica).
template <int DT, int RT>
__global__ __launch_bounds__(256) void k_sky_step(
    int64_t n, int R, int64_t rows_per_wg, int64_t G, const int64_t *__restrict__ s_off,
    const int32_t *__restrict__ s_lo, const int32_t *__restrict__ s_len, const uint8_t *__restrict__ s_val,
    const int32_t *__restrict__ row_chunk_ptr, const float *__restrict__ hub_part,
    const float *__restrict__ x_in, float *__restrict__ x_out,
    float *__restrict__ y, StepArgs sa) {
    constexpr int RPW = 64 / RT;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane / RT, rr = lane % RT;
    const int64_t blk = xcd_remap(blockIdx.x, G);
    const int64_t row_begin = blk * rows_per_wg;
    const int64_t row_end = row_begin + rows_per_wg < n ? row_begin + rows_per_wg : n;
    const int64_t r = (int64_t)blockIdx.y * RT + rr;
    const float coef = sa.a0 - sa.pump[sa.k];
    for (int64_t ub = row_begin + wave * RPW; ub < row_end; ub += 4 * RPW) {
        const int64_t u = ub + sub;
        if (u >= row_end) continue;
        const int32_t lo = s_lo[u];
        const int32_t len = s_len[u];
        const int64_t off = s_off[u];
        float z = 0.f;
        const float *xc = x_in + (int64_t)lo * R + r;
#pragma unroll 8
        for (int e = 0; e < len; ++e) z += ld_val<DT>(s_val, off + e) * coupling_value(xc[(int64_t)e * R], sa.discrete);
        if (row_chunk_ptr)
            for (int c = row_chunk_ptr[u]; c < row_chunk_ptr[u + 1]; ++c) z += hub_part[(int64_t)c * R + r];
        z = with_field(z, u, sa);
        const int64_t idx = u * R + r;
        float xv = x_in[idx], yv = y[idx];
        bsb_update(z, xv, yv, coef, sa);
        y[idx] = yv;
        x_out[idx] = xv;
        store_lr_copy(sa, idx, xv);
    }
}

// One column of a band block (kBandRows values) through the scalar cache: the address is
// wave-uniform, so the values arrive in SGPRs and feed the FMAs directly.
template <int DT>
__device__ inline void band_column(const uint8_t *bb_val, int64_t e0, float (&v)[kBandRows]) {
    typedef const __attribute__((address_space(4))) uint32_t cu32;
    if constexpr (DT == QH_F32) {
        cu32 *q = (cu32 *)(bb_val + e0 * 4);
#pragma unroll
        for (int i = 0; i < kBandRows; ++i) v[i] = __uint_as_float(q[i]);
    } else {
        cu32 *q = (cu32 *)(bb_val + e0 * 2);
#pragma unroll
        for (int i = 0; i < kBandRows / 2; ++i) {
            const uint32_t w = q[i];
            if constexpr (DT == QH_F16) {
                v[2 * i] = f16_bits_to_f32((uint16_t)w);
                v[2 * i + 1] = f16_bits_to_f32((uint16_t)(w >> 16));
            } else {
                v[2 * i] = __uint_as_float(w << 16);
                v[2 * i + 1] = __uint_as_float(w & 0xffff0000u);
            }
        }
    }
}

// Rows of band block blk for replica r after the band columns: the long-range chunk
// partials of each row (in chunk order) join the band sum z, then the fused update.
// my_cp: lanes 0..kBandRows hold row_chunk_ptr of rows blk*kBandRows + lane.
// NT: the state goes out with non-temporal stores (graphs with long-range rows, where it
// leaves the L2 to the long-range gathers; measured on the Pore-C workload).
// FLD = false compiles the deformation field out (launches without one).
template <bool NT, bool FLD = true>
__device__ inline void band_block_finish(int64_t blk, int64_t n, int64_t R, int64_t r, const float (&z)[kBandRows],
                                         const float (&xo)[kBandRows], const float (&yo)[kBandRows], int32_t my_cp,
                                         const int32_t *__restrict__ row_chunk_ptr,
                                         const float *__restrict__ hub_part, float *x_out, float *y, float coef,
                                         const StepArgs &sa) {
    constexpr int RB = kBandRows;
    // the first chunk partial of every long-range row, all sixteen loads in flight together
    float p0[RB];
    if (row_chunk_ptr) {
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int32_t cb = __builtin_amdgcn_readlane(my_cp, i), ce = __builtin_amdgcn_readlane(my_cp, i + 1);
            p0[i] = (blk * RB + i < n && cb < ce) ? hub_part[(int64_t)cb * R + r] : 0.f;
        }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int64_t u = blk * RB + i;
        if (u >= n) break;
        float zi = z[i];
        if (row_chunk_ptr) {                   // long-range rows: chunk partials, in order
            const int32_t cb = __builtin_amdgcn_readlane(my_cp, i), ce = __builtin_amdgcn_readlane(my_cp, i + 1);
            if (cb < ce) {
                zi += p0[i];
                // hub rows have many chunks: eight loads in flight at a time, added in order
                int c = cb + 1;
                for (; c + 8 <= ce; c += 8) {
                    float v[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = hub_part[(int64_t)(c + k) * R + r];
#pragma unroll
                    for (int k = 0; k < 8; ++k) zi += v[k];
                }
                for (; c < ce; ++c) zi += hub_part[(int64_t)c * R + r];
            }
        }
        if constexpr (FLD) zi = with_field(zi, u, sa);
        const int64_t idx = u * R + r;
        float xv = xo[i], yv = yo[i];
        bsb_update(zi, xv, yv, coef, sa);
        if constexpr (NT) {
            __builtin_nontemporal_store(yv, &y[idx]);
            __builtin_nontemporal_store(xv, &x_out[idx]);
        } else {
            y[idx] = yv;
            x_out[idx] = xv;
        }
        store_lr_copy(sa, idx, xv);
    }
}

// Register-tiled band step (R a multiple of 64; lane = replica).  Wave = one band block
// of kBandRows consecutive rows: it walks the block's union column range once, loads
// each x row once and applies it to all kBandRows accumulators with one column of the
// block (kBandRows values, wave-uniform, so they arrive through scalar loads).  The
// long-range lists of the block's rows follow, then the fused update.
// One band block of rows [blk*16, blk*16 + 16) for the lane's replica r (inactive lanes
// skip every memory access).  Shared by the per-step and batched kernels.
template <int DT, bool NT = false, bool FLD = true>
__device__ inline void band_block_step(int64_t blk, int64_t n, int64_t R, int64_t r, bool active,
                                       const int64_t *__restrict__ bb_off, const int32_t *__restrict__ bb_lo,
                                       const int32_t *__restrict__ bb_w, const uint8_t *__restrict__ bb_val,
                                       const int32_t *__restrict__ row_chunk_ptr, const float *__restrict__ hub_part,
                                       const float *x_in, float *x_out, float *y, float coef, const StepArgs &sa) {
    constexpr int RB = kBandRows;
    // blk is wave-uniform, so are the block's extents: keep them (and the band loop) scalar
    const int32_t L = __builtin_amdgcn_readfirstlane(bb_lo[blk]), W = __builtin_amdgcn_readfirstlane(bb_w[blk]);
    const int64_t off = (int64_t)__builtin_amdgcn_readfirstlane((int32_t)bb_off[blk]) |
                        ((int64_t)__builtin_amdgcn_readfirstlane((int32_t)(bb_off[blk] >> 32)) << 32);
    float z[RB], xo[RB], yo[RB];
    // long-range rows: the chunk range of every row (lanes 0..RB load row_chunk_ptr once),
    // issued first so that the band loop never waits on it
    int32_t my_cp = 0;
    if (row_chunk_ptr) {
        const int lane = threadIdx.x & 63;
        if (lane <= RB && blk * RB + lane <= n) my_cp = row_chunk_ptr[blk * RB + lane];
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        z[i] = 0.f;
        const int64_t u = blk * RB + i;       // own state first: its latency hides under the band loop
        xo[i] = (active && u < n) ? x_in[u * R + r] : 0.f;
        // y is read once per step: a non-temporal load keeps it from displacing x rows that
        // neighbouring blocks still read (measured 0.7 % faster on the chromosome graph)
        yo[i] = (active && u < n) ? __builtin_nontemporal_load(&y[u * R + r]) : 0.f;
    }
    // inactive lanes read replica 0 of the same rows (always in bounds) and weigh it by 0:
    // no divergent branch around the loads (|x| <= 1, so the product is an exact 0)
    // (x is device memory: global loads, so that the wait for the scalar band values does
    // not also wait for them, as it would for flat loads)
    typedef const __attribute__((address_space(1))) float gfloat;
    gfloat *xc = (gfloat *)(x_in + (int64_t)L * R + (active ? r : 0));
    const float live = active ? 1.f : 0.f;
    // eight columns per round keep eight x-row loads (and their scalar band values) in flight
    // per wave (four: 3-4 % slower on the chromosome graph and the batched SNP blocks)
#pragma unroll 8
    for (int32_t j = 0; j < W; ++j) {
        const float xj = coupling_value(xc[(int64_t)j * R], sa.discrete) * live;
        const int64_t e0 = off + (int64_t)j * RB;
        float val[RB];
        band_column<DT>(bb_val, e0, val);
#pragma unroll
        for (int i = 0; i < RB; ++i) z[i] += val[i] * xj;
    }
    if (!active) return;
#pragma unroll
    for (int i = 0; i < RB; ++i) z[i] *= sa.bscale;   // exact: a power of two
    band_block_finish<NT, FLD>(blk, n, R, r, z, xo, yo, my_cp, row_chunk_ptr, hub_part, x_out, y, coef, sa);
}

// The same band block on the matrix cores: a band block is a dense 16 x W matrix stored
// column-major, which is exactly the A-operand order of v_mfma_f32_16x16x4f32 (lane l
// holds row l % 16 of column l / 16), so four columns arrive with one 64-lane load; x rows
// L + j .. L + j + 3 of 16 replicas are the B operand.  NB = 16-replica blocks per wave
// (all 64 lanes busy for any replica count).  Values enter in FP32 (16-bit codes widened
// exactly); the MFMA sums each group of four columns before adding it, so results match
// the FMA kernels to FP32 rounding, not bit for bit.  Output: lane l owns rows
// 4 (l / 16) .. + 3 of the block and replica r0 + 16 b + l % 16.
template <int DT, int NB>
__device__ inline void band_block_step_mfma(int64_t blk, int64_t n, int64_t R, int64_t r0,
                                            const int64_t *__restrict__ bb_off, const int32_t *__restrict__ bb_lo,
                                            const int32_t *__restrict__ bb_w, const uint8_t *__restrict__ bb_val,
                                            const int32_t *__restrict__ row_chunk_ptr,
                                            const float *__restrict__ hub_part, const float *x_in, float *x_out,
                                            float *y, float coef, const StepArgs &sa) {
    constexpr int RB = kBandRows;
    const int lane = threadIdx.x & 63, l16 = lane & 15, g4 = lane >> 4;
    const int32_t L = bb_lo[blk], W = bb_w[blk];
    const int64_t off = bb_off[blk];
    const int64_t rowbase = blk * RB + 4 * g4;
    int32_t my_cp = 0;
    if (row_chunk_ptr && lane <= RB && blk * RB + lane <= n) my_cp = row_chunk_ptr[blk * RB + lane];
    float xo[NB][4], yo[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t u = rowbase + q;
            xo[b][q] = u < n ? x_in[u * R + r0 + b * 16 + l16] : 0.f;
            yo[b][q] = u < n ? y[u * R + r0 + b * 16 + l16] : 0.f;
        }
    float4_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = float4_t{0.f, 0.f, 0.f, 0.f};
    // columns j .. j + 15 per round: four MFMA K-steps with their loads in flight together
    for (int32_t j = 0; j < W; j += 16) {
        float av[4], bv[4][NB];
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
            const int32_t col = j + kq * 4 + g4;
            const bool in = col < W;
            av[kq] = in ? ld_val<DT>(bb_val, off + (int64_t)col * RB + l16) : 0.f;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                bv[kq][b] = in ? coupling_value(x_in[(int64_t)(L + col) * R + r0 + b * 16 + l16], sa.discrete) : 0.f;
        }
#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kq], bv[kq][b], acc[b], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t u = rowbase + q;
        // chunk range of row u (row 4 g4 + q of the block): from lanes 4 g4 + q and + 1
        const int32_t cb = __shfl(my_cp, 4 * g4 + q), ce = __shfl(my_cp, 4 * g4 + q + 1);
        if (u >= n) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t r = r0 + b * 16 + l16;
            float zi = acc[b][q] * sa.bscale;
            if (row_chunk_ptr)
                for (int c = cb; c < ce; ++c) zi += hub_part[(int64_t)c * R + r];
            zi = with_field(zi, u, sa);
            const int64_t idx = u * R + r;
            float xv = xo[b][q], yv = yo[b][q];
            bsb_update(zi, xv, yv, coef, sa);
            y[idx] = yv;
            x_out[idx] = xv;
            store_lr_copy(sa, idx, xv);
        }
    }
}

template <int DT, int NB>
__global__ __launch_bounds__(256) void k_band_step_mfma(
    int64_t n, int R, int64_t n_bblk, int64_t G, const int64_t *__restrict__ bb_off,
    const int32_t *__restrict__ bb_lo, const int32_t *__restrict__ bb_w, const uint8_t *__restrict__ bb_val,
    const int32_t *__restrict__ row_chunk_ptr, const float *__restrict__ hub_part,
    const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ y, StepArgs sa) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t blk = xcd_remap(blockIdx.x, G) * 4 + wave;
    if (blk >= n_bblk) return;
    band_block_step_mfma<DT, NB>(blk, n, R, (int64_t)blockIdx.y * NB * 16, bb_off, bb_lo, bb_w, bb_val,
                                 row_chunk_ptr, hub_part, x_in, x_out, y, sa.a0 - sa.pump[sa.k], sa);
}

template <int DT, bool NT, bool FLD>
__global__ __launch_bounds__(64) void k_band_step(
    int64_t n, int R, int64_t n_bblk, int64_t G, const int64_t *__restrict__ bb_off,
    const int32_t *__restrict__ bb_lo, const int32_t *__restrict__ bb_w, const uint8_t *__restrict__ bb_val,
    const int32_t *__restrict__ row_chunk_ptr, const float *__restrict__ hub_part,
    const float *__restrict__ x_in, float *__restrict__ x_out,
    float *__restrict__ y, StepArgs sa) {
    const int lane = threadIdx.x;
    const int64_t blk = xcd_remap(blockIdx.x, G);
    if (blk >= n_bblk) return;
    const int64_t r = (int64_t)blockIdx.y * 64 + lane;
    band_block_step<DT, NT, FLD>(blk, n, R, r, true, bb_off, bb_lo, bb_w, bb_val, row_chunk_ptr, hub_part, x_in,
                                 x_out, y, sa.a0 - sa.pump[sa.k], sa);
}

// ---------------------------------------------------------------------------
// batched blocks: one persistent launch, whole blocks per workgroup
// ---------------------------------------------------------------------------

// Initial state of one block by one workgroup: the single-graph counter layout with the
// block's n, and the 16-bit product copy for dense 16/8-bit blocks.
template <int64_t R>
__device__ inline void block_init(const BlockDesc &B, uint64_t seed, int tid) {
    const int64_t n = B.n;
    for (int64_t t = tid; t < n * R; t += 256) {
        const int64_t i = t / R, r = t - i * R;
        const uint64_t c = 2ull * ((uint64_t)r * (uint64_t)n + (uint64_t)i);
        const float xv = (float)(0.2 * ((double)(sm64_draw(seed, c) >> 11) * 0x1.0p-53) - 0.1);
        B.x[t] = xv;
        B.y[t] = (float)(0.2 * ((double)(sm64_draw(seed, c + 1) >> 11) * 0x1.0p-53) - 0.1);
        if (B.kind == 0 && B.dtype != QH_F32) {
            const float cv = coupling_value(xv, B.discrete);
            B.h0[((i >> 3) * R + r) * 8 + (i & 7)] = B.dtype == QH_BF16 ? f32_to_bf16_rne(cv) : f32_to_f16_rne(cv);
        }
    }
    __syncthreads();
}

// Each workgroup runs its scheduled blocks one after another; a block's steps are
// separated by workgroup barriers only, because no other workgroup touches its state.
// Dense blocks use the tile product of the per-step kernel (wave w: rows 16w.. of every
// row tile), SNP blocks the band step; arithmetic and order match the single-graph
// kernels, so a block's result equals its single-graph solve bit for bit.
template <int NB>
__global__ __launch_bounds__(256) void k_batched(const BlockDesc *__restrict__ blocks,
                                                 const int32_t *__restrict__ sched_ptr,
                                                 const int32_t *__restrict__ sched, int steps, float dt, float a0,
                                                 const float *__restrict__ pump, uint64_t seed) {
    constexpr int64_t R = NB * 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int k = sched_ptr[blockIdx.x]; k < sched_ptr[blockIdx.x + 1]; ++k) {
        const BlockDesc B = blocks[sched[k]];
        const int64_t n = B.n;
        float *xb = B.x, *yb = B.y;
        block_init<R>(B, seed, tid);
        const bool dense16 = B.kind == 0 && B.dtype != QH_F32;
        StepArgs sa{B.c0, dt, a0, pump, 0, B.discrete, B.bscale, B.field};
        float *cur = xb, *oth = B.xs;
        for (int s = 0; s < steps; ++s) {
            sa.k = s;
            const float coef = a0 - pump[s];
            if (B.kind == 0) {
                const uint16_t *hin = (s & 1) ? B.h1 : B.h0;
                uint16_t *hout = (s & 1) ? B.h0 : B.h1;
                float *xin = dense16 ? xb : cur, *xout = dense16 ? xb : oth;
                for (int64_t rt = 0; rt < B.n_rt; ++rt) {
                    const int64_t rowbase = rt * kTile + wave * 16 + 4 * (lane >> 4);
                    float xo[NB][4], yo[NB][4];
                    float4_t acc[NB];
                    dense_load_state<NB>(xo, yo, rowbase, n, xin, yb, R, 0, lane);
#define QH_BD(DTV)                                                                                              \
    dense_product<DTV, NB>(acc, B.t_ptr[rt], B.t_ptr[rt + 1], B.t_col, B.t_val, xin, hin, R, 0, wave, lane,   \
                           sa.discrete);                                                                     \
    dense_update<DTV, NB>(acc, xo, yo, rowbase, n, R, 0, lane, B.row_scale, xout, yb, hout, coef, sa)
                    switch (B.dtype) {
                        case QH_F32: QH_BD(QH_F32); break;
                        case QH_F16: QH_BD(QH_F16); break;
                        case QH_BF16: QH_BD(QH_BF16); break;
                        default: QH_BD(QH_FP8_ROWSCALE); break;
                    }
#undef QH_BD
                }
            } else {
                const bool active = lane < R;
                for (int64_t bb = wave; bb < B.n_bblk; bb += 4) {
#define QH_BB(DTV)                                                                                          \
    band_block_step<DTV>(bb, n, R, lane, active, B.bb_off, B.bb_lo, B.bb_w, B.bb_val, nullptr, nullptr,   \
                         cur, oth, yb, coef, sa)
                    switch (B.dtype) {
                        case QH_F32: QH_BB(QH_F32); break;
                        case QH_F16: QH_BB(QH_F16); break;
                        default: QH_BB(QH_BF16); break;
                    }
#undef QH_BB
                }
            }
            __syncthreads();
            if (!dense16) { float *t = cur; cur = oth; oth = t; }
        }
        // the ping-pong paths may end in the scratch half
        if (!dense16 && cur != xb)
            for (int64_t t = tid; t < n * R; t += 256) xb[t] = cur[t];
        __syncthreads();
    }
}

// One step of every block of one class (storage kind x dtype) in one launch.  Work item
// = one row tile of a dense block (the k_dense_step workgroup) or four band blocks of an
// SNP block (one per wave, lanes r < R active); items of one block are adjacent, and the
// XCD remap keeps them on one XCD.  Ping-pong halves follow the single-graph solve (step k
// reads half k & 1).  One instantiation per class keeps each one's register budget (and
// occupancy) that of its own path.
template <int KIND, int DT, int NB>
__global__ __launch_bounds__(256) void k_batched_step(const BlockDesc *__restrict__ blocks,
                                                      const int2 *__restrict__ items, XcdSplit xs, int k,
                                                      float dt, float a0, const float *__restrict__ pump) {
    constexpr int64_t R = NB * 16;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int64_t item = xs.off[xcd] + blockIdx.x / kXcds;
    if (item >= xs.off[xcd + 1]) return;
    const int2 I = items[item];
    const BlockDesc &B = blocks[I.x];
    const StepArgs sa{B.c0, dt, a0, pump, k, B.discrete, B.bscale, B.field};
    const float coef = a0 - pump[k];
    const int cur = k & 1;
    const int64_t n = B.n;
    if constexpr (KIND == 0) {
        constexpr bool d16 = DT != QH_F32;
        const uint16_t *hin = cur ? B.h1 : B.h0;
        uint16_t *hout = cur ? B.h0 : B.h1;
        float *xin = d16 ? B.x : (cur ? B.xs : B.x);
        float *xout = d16 ? B.x : (cur ? B.x : B.xs);
        const int64_t rt = I.y;
        const int64_t rowbase = rt * kTile + wave * 16 + 4 * (lane >> 4);
        float xo[NB][4], yo[NB][4];
        float4_t acc[NB];
        dense_load_state<NB>(xo, yo, rowbase, n, xin, B.y, R, 0, lane);
        dense_product<DT, NB>(acc, B.t_ptr[rt], B.t_ptr[rt + 1], B.t_col, B.t_val, xin, hin, R, 0, wave, lane,
                              sa.discrete);
        dense_update<DT, NB>(acc, xo, yo, rowbase, n, R, 0, lane, B.row_scale, xout, B.y, hout, coef, sa);
    } else {
        const int64_t bb = (int64_t)I.y * 4 + wave;
        if (bb >= B.n_bblk) return;
        const float *xin = cur ? B.xs : B.x;
        float *xout = cur ? B.x : B.xs;
        band_block_step<DT>(bb, n, R, lane, lane < R, B.bb_off, B.bb_lo, B.bb_w, B.bb_val, nullptr, nullptr, xin,
                            xout, B.y, coef, sa);
    }
}

// Product of S 16-row strips (s0 .. s0 + S - 1) of one 64-row tile by one wave: the strips
// share the B fragments (the 16-bit copy of x), which the wave loads once per stored tile
// instead of once per strip.  Strip s's MFMAs run in dense_product's order (tile, column
// half, replica block), and a slot past t_end adds an exact zero there (an accumulator that
// starts at +0 never becomes -0), so each strip's sum equals the four-wave product's bit for
// bit whatever U and S are.  The tiles are read once per step: non-temporal loads keep them
// from displacing the x copies other row tiles still read (1.7 % faster on the batch).
// Measured on the 3,000-block batch at R = 32 (dense FP8 class per step): U = 2, S = 4
// 1,059 us; U = 4 1,066 us; S = 2 (two waves per row tile, B loaded twice) 1,229 us.
template <int DT, int NB, int U, int S>
__device__ inline void dense_product_rowtile(float4_t (&acc)[S][NB], int t_beg, int t_end, int s0,
                                             const int32_t *__restrict__ t_col, const uint8_t *__restrict__ t_val,
                                             const uint16_t *__restrict__ h_in, int64_t R, int lane) {
    static_assert(DT != QH_F32, "the whole-tile product takes 16/8-bit tiles");
    const int l16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int s4 = 0; s4 < S; ++s4)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[s4][b] = float4_t{0.f, 0.f, 0.f, 0.f};
    using RawA = typename std::conditional<DT == QH_FP8_ROWSCALE, uint2, half8_t>::type;
    for (int t = t_beg; t < t_end; t += U) {
        RawA a[U][2 * S];
        half8_t bv[U][2][NB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int tt = t + u < t_end ? t + u : t_end - 1;
            const int64_t j0 = (int64_t)t_col[tt] * kTile;
#pragma unroll
            for (int f = 0; f < 2 * S; ++f) {
                const int fr = 2 * s0 + f;
                if constexpr (DT == QH_FP8_ROWSCALE) {
                    typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
                    const u32x2_t *pa = (const u32x2_t *)(t_val + (int64_t)tt * kTileElems + ((fr * 64 + lane) << 3));
                    const u32x2_t v = __builtin_nontemporal_load(pa);
                    a[u][f] = make_uint2(v.x, v.y);
                } else {
                    const half8_t *pa =
                        (const half8_t *)((const uint16_t *)t_val + (int64_t)tt * kTileElems + ((fr * 64 + lane) << 3));
                    a[u][f] = __builtin_nontemporal_load(pa);
                }
            }
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const int64_t jg = (j0 + kb * 32) / 8 + g4;
#pragma unroll
                for (int b = 0; b < NB; ++b) bv[u][kb][b] = *(const half8_t *)(h_in + (jg * R + b * 16 + l16) * 8);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (t + u >= t_end) break;        // wave-uniform: past the row tile's last stored tile
#pragma unroll
            for (int s4 = 0; s4 < S; ++s4)
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    half8_t av;
                    if constexpr (DT == QH_FP8_ROWSCALE) av = e4m3x8_to_f16_scaled(a[u][s4 * 2 + kb]);
                    else av = a[u][s4 * 2 + kb];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if constexpr (DT == QH_BF16) {
                            bf16x8_t aw, bw;
                            __builtin_memcpy(&aw, &av, 16);
                            __builtin_memcpy(&bw, &bv[u][kb][b], 16);
                            acc[s4][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bw, acc[s4][b], 0, 0, 0);
                        } else {
                            acc[s4][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv[u][kb][b], acc[s4][b], 0, 0, 0);
                        }
                    }
                }
        }
    }
}

// One step of the dense 16/8-bit blocks of one class: work item = (block, row tile), one wave
// each, four per workgroup, taken from the list of the XCD that runs the workgroup (adjacent
// items of a block share its x columns in the CU's cache and the XCD's L2).  The same
// arithmetic as k_batched_step's dense path.
template <int DT, int NB>
__global__ __launch_bounds__(256) void k_batched_rowtile(const BlockDesc *__restrict__ blocks,
                                                         const int2 *__restrict__ items, XcdSplit xs, int k,
                                                         float dt, float a0, const float *__restrict__ pump) {
    constexpr int S = 4;   // strips per wave: the whole row tile
    constexpr int64_t R = NB * 16;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int64_t item = xs.off[xcd] + (int64_t)(blockIdx.x / kXcds) * 4 + wave;
    if (item >= xs.off[xcd + 1]) return;
    const int s0 = 0;
    const int2 I = items[item];
    const BlockDesc &B = blocks[I.x];
    const StepArgs sa{B.c0, dt, a0, pump, k, B.discrete, B.bscale, B.field};
    const float coef = a0 - pump[k];
    const int cur = k & 1;
    const uint16_t *hin = cur ? B.h1 : B.h0;
    uint16_t *hout = cur ? B.h0 : B.h1;
    const int64_t rt = I.y;
    float4_t acc[S][NB];
    dense_product_rowtile<DT, NB, 2, S>(acc, B.t_ptr[rt], B.t_ptr[rt + 1], s0, B.t_col, B.t_val, hin, R, lane);
#pragma unroll
    for (int s4 = 0; s4 < S; ++s4) {
        const int64_t rowbase = rt * kTile + (s0 + s4) * 16 + 4 * (lane >> 4);
        float xo[NB][4], yo[NB][4];
        dense_load_state<NB>(xo, yo, rowbase, B.n, B.x, B.y, R, 0, lane);
        dense_update<DT, NB>(acc[s4], xo, yo, rowbase, B.n, R, 0, lane, B.row_scale, B.x, B.y, hout, coef, sa);
    }
}

template <int NB>
__global__ __launch_bounds__(256) void k_batched_init(const BlockDesc *__restrict__ blocks, uint64_t seed) {
    block_init<NB * 16>(blocks[blockIdx.x], seed, threadIdx.x);
}

// classes: 0-3 dense F32/F16/BF16/FP8, 4-6 band F32/F16/BF16 (kBatchClasses in total)
// Workgroups of one class's launch: kXcds times the longest XCD list (in workgroups of
// `per` items), so that workgroup q * kXcds + x serves XCD x's q-th group.
static unsigned xcd_grid(const XcdSplit &xs, int per) {
    int64_t m = 0;
    for (int x = 0; x < kXcds; ++x) m = std::max(m, ceil_div(xs.off[x + 1] - xs.off[x], per));
    return (unsigned)(m * kXcds);
}

template <int NB>
static void launch_class(int cls, hipStream_t st, const BlockDesc *blocks, const int2 *items, const XcdSplit &xs,
                         int k, float dt, float a0, const float *pump) {
#define QH_CLS(KD, DTV)                                                                                  \
    hipLaunchKernelGGL((k_batched_step<KD, DTV, NB>), dim3(xcd_grid(xs, 1)), dim3(256), 0, st, blocks, items, xs, \
                       k, dt, a0, pump)
#define QH_RT(DTV)                                                                                           \
    hipLaunchKernelGGL((k_batched_rowtile<DTV, NB>), dim3(xcd_grid(xs, 4)), dim3(256), 0, st, blocks, items, xs, \
                       k, dt, a0, pump)
    switch (cls) {
        case 0: QH_CLS(0, QH_F32); break;
        case 1: QH_RT(QH_F16); break;
        case 2: QH_RT(QH_BF16); break;
        case 3: QH_RT(QH_FP8_ROWSCALE); break;
        case 4: QH_CLS(1, QH_F32); break;
        case 5: QH_CLS(1, QH_F16); break;
        default: QH_CLS(1, QH_BF16); break;
    }
#undef QH_RT
#undef QH_CLS
}

// Side stream of a device for the SNP band classes of a batched solve (default priority,
// non-blocking), with the two events that fork it from and join it to the caller's stream;
// one set per device, created once and kept for the life of the process (a captured graph
// may refer to them until it is instantiated).
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
static SideStream &side_stream(int dev) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static SideStream sides[kMaxDevices];
    if (dev < 0 || dev >= kMaxDevices) fail(QH_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(mu);
    SideStream &s = sides[dev];
    if (!s.stream) {
        QH_HIP(hipEventCreateWithFlags(&s.fork, hipEventDisableTiming));
        QH_HIP(hipEventCreateWithFlags(&s.join, hipEventDisableTiming));
        QH_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
    }
    return s;
}

// The dense classes (bound by HBM bandwidth) and the band classes (bound by load latency)
// touch disjoint blocks, so their step chains run concurrently: the band classes go to a
// side stream forked from `st` after the initial state and joined back before return (a
// capture of `st` records the same fork and join as two parallel chains).  Each block's
// launches stay in step order on its own stream, so the results do not depend on it.
void launch_batched_steps(int R, int nb, const BlockDesc *blocks, const int2 *items, const int64_t *class_ptr,
                          const XcdSplit *splits, int steps, float dt, float a0, const float *pump, uint64_t seed,
                          hipStream_t st) {
    bool dense = false, band = false;
    for (int c = 0; c < kBatchClasses; ++c)
        if (class_ptr[c + 1] > class_ptr[c]) (c < 4 ? dense : band) = true;
    const bool fork = dense && band && steps > 0;
    hipStream_t sb = st;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    if (fork) {
        int dev = 0;
        QH_HIP(hipGetDevice(&dev));
        SideStream &side = side_stream(dev);
        sb = side.stream;
        ev_fork = side.fork;
        ev_join = side.join;
    }
    {
#define QH_BSTEPS(NBV)                                                                                    \
    do {                                                                                                  \
        hipLaunchKernelGGL(k_batched_init<NBV>, dim3(nb), dim3(256), 0, st, blocks, seed);               \
        QH_CHECK_LAUNCH();                                                                                \
        if (fork) {                                                                                       \
            QH_HIP(hipEventRecord(ev_fork, st));                                                          \
            QH_HIP(hipStreamWaitEvent(sb, ev_fork, 0));                                                   \
        }                                                                                                 \
        for (int k = 0; k < steps; ++k)                                                                  \
            for (int c = 0; c < kBatchClasses; ++c)                                                      \
                if (class_ptr[c + 1] > class_ptr[c])                                                     \
                    launch_class<NBV>(c, c < 4 ? st : sb, blocks, items + class_ptr[c], splits[c], k, dt, a0, \
                                      pump);                                                             \
        if (fork) {                                                                                       \
            QH_HIP(hipEventRecord(ev_join, sb));                                                          \
            QH_HIP(hipStreamWaitEvent(st, ev_join, 0));                                                   \
        }                                                                                                 \
    } while (0)
        switch (R) {
            case 16: QH_BSTEPS(1); break;
            case 32: QH_BSTEPS(2); break;
            case 64: QH_BSTEPS(4); break;
            default: fail(QH_EUNSUPPORTED, "batched solves take 16, 32 or 64 replicas");
        }
#undef QH_BSTEPS
        QH_CHECK_LAUNCH();
    }
}

void launch_batched(int R, int workers, const BlockDesc *blocks, const int32_t *sched_ptr, const int32_t *sched,
                    int steps, float dt, float a0, const float *pump, uint64_t seed, hipStream_t st) {
#define QH_BATCH(NBV)                                                                                          \
    hipLaunchKernelGGL(k_batched<NBV>, dim3(workers), dim3(256), 0, st, blocks, sched_ptr, sched, steps, dt, a0, \
                       pump, seed)
    switch (R) {
        case 16: QH_BATCH(1); break;
        case 32: QH_BATCH(2); break;
        case 64: QH_BATCH(4); break;
        default: fail(QH_EUNSUPPORTED, "batched solves take 16, 32 or 64 replicas");
    }
#undef QH_BATCH
    QH_CHECK_LAUNCH();
}

int batched_workers_per_cu(int R) {
    int occ = 0;
    hipError_t e = hipSuccess;
    switch (R) {
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batched<1>, 256, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batched<2>, 256, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batched<4>, 256, 0); break;
    }
    if (e != hipSuccess) { (void)hipGetLastError(); occ = 1; }
    return std::max(occ, 1);
}

__global__ void k_copy_state_in(int64_t n, int R, const float *__restrict__ src, float *__restrict__ dst) {
    int64_t total = n * R;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

static int grid_for(int64_t n, int block = 256, int64_t cap = 65536) {
    int64_t g = ceil_div(n, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}


// 16-bit SNP graphs with long-range rows gather x from a binary16 copy (F32 graphs from x)
static bool lr_copy(const qh_graph *g) {
    return g->storage == QH_STORE_SKYLINE && g->l_nnz > 0 && g->dtype != QH_F32;
}

// Clearing of new plans' state buffers: one memset each, or, between begin_plan_zeroing
// and end_plan_zeroing on this thread (the batched solve creating thousands of plans), one
// kernel over the collected list.
static thread_local std::vector<std::pair<void *, size_t>> *t_plan_zero = nullptr;

template <class T>
static void plan_zero(DevBuf<T> &b, hipStream_t st) {
    if (t_plan_zero) t_plan_zero->push_back({(void *)b.p, b.bytes()});
    else b.zero(st);
}

// one workgroup per buffer; the allocator's blocks are 256-byte aligned and the buffers
// hold 2- or 4-byte elements
__global__ void k_zero_buffers(const uint64_t *__restrict__ ptr, const uint64_t *__restrict__ bytes) {
    uint8_t *p = (uint8_t *)ptr[blockIdx.x];
    const uint64_t nb = bytes[blockIdx.x];
    const uint64_t n16 = nb / 16;
    for (uint64_t i = threadIdx.x; i < n16; i += blockDim.x) ((uint4 *)p)[i] = make_uint4(0, 0, 0, 0);
    for (uint64_t i = n16 * 16 + threadIdx.x; i < nb; i += blockDim.x) p[i] = 0;
}

void begin_plan_zeroing(std::vector<std::pair<void *, size_t>> &list) { t_plan_zero = &list; }

void end_plan_zeroing(std::vector<std::pair<void *, size_t>> &list, DevBuf<uint64_t> &table, hipStream_t st) {
    t_plan_zero = nullptr;
    const size_t m = list.size();
    if (!m) return;
    if (m > 0x7fffffffu) fail(QH_EUNSUPPORTED, "too many buffers to clear");
    std::vector<uint64_t> h(2 * m);
    for (size_t i = 0; i < m; ++i) {
        h[i] = (uint64_t)(uintptr_t)list[i].first;
        h[m + i] = (uint64_t)list[i].second;
    }
    table.alloc(2 * m);
    table.upload(h.data(), 2 * m, st);
    hipLaunchKernelGGL(k_zero_buffers, dim3((unsigned)m), dim3(256), 0, st, table.p, table.p + m);
    QH_CHECK_LAUNCH();
    QH_HIP(hipStreamSynchronize(st));   // the host table goes out of scope
}

SolvePlan &solve_plan(const qh_graph *gc, int R, hipStream_t st) {
    qh_graph *g = const_cast<qh_graph *>(gc);
    auto it = g->plans.find(R);
    if (it != g->plans.end()) return *it->second;
    std::unique_ptr<SolvePlan> p(new SolvePlan());
    p->R = R;
    p->n_pad = ceil_div(std::max<int64_t>(g->n, 1), kTile) * kTile;
    size_t st_elems = (size_t)p->n_pad * R;
    p->xa.alloc(st_elems);
    plan_zero(p->xa, st);
    p->y.alloc(st_elems);
    plan_zero(p->y, st);
    bool dense16 = g->storage == QH_STORE_DENSE && g->dtype != QH_F32;
    if (!dense16) {
        p->xb.alloc(st_elems);
        plan_zero(p->xb, st);
        if (lr_copy(g)) {
            p->la.alloc(st_elems);
            plan_zero(p->la, st);
            p->lb.alloc(st_elems);
            plan_zero(p->lb, st);
        }
    } else {
        p->ha.alloc(st_elems);
        plan_zero(p->ha, st);
        p->hb.alloc(st_elems);
        plan_zero(p->hb, st);
    }
    alloc_readout_scratch(*p, g->n, g->n_comp, g->n_chunks, R);
    if (g->n_hub_chunks) p->hub_part.alloc((size_t)g->n_hub_chunks * R);
    SolvePlan &ref = *p;
    g->plans[R] = std::move(p);
    return ref;
}

// Launch one step k of the schedule.  `cur` selects the ping-pong half holding x (or h).
static void launch_step(const qh_graph *g, SolvePlan &p, const StepArgs &sa, int cur, hipStream_t st) {
    const int R = p.R;
    const int64_t n = g->n;
    if (g->storage == QH_STORE_DENSE) {
        const int RT = R >= 64 ? p.run_rt : R;
        const int64_t G = g->n_rt * (R / RT);
        if (G == 0) return;
        float *xin = cur ? p.xb.p : p.xa.p;
        float *xout = cur ? p.xa.p : p.xb.p;
        const uint16_t *hin = cur ? p.hb.p : p.ha.p;
        uint16_t *hout = cur ? p.ha.p : p.hb.p;
#define QH_DENSE(DTV, NBV, UV)                                                                              \
    hipLaunchKernelGGL((k_dense_step<DTV, NBV, UV>), dim3((unsigned)G), dim3(256), 0, st, n, R, g->n_rt, G,     \
                       g->t_ptr.p, g->t_col.p, g->t_val.p, g->row_scale.p,                                   \
                       DTV == QH_F32 ? xin : p.xa.p, DTV == QH_F32 ? xout : p.xa.p, p.y.p, hin, hout, sa)
#define QH_DENSE_NB(DTV)                                  \
    do {                                                  \
        if (RT == 16) QH_DENSE(DTV, 1, 4);                \
        else if (RT == 32) QH_DENSE(DTV, 2, 4);           \
        else if (p.run_depth == 4) QH_DENSE(DTV, 4, 4);   \
        else QH_DENSE(DTV, 4, 2);                         \
    } while (0)
        switch (g->dtype) {
            case QH_F32: QH_DENSE_NB(QH_F32); break;
            case QH_F16: QH_DENSE_NB(QH_F16); break;
            case QH_BF16: QH_DENSE_NB(QH_BF16); break;
            case QH_FP8_ROWSCALE: QH_DENSE_NB(QH_FP8_ROWSCALE); break;
        }
#undef QH_DENSE_NB
#undef QH_DENSE
        QH_CHECK_LAUNCH();
        return;
    }
    // skyline
    const int RT = R >= 64 ? 64 : R;
    const int64_t rows_per_wg = 64;
    const int64_t nblk = ceil_div(n, rows_per_wg);
    if (nblk == 0) return;
    const float *xin = cur ? p.xb.p : p.xa.p;
    float *xout = cur ? p.xa.p : p.xb.p;
    const bool lr = g->l_nnz > 0;
    // 16-bit graphs with long-range rows: the step also writes a binary16 copy of the new x,
    // which the next step's long-range gathers read
    const bool lh = lr && p.la.p != nullptr;
    StepArgs sl = sa;
    if (lh) sl.lr_out = cur ? p.la.p : p.lb.p;
    const uint16_t *lhin = lh ? (cur ? p.lb.p : p.la.p) : nullptr;
    dim3 grid((unsigned)nblk, (unsigned)(R / RT));
#define QH_HUB(DTV, RTV, H16V)                                                                                  \
    hipLaunchKernelGGL((k_hub_partials<DTV, RTV, H16V>), dim3((unsigned)grid_for(g->n_hub_chunks, 4 * (64 / RTV), 4096), \
                                                        (unsigned)(R / RTV)),                                       \
                       dim3(256), 0, st, g->n_hub_chunks, R, g->hub_chunk_beg.p, g->hub_chunk_end.p, g->l_col.p,   \
                       g->l_val.p, xin, lhin, p.hub_part.p, sa.discrete)
#define QH_PK(DTV, H16V)                                                                                        \
    hipLaunchKernelGGL((k_lr_packets<DTV, H16V>), dim3((unsigned)grid_for(g->n_lr_pk, 4, 1 << 20), (unsigned)(R / 64)),  \
                       dim3(256), 0, st, g->n_lr_pk, R, g->lr_pk_ptr.p, g->hub_chunk_beg.p, g->hub_chunk_end.p,     \
                       g->l_col.p, g->l_val.p, xin, lhin, p.hub_part.p, sa.discrete)
#define QH_SKY(DTV, RTV)                                                                                       \
    hipLaunchKernelGGL((k_sky_step<DTV, RTV>), grid, dim3(256), 0, st, n, R, rows_per_wg, nblk, g->s_off.p,    \
                       g->s_lo.p, g->s_len.p, g->s_val.p, lr ? g->row_chunk_ptr.p : nullptr, p.hub_part.p, xin, \
                       xout, p.y.p, sl)
    // step kernel: band blocks on FMAs (64-replica tiles), band blocks on MFMAs, or per row
    int sk = p.sky_kernel;
    if (sk == kSkyBandFma && !(RT == 64 && g->n_bblk > 0)) sk = kSkyRows;
    if (sk == kSkyBandMfma && g->n_bblk == 0) sk = kSkyRows;
    const int64_t GB = ceil_div(g->n_bblk, 4);
    // the FMA band kernel: one wave (one band block) per workgroup, which measured about 1 %
    // faster than four on both SNP workloads (finer grains, a shorter tail)
#define QH_BAND_K(DTV, NTV, FLDV)                                                                                 \
    hipLaunchKernelGGL((k_band_step<DTV, NTV, FLDV>), dim3((unsigned)g->n_bblk, (unsigned)(R / 64)), dim3(64), 0, \
                       st, n, R, g->n_bblk, g->n_bblk, g->bb_off.p, g->bb_lo.p, g->bb_w.p, g->bb_val.p,                         \
                       lr ? g->row_chunk_ptr.p : nullptr, p.hub_part.p, xin, xout, p.y.p, sl)
#define QH_BAND_NT(DTV, NTV)                                            \
    do {                                                                \
        if (sa.field) QH_BAND_K(DTV, NTV, true);                        \
        else QH_BAND_K(DTV, NTV, false);                                \
    } while (0)
#define QH_BAND(DTV)                                                    \
    do {                                                                \
        if (lr) QH_BAND_NT(DTV, true);                                  \
        else QH_BAND_NT(DTV, false);                                    \
    } while (0)
#define QH_BANDM(DTV, NBV)                                                                                      \
    hipLaunchKernelGGL((k_band_step_mfma<DTV, NBV>), dim3((unsigned)GB, (unsigned)(R / (NBV * 16))), dim3(256), 0, \
                       st, n, R, g->n_bblk, GB, g->bb_off.p, g->bb_lo.p, g->bb_w.p, g->bb_val.p,                \
                       lr ? g->row_chunk_ptr.p : nullptr, p.hub_part.p, xin, xout, p.y.p, sl)
#define QH_LR(DTV)                                                      \
    do {                                                                \
        if (!lr) break;                                                 \
        if (lh) {                                                       \
            if (RT == 16) QH_HUB(DTV, 16, true);                        \
            else if (RT == 32) QH_HUB(DTV, 32, true);                   \
            else QH_PK(DTV, true);                                      \
        } else {                                                        \
            if (RT == 16) QH_HUB(DTV, 16, false);                       \
            else if (RT == 32) QH_HUB(DTV, 32, false);                  \
            else QH_PK(DTV, false);                                     \
        }                                                               \
    } while (0)
#define QH_SKY_RT(DTV)                                                  \
    do {                                                                \
        QH_LR(DTV);                                                     \
        if (sk == kSkyBandMfma) {                                       \
            if (g->bb_dtype == QH_F16) {                                \
                if (RT == 16) QH_BANDM(QH_F16, 1);                      \
                else if (RT == 32) QH_BANDM(QH_F16, 2);                 \
                else QH_BANDM(QH_F16, 4);                               \
            } else {                                                    \
                if (RT == 16) QH_BANDM(DTV, 1);                         \
                else if (RT == 32) QH_BANDM(DTV, 2);                    \
                else QH_BANDM(DTV, 4);                                  \
            }                                                           \
        } else if (sk == kSkyBandFma) {                                 \
            if (g->bb_dtype == QH_F16) QH_BAND(QH_F16);                 \
            else QH_BAND(DTV);                                          \
        } else if (RT == 16) QH_SKY(DTV, 16);                           \
        else if (RT == 32) QH_SKY(DTV, 32);                             \
        else QH_SKY(DTV, 64);                                           \
    } while (0)
    switch (g->dtype) {
        case QH_F32: QH_SKY_RT(QH_F32); break;
        case QH_F16: QH_SKY_RT(QH_F16); break;
        case QH_BF16: QH_SKY_RT(QH_BF16); break;
        default: fail(QH_EUNSUPPORTED, "dtype not offered on skyline storage");
    }
#undef QH_SKY_RT
#undef QH_LR
#undef QH_BANDM
#undef QH_BAND
#undef QH_BAND_NT
#undef QH_BAND_K
#undef QH_SKY
#undef QH_PK
#undef QH_HUB
    QH_CHECK_LAUNCH();
}

static bool x_pingpong(const qh_graph *g) { return !(g->storage == QH_STORE_DENSE && g->dtype != QH_F32); }

// Launch steps [kb, ke); returns the ping-pong half that holds the final state.
static int run_steps(const qh_graph *g, SolvePlan &p, const qh_bsb_opts *o, const float *pump, double c0, double a0,
                     int kb, int ke, hipStream_t st) {
    StepArgs sa;
    sa.c0 = (float)c0;
    sa.dt = (float)o->dt;
    sa.a0 = (float)a0;
    sa.pump = pump;
    sa.discrete = o->variant == 1;
    sa.bscale = g->bb_scale;
    sa.field = o->field;
    int cur = 0;
    for (int k = kb; k < ke; ++k) {
        sa.k = k;
        launch_step(g, p, sa, cur, st);
        cur ^= 1;
    }
    return cur;
}

// The copies of x that the step kernels read besides x itself, made from xa: the dense
// paths' 16-bit product copy (ha), or the binary16 copy of the long-range gathers (la).
static void x_to_h(const qh_graph *g, SolvePlan &p, int64_t n, int R, int discrete, hipStream_t st) {
    const int64_t nR = n * R;
    if (!nR) return;
    if (x_pingpong(g)) {
        if (lr_copy(g)) {
            hipLaunchKernelGGL(k_x_to_lh, dim3(grid_for(nR)), dim3(256), 0, st, nR, p.xa.p, p.la.p, discrete);
            QH_CHECK_LAUNCH();
        }
        return;
    }
    if (g->dtype == QH_BF16)
        hipLaunchKernelGGL(k_x_to_h<true>, dim3(grid_for(nR)), dim3(256), 0, st, n, R, p.xa.p, p.ha.p, discrete);
    else
        hipLaunchKernelGGL(k_x_to_h<false>, dim3(grid_for(nR)), dim3(256), 0, st, n, R, p.xa.p, p.ha.p, discrete);
    QH_CHECK_LAUNCH();
}

// Clears the persistent plan's step flags and error word (a kernel rather than a memset,
// so that a caller capturing the stream into a graph records no memset node).
__global__ void k_zero_i32(int64_t n, int *__restrict__ p) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Steps [kb, ke) in one cooperative launch; the state is in p.xa / p.y / p.ha.
static void run_persistent(const qh_graph *g, SolvePlan &p, const float *pump, double c0, double dt, double a0,
                           int kb, int ke, int discrete, const float *field, int coherent, hipStream_t st) {
    PersistPlan &pp = *p.pp;
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for((int64_t)pp.flags.n)), dim3(256), 0, st, (int64_t)pp.flags.n,
                       pp.flags.p);
    QH_CHECK_LAUNCH();
    PersistArgs pa{};
    pa.n = g->n;
    pa.R = p.R;
    pa.kb = kb;
    pa.ke = ke;
    pa.ng = pp.ng;
    pa.wpg = pp.wpg;
    pa.wg_rt = pp.wg_rt.p;
    pa.t_ptr = g->t_ptr.p;
    pa.t_val = g->t_val.p;
    pa.row_scale = g->row_scale.p;
    pa.wg_ct_ptr = pp.wg_ct_ptr.p;
    pa.wg_ct = pp.wg_ct.p;
    pa.tile_slot = pp.tile_slot.p;
    pa.nbr_ptr = pp.nbr_ptr.p;
    pa.nbr = pp.nbr.p;
    pa.x = p.xa.p;
    pa.y = p.y.p;
    pa.h0 = p.ha.p;
    pa.h1 = p.hb.p;
    pa.flags = pp.flags.p;
    pa.err = pp.flags.p + (int64_t)pp.ng * pp.wpg + 32;
    pa.c0 = (float)c0;
    pa.dt = (float)dt;
    pa.a0 = (float)a0;
    pa.pump = pump;
    pa.discrete = discrete;
    pa.field = field;
    pa.lds_j_bytes = pp.lds_j_bytes;
    pa.lds_tab_off = pp.lds_tab_off;
    pa.max_wg_tiles = pp.max_wg_tiles;
    pa.max_ct = pp.max_ct;
    pa.max_polls = (int64_t)1 << 27;
    launch_persistent(g, pp, pa, coherent, st);
    int32_t err = 0;
    QH_HIP(hipMemcpyAsync(&err, pa.err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    QH_HIP(hipStreamSynchronize(st));
    if (err) fail(QH_EHIP, "persistent bSB kernel: a neighbour wait exceeded its poll limit");
}

// Autotuner for plan 0 on dense 16/8-bit graphs: time a short run of each candidate on
// scratch state -- one fused kernel per step, and the persistent launch -- and keep the
// faster.  Both compute bit-identical results, so the choice only affects speed.
static void autotune_dense(const qh_graph *g, SolvePlan &p, const qh_bsb_opts *o, const float *pump, double c0,
                           double a0, hipStream_t st) {
    const int64_t n = g->n;
    const int R = p.R;
    const int nt = std::min(o->steps, 64);
    const bool pers_ok = p.pp && p.pp->ok;
    // per-step candidates (replica tile, tiles in flight for 64-replica tiles: 64 + depth 4
    // is coded as 65), then 0 = persistent
    std::vector<int> cands;
    if (R >= 64) cands = {64, 65, 32, 16};
    else cands = {R};
    if (pers_ok) { cands.push_back(0); cands.push_back(-1); }   // persistent: fences; coherent accesses
    p.tuned_plan = 1;
    p.tuned_rt = cands[0];
    p.tuned_depth = 2;
    p.run_rt = R >= 64 ? 64 : R;
    p.run_depth = 2;
    if (cands.size() == 1) return;          // nothing to choose
    hipEvent_t e0, e1;
    QH_HIP(hipEventCreate(&e0));
    QH_HIP(hipEventCreate(&e1));
    float best = 0.0f, best_step = 0.0f;
    bool first = true;
    for (int cand : cands) {
        if (cand > 0) {
            p.run_rt = cand == 65 ? 64 : cand;
            p.run_depth = cand == 65 ? 4 : 2;
        }
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {   // the first repetition warms caches and code
            hipLaunchKernelGGL(k_init, dim3(grid_for(n * R)), dim3(256), 0, st, (uint64_t)0x5eed, n, R, p.xa.p,
                               p.y.p);
            QH_CHECK_LAUNCH();
            if (!x_pingpong(g)) x_to_h(g, p, n, R, o->variant == 1, st);
            QH_HIP(hipEventRecord(e0, st));
            if (cand > 0) run_steps(g, p, o, pump, c0, a0, 0, nt, st);
            else run_persistent(g, p, pump, c0, o->dt, a0, 0, nt, o->variant == 1, o->field, cand < 0, st);
            QH_HIP(hipEventRecord(e1, st));
            QH_HIP(hipEventSynchronize(e1));
        }
        QH_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (cand > 0 && (best_step == 0.0f || ms < best_step)) {
            best_step = ms;
            p.tuned_rt = p.run_rt;
            p.tuned_depth = p.run_depth;
            p.tuned_us[0] = ms * 1000.0f / nt;
        }
        if (cand == 0) p.tuned_us[1] = ms * 1000.0f / nt;
        if (cand < 0) p.tuned_us_coh = ms * 1000.0f / nt;
        if (first || ms < best) {
            best = ms;
            p.tuned_plan = cand > 0 ? 1 : 2;
            if (cand <= 0) p.tuned_coh = cand < 0;
        }
        first = false;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p.run_rt = p.tuned_rt;
    p.run_depth = p.tuned_depth;
}

// SNP graphs: time the two band kernels (64 steps each from a seeded state) and keep the
// faster; the band FMA kernel needs 64-replica tiles.
static void autotune_sky(const qh_graph *g, SolvePlan &p, const qh_bsb_opts *o, const float *pump, double c0,
                         double a0, hipStream_t st) {
    const int64_t n = g->n;
    const int R = p.R;
    const int nt = std::min(o->steps, 64);
    std::vector<int> cands;
    if (R >= 64) cands.push_back(kSkyBandFma);
    cands.push_back(kSkyBandMfma);
    p.sky_tuned = true;
    p.sky_best = cands[0];
    if (g->n_bblk == 0) { p.sky_best = kSkyRows; return; }
    hipEvent_t e0, e1;
    QH_HIP(hipEventCreate(&e0));
    QH_HIP(hipEventCreate(&e1));
    float best = 0.0f;
    for (size_t i = 0; i < cands.size(); ++i) {
        p.sky_kernel = cands[i];
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {   // the first repetition warms caches and code
            hipLaunchKernelGGL(k_init, dim3(grid_for(n * R)), dim3(256), 0, st, (uint64_t)0x5eed, n, R, p.xa.p,
                               p.y.p);
            QH_CHECK_LAUNCH();
            x_to_h(g, p, n, R, o->variant == 1, st);
            QH_HIP(hipEventRecord(e0, st));
            run_steps(g, p, o, pump, c0, a0, 0, nt, st);
            QH_HIP(hipEventRecord(e1, st));
            QH_HIP(hipEventSynchronize(e1));
        }
        QH_HIP(hipEventElapsedTime(&ms, e0, e1));
        p.sky_us[cands[i]] = ms * 1000.0f / nt;
        if (i == 0 || ms < best) {
            best = ms;
            p.sky_best = cands[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

// Eq. (5): E(s) = -1/2 s'Js = W - 2 cut(s), with W = -1/2 sum_ab J_ab
__global__ void k_energy(double W, const double *__restrict__ cut, double *__restrict__ e) {
    if (threadIdx.x == 0) e[0] = W - 2.0 * cut[0];
}

const float *linear_pump(SolvePlan &p, int steps, hipStream_t st) {
    if (p.pump_steps != steps) {
        p.pump_lin.alloc(steps);
        hipLaunchKernelGGL(k_pump_linear, dim3(grid_for(steps)), dim3(256), 0, st, steps, p.pump_lin.p);
        QH_CHECK_LAUNCH();
        p.pump_steps = steps;
    }
    return p.pump_lin.p;
}

// Runs the plan-0 autotuner for (graph, opts->replicas) without a solve and returns the
// choice as explicit options (plan, replica_tile, tiles_in_flight, persistent_sync) that
// make a later qh_bsb_solve skip the tuning and run the same kernels.
void autotune(const qh_graph *g, const qh_bsb_opts *o, qh_bsb_opts *chosen, float *us, hipStream_t st) {
    int cur_dev = 0;
    QH_HIP(hipGetDevice(&cur_dev));
    if (cur_dev != g->device) fail(QH_EINVAL, "graph lives on device %d, current device is %d", g->device, cur_dev);
    const int R = o->replicas;
    SolvePlan &p = solve_plan(g, R, st);
    const double c0 = o->c0 > 0.0 ? o->c0 : g->c0_auto;
    const double a0 = o->a0 > 0.0 ? o->a0 : 1.0;
    const float *pump = o->pump ? o->pump : linear_pump(p, o->steps, st);
    *chosen = *o;
    chosen->replica_tile = 0;
    chosen->tiles_in_flight = 0;
    chosen->persistent_sync = 0;
    us[0] = us[1] = 0.0f;
    if (g->n == 0) { chosen->plan = 1; return; }
    if (g->storage == QH_STORE_DENSE) {
        const bool dense16 = !x_pingpong(g);
        if (dense16 && !p.pp_tried) {
            p.pp = std::make_shared<PersistPlan>();
            build_persistent_plan(g, R, *p.pp, st);
            p.pp_tried = true;
        }
        if (!p.tuned_plan) autotune_dense(g, p, o, pump, c0, a0, st);
        if (dense16 && p.pp && p.pp->ok && p.tuned_plan == 2) {
            chosen->plan = 2;
            chosen->persistent_sync = p.tuned_coh ? 2 : 1;
            us[0] = p.tuned_coh ? p.tuned_us_coh : p.tuned_us[1];
        } else {
            chosen->plan = 1;
            if (R >= 64) {
                chosen->replica_tile = p.tuned_rt ? p.tuned_rt : 64;
                if (chosen->replica_tile == 64) chosen->tiles_in_flight = p.tuned_depth;
            }
            us[0] = p.tuned_us[0];
        }
    } else {
        if (!p.sky_tuned) autotune_sky(g, p, o, pump, c0, a0, st);
        chosen->plan = p.sky_best == kSkyBandMfma ? 5 : p.sky_best == kSkyBandFma ? 4 : 3;
        us[0] = p.sky_us[kSkyBandFma];
        us[1] = p.sky_us[kSkyBandMfma];
    }
}

void bsb_solve(const qh_graph *g, const qh_bsb_opts *o, qh_result *res, hipStream_t st) {
    int cur_dev = 0;
    QH_HIP(hipGetDevice(&cur_dev));
    if (cur_dev != g->device) fail(QH_EINVAL, "graph lives on device %d, current device is %d", g->device, cur_dev);
    const int R = o->replicas;
    const int64_t n = g->n;
    SolvePlan &p = solve_plan(g, R, st);
    const int kb = o->step_begin, ke = o->step_end == 0 ? o->steps : o->step_end;
    const double c0 = o->c0 > 0.0 ? o->c0 : g->c0_auto;
    const double a0 = o->a0 > 0.0 ? o->a0 : 1.0;
    const float *pump = o->pump ? o->pump : linear_pump(p, o->steps, st);
    const int64_t nR = n * R;
    const bool dense16 = !x_pingpong(g);
    const bool dense = g->storage == QH_STORE_DENSE;
    if (dense && o->plan >= 3) fail(QH_EINVAL, "plans 3-5 choose the step kernel of SNP (skyline) graphs");
    if (!dense) {
        // SNP graphs: plan 3 per-row kernel, 4 band blocks on FMAs, 5 band blocks on MFMAs;
        // plan 0 times the two band kernels on this graph once, plan 1 keeps that choice
        // (band FMAs when never tuned)
        int want = o->plan == 3 ? kSkyRows : o->plan == 4 ? kSkyBandFma : o->plan == 5 ? kSkyBandMfma : -1;
        if (want < 0) {
            if (o->plan == 0 && !p.sky_tuned && ke > kb && n > 0) autotune_sky(g, p, o, pump, c0, a0, st);
            want = p.sky_tuned ? p.sky_best : kSkyBandFma;
        }
        if (p.sky_kernel != want) {
            // the captured step loop launches the other kernel: drop it
            p.sky_kernel = want;
            if (p.exec) { (void)hipGraphExecDestroy(p.exec); p.exec = nullptr; }
            if (p.graph) { (void)hipGraphDestroy(p.graph); p.graph = nullptr; }
        }
    }

    // the step loop: the persistent dense plan (plan 2), one fused kernel per step (plan 1,
    // optionally replayed from a captured hipGraph), or the autotuner's choice (plan 0)
    int final_half = 0;
    bool persistent = false;
    const bool want_persistent = o->plan == 0 || o->plan == 2;
    if (dense && ke > kb && n > 0) {
        if (dense16 && want_persistent && !p.pp_tried) {
            p.pp = std::make_shared<PersistPlan>();
            build_persistent_plan(g, R, *p.pp, st);
            p.pp_tried = true;
        }
        if (o->plan == 0 && !p.tuned_plan) autotune_dense(g, p, o, pump, c0, a0, st);
        if (dense16 && want_persistent && p.pp->ok) persistent = o->plan == 2 || p.tuned_plan == 2;
    }
    // replica tile of the per-step dense kernel: the caller's, else the tuned one, else 64
    p.run_rt = R < 64 ? R : o->replica_tile ? o->replica_tile : p.tuned_rt ? p.tuned_rt : 64;
    p.run_depth = o->tiles_in_flight ? o->tiles_in_flight
                                     : (!o->replica_tile && p.tuned_rt == p.run_rt) ? p.tuned_depth : 2;
    if (o->plan == 2 && !persistent)
        fail(QH_EUNSUPPORTED, "the persistent plan does not apply to this graph and replica count");
    // initial state into xa / y (after any tuning, which uses the same buffers)
    auto load_state = [&]() {
        if (o->init) {
            if (nR) {
                hipLaunchKernelGGL(k_init, dim3(grid_for(nR)), dim3(256), 0, st, o->seed, n, R, p.xa.p, p.y.p);
                QH_CHECK_LAUNCH();
            }
        } else if (nR) {
            hipLaunchKernelGGL(k_copy_state_in, dim3(grid_for(nR)), dim3(256), 0, st, n, R, res->x, p.xa.p);
            hipLaunchKernelGGL(k_copy_state_in, dim3(grid_for(nR)), dim3(256), 0, st, n, R, res->y, p.y.p);
            QH_CHECK_LAUNCH();
        }
        x_to_h(g, p, n, R, o->variant == 1, st);
    };
    load_state();
    if (ke > kb && n > 0) p.last_plan = persistent ? 2 : 1;
    const int coherent = o->persistent_sync == 2 || (o->persistent_sync == 0 && p.tuned_coh);
    if (persistent) p.last_coh = coherent;
    if (o->eval_every > 0) {
        // read out after every eval_every steps: the step loop runs in ranges, each starting
        // from the state the previous one left in xa / y (and the 16-bit copy made from xa,
        // the same bits the step kernels write), so the trajectory is that of one range
        const int m = o->eval_every;
        EvalArgs ev;
        ev.W = g->total_weight;
        int k0 = kb;
        for (ev.index = 0;; ++ev.index) {
            const int k1 = (int)std::min<int64_t>(ke, (int64_t)k0 + m);
            int fh = 0;
            if (k1 > k0 && n > 0) {
                if (persistent) run_persistent(g, p, pump, c0, o->dt, a0, k0, k1, o->variant == 1, o->field, coherent, st);
                else fh = run_steps(g, p, o, pump, c0, a0, k0, k1, st);
            }
            if (fh && !dense16 && nR)   // ping-pong paths: the range ended in the second half
                QH_HIP(hipMemcpyAsync(p.xa.p, p.xb.p, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
            ev.last = k1 >= ke;
            ev.energy_row = res->energy ? res->energy + (int64_t)ev.index * R : nullptr;
            if (ev.last) {
                if (res->x && nR) QH_HIP(hipMemcpyAsync(res->x, p.xa.p, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
                if (res->y && nR) QH_HIP(hipMemcpyAsync(res->y, p.y.p, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
            }
            readout(view_of(g), p, R, p.xa.p, p.y.p, res, o->greedy != 0, st, ev.last, &ev);
            if (ev.last) break;
            x_to_h(g, p, n, R, o->variant == 1, st);
            k0 = k1;
        }
        if (res->best_energy) {
            hipLaunchKernelGGL(k_energy, dim3(1), dim3(64), 0, st, g->total_weight, res->best_cut, res->best_energy);
            QH_CHECK_LAUNCH();
        }
        return;
    }
    if (persistent) {
        run_persistent(g, p, pump, c0, o->dt, a0, kb, ke, o->variant == 1, o->field, coherent, st);
    } else if (ke > kb && n > 0) {
        if (o->use_graph) {
            auto key = std::make_tuple(kb, ke, (int)g->dtype, c0, o->dt, a0, pump, R,
                                       (p.run_rt * 8 + p.run_depth) * 2 + (o->variant == 1), o->field);
            if (!p.exec || p.graph_key != key) {
                if (p.exec) { (void)hipGraphExecDestroy(p.exec); p.exec = nullptr; }
                if (p.graph) { (void)hipGraphDestroy(p.graph); p.graph = nullptr; }
                hipStream_t cs;
                QH_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                QH_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                try {
                    run_steps(g, p, o, pump, c0, a0, kb, ke, cs);
                } catch (...) {
                    hipGraph_t junk = nullptr;
                    (void)hipStreamEndCapture(cs, &junk);
                    if (junk) (void)hipGraphDestroy(junk);
                    (void)hipStreamDestroy(cs);
                    throw;
                }
                QH_HIP(hipStreamEndCapture(cs, &p.graph));
                QH_HIP(hipStreamDestroy(cs));
                QH_HIP(hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0));
                p.graph_key = key;
            }
            QH_HIP(hipGraphLaunch(p.exec, st));
            final_half = (ke - kb) & 1;
        } else {
            final_half = run_steps(g, p, o, pump, c0, a0, kb, ke, st);
        }
    }
    const float *xfin = (!dense16 && final_half) ? p.xb.p : p.xa.p;
    if (res->x && nR) QH_HIP(hipMemcpyAsync(res->x, xfin, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (res->y && nR) QH_HIP(hipMemcpyAsync(res->y, p.y.p, nR * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (!o->readout) return;
    if (res->energy) {
        EvalArgs ev;   // one evaluation, after the last step
        ev.W = g->total_weight;
        ev.energy_row = res->energy;
        readout(view_of(g), p, R, xfin, p.y.p, res, o->greedy != 0, st, true, &ev);
    } else {
        readout(view_of(g), p, R, xfin, p.y.p, res, o->greedy != 0, st);
    }
    if (res->best_energy) {
        hipLaunchKernelGGL(k_energy, dim3(1), dim3(64), 0, st, g->total_weight, res->best_cut, res->best_energy);
        QH_CHECK_LAUNCH();
    }
}



}  // namespace qh

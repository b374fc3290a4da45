// Number formats of the stored couplings and of the product copy of x.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qh {

// Round an FP64 value once, to nearest with ties to even, onto the grid of a
// binary format with `p` fraction bits and minimum normal exponent `emin`.
// Values above `vmax` saturate (sat = true) or become infinity.
__host__ __device__ inline double round_grid(double v, int p, int emin, double vmax, bool sat) {
    double a = fabs(v);
    if (a == 0.0 || !(a == a)) return v;
    int ex;
    (void)frexp(a, &ex);           // a = m 2^ex, m in [0.5, 1)
    int e = ex - 1;
    if (e < emin) e = emin;
    double k = rint(ldexp(a, p - e));   // exact scaling, ties-to-even
    double r = ldexp(k, e - p);
    if (r > vmax) r = sat ? vmax : INFINITY;
    return copysign(r, v);
}

__host__ __device__ inline uint16_t f64_to_f16_bits(double v) {
    double r = round_grid(v, 10, -14, 65504.0, false);
    _Float16 h = (_Float16)(float)r;   // exact: r is representable
    uint16_t b;
    __builtin_memcpy(&b, &h, 2);
    return b;
}

__host__ __device__ inline uint16_t f64_to_bf16_bits(double v) {
    double r = round_grid(v, 7, -126, 3.3895313892515355e38, false);
    float f = (float)r;                // exact
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float f64_to_f32(double v) { return (float)v; }

// OCP E4M3 (bias 7, largest finite 448, saturating).
__host__ __device__ inline uint8_t f64_to_e4m3_bits(double v) {
    double r = round_grid(v, 3, -6, 448.0, true);
    uint8_t sign = (r < 0 || (r == 0 && signbit(r))) ? 0x80 : 0;
    double a = fabs(r);
    if (a == 0.0) return sign;
    int ex;
    double m = frexp(a, &ex);
    int e = ex - 1;
    uint32_t code;
    if (e >= -6) {
        uint32_t frac = (uint32_t)rint((2.0 * m - 1.0) * 8.0);
        code = ((uint32_t)(e + 7) << 3) | frac;
    } else {
        code = (uint32_t)rint(ldexp(a, 9));
    }
    return (uint8_t)(sign | code);
}

__host__ __device__ inline float f16_bits_to_f32(uint16_t b) {
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    return (float)h;
}

__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// E4M3 code -> binary16 bits holding (code value) * 2^-8, exact for every finite code.
__host__ __device__ inline uint16_t e4m3_to_f16_bits_scaled(uint8_t c) {
    return (uint16_t)(((uint16_t)(c & 0x80) << 8) | ((uint16_t)(c & 0x7F) << 7));
}

// Eight E4M3 codes (c.x bytes 0-3, then c.y bytes 0-3) -> eight binary16 values holding
// (code value) * 2^-8, in that order, by the hardware conversion: the same bits as
// e4m3_to_f16_bits_scaled for every finite code (the scaled values are exact in binary16).
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
__device__ inline f16x8_t e4m3x8_to_f16_scaled(uint2 c) {
    const auto p0 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(c.x, 0.00390625f, false);
    const auto p1 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(c.x, 0.00390625f, true);
    const auto p2 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(c.y, 0.00390625f, false);
    const auto p3 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(c.y, 0.00390625f, true);
    uint32_t w[4];
    __builtin_memcpy(&w[0], &p0, 4);
    __builtin_memcpy(&w[1], &p1, 4);
    __builtin_memcpy(&w[2], &p2, 4);
    __builtin_memcpy(&w[3], &p3, 4);
    f16x8_t r;
    __builtin_memcpy(&r, w, 16);
    return r;
}

__host__ __device__ inline double e4m3_bits_to_f64(uint8_t c) {
    return (double)f16_bits_to_f32(e4m3_to_f16_bits_scaled(c)) * 256.0;
}

// float -> bfloat16, round to nearest even (finite inputs).
__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline uint16_t f32_to_f16_rne(float f) {
    _Float16 h = (_Float16)f;
    uint16_t b;
    __builtin_memcpy(&b, &h, 2);
    return b;
}

// Dense tile layouts.  A 64x64 tile is stored in the register order of the MFMA
// A operand so that each lane loads its fragment with one contiguous load.
//  16/8-bit (v_mfma_f32_16x16x32_{f16,bf16}): fragment (rb, kb) covers rows 16rb..,
//    cols 32kb..; lane l holds row l%16, cols 8(l/16)..+8.
//  32-bit (v_mfma_f32_16x16x4f32): block (rb, kq) covers rows 16rb.., cols 16kq..;
//    lane l holds, for the 4 k-steps ks = 4kq..4kq+3, row l%16 and col 4ks + l/16.
__host__ __device__ inline void tile_pos16(int idx, int &i, int &j) {
    int e = idx & 7, lane = (idx >> 3) & 63, frag = idx >> 9;
    int rb = frag >> 1, kb = frag & 1;
    i = rb * 16 + (lane & 15);
    j = kb * 32 + 8 * (lane >> 4) + e;
}
__host__ __device__ inline int tile_idx16(int i, int j) {
    int rb = i >> 4, kb = j >> 5;
    int lane = ((j & 31) >> 3) * 16 + (i & 15);
    return (((rb * 2 + kb) * 64 + lane) << 3) + (j & 7);
}
__host__ __device__ inline void tile_pos32(int idx, int &i, int &j) {
    int e4 = idx & 3, lane = (idx >> 2) & 63, blk = idx >> 8;
    int rb = blk >> 2, kq = blk & 3;
    int ks = kq * 4 + e4;
    i = rb * 16 + (lane & 15);
    j = ks * 4 + (lane >> 4);
}
__host__ __device__ inline int tile_idx32(int i, int j) {
    int rb = i >> 4, ks = j >> 2;
    int lane = (j & 3) * 16 + (i & 15);
    int kq = ks >> 2, e4 = ks & 3;
    return (((rb * 4 + kq) * 64 + lane) << 2) + e4;
}

}  // namespace qh

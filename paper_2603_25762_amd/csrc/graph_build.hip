// Graph construction: ternary encoding (Eq. 1), read-graph conflict / signed
// weights (Eqs. 2-3), SNP-graph log-likelihood weights (Eqs. 9-14), the FP64
// master CSR, connected components, and the storage copies used by the step
// kernels (dense MFMA-ordered tiles, skyline band + long-range CSR) in the
// requested number format.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <numeric>

#include <rocprim/rocprim.hpp>

#include "formats.h"

#include "internal.h"

namespace qh {

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------

// Eq. (1): M = +1 where the observed allele is the one placed on H1, else -1; the graph's
// own copy of the initial H1 (S entries) is written on the way.
__global__ void k_encode(int64_t nobs, const int32_t *__restrict__ snp,
                         const uint8_t *__restrict__ allele, const uint8_t *__restrict__ init_h1,
                         int8_t *__restrict__ M, int64_t S, uint8_t *__restrict__ h1_copy) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nobs;
         t += (int64_t)gridDim.x * blockDim.x)
        M[t] = (allele[t] == init_h1[snp[t]]) ? 1 : -1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x)
        h1_copy[i] = init_h1[i];
}

// Initial state of the SNP structure pass in one buffer: the long-range pair counter (64-bit,
// words 0-1), then lo, hi and the union-find parents (n each), every vertex its own.
__global__ void k_structure_init(int64_t n, int32_t *__restrict__ buf) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * n + 2;
         i += (int64_t)gridDim.x * blockDim.x)
        buf[i] = i < 2 ? 0 : (int32_t)((i - 2) % n);
}

__global__ void k_gather_i8(int64_t n, const int64_t *__restrict__ idx, const int8_t *__restrict__ src,
                            int8_t *__restrict__ dst) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[idx[t]];
}

// ---------------------------------------------------------------------------
// device structure pass of read graphs: validation, coverage lists, components
// ---------------------------------------------------------------------------

// Per fragment: frag_ptr non-decreasing, SNP indices in range and strictly ascending,
// alleles 0/1.  err[k] = lowest offending fragment + 1 for check k (all ones when none);
// err[4] = frag_ptr[F] (the observation count) and err[5] = frag_ptr[0], so that one copy
// brings everything back.  With frag_ptr[0] != 0 or a count outside [0, 2^31) nothing else
// is read (the host reports those).
__global__ void k_validate_frags(int64_t F, const int64_t *__restrict__ fp, const int32_t *__restrict__ snp,
                                 const uint8_t *__restrict__ allele, int32_t n_snp,
                                 unsigned long long *__restrict__ err) {
    const int64_t nobs = fp[F], fp0 = fp[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        err[4] = (unsigned long long)nobs;
        err[5] = (unsigned long long)fp0;
    }
    if (fp0 != 0 || nobs < 0 || nobs > INT32_MAX) return;
    // one wave per fragment, a lane per observation: the loads of a fragment go out together
    const int lane = threadIdx.x & 63;
    const int64_t wpb = blockDim.x >> 6;
    for (int64_t f = blockIdx.x * wpb + (threadIdx.x >> 6); f < F; f += (int64_t)gridDim.x * wpb) {
        const int64_t b = fp[f], e = fp[f + 1];
        const unsigned long long tag = (unsigned long long)f + 1;
        if (e < b || b < 0 || e > nobs) {
            if (lane == 0) atomicMin(&err[0], tag);
            continue;
        }
        for (int64_t t = b + lane; t < e; t += 64) {
            const int32_t j = snp[t];
            const int32_t prev = t > b ? snp[t - 1] : INT32_MIN;
            if (j < 0 || j >= n_snp) atomicMin(&err[1], tag);
            else if (t > b && j <= prev) atomicMin(&err[2], tag);
            if (allele[t] > 1) atomicMin(&err[3], tag);
        }
    }
}

__global__ void k_obs_frag(int64_t F, const int64_t *__restrict__ fp, int32_t *__restrict__ obs_frag,
                           int32_t *__restrict__ obs_idx) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x)
        for (int64_t t = fp[f]; t < fp[f + 1]; ++t) {
            obs_frag[t] = (int32_t)f;
            obs_idx[t] = (int32_t)t;
        }
}

// cov_ptr[j] = first position of SNP j in the SNP-sorted observations (lower bound)
__global__ void k_cov_ptr(int32_t S, int64_t nobs, const int32_t *__restrict__ sorted_snp,
                          int64_t *__restrict__ cov_ptr) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= S; j += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = nobs;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted_snp[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        cov_ptr[j] = lo;
    }
}

__global__ void k_cov_fill(int64_t nobs, const int32_t *__restrict__ sorted_obs, const int32_t *__restrict__ obs_frag,
                           const int8_t *__restrict__ M, int32_t *__restrict__ cov_frag, int8_t *__restrict__ cov_M) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nobs; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t t = sorted_obs[p];
        cov_frag[p] = obs_frag[t];
        cov_M[p] = M[t];
    }
}

// Union-find with lock-free hooking: a root is hooked under a smaller root by CAS, so the
// root of every tree is its smallest vertex.  Parent reads bypass stale cache lines.
__device__ inline int32_t duf_parent(int32_t *p, int32_t x) {
    return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root with path splitting: every visited non-root is pointed at its grandparent.  Parents
// only ever point at smaller indices (hooks and splits alike), so every walk ends, and a
// split never touches a root, so it cannot race with a hook.
__device__ inline int32_t duf_root(int32_t *p, int32_t x) {
    while (true) {
        const int32_t y = duf_parent(p, x);
        if (y == x) return x;
        const int32_t z = duf_parent(p, y);
        if (z != y) __hip_atomic_store(p + x, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = y;
    }
}

// The same walk through cached parent reads, which may be stale: a stale parent of x is an
// earlier parent, and every earlier parent is still an ancestor (parents only move towards
// the root), so the walk ends at a vertex that was a root once; splits still go out as
// device-coherent stores (plain stores never touch the parent array).
__device__ inline int32_t duf_root_cached(int32_t *p, int32_t x) {
    while (true) {
        const int32_t y = p[x];
        if (y == x) return x;
        const int32_t z = p[y];
        if (z != y) __hip_atomic_store(p + x, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = y;
    }
}

// Joins the trees of x and y: the larger root is hooked under the smaller by
// compare-and-swap.  The first attempt walks through cached reads; a hook that fails (the
// walk ended at a vertex that is no longer a root) walks again with device-coherent reads.
__device__ inline void duf_link(int32_t *p, int32_t x, int32_t y) {
    bool coherent = false;
    while (true) {
        x = coherent ? duf_root(p, x) : duf_root_cached(p, x);
        y = coherent ? duf_root(p, y) : duf_root_cached(p, y);
        if (x == y) return;        // both are descendants of that vertex: one tree already
        if (x < y) { const int32_t t = x; x = y; y = t; }
        if (atomicCAS(p + x, x, y) == x) return;   // x was a root and now hangs under y
        coherent = true;
    }
}

__global__ void k_uf_init(int64_t n, int32_t *__restrict__ p) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// fragments that share a SNP are linked along its coverage list: one thread per position
// q of the SNP-sorted observations links cov_frag[q - 1] and cov_frag[q] of the same SNP
__global__ void k_uf_link(int64_t nobs, const int32_t *__restrict__ sorted_snp, const int32_t *__restrict__ cov_frag,
                          int32_t *p) {
    for (int64_t q = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nobs;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (sorted_snp[q] != sorted_snp[q - 1]) continue;
        duf_link(p, cov_frag[q - 1], cov_frag[q]);
    }
}

__global__ void k_uf_flatten(int64_t n, int32_t *p) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = duf_root(p, (int32_t)i);
}

// ---------------------------------------------------------------------------
// device structure pass of SNP graphs: kept observations, skyline extents,
// long-range pair set, components
// ---------------------------------------------------------------------------

// kept observations (Phred > 3) per fragment; cnt has F + 1 entries (cnt[F] = 0) so that
// its exclusive scan is the fragment pointer of the kept list
__global__ void k_kept_count(int64_t F, const int64_t *__restrict__ fp, const uint8_t *__restrict__ phred,
                             int64_t *__restrict__ cnt) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f <= F; f += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        if (f < F)
            for (int64_t t = fp[f]; t < fp[f + 1]; ++t) c += phred[t] > 3;
        cnt[f] = c;
    }
}

__global__ void k_kept_fill(int64_t F, const int64_t *__restrict__ fp, const uint8_t *__restrict__ phred,
                            const int64_t *__restrict__ kept_ptr, int64_t *__restrict__ kept_obs,
                            int32_t *__restrict__ kept_frag) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        int64_t q = kept_ptr[f];
        for (int64_t t = fp[f]; t < fp[f + 1]; ++t)
            if (phred[t] > 3) {
                kept_obs[q] = t;
                kept_frag[q] = (int32_t)f;
                ++q;
            }
    }
}

// Per kept observation a of fragment f (SNP u = u_a): the pairs (a, b), a < b <= a + L with
// L = floor(k (|S_f| - 1) / 10).  In-band pairs (v - u <= band_limit, or no limit) widen
// the skyline: hi[u] >= the largest in-band v, lo[v] <= u; the others are long-range
// (counted in pass 0, written as both directed keys u n + v and v n + u in pass 1).
// Consecutive kept SNPs of a fragment with L >= 1 are linked for the components.
__global__ void k_snp_structure(int64_t n_kept, const int64_t *__restrict__ kept_obs,
                                const int32_t *__restrict__ kept_frag, const int64_t *__restrict__ kept_ptr,
                                const int32_t *__restrict__ snp, int linkage_k, int32_t band_limit, int64_t n,
                                int32_t *__restrict__ lo, int32_t *__restrict__ hi, int32_t *uf,
                                unsigned long long *__restrict__ lr_count, uint64_t *__restrict__ lr_keys, int pass) {
    for (int64_t kk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; kk < n_kept;
         kk += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f = kept_frag[kk];
        const int64_t base = kept_ptr[f], ns = kept_ptr[f + 1] - base;
        if (ns < 2) continue;
        const int64_t L = (int64_t)linkage_k * (ns - 1) / 10;
        if (L < 1) continue;
        const int64_t a = kk - base;
        const int32_t u = snp[kept_obs[kk]];
        const int64_t bmax = a + L < ns - 1 ? a + L : ns - 1;
        if (pass == 0) {
            if (a > 0) duf_link(uf, snp[kept_obs[kk - 1]], u);   // the previous kept SNP of the fragment
            int32_t vmax = -1;
            unsigned long long nlr = 0;
            for (int64_t b = a + 1; b <= bmax; ++b) {
                const int32_t v = snp[kept_obs[base + b]];
                if (band_limit == 0 || v - u <= band_limit) vmax = v;
                else ++nlr;
            }
            if (vmax >= 0) atomicMax(hi + u, vmax);
            // lo[u]: the smallest partner w < u in band among a' in [a - L, a)
            const int64_t a0 = a - L > 0 ? a - L : 0;
            for (int64_t b = a0; b < a; ++b) {
                const int32_t w = snp[kept_obs[base + b]];
                if (band_limit == 0 || u - w <= band_limit) { atomicMin(lo + u, w); break; }
            }
            if (nlr) atomicAdd(lr_count, nlr);
        } else {
            for (int64_t b = a + 1; b <= bmax; ++b) {
                const int32_t v = snp[kept_obs[base + b]];
                if (band_limit == 0 || v - u <= band_limit) continue;
                const unsigned long long at = atomicAdd(lr_count, 2ull);
                lr_keys[at] = (uint64_t)u * (uint64_t)n + (uint64_t)v;
                lr_keys[at + 1] = (uint64_t)v * (uint64_t)n + (uint64_t)u;
            }
        }
    }
}

// long-range CSR from the sorted, unique directed keys: l_ptr[u] = first key of row u
__global__ void k_lr_csr(int64_t n, int64_t l_nnz, const uint64_t *__restrict__ keys, int64_t *__restrict__ l_ptr,
                         int32_t *__restrict__ l_col) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n || i < l_nnz;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i <= n) {
            const uint64_t key = (uint64_t)i * (uint64_t)n;
            int64_t a = 0, b = l_nnz;
            while (a < b) {
                const int64_t m = (a + b) >> 1;
                if (keys[m] < key) a = m + 1;
                else b = m;
            }
            l_ptr[i] = a;
        }
        if (i < l_nnz) l_col[i] = (int32_t)(keys[i] % (uint64_t)n);
    }
}

// Eqs. (2)-(3): every ordered pair of fragments covering SNP column j adds its
// per-column term.  conflict: 1[M_a M_b = -1] (stored as A); signed: M_a M_b (J).
__global__ void k_read_pairs(int32_t n_cols, const int64_t *__restrict__ cov_ptr,
                             const int32_t *__restrict__ cov_frag, const int8_t *__restrict__ cov_M,
                             int32_t *__restrict__ W, int64_t F, int conflict) {
    for (int64_t j = blockIdx.x; j < n_cols; j += gridDim.x) {
        int64_t b = cov_ptr[j], c = cov_ptr[j + 1] - b;
        for (int64_t t = threadIdx.x; t < c * c; t += blockDim.x) {
            int64_t p = t / c, q = t - p * c;
            if (p == q) continue;
            int prod = (int)cov_M[b + p] * (int)cov_M[b + q];
            int v = conflict ? (prod == -1 ? 1 : 0) : prod;
            if (v) atomicAdd(&W[(int64_t)cov_frag[b + p] * F + cov_frag[b + q]], v);
        }
    }
}

// Rows of Eqs. (2)-(3), one workgroup per fragment p: the row's F counters live in LDS;
// for every SNP j of p and every fragment q on j's coverage list (q != p) the row adds
// M_pj M_qj (signed kind) or 1 where the two disagree (conflict kind) with an LDS atomic,
// then goes out whole, zeros included.  p's observations are taken kRowObs at a time:
// their coverage lists are concatenated (offsets in LDS) and the items split evenly over
// the workgroup.  Integer sums, so the order of the additions does not matter.
constexpr int kRowObs = 256;
constexpr int64_t kRowLdsMaxF = 36864;   // F int32 counters per workgroup (144 KB of LDS)
__global__ __launch_bounds__(256) void k_read_rows(int64_t F, const int64_t *__restrict__ fp,
                                                   const int32_t *__restrict__ snp, const int8_t *__restrict__ M,
                                                   const int64_t *__restrict__ cov_ptr,
                                                   const int32_t *__restrict__ cov_frag,
                                                   const int8_t *__restrict__ cov_M, int32_t *__restrict__ W,
                                                   int conflict) {
    extern __shared__ int32_t row[];            // [F]
    __shared__ int64_t cbeg[kRowObs];           // coverage list of each observation of the chunk
    __shared__ int32_t coff[kRowObs + 1];       // offsets of the lists in the concatenation
    __shared__ int8_t cm[kRowObs];              // M_pj
    const int tid = threadIdx.x;
    for (int64_t p = blockIdx.x; p < F; p += gridDim.x) {
        for (int64_t q = tid; q < F; q += 256) row[q] = 0;
        const int64_t t0 = fp[p], t1 = fp[p + 1];
        for (int64_t base = t0; base < t1; base += kRowObs) {
            const int nb = (int)(t1 - base < kRowObs ? t1 - base : kRowObs);
            if (tid < nb) {
                const int32_t j = snp[base + tid];
                const int64_t b = cov_ptr[j];
                cbeg[tid] = b;
                coff[tid + 1] = (int32_t)(cov_ptr[j + 1] - b);
                cm[tid] = M[base + tid];
            }
            __syncthreads();    // (also: the zeroed row before the first atomic)
            if (tid == 0) {
                coff[0] = 0;
                for (int k = 0; k < nb; ++k) coff[k + 1] += coff[k];
            }
            __syncthreads();
            const int total = coff[nb];
            for (int i = tid; i < total; i += 256) {
                int lo = 0, hi = nb;            // the last observation k with coff[k] <= i
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (coff[mid] <= i) lo = mid;
                    else hi = mid;
                }
                const int64_t c = cbeg[lo] + (i - coff[lo]);
                const int32_t q = cov_frag[c];
                if (q == p) continue;
                const int prod = (int)cm[lo] * (int)cov_M[c];
                const int v = conflict ? (prod == -1 ? 1 : 0) : prod;
                if (v) atomicAdd(&row[q], v);
            }
            __syncthreads();    // the chunk's tables are read before the next chunk writes them
        }
        __syncthreads();
        for (int64_t q = tid; q < F; q += 256) W[p * F + q] = row[q];
        __syncthreads();        // the row is written out before the next fragment clears it
    }
}

// Nonzero count per row of a dense int32 matrix (one wave per row).
__global__ void k_dense_row_nnz(int64_t F, const int32_t *__restrict__ W, int64_t *__restrict__ cnt) {
    int lane = threadIdx.x & 63;
    int64_t row = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= F) return;
    int64_t c = 0;
    for (int64_t col = lane; col < F; col += 64) c += (W[row * F + col] != 0);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if (lane == 0) cnt[row] = c;
}

// Ordered compaction of the nonzeros of each dense row into the master CSR.
__global__ void k_dense_row_fill(int64_t F, const int32_t *__restrict__ W, int negate,
                                 const int64_t *__restrict__ ptr, int32_t *__restrict__ col,
                                 double *__restrict__ val) {
    int lane = threadIdx.x & 63;
    int64_t row = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= F) return;
    int64_t out = ptr[row];
    for (int64_t c0 = 0; c0 < F; c0 += 64) {
        int64_t c = c0 + lane;
        int w = c < F ? W[row * F + c] : 0;
        uint64_t mask = __ballot(w != 0);
        if (w != 0) {
            int before = __popcll(mask & ((1ull << lane) - 1ull));
            col[out + before] = (int32_t)c;
            val[out + before] = negate ? -(double)w : (double)w;
        }
        out += __popcll(mask);
    }
}

// Occupancy of each 64x64 tile of a dense matrix.
__global__ void k_tile_occupancy(int64_t F, int64_t n_rt, const int32_t *__restrict__ W,
                                 uint8_t *__restrict__ occ) {
    int64_t rt = blockIdx.y, ct = blockIdx.x;
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int found = 0;
    for (int e = threadIdx.x; e < kTileElems; e += blockDim.x) {
        int64_t i = rt * kTile + (e >> 6), j = ct * kTile + (e & 63);
        if (i < F && j < F && W[i * F + j] != 0) found = 1;
    }
    if (found) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) occ[rt * n_rt + ct] = (uint8_t)any;
}

// Per-row max |J| over the master CSR (one wave per row, coalesced; a maximum does not
// depend on the order it is taken in).
__global__ void k_row_absmax(int64_t n, const int64_t *__restrict__ ptr,
                             const double *__restrict__ val, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    for (int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < n;
         r += (int64_t)gridDim.x * (blockDim.x >> 6)) {
        double m = 0.0;
        for (int64_t e = ptr[r] + lane; e < ptr[r + 1]; e += 64) m = fmax(m, fabs(val[e]));
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
        if (lane == 0) out[r] = m;
    }
}

// Per-row sum |J| (greedy tolerance for float weights).
__global__ void k_row_abssum(int64_t n, const int64_t *__restrict__ ptr,
                             const double *__restrict__ val, double *__restrict__ out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        double m = 0.0;
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) m += fabs(val[e]);
        out[r] = m;
    }
}

// FP8 row scale s_i = RNE_f32(max_j |J_ij| / 448); the kernels use 256 s_i because the
// code decode yields code * 2^-8.
__global__ void k_fp8_scales(int64_t n, const double *__restrict__ rmax, float *__restrict__ scale,
                             float *__restrict__ scale_dec) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        float s = (float)(rmax[r] / 448.0);
        scale[r] = s;
        scale_dec[r] = s * 256.0f;
    }
}

// Pack the stored tiles of a dense matrix in MFMA fragment order and number format.
__global__ void k_pack_tiles(int64_t F, const int32_t *__restrict__ W, int negate,
                             const int32_t *__restrict__ tile_row, const int32_t *__restrict__ tile_col,
                             int dtype, const float *__restrict__ scale, uint8_t *__restrict__ out) {
    int64_t t = blockIdx.x;
    int64_t rt = tile_row[t], ct = tile_col[t];
    for (int idx = threadIdx.x; idx < kTileElems; idx += blockDim.x) {
        int i, j;
        if (dtype == QH_F32) tile_pos32(idx, i, j);
        else tile_pos16(idx, i, j);
        int64_t gi = rt * kTile + i, gj = ct * kTile + j;
        double v = 0.0;
        if (gi < F && gj < F) {
            int w = W[gi * F + gj];
            v = negate ? -(double)w : (double)w;
        }
        int64_t o = t * kTileElems + idx;
        switch (dtype) {
            case QH_F32: ((float *)out)[o] = f64_to_f32(v); break;
            case QH_F16: ((uint16_t *)out)[o] = f64_to_f16_bits(v); break;
            case QH_BF16: ((uint16_t *)out)[o] = f64_to_bf16_bits(v); break;
            case QH_FP8_ROWSCALE: {
                double s = gi < F ? (double)scale[gi] : 0.0;
                out[o] = s > 0.0 ? f64_to_e4m3_bits(v / s) : (uint8_t)0;
                break;
            }
        }
    }
}

// ---- SNP graph (Eqs. 9-14) -------------------------------------------------

// In-place conversion of fixed-point sums (int64 multiples of 2^-40) to FP64.
__global__ void k_fixed_to_f64(int64_t n, double *__restrict__ v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const long long q = __builtin_bit_cast(long long, v[i]);
        v[i] = (double)q * 0x1p-40;
    }
}

// kept observations of a fragment whose SNP index, allele code, Phred confidence and skyline
// row base k_snp_pairs stages in LDS (a longer fragment's later partners come from memory)
constexpr int kFragLds = 512;

// Eqs. (9), (11)-(13) with the per-fragment factor alpha and the 1/(|S_i|-1)
// normalisation of Eq. (14).  J = -w, so each pair term enters J with a + sign.
// One wave per fragment f and a lane per kept observation (rank a), which handles the
// pairs (a, b) with a < b <= a + L of the fragment.  In fixed-point mode a term of magnitude
// 2^20 or more cannot be represented: *clamped is set and the build fails.
__global__ __launch_bounds__(256) void k_snp_pairs(int64_t F, const int64_t *__restrict__ kept_obs,
                                                   const int64_t *__restrict__ kept_ptr,
                                                   const int32_t *__restrict__ snp, const int8_t *__restrict__ M,
                                                   const uint8_t *__restrict__ phred,
                                                   const double *__restrict__ alpha,
                                                   const double *__restrict__ qconf, int linkage_k,
                                                   int32_t band_limit, const int64_t *__restrict__ s_off,
                                                   const int32_t *__restrict__ s_lo, double *__restrict__ s_val64,
                                                   const int64_t *__restrict__ l_ptr,
                                                   const int32_t *__restrict__ l_col, double *__restrict__ l_val64,
                                                   int fixed, int32_t *__restrict__ clamped) {
    __shared__ double s_q[4][kFragLds];
    __shared__ int64_t s_rb[4][kFragLds];   // skyline row base s_off[u] - s_lo[u] of each SNP
    __shared__ int32_t s_u[4][kFragLds];
    __shared__ int8_t s_m[4][kFragLds];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *sq = s_q[wave];
    int64_t *srb = s_rb[wave];
    int32_t *su = s_u[wave];
    int8_t *sm = s_m[wave];
    for (int64_t f0 = (int64_t)blockIdx.x * 4; f0 < F; f0 += (int64_t)gridDim.x * 4) {
        const int64_t f = f0 + wave;
        int64_t base = 0, ns = 0;
        if (f < F) {
            base = kept_ptr[f];
            ns = kept_ptr[f + 1] - base;
        }
        if (ns >= 2)
            for (int64_t a = lane; a < ns && a < kFragLds; a += 64) {
                const int64_t t = kept_obs[base + a];
                const int32_t u = snp[t];
                su[a] = u;
                sm[a] = M[t];
                sq[a] = qconf[phred[t]];
                srb[a] = s_off[u] - s_lo[u];
            }
        __syncthreads();
        const int64_t L = ns >= 2 ? (int64_t)linkage_k * (ns - 1) / 10 : 0;
        const double af = (ns >= 2 && alpha) ? alpha[f] : 1.0;
        for (int64_t a = lane; L >= 1 && a < ns; a += 64) {
            const bool sa = a < kFragLds;
            const int64_t ta = sa ? 0 : kept_obs[base + a];
            const int32_t u = sa ? su[a] : snp[ta];
            const int Mu = sa ? sm[a] : M[ta];
            const double qu = sa ? sq[a] : qconf[phred[ta]];
            const int64_t rbu = sa ? srb[a] : s_off[u] - s_lo[u];
            const int64_t bmax = a + L < ns - 1 ? a + L : ns - 1;
            for (int64_t b = a + 1; b <= bmax; ++b) {
                const bool sb = b < kFragLds;
                const int64_t tb = sb ? 0 : kept_obs[base + b];
                const int32_t v = sb ? su[b] : snp[tb];
                const int Mv = sb ? sm[b] : M[tb];
                const double qv = sb ? sq[b] : qconf[phred[tb]];
                const double p_cis = qu * qv + (1.0 - qu) * (1.0 - qv);
                const double p_trans = qu * (1.0 - qv) + (1.0 - qu) * qv;
                const double sgn = (Mu * Mv > 0) ? 1.0 : -1.0;
                const double l = sgn * log10(p_cis / p_trans);
                const double term = af * l / (double)(ns - 1);   // enters J = -w with + sign
                // fixed = 1: the term as a multiple of 2^-40 (|term| clamped to 2^20), summed with
                // integer atomics, whose result does not depend on the order of the additions
                const double tc = term < -0x1p20 ? -0x1p20 : (term > 0x1p20 ? 0x1p20 : term);
                if (fixed && !(fabs(term) < 0x1p20)) *clamped = 1;
                const unsigned long long tq = (unsigned long long)(long long)__builtin_rint(tc * 0x1p40);
                auto add = [&](double *p) {
                    if (fixed) atomicAdd((unsigned long long *)p, tq);
                    else unsafeAtomicAdd(p, term);
                };
                if (band_limit == 0 || v - u <= band_limit) {
                    add(&s_val64[rbu + v]);
                    add(&s_val64[(sb ? srb[b] : s_off[v] - s_lo[v]) + u]);
                } else {
                    int64_t lo = l_ptr[u], hi = l_ptr[u + 1];
                    while (lo < hi) { int64_t m = (lo + hi) >> 1; if (l_col[m] < v) lo = m + 1; else hi = m; }
                    add(&l_val64[lo]);
                    lo = l_ptr[v]; hi = l_ptr[v + 1];
                    while (lo < hi) { int64_t m = (lo + hi) >> 1; if (l_col[m] < u) lo = m + 1; else hi = m; }
                    add(&l_val64[lo]);
                }
            }
        }
        __syncthreads();
    }
}

// Nonzeros per row of skyline + long-range.
__global__ void k_sky_row_nnz(int64_t n, const int64_t *__restrict__ s_off, const int32_t *__restrict__ s_len,
                              const double *__restrict__ s_val64, const int64_t *__restrict__ l_ptr,
                              const double *__restrict__ l_val64, int64_t *__restrict__ cnt) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        for (int64_t e = 0; e < s_len[u]; ++e) c += (s_val64[s_off[u] + e] != 0.0);
        if (l_ptr)
            for (int64_t e = l_ptr[u]; e < l_ptr[u + 1]; ++e) c += (l_val64[e] != 0.0);
        cnt[u] = c;
    }
}

__global__ void k_sky_row_fill(int64_t n, const int64_t *__restrict__ s_off, const int32_t *__restrict__ s_lo,
                               const int32_t *__restrict__ s_len, const double *__restrict__ s_val64,
                               const int64_t *__restrict__ l_ptr, const int32_t *__restrict__ l_col,
                               const double *__restrict__ l_val64, const int64_t *__restrict__ m_ptr,
                               int32_t *__restrict__ m_col, double *__restrict__ m_val) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        int64_t o = m_ptr[u];
        int32_t lo = s_lo[u];
        int64_t le = l_ptr ? l_ptr[u] : 0, lend = l_ptr ? l_ptr[u + 1] : 0;
        for (; le < lend && l_col[le] < lo; ++le)
            if (l_val64[le] != 0.0) { m_col[o] = l_col[le]; m_val[o] = l_val64[le]; ++o; }
        for (int64_t e = 0; e < s_len[u]; ++e) {
            double v = s_val64[s_off[u] + e];
            if (v != 0.0) { m_col[o] = lo + (int32_t)e; m_val[o] = v; ++o; }
        }
        for (; le < lend; ++le)
            if (l_val64[le] != 0.0) { m_col[o] = l_col[le]; m_val[o] = l_val64[le]; ++o; }
    }
}

// FP64 -> stored number format (elementwise, RNE).
// flush: magnitudes below it store as 0 (BF16 SNP storage, see the caller); 0 = none
__global__ void k_quantize(int64_t n, const double *__restrict__ src, int dtype, uint8_t *__restrict__ dst,
                           double flush) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        double v = src[t];
        if (fabs(v) < flush) v = 0.0;
        switch (dtype) {
            case QH_F32: ((float *)dst)[t] = (float)v; break;
            case QH_F16: ((uint16_t *)dst)[t] = f64_to_f16_bits(v); break;
            case QH_BF16: ((uint16_t *)dst)[t] = f64_to_bf16_bits(v); break;
        }
    }
}

// Band blocks: element (block b, column offset j, row i) = J[16b + i][bb_lo[b] + j], zero
// outside the row's skyline range (and on the diagonal, which is zero anyway).
// Largest |value| of an FP64 array, as the bits of a non-negative double (which order like
// the values), reduced over the wave before one atomic.
__global__ void k_absmax_bits(int64_t m, const double *__restrict__ v, unsigned long long *__restrict__ out) {
    unsigned long long hi = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v[e]));
        hi = b > hi ? b : hi;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(hi, d);
        hi = o > hi ? o : hi;
    }
    if ((threadIdx.x & 63) == 0 && hi) atomicMax(out, hi);
}

// Exponent range of nonzero BF16 band values: ext[0] = largest biased exponent, ext[1] =
// smallest (a BF16 subnormal counts as exponent 0, which no scale can bring into range).
__global__ void k_band_exp_range(int64_t m, const uint16_t *__restrict__ v, int32_t *__restrict__ ext) {
    int32_t hi = -1, lo = 1 << 30;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t b = v[e] & 0x7fff;
        if (!b) continue;
        const int32_t ex = b >> 7;
        hi = max(hi, ex);
        lo = min(lo, ex);
    }
    // wave-wide max / min first: one pair of atomics per wave
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        hi = max(hi, __shfl_xor(hi, d));
        lo = min(lo, __shfl_xor(lo, d));
    }
    if ((threadIdx.x & 63) == 0 && hi >= 0) {
        atomicMax(&ext[0], hi);
        atomicMin(&ext[1], lo);
    }
}

// BF16 band values -> binary16 of value * 2^shift, exact when the exponent range allows it.
__global__ void k_band_bf16_to_f16(int64_t m, uint16_t *__restrict__ v, int shift) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        v[e] = f32_to_f16_rne(ldexpf(bf16_bits_to_f32(v[e]), shift));
}

__global__ void k_pack_band(int64_t n, int64_t n_bblk, const int64_t *__restrict__ s_off,
                            const int32_t *__restrict__ s_lo, const int32_t *__restrict__ s_len,
                            const double *__restrict__ s_val64, const int64_t *__restrict__ bb_off,
                            const int32_t *__restrict__ bb_lo, const int32_t *__restrict__ bb_w, int dtype,
                            uint8_t *__restrict__ out, double flush) {
    for (int64_t b = blockIdx.x; b < n_bblk; b += gridDim.x) {
        const int64_t cnt = (int64_t)bb_w[b] * kBandRows;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int64_t j = e / kBandRows, i = e - j * kBandRows;
            const int64_t u = b * kBandRows + i, c = bb_lo[b] + j;
            double v = 0.0;
            if (u < n && c >= s_lo[u] && c < s_lo[u] + s_len[u]) v = s_val64[s_off[u] + (c - s_lo[u])];
            if (fabs(v) < flush) v = 0.0;
            const int64_t o = bb_off[b] + e;
            switch (dtype) {
                case QH_F32: ((float *)out)[o] = (float)v; break;
                case QH_F16: ((uint16_t *)out)[o] = f64_to_f16_bits(v); break;
                case QH_BF16: ((uint16_t *)out)[o] = f64_to_bf16_bits(v); break;
            }
        }
    }
}

// Deterministic partial sums of squares (fixed grid, fixed order per block).
// part[b] = sum of v[t] (sq = 0) or v[t]^2 (sq = 1) over block b's contiguous range, in a
// fixed order (a deterministic total once the host adds the parts in order)
__global__ void k_sum_partial(int64_t n, const double *__restrict__ v, double *__restrict__ part, int sq) {
    __shared__ double sh[256];
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    int64_t b = blockIdx.x * per, e = b + per < n ? b + per : n;
    double acc = 0.0;
    for (int64_t t = b + threadIdx.x; t < e; t += blockDim.x) acc += sq ? v[t] * v[t] : v[t];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sumsq_partial(int64_t n, const double *__restrict__ v, double *__restrict__ part) {
    __shared__ double sh[256];
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    int64_t b = blockIdx.x * per, e = b + per < n ? b + per : n;
    double acc = 0.0;
    for (int64_t t = b + threadIdx.x; t < e; t += blockDim.x) acc += v[t] * v[t];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ---- export ----------------------------------------------------------------

__global__ void k_export_csr(int64_t r0, int64_t r1, int64_t n, const int64_t *__restrict__ ptr,
                             const int32_t *__restrict__ col, const double *__restrict__ val,
                             double *__restrict__ out) {
    for (int64_t r = r0 + blockIdx.x; r < r1; r += gridDim.x)
        for (int64_t e = ptr[r] + threadIdx.x; e < ptr[r + 1]; e += blockDim.x)
            out[(r - r0) * n + col[e]] = val[e];
}

__global__ void k_export_tiles(int64_t r0, int64_t r1, int64_t n, const int32_t *__restrict__ t_ptr,
                               const int32_t *__restrict__ t_col, const uint8_t *__restrict__ t_val,
                               int dtype, const float *__restrict__ scale, double *__restrict__ out) {
    for (int64_t r = r0 + blockIdx.x; r < r1; r += gridDim.x) {
        int64_t rt = r / kTile;
        int i = (int)(r - rt * kTile);
        for (int64_t t = t_ptr[rt]; t < t_ptr[rt + 1]; ++t) {
            int64_t ct = t_col[t];
            for (int j = threadIdx.x; j < kTile; j += blockDim.x) {
                int64_t c = ct * kTile + j;
                if (c >= n) continue;
                int64_t o = t * kTileElems + (dtype == QH_F32 ? tile_idx32(i, j) : tile_idx16(i, j));
                double v = 0.0;
                switch (dtype) {
                    case QH_F32: v = ((const float *)t_val)[o]; break;
                    case QH_F16: v = f16_bits_to_f32(((const uint16_t *)t_val)[o]); break;
                    case QH_BF16: v = bf16_bits_to_f32(((const uint16_t *)t_val)[o]); break;
                    // scale holds 256 s_i; the f16 expansion holds code * 2^-8
                    case QH_FP8_ROWSCALE:
                        v = (double)f16_bits_to_f32(e4m3_to_f16_bits_scaled(t_val[o])) * (double)scale[r];
                        break;
                }
                out[(r - r0) * n + c] = v;
            }
        }
    }
}

__device__ inline double load_stored(const uint8_t *p, int64_t e, int dtype) {
    switch (dtype) {
        case QH_F32: return ((const float *)p)[e];
        case QH_F16: return f16_bits_to_f32(((const uint16_t *)p)[e]);
        case QH_BF16: return bf16_bits_to_f32(((const uint16_t *)p)[e]);
    }
    return 0.0;
}

__global__ void k_export_sky(int64_t r0, int64_t r1, int64_t n, const int64_t *__restrict__ s_off,
                             const int32_t *__restrict__ s_lo, const int32_t *__restrict__ s_len,
                             const uint8_t *__restrict__ s_val, const int64_t *__restrict__ l_ptr,
                             const int32_t *__restrict__ l_col, const uint8_t *__restrict__ l_val, int dtype,
                             double *__restrict__ out) {
    for (int64_t r = r0 + blockIdx.x; r < r1; r += gridDim.x) {
        for (int64_t e = threadIdx.x; e < s_len[r]; e += blockDim.x)
            out[(r - r0) * n + s_lo[r] + e] = load_stored(s_val, s_off[r] + e, dtype);
        if (l_ptr)
            for (int64_t e = l_ptr[r] + threadIdx.x; e < l_ptr[r + 1]; e += blockDim.x)
                out[(r - r0) * n + l_col[e]] = load_stored(l_val, e, dtype);
    }
}

// ---- Eq. (15) ---------------------------------------------------------------

__global__ void k_flip_csr(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           double *__restrict__ val, const int8_t *__restrict__ s) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e)
            if (s[r] != s[col[e]]) val[e] = -val[e];
}

__device__ inline void negate_stored(uint8_t *p, int64_t e, int dtype) {
    if (dtype == QH_F32) ((uint32_t *)p)[e] ^= 0x80000000u;
    else ((uint16_t *)p)[e] ^= 0x8000u;
}

__global__ void k_flip_sky(int64_t n, const int64_t *__restrict__ s_off, const int32_t *__restrict__ s_lo,
                           const int32_t *__restrict__ s_len, uint8_t *__restrict__ s_val,
                           const int64_t *__restrict__ l_ptr, const int32_t *__restrict__ l_col,
                           uint8_t *__restrict__ l_val, int dtype, const int8_t *__restrict__ s) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = 0; e < s_len[r]; ++e)
            if (s[r] != s[s_lo[r] + e]) negate_stored(s_val, s_off[r] + e, dtype);
        if (l_ptr)
            for (int64_t e = l_ptr[r]; e < l_ptr[r + 1]; ++e)
                if (s[r] != s[l_col[e]]) negate_stored(l_val, e, dtype);
    }
}

__global__ void k_flip_band(int64_t n, int64_t n_bblk, const int64_t *__restrict__ bb_off,
                            const int32_t *__restrict__ bb_lo, const int32_t *__restrict__ bb_w, uint8_t *__restrict__ val,
                            int dtype, const int8_t *__restrict__ s) {
    for (int64_t b = blockIdx.x; b < n_bblk; b += gridDim.x) {
        const int64_t cnt = (int64_t)bb_w[b] * kBandRows;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            const int64_t j = e / kBandRows, i = e - j * kBandRows;
            const int64_t u = b * kBandRows + i, c = bb_lo[b] + j;
            if (u < n && s[u] != s[c]) negate_stored(val, bb_off[b] + e, dtype);
        }
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

static int grid_for(int64_t n, int block = 256, int64_t cap = 65536) {
    int64_t g = ceil_div(n, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Several host arrays into device buffers with one host-to-device copy: the arrays are
// packed 16-byte aligned behind a table of (destination, offset, bytes), copied in one
// piece and scattered by one kernel, a workgroup per array.  As with any upload, the
// stream is synchronised before the object (which owns the packed host copy and the
// device staging block) goes out of scope.
struct PackSeg {
    uint64_t dst, off, bytes;
};
constexpr int kPackSegs = 16;
constexpr size_t kPackTable = kPackSegs * sizeof(PackSeg);   // a multiple of 16

__global__ void k_scatter(const uint8_t *__restrict__ blob) {
    const PackSeg sg = ((const PackSeg *)blob)[blockIdx.x];
    const uint8_t *src = blob + kPackTable + sg.off;
    uint8_t *dst = (uint8_t *)sg.dst;   // device buffers start 256-byte aligned
    const uint64_t n16 = sg.bytes / 16;
    for (uint64_t i = threadIdx.x; i < n16; i += blockDim.x) ((uint4 *)dst)[i] = ((const uint4 *)src)[i];
    for (uint64_t i = n16 * 16 + threadIdx.x; i < sg.bytes; i += blockDim.x) dst[i] = src[i];
}

class PackedUpload {
  public:
    PackedUpload() : blob_(kPackTable, 0) {}
    PackedUpload(const PackedUpload &) = delete;
    PackedUpload &operator=(const PackedUpload &) = delete;
    // a build that fails between the flush and its caller's synchronisation unwinds
    // through here: wait for the copy before the host and staging blocks are released
    ~PackedUpload() {
        if (st_ && std::uncaught_exceptions()) (void)hipStreamSynchronize(st_);
    }
    template <class T>
    void add(DevBuf<T> &dst, const T *src, size_t count) {
        if (!count) return;
        if (segs_ == kPackSegs) fail(QH_EHIP, "packed upload: more than %d arrays", kPackSegs);
        const size_t bytes = count * sizeof(T);
        const size_t at = (blob_.size() + 15) & ~(size_t)15;
        blob_.resize(at + bytes);
        std::memcpy(blob_.data() + at, src, bytes);
        const PackSeg sg{(uint64_t)(uintptr_t)dst.p, (uint64_t)(at - kPackTable), (uint64_t)bytes};
        std::memcpy(blob_.data() + segs_ * sizeof(PackSeg), &sg, sizeof(sg));
        ++segs_;
    }
    // queues the copy and the scatter on `st`; once per object
    void flush(hipStream_t st) {
        if (!segs_) return;
        st_ = st;
        stage_.alloc(blob_.size());
        QH_HIP(hipMemcpyAsync(stage_.p, blob_.data(), blob_.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)segs_), dim3(256), 0, st, stage_.p);
        QH_CHECK_LAUNCH();
    }

  private:
    std::vector<uint8_t> blob_;
    int segs_ = 0;
    hipStream_t st_ = nullptr;
    DevBuf<uint8_t> stage_;   // (declared last: released first, after the wait above)
};

// Eq. (9) per integer Phred score, q = 1 - 10^(-Q/10) for Q = 0..255: one table per device,
// computed and uploaded once and kept for the life of the process.
static const double *qconf_table() {
    static std::mutex mu;
    static std::map<int, double *> tables;
    int dev = 0;
    QH_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    double *&t = tables[dev];
    if (!t) {
        double h[256];
        for (int q = 0; q < 256; ++q) h[q] = 1.0 - std::pow(10.0, -(double)q / 10.0);
        double *d = nullptr;
        QH_HIP(hipMalloc(&d, sizeof(h)));
        if (hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(d);
            fail(QH_EHIP, "Phred table upload failed");
        }
        t = d;
    }
    return t;
}

static int32_t uf_find(std::vector<int32_t> &p, int32_t x) {
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}


int64_t label_components(int64_t n, std::vector<int32_t> &parent, std::vector<int32_t> &comp) {
    std::vector<int32_t> size(n, 0), label(n, -1);
    for (int64_t i = 0; i < n; ++i) size[uf_find(parent, (int32_t)i)]++;
    comp.assign(n, -1);
    int32_t next = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t r = uf_find(parent, (int32_t)i);
        if (size[r] < 2) continue;
        if (label[r] < 0) label[r] = next++;
        comp[i] = label[r];
    }
    return next;
}

static constexpr int kChunkVerts = 32;

void upload_components(qh_graph *g, const std::vector<int32_t> &comp, int64_t n_comp, hipStream_t st) {
    int64_t n = g->n;
    g->n_comp = n_comp;
    PackedUpload pu;
    g->comp.alloc(n);
    pu.add(g->comp, comp.data(), n);
    std::vector<int32_t> first(n_comp, -1);
    std::vector<int64_t> cnt(n_comp + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        if (comp[i] >= 0) {
            if (first[comp[i]] < 0) first[comp[i]] = (int32_t)i;
            cnt[comp[i] + 1]++;
        }
    g->largest_comp = 0;
    for (int64_t c = 0; c < n_comp; ++c) g->largest_comp = std::max(g->largest_comp, cnt[c + 1]);
    for (int64_t c = 0; c < n_comp; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> order(cnt[n_comp]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        if (comp[i] >= 0) order[fill[comp[i]]++] = (int32_t)i;
    std::vector<int32_t> ccomp, cbeg, cend, cptr(n_comp + 1, 0);
    for (int64_t c = 0; c < n_comp; ++c) {
        cptr[c] = (int32_t)ccomp.size();
        for (int64_t b = cnt[c]; b < cnt[c + 1]; b += kChunkVerts) {
            ccomp.push_back((int32_t)c);
            cbeg.push_back((int32_t)b);
            cend.push_back((int32_t)std::min<int64_t>(b + kChunkVerts, cnt[c + 1]));
        }
    }
    cptr[n_comp] = (int32_t)ccomp.size();
    g->n_chunks = (int64_t)ccomp.size();
    g->comp_first.alloc(n_comp);
    pu.add(g->comp_first, first.data(), n_comp);
    g->n_ord = (int64_t)order.size();
    g->comp_order.alloc(order.size());
    pu.add(g->comp_order, order.data(), order.size());
    g->chunk_comp.alloc(ccomp.size());
    pu.add(g->chunk_comp, ccomp.data(), ccomp.size());
    g->chunk_begin.alloc(cbeg.size());
    pu.add(g->chunk_begin, cbeg.data(), cbeg.size());
    g->chunk_end.alloc(cend.size());
    pu.add(g->chunk_end, cend.data(), cend.size());
    g->comp_chunk_ptr.alloc(n_comp + 1);
    pu.add(g->comp_chunk_ptr, cptr.data(), n_comp + 1);
    pu.flush(st);
    QH_HIP(hipStreamSynchronize(st));  // the packed host copy goes out of scope
}


// ---------------------------------------------------------------------------
// read graph
// ---------------------------------------------------------------------------

// The device-memory cap of a graph: fail with ENOMEM before allocating `more` bytes of
// owned storage when the graph would then exceed it (owned = the buffers counted in
// device_bytes; `have` = what it already owns).
static void charge(const qh_graph *g, int64_t have, int64_t more, const char *what) {
    if (g->max_bytes > 0 && have + more > g->max_bytes)
        fail(QH_ENOMEM, "graph needs more than max_device_bytes = %lld (%s: %lld bytes on top of %lld)",
             (long long)g->max_bytes, what, (long long)more, (long long)have);
}

static void pack_dense_storage(qh_graph *g, const int32_t *W, int negate, hipStream_t st) {
    int64_t F = g->n;
    int64_t n_rt = ceil_div(F, kTile);
    g->n_rt = n_rt;
    DevBuf<uint8_t> occ(n_rt * n_rt);
    if (n_rt > 0) {
        hipLaunchKernelGGL(k_tile_occupancy, dim3((unsigned)n_rt, (unsigned)n_rt), dim3(256), 0, st, F,
                           n_rt, W, occ.p);
        QH_CHECK_LAUNCH();
    }
    auto occ_h = download(occ.p, n_rt * n_rt, st);
    std::vector<int32_t> tptr(n_rt + 1, 0), tcol, trow;
    for (int64_t rt = 0; rt < n_rt; ++rt) {
        tptr[rt] = (int32_t)tcol.size();
        for (int64_t ct = 0; ct < n_rt; ++ct)
            if (occ_h[rt * n_rt + ct]) { tcol.push_back((int32_t)ct); trow.push_back((int32_t)rt); }
    }
    tptr[n_rt] = (int32_t)tcol.size();
    g->n_tiles = (int64_t)tcol.size();
    PackedUpload pu;
    g->t_ptr.alloc(n_rt + 1);
    pu.add(g->t_ptr, tptr.data(), n_rt + 1);
    g->t_col.alloc(tcol.size());
    pu.add(g->t_col, tcol.data(), tcol.size());
    DevBuf<int32_t> trow_d(trow.size());
    pu.add(trow_d, trow.data(), trow.size());
    pu.flush(st);
    charge(g, (int64_t)(g->m_ptr.bytes() + g->m_col.bytes() + g->m_val.bytes()),
           std::max<int64_t>(g->n_tiles, 1) * kTileElems * dtype_bytes(g->dtype), "dense tiles");
    g->t_val.alloc((size_t)std::max<int64_t>(g->n_tiles, 1) * kTileElems * dtype_bytes(g->dtype));
    if (g->dtype == QH_FP8_ROWSCALE) {
        DevBuf<double> rmax(F);
        DevBuf<float> scale(F);
        g->row_scale.alloc(F);
        if (F) {
            hipLaunchKernelGGL(k_row_absmax, dim3(grid_for(F, 4)), dim3(256), 0, st, F, g->m_ptr.p, g->m_val.p,
                               rmax.p);
            hipLaunchKernelGGL(k_fp8_scales, dim3(grid_for(F)), dim3(256), 0, st, F, rmax.p, scale.p,
                               g->row_scale.p);
            QH_CHECK_LAUNCH();
        }
        if (g->n_tiles) {
            hipLaunchKernelGGL(k_pack_tiles, dim3((unsigned)g->n_tiles), dim3(256), 0, st, F, W, negate,
                               trow_d.p, g->t_col.p, g->dtype, scale.p, g->t_val.p);
            QH_CHECK_LAUNCH();
        }
        QH_HIP(hipStreamSynchronize(st));
    } else if (g->n_tiles) {
        hipLaunchKernelGGL(k_pack_tiles, dim3((unsigned)g->n_tiles), dim3(256), 0, st, F, W, negate, trow_d.p,
                           g->t_col.p, g->dtype, (const float *)nullptr, g->t_val.p);
        QH_CHECK_LAUNCH();
        QH_HIP(hipStreamSynchronize(st));
    } else {
        QH_HIP(hipStreamSynchronize(st));   // the uploads' host vectors go out of scope
    }
}

// Observation count (frag_ptr[F]) and validation of the fragment CSR on the device; only
// the count and four error words come back to the host.
static int64_t validate_fragments(const qh_reads *r, int32_t S, hipStream_t st) {
    const int64_t F = r->n_frag;
    int64_t nobs = 0;
    if (F > 0) {
        DevBuf<unsigned long long> err(6);
        QH_HIP(hipMemsetAsync(err.p, 0xFF, 4 * sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_validate_frags, dim3(grid_for(F, 4)), dim3(256), 0, st, F, r->frag_ptr, r->snp, r->allele,
                           S, err.p);
        QH_CHECK_LAUNCH();
        unsigned long long eh[6];
        QH_HIP(hipMemcpyAsync(eh, err.p, sizeof(eh), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
        nobs = (int64_t)eh[4];
        if ((int64_t)eh[5] != 0) fail(QH_EINVAL, "frag_ptr[0] must be 0");
        if (nobs < 0) fail(QH_EINVAL, "frag_ptr decreases");
        if (nobs > INT32_MAX) fail(QH_EUNSUPPORTED, "more than 2^31 observations");
        if (eh[0] != ~0ull) fail(QH_EINVAL, "frag_ptr decreases at fragment %llu", eh[0] - 1);
        if (eh[1] != ~0ull) fail(QH_EINVAL, "fragment %llu: SNP index out of range", eh[1] - 1);
        if (eh[2] != ~0ull) fail(QH_EINVAL, "fragment %llu: SNP indices not strictly ascending", eh[2] - 1);
        if (eh[3] != ~0ull) fail(QH_EINVAL, "fragment %llu: allele must be 0 or 1", eh[3] - 1);
    }

    return nobs;
}

void build_read_graph(qh_graph *g, const qh_reads *r, const qh_snps *s, hipStream_t st) {
    int64_t F = r->n_frag;
    int32_t S = s->n_snp;
    if (F > 46340) fail(QH_EUNSUPPORTED, "dense read graphs are limited to 46340 fragments");
    g->n = F;
    g->integer = true;
    const int64_t nobs = validate_fragments(r, S, st);

    // encode, then per-SNP coverage lists (fragments ascending): a stable sort of the
    // observations by SNP keeps the fragment order inside every list
    DevBuf<int8_t> M(nobs);
    g->cov_ptr.alloc(S + 1);
    g->cov_frag.alloc(nobs);
    g->cov_M.alloc(nobs);
    g->init_h1.alloc(S);
    DevBuf<int32_t> keys_out;   // SNP of every position of the sorted observations
    if (nobs) {
        hipLaunchKernelGGL(k_encode, dim3(grid_for(std::max<int64_t>(nobs, S))), dim3(256), 0, st, nobs, r->snp,
                           r->allele, s->init_h1, M.p, (int64_t)S, g->init_h1.p);
        keys_out.alloc(nobs);
        DevBuf<int32_t> obs_frag(nobs), obs_idx(nobs), vals_out(nobs);
        hipLaunchKernelGGL(k_obs_frag, dim3(grid_for(F)), dim3(256), 0, st, F, r->frag_ptr, obs_frag.p, obs_idx.p);
        QH_CHECK_LAUNCH();
        int bits = 1;
        while (bits < 31 && (1ll << bits) < (int64_t)S) ++bits;
        size_t tmp_bytes = 0;
        QH_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, (const int32_t *)r->snp, keys_out.p,
                                         (const int32_t *)obs_idx.p, vals_out.p, (size_t)nobs, 0, bits, st));
        DevBuf<uint8_t> tmp(std::max<size_t>(tmp_bytes, 1));
        QH_HIP(rocprim::radix_sort_pairs(tmp.p, tmp_bytes, (const int32_t *)r->snp, keys_out.p,
                                         (const int32_t *)obs_idx.p, vals_out.p, (size_t)nobs, 0, bits, st));
        hipLaunchKernelGGL(k_cov_ptr, dim3(grid_for(S + 1)), dim3(256), 0, st, S, nobs, keys_out.p, g->cov_ptr.p);
        hipLaunchKernelGGL(k_cov_fill, dim3(grid_for(nobs)), dim3(256), 0, st, nobs, vals_out.p, obs_frag.p, M.p,
                           g->cov_frag.p, g->cov_M.p);
        QH_CHECK_LAUNCH();
        QH_HIP(hipStreamSynchronize(st));   // sort scratch is released on scope exit
    } else {
        g->cov_ptr.zero(st);
    }

    // components: fragments sharing a SNP are linked (device union-find, root = smallest
    // fragment, so the labels follow the order of each component's first fragment)
    std::vector<int32_t> parent(F);
    if (F) {
        DevBuf<int32_t> par(F);
        hipLaunchKernelGGL(k_uf_init, dim3(grid_for(F)), dim3(256), 0, st, F, par.p);
        if (nobs > 1)
            hipLaunchKernelGGL(k_uf_link, dim3(grid_for(nobs)), dim3(256), 0, st, nobs, keys_out.p, g->cov_frag.p,
                               par.p);
        hipLaunchKernelGGL(k_uf_flatten, dim3(grid_for(F)), dim3(256), 0, st, F, par.p);
        QH_CHECK_LAUNCH();
        QH_HIP(hipMemcpyAsync(parent.data(), par.p, F * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
    }
    std::vector<int32_t> comp;
    int64_t n_comp = label_components(F, parent, comp);
    upload_components(g, comp, n_comp, st);

    if (S && !nobs) QH_HIP(hipMemcpyAsync(g->init_h1.p, s->init_h1, S, hipMemcpyDeviceToDevice, st));

    // Eqs. (2)-(3) into a dense int32 matrix
    int conflict = g->kind == QH_READ_CONFLICT;
    DevBuf<int32_t> W((size_t)std::max<int64_t>(F * F, 1));
    if (F && F <= kRowLdsMaxF) {   // every row written whole
        if (F * (int64_t)sizeof(int32_t) > 65536)
            QH_HIP(hipFuncSetAttribute((const void *)k_read_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kRowLdsMaxF * sizeof(int32_t))));
        hipLaunchKernelGGL(k_read_rows, dim3((unsigned)std::min<int64_t>(F, 1 << 20)), dim3(256),
                           (unsigned)(F * sizeof(int32_t)), st, F, r->frag_ptr, r->snp, M.p, g->cov_ptr.p,
                           g->cov_frag.p, g->cov_M.p, W.p, conflict);
        QH_CHECK_LAUNCH();
    } else {
        W.zero(st);
        if (S && F) {
            hipLaunchKernelGGL(k_read_pairs, dim3((unsigned)std::min<int64_t>(S, 1 << 20)), dim3(256), 0, st, S,
                               g->cov_ptr.p, g->cov_frag.p, g->cov_M.p, W.p, F, conflict);
            QH_CHECK_LAUNCH();
        }
    }
    // master CSR (J = -A for the conflict kind)
    DevBuf<int64_t> cnt(F);
    int waves_per_block = 4;
    if (F) {
        hipLaunchKernelGGL(k_dense_row_nnz, dim3((unsigned)ceil_div(F, waves_per_block)), dim3(256), 0, st, F,
                           W.p, cnt.p);
        QH_CHECK_LAUNCH();
    }
    auto cnt_h = download(cnt.p, F, st);
    std::vector<int64_t> ptr(F + 1, 0);
    for (int64_t i = 0; i < F; ++i) ptr[i + 1] = ptr[i] + cnt_h[i];
    g->nnz = ptr[F];
    charge(g, 0, (F + 1) * 8 + g->nnz * 12, "FP64 master weights");
    g->m_ptr.alloc(F + 1);
    g->m_ptr.upload(ptr.data(), F + 1, st);
    g->m_col.alloc(g->nnz);
    g->m_val.alloc(g->nnz);
    if (F) {
        hipLaunchKernelGGL(k_dense_row_fill, dim3((unsigned)ceil_div(F, waves_per_block)), dim3(256), 0, st, F,
                           W.p, conflict, g->m_ptr.p, g->m_col.p, g->m_val.p);
        QH_CHECK_LAUNCH();
    }
    pack_dense_storage(g, W.p, conflict, st);
    QH_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// SNP graph
// ---------------------------------------------------------------------------

void build_snp_graph(qh_graph *g, const qh_reads *r, const qh_snps *s, int linkage_k, int band_limit,
                     hipStream_t st) {
    int64_t F = r->n_frag;
    int32_t n = s->n_snp;
    g->n = n;
    g->integer = false;
    g->band_limit = band_limit;
    const int64_t nobs = validate_fragments(r, n, st);

    // kept observations (Phred > 3), per fragment in SNP order
    DevBuf<int64_t> kept_ptr_d(F + 1);
    int64_t n_kept = 0;
    {
        DevBuf<int64_t> kcnt(F + 1);
        hipLaunchKernelGGL(k_kept_count, dim3(grid_for(F + 1)), dim3(256), 0, st, F, r->frag_ptr, r->phred, kcnt.p);
        QH_CHECK_LAUNCH();
        size_t tb = 0;
        QH_HIP(rocprim::exclusive_scan(nullptr, tb, kcnt.p, kept_ptr_d.p, (int64_t)0, (size_t)(F + 1),
                                       rocprim::plus<int64_t>(), st));
        DevBuf<uint8_t> tmp(std::max<size_t>(tb, 1));
        QH_HIP(rocprim::exclusive_scan(tmp.p, tb, kcnt.p, kept_ptr_d.p, (int64_t)0, (size_t)(F + 1),
                                       rocprim::plus<int64_t>(), st));
        QH_HIP(hipMemcpyAsync(&n_kept, kept_ptr_d.p + F, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
    }
    DevBuf<int64_t> kept_obs_d(n_kept);
    DevBuf<int32_t> kept_frag_d(n_kept);
    if (n_kept) {
        hipLaunchKernelGGL(k_kept_fill, dim3(grid_for(F)), dim3(256), 0, st, F, r->frag_ptr, r->phred, kept_ptr_d.p,
                           kept_obs_d.p, kept_frag_d.p);
        QH_CHECK_LAUNCH();
    }

    // structure on the device: skyline extents, components, long-range pair set
    std::vector<int32_t> lo(n), hi(n), parent(n);
    int64_t l_nnz = 0;
    {
        // one buffer (and one copy back): the pair counter, lo, hi and the parents
        DevBuf<int32_t> sb(3 * (size_t)n + 2);
        unsigned long long *lrc = (unsigned long long *)sb.p;   // device blocks are 256-byte aligned
        int32_t *lo_p = sb.p + 2, *hi_p = lo_p + n, *uf_p = hi_p + n;
        hipLaunchKernelGGL(k_structure_init, dim3(grid_for(3 * (int64_t)n + 2)), dim3(256), 0, st, (int64_t)n,
                           sb.p);
        QH_CHECK_LAUNCH();
        if (n_kept) {
            hipLaunchKernelGGL(k_snp_structure, dim3(grid_for(n_kept)), dim3(256), 0, st, n_kept, kept_obs_d.p,
                               kept_frag_d.p, kept_ptr_d.p, r->snp, linkage_k, (int32_t)band_limit, (int64_t)n,
                               lo_p, hi_p, uf_p, lrc, (uint64_t *)nullptr, 0);
            QH_CHECK_LAUNCH();
        }
        if (n) {
            hipLaunchKernelGGL(k_uf_flatten, dim3(grid_for(n)), dim3(256), 0, st, (int64_t)n, uf_p);
            QH_CHECK_LAUNCH();
        }
        std::vector<int32_t> sh(3 * (size_t)n + 2);
        QH_HIP(hipMemcpyAsync(sh.data(), sb.p, sh.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
        unsigned long long n_lr_pairs = 0;
        std::memcpy(&n_lr_pairs, sh.data(), sizeof(n_lr_pairs));
        std::copy(sh.begin() + 2, sh.begin() + 2 + n, lo.begin());
        std::copy(sh.begin() + 2 + n, sh.begin() + 2 + 2 * (size_t)n, hi.begin());
        std::copy(sh.begin() + 2 + 2 * (size_t)n, sh.end(), parent.begin());
        // long-range keys u n + v of both directions, sorted and unique
        const int64_t n_dir = 2 * (int64_t)n_lr_pairs;
        g->l_ptr.alloc(n + 1);
        if (n_dir) {
            DevBuf<uint64_t> keys(n_dir), sorted(n_dir), uniq(n_dir);
            QH_HIP(hipMemsetAsync(lrc, 0, sizeof(unsigned long long), st));
            hipLaunchKernelGGL(k_snp_structure, dim3(grid_for(n_kept)), dim3(256), 0, st, n_kept, kept_obs_d.p,
                               kept_frag_d.p, kept_ptr_d.p, r->snp, linkage_k, (int32_t)band_limit, (int64_t)n,
                               lo_p, hi_p, uf_p, lrc, keys.p, 1);
            QH_CHECK_LAUNCH();
            int bits = 1;
            while (bits < 64 && ((uint64_t)1 << bits) < (uint64_t)n * (uint64_t)n) ++bits;
            size_t tb = 0;
            QH_HIP(rocprim::radix_sort_keys(nullptr, tb, keys.p, sorted.p, (size_t)n_dir, 0, bits, st));
            DevBuf<uint8_t> tmp(std::max<size_t>(tb, 1));
            QH_HIP(rocprim::radix_sort_keys(tmp.p, tb, keys.p, sorted.p, (size_t)n_dir, 0, bits, st));
            DevBuf<size_t> n_unique(1);
            size_t tu = 0;
            QH_HIP(rocprim::unique(nullptr, tu, sorted.p, uniq.p, n_unique.p, (size_t)n_dir,
                                   rocprim::equal_to<uint64_t>(), st));
            DevBuf<uint8_t> tmp2(std::max<size_t>(tu, 1));
            QH_HIP(rocprim::unique(tmp2.p, tu, sorted.p, uniq.p, n_unique.p, (size_t)n_dir,
                                   rocprim::equal_to<uint64_t>(), st));
            size_t nu = 0;
            QH_HIP(hipMemcpyAsync(&nu, n_unique.p, sizeof(size_t), hipMemcpyDeviceToHost, st));
            QH_HIP(hipStreamSynchronize(st));
            l_nnz = (int64_t)nu;
            g->l_col.alloc(l_nnz);
            hipLaunchKernelGGL(k_lr_csr, dim3(grid_for(std::max<int64_t>(n + 1, l_nnz))), dim3(256), 0, st,
                               (int64_t)n, l_nnz, uniq.p, g->l_ptr.p, g->l_col.p);
            QH_CHECK_LAUNCH();
            QH_HIP(hipStreamSynchronize(st));   // sort scratch is released on scope exit
        } else {
            g->l_ptr.zero(st);
            g->l_col.alloc(0);
        }
    }
    g->l_nnz = l_nnz;
    std::vector<int32_t> comp;
    int64_t n_comp = label_components(n, parent, comp);
    upload_components(g, comp, n_comp, st);

    std::vector<int64_t> off(n);
    std::vector<int32_t> len(n);
    int64_t slots = 0;
    for (int32_t u = 0; u < n; ++u) {
        off[u] = slots;
        len[u] = hi[u] - lo[u] + 1;
        slots += len[u];
    }
    g->s_slots = slots;
    std::vector<int64_t> lptr(n + 1, 0);
    if (l_nnz) lptr = download(g->l_ptr.p, n + 1, st);

    // long-range rows split into chunks of at most kHubChunk entries (chunks tile the
    // long-range entries in row order); consecutive chunks grouped into packets of at most
    // 64 entries, one wave each
    {
        std::vector<int32_t> rptr(n + 1, 0), pk;
        std::vector<int64_t> cbeg, cend;
        int64_t pk_entries = 0;
        for (int32_t u = 0; u < n; ++u) {
            for (int64_t b = lptr[u]; b < lptr[u + 1]; b += kHubChunk) {
                const int64_t e = std::min<int64_t>(b + kHubChunk, lptr[u + 1]);
                if (pk.empty() || pk_entries + (e - b) > 64) {
                    pk.push_back((int32_t)cbeg.size());
                    pk_entries = 0;
                }
                pk_entries += e - b;
                cbeg.push_back(b);
                cend.push_back(e);
            }
            rptr[u + 1] = (int32_t)cbeg.size();
        }
        pk.push_back((int32_t)cbeg.size());
        g->n_hub_chunks = (int64_t)cbeg.size();
        g->n_lr_pk = (int64_t)pk.size() - 1;
        PackedUpload pu;
        g->row_chunk_ptr.alloc(n + 1);
        pu.add(g->row_chunk_ptr, rptr.data(), n + 1);
        g->hub_chunk_beg.alloc(cbeg.size());
        pu.add(g->hub_chunk_beg, cbeg.data(), cbeg.size());
        g->hub_chunk_end.alloc(cend.size());
        pu.add(g->hub_chunk_end, cend.data(), cend.size());
        g->lr_pk_ptr.alloc(pk.size());
        pu.add(g->lr_pk_ptr, pk.data(), pk.size());
        pu.flush(st);
        QH_HIP(hipStreamSynchronize(st));
    }

    // device structure (the packed copy lives to the end of the build, past its last sync)
    PackedUpload pu_sky;
    g->s_off.alloc(n);
    pu_sky.add(g->s_off, off.data(), n);
    g->s_lo.alloc(n);
    pu_sky.add(g->s_lo, lo.data(), n);
    g->s_len.alloc(n);
    pu_sky.add(g->s_len, len.data(), n);
    pu_sky.flush(st);
    const double *qconf = qconf_table();

    DevBuf<int8_t> M(nobs);
    g->init_h1.alloc(n);
    if (nobs || n) {
        hipLaunchKernelGGL(k_encode, dim3(grid_for(std::max<int64_t>(nobs, n))), dim3(256), 0, st, nobs, r->snp,
                           r->allele, s->init_h1, M.p, (int64_t)n, g->init_h1.p);
        QH_CHECK_LAUNCH();
    }

    DevBuf<double> s_val64(slots), l_val64(l_nnz);
    s_val64.zero(st);
    l_val64.zero(st);
    if (n_kept) {
        DevBuf<int32_t> clamped(1);
        clamped.zero(st);
        hipLaunchKernelGGL(k_snp_pairs, dim3(grid_for(F, 4, 1 << 20)), dim3(256), 0, st, F,
                           kept_obs_d.p, kept_ptr_d.p, r->snp, M.p, r->phred, r->alpha, qconf,
                           linkage_k, (int32_t)band_limit, g->s_off.p, g->s_lo.p, s_val64.p, g->l_ptr.p,
                           g->l_col.p, l_val64.p, g->deterministic, clamped.p);
        QH_CHECK_LAUNCH();
        if (g->deterministic) {
            if (download(clamped.p, 1, st)[0])
                fail(QH_ENUMERIC, "deterministic build: an Eq. (14) term reaches 2^20 in magnitude, beyond the "
                                  "fixed-point range (build with deterministic = 0)");
            if (slots) hipLaunchKernelGGL(k_fixed_to_f64, dim3(grid_for(slots)), dim3(256), 0, st, (int64_t)slots,
                                          s_val64.p);
            if (l_nnz) hipLaunchKernelGGL(k_fixed_to_f64, dim3(grid_for(l_nnz)), dim3(256), 0, st, (int64_t)l_nnz,
                                          l_val64.p);
            QH_CHECK_LAUNCH();
        }
    }
    // master CSR
    DevBuf<int64_t> cnt(n);
    const int64_t *lp = l_nnz ? g->l_ptr.p : nullptr;
    if (n) {
        hipLaunchKernelGGL(k_sky_row_nnz, dim3(grid_for(n)), dim3(256), 0, st, (int64_t)n, g->s_off.p, g->s_len.p,
                           s_val64.p, lp, l_val64.p, cnt.p);
        QH_CHECK_LAUNCH();
    }
    auto cnt_h = download(cnt.p, n, st);
    std::vector<int64_t> mptr(n + 1, 0);
    for (int32_t u = 0; u < n; ++u) mptr[u + 1] = mptr[u] + cnt_h[u];
    g->nnz = mptr[n];
    charge(g, 0, ((int64_t)n + 1) * 8 + g->nnz * 12, "FP64 master weights");
    g->m_ptr.alloc(n + 1);
    g->m_ptr.upload(mptr.data(), n + 1, st);
    g->m_col.alloc(g->nnz);
    g->m_val.alloc(g->nnz);
    if (n) {
        hipLaunchKernelGGL(k_sky_row_fill, dim3(grid_for(n)), dim3(256), 0, st, (int64_t)n, g->s_off.p, g->s_lo.p,
                           g->s_len.p, s_val64.p, lp, g->l_col.p, l_val64.p, g->m_ptr.p, g->m_col.p, g->m_val.p);
        QH_CHECK_LAUNCH();
    }
    // storage copy.  BF16 storage flushes magnitudes below 2^(E - 31), E the exponent of the
    // largest |weight|, to zero: such entries are FP64 rounding residue of Eq. 14 sums whose
    // terms cancel (or weights 2^-31 of the largest and below), and without them every BF16
    // value fits one scaled binary16 encoding of the band (32 binades).
    int eb = dtype_bytes(g->dtype);
    double flush = 0.0;
    if (g->dtype == QH_BF16 && (slots || l_nnz)) {
        DevBuf<unsigned long long> mx(1);
        mx.zero(st);
        if (slots)
            hipLaunchKernelGGL(k_absmax_bits, dim3(grid_for(slots)), dim3(256), 0, st, slots, s_val64.p, mx.p);
        if (l_nnz)
            hipLaunchKernelGGL(k_absmax_bits, dim3(grid_for(l_nnz)), dim3(256), 0, st, l_nnz, l_val64.p, mx.p);
        QH_CHECK_LAUNCH();
        unsigned long long bits = 0;
        QH_HIP(hipMemcpyAsync(&bits, mx.p, sizeof(bits), hipMemcpyDeviceToHost, st));
        QH_HIP(hipStreamSynchronize(st));
        double wmax;
        std::memcpy(&wmax, &bits, sizeof(wmax));
        if (wmax > 0.0) {
            int ex = 0;
            std::frexp(wmax, &ex);                 // wmax = f * 2^ex, f in [0.5, 1)
            flush = std::ldexp(1.0, ex - 1 - 31);
        }
    }
    g->snp_flush = flush;
    g->s_val.alloc((size_t)slots * eb);
    g->l_val.alloc((size_t)std::max<int64_t>(l_nnz, 1) * eb);
    if (slots) {
        hipLaunchKernelGGL(k_quantize, dim3(grid_for(slots)), dim3(256), 0, st, slots, s_val64.p, g->dtype,
                           g->s_val.p, flush);
        QH_CHECK_LAUNCH();
    }
    if (l_nnz) {
        hipLaunchKernelGGL(k_quantize, dim3(grid_for(l_nnz)), dim3(256), 0, st, l_nnz, l_val64.p, g->dtype,
                           g->l_val.p, flush);
        QH_CHECK_LAUNCH();
    }
    // band blocks for the register-tiled step kernel
    {
        const int64_t nb = ceil_div(n, kBandRows);
        std::vector<int32_t> blo(nb), bw(nb);
        std::vector<int64_t> boff(nb + 1, 0);
        for (int64_t b = 0; b < nb; ++b) {
            int32_t L = INT32_MAX, H = -1;
            for (int64_t u = b * kBandRows; u < std::min<int64_t>(n, (b + 1) * kBandRows); ++u) {
                L = std::min(L, lo[u]);
                H = std::max(H, hi[u]);
            }
            blo[b] = L;
            bw[b] = H - L + 1;
            boff[b + 1] = boff[b] + (int64_t)bw[b] * kBandRows;
        }
        g->n_bblk = nb;
        g->bb_elems = boff[nb];
        PackedUpload pu;
        g->bb_off.alloc(nb + 1);
        pu.add(g->bb_off, boff.data(), nb + 1);
        g->bb_lo.alloc(nb);
        pu.add(g->bb_lo, blo.data(), nb);
        g->bb_w.alloc(nb);
        pu.add(g->bb_w, bw.data(), nb);
        pu.flush(st);
        charge(g, (int64_t)(g->m_ptr.bytes() + g->m_col.bytes() + g->m_val.bytes()),
               std::max<int64_t>(boff[nb], 1) * eb, "band blocks");
        g->bb_val.alloc((size_t)std::max<int64_t>(boff[nb], 1) * eb);
        g->bb_dtype = g->dtype;
        if (nb) {
            hipLaunchKernelGGL(k_pack_band, dim3((unsigned)std::min<int64_t>(nb, 1 << 20)), dim3(256), 0, st,
                               (int64_t)n, nb, g->s_off.p, g->s_lo.p, g->s_len.p, s_val64.p, g->bb_off.p, g->bb_lo.p,
                               g->bb_w.p, g->dtype, g->bb_val.p, flush);
            QH_CHECK_LAUNCH();
            if (g->dtype == QH_BF16) {
                // a BF16 value 1.m x 2^E (7 fraction bits) is exact in binary16 after scaling by
                // 2^s when E + s <= 15 and E - 7 + s >= -24: one s serves every value when the
                // exponents span at most 32 binades; take the largest such s
                const int32_t init[2] = {-1, 1 << 30};
                DevBuf<int32_t> ext(2);
                ext.upload(init, 2, st);
                hipLaunchKernelGGL(k_band_exp_range, dim3(grid_for(boff[nb])), dim3(256), 0, st, boff[nb],
                                   (const uint16_t *)g->bb_val.p, ext.p);
                QH_CHECK_LAUNCH();
                int32_t hl[2];
                QH_HIP(hipMemcpyAsync(hl, ext.p, sizeof(hl), hipMemcpyDeviceToHost, st));
                QH_HIP(hipStreamSynchronize(st));
                const int e_max = hl[0] - 127, e_min = hl[1] - 127;
                if (hl[0] < 0) {
                    g->bb_dtype = QH_F16;          // all zeros
                } else if (hl[1] > 0 && e_max - e_min <= 32 && e_max >= -45 && e_max <= 75) {
                    const int shift = 15 - e_max;       // |shift| <= 60: the scale stays a normal float
                    hipLaunchKernelGGL(k_band_bf16_to_f16, dim3(grid_for(boff[nb])), dim3(256), 0, st, boff[nb],
                                       (uint16_t *)g->bb_val.p, shift);
                    QH_CHECK_LAUNCH();
                    g->bb_dtype = QH_F16;
                    g->bb_scale = std::ldexp(1.0f, -shift);
                }
            }
        }
        QH_HIP(hipStreamSynchronize(st));   // the uploads' host vectors go out of scope
    }
    QH_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// shared finishing steps
// ---------------------------------------------------------------------------

// W = -1/2 sum_ab J_ab over the master values (Eq. 5: E(s) = W - 2 cut(s)), summed in a fixed
// order (1,024 strided partials, then the partials in index order), so equal weights give an
// equal W bit for bit.
static void refresh_total_weight(qh_graph *g, hipStream_t st) {
    g->total_weight = 0.0;
    if (!g->nnz) return;
    const int parts = 1024;
    DevBuf<double> part(parts);
    hipLaunchKernelGGL(k_sum_partial, dim3(parts), dim3(256), 0, st, g->nnz, g->m_val.p, part.p, 0);
    QH_CHECK_LAUNCH();
    auto pw = download(part.p, parts, st);
    double sj = 0.0;
    for (double v : pw) sj += v;
    g->total_weight = -0.5 * sj;
}

void finalize_graph(qh_graph *g, hipStream_t st) {
    // W (as refresh_total_weight), c0 = 0.5 / (sigma sqrt(n)) with sigma^2 = sum J^2 /
    // (n (n - 1)), and the greedy tolerance of float weights: the partial sums and row sums
    // of all three come back in one copy
    const int parts = 1024;
    const int64_t nrs = (!g->integer && g->n) ? g->n : 0;
    g->total_weight = 0.0;
    if (g->nnz || nrs) {
        DevBuf<double> buf(2 * parts + nrs);
        if (g->nnz) {
            hipLaunchKernelGGL(k_sum_partial, dim3(parts), dim3(256), 0, st, g->nnz, g->m_val.p, buf.p, 0);
            hipLaunchKernelGGL(k_sumsq_partial, dim3(parts), dim3(256), 0, st, g->nnz, g->m_val.p, buf.p + parts);
        }
        if (nrs)
            hipLaunchKernelGGL(k_row_abssum, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->m_ptr.p, g->m_val.p,
                               buf.p + 2 * parts);
        QH_CHECK_LAUNCH();
        auto h = download(buf.p, (size_t)(2 * parts + nrs), st);
        if (g->nnz) {
            double sj = 0.0, ss = 0.0;
            for (int i = 0; i < parts; ++i) sj += h[i];
            for (int i = 0; i < parts; ++i) ss += h[parts + i];
            g->total_weight = -0.5 * sj;
            if (ss > 0.0 && g->n >= 2) {
                double sigma = std::sqrt(ss / ((double)g->n * (double)(g->n - 1)));
                g->c0_auto = 0.5 / (sigma * std::sqrt((double)g->n));
            }
        }
        if (nrs) {
            double m = 0.0;
            for (int64_t i = 0; i < nrs; ++i) m = std::max(m, h[2 * parts + i]);
            g->greedy_eps = 1e-12 * m;
        }
    }
    g->device_bytes = (int64_t)(g->m_ptr.bytes() + g->m_col.bytes() + g->m_val.bytes() + g->comp.bytes() +
                                g->comp_first.bytes() + g->comp_order.bytes() + g->chunk_comp.bytes() +
                                g->chunk_begin.bytes() + g->chunk_end.bytes() + g->comp_chunk_ptr.bytes() +
                                g->t_ptr.bytes() + g->t_col.bytes() + g->t_val.bytes() +
                                g->row_scale.bytes() + g->s_off.bytes() + g->s_lo.bytes() + g->s_len.bytes() +
                                g->s_val.bytes() + g->bb_off.bytes() + g->bb_lo.bytes() + g->bb_w.bytes() +
                                g->bb_val.bytes() + g->l_ptr.bytes() + g->l_col.bytes() + g->l_val.bytes() +
                                g->row_chunk_ptr.bytes() + g->hub_chunk_beg.bytes() + g->hub_chunk_end.bytes() +
                                g->lr_pk_ptr.bytes() + g->cov_ptr.bytes() + g->cov_frag.bytes() +
                                g->cov_M.bytes() + g->init_h1.bytes());
    charge(g, g->device_bytes, 0, "the finished graph");
}

void export_master_rows(const qh_graph *g, int64_t r0, int64_t r1, double *out, hipStream_t st) {
    if (r1 <= r0) return;
    QH_HIP(hipMemsetAsync(out, 0, (size_t)(r1 - r0) * g->n * sizeof(double), st));
    hipLaunchKernelGGL(k_export_csr, dim3((unsigned)std::min<int64_t>(r1 - r0, 65536)), dim3(256), 0, st, r0,
                       r1, g->n, g->m_ptr.p, g->m_col.p, g->m_val.p, out);
    QH_CHECK_LAUNCH();
}

void export_stored_rows(const qh_graph *g, int64_t r0, int64_t r1, double *out, hipStream_t st) {
    if (r1 <= r0) return;
    QH_HIP(hipMemsetAsync(out, 0, (size_t)(r1 - r0) * g->n * sizeof(double), st));
    unsigned grid = (unsigned)std::min<int64_t>(r1 - r0, 65536);
    if (g->storage == QH_STORE_DENSE) {
        if (!g->n_tiles) return;
        hipLaunchKernelGGL(k_export_tiles, dim3(grid), dim3(64), 0, st, r0, r1, g->n, g->t_ptr.p, g->t_col.p,
                           g->t_val.p, g->dtype, g->row_scale.p, out);
    } else {
        hipLaunchKernelGGL(k_export_sky, dim3(grid), dim3(64), 0, st, r0, r1, g->n, g->s_off.p, g->s_lo.p,
                           g->s_len.p, g->s_val.p, g->l_nnz ? g->l_ptr.p : nullptr, g->l_col.p, g->l_val.p,
                           g->dtype, out);
    }
    QH_CHECK_LAUNCH();
}

void flip_crossing(qh_graph *g, const int8_t *spins, hipStream_t st) {
    if (g->storage != QH_STORE_SKYLINE) fail(QH_EUNSUPPORTED, "flip_crossing is offered on SNP graphs");
    if (!g->n) return;
    hipLaunchKernelGGL(k_flip_csr, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->m_ptr.p, g->m_col.p,
                       g->m_val.p, spins);
    hipLaunchKernelGGL(k_flip_sky, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->s_off.p, g->s_lo.p,
                       g->s_len.p, g->s_val.p, g->l_nnz ? g->l_ptr.p : nullptr, g->l_col.p, g->l_val.p, g->dtype,
                       spins);
    if (g->n_bblk)
        hipLaunchKernelGGL(k_flip_band, dim3((unsigned)std::min<int64_t>(g->n_bblk, 1 << 20)), dim3(256), 0, st,
                           g->n, g->n_bblk, g->bb_off.p, g->bb_lo.p, g->bb_w.p, g->bb_val.p, g->bb_dtype, spins);
    QH_CHECK_LAUNCH();
    // the flipped edges change W = -1/2 sum J (by twice their old weight); c0 depends on J^2
    // only and the greedy tolerance on |J|, so they stay.  Solve plans hold no copy of J.
    refresh_total_weight(g, st);
}

}  // namespace qh

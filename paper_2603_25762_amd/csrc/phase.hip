// Haplotype reconstruction from spins.
//  Read graphs: per-SNP vote counts of Eqs. (7)-(8) and the hierarchical rule of
//  "Consistency processing", written in closed form: with d_l = c_l^+ - c_l^-,
//  the subset with the larger |d_l| (S1 on ties) keeps its majority and the other
//  subset takes the complement; d_1 = d_2 = 0 filters the SNP.  Opposing
//  majorities and one-sided majorities are special cases of the same rule.
//  SNP graphs: one parity round, Eqs. (16)-(17).
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace qh {

// Counters of qh_phase_noalloc: the s = +1 and s = -1 vertex counts of up to
// kNoAllocMaxComp components, in device memory that the library never allocates at run
// time.  Each device holds its own copy for the life of the process; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr int64_t kNoAllocMaxComp = (int64_t)1 << 19;
static __device__ __align__(256) int32_t scratch[2 * kNoAllocMaxComp];

__global__ void k_phase_vote(int32_t n_snp, const int64_t *__restrict__ cov_ptr, const int32_t *__restrict__ cov_frag,
                             const int8_t *__restrict__ cov_M, const int32_t *__restrict__ comp,
                             const int8_t *__restrict__ spins, const uint8_t *__restrict__ init_h1,
                             int8_t *__restrict__ h1, int32_t *__restrict__ block) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_snp;
         j += (int64_t)gridDim.x * blockDim.x) {
        int d1 = 0, d2 = 0, blk = -1;
        for (int64_t p = cov_ptr[j]; p < cov_ptr[j + 1]; ++p) {
            int f = cov_frag[p];
            int c = comp[f];
            if (c < 0) continue;
            blk = c;
            int m = cov_M[p];
            if (spins[f] > 0) d1 += m; else d2 += m;
        }
        block[j] = blk;
        const int H1 = init_h1[j], H2 = 1 - H1;
        if (d1 == 0 && d2 == 0) { h1[j] = -1; continue; }
        int a1 = d1 < 0 ? -d1 : d1, a2 = d2 < 0 ? -d2 : d2;
        if (a1 >= a2) h1[j] = (int8_t)(d1 > 0 ? H1 : H2);
        else h1[j] = (int8_t)(d2 > 0 ? H2 : H1);
    }
}

__global__ void k_comp_sizes(int64_t n, const int32_t *__restrict__ comp, const int8_t *__restrict__ spins,
                             int32_t *__restrict__ plus, int32_t *__restrict__ minus) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        int c = comp[u];
        if (c < 0) continue;
        if (spins[u] > 0) atomicAdd(&plus[c], 1); else atomicAdd(&minus[c], 1);
    }
}

__global__ void k_phase_parity(int64_t n, const int32_t *__restrict__ comp, const int8_t *__restrict__ spins,
                               const int32_t *__restrict__ plus, const int32_t *__restrict__ minus,
                               const uint8_t *__restrict__ init_h1, int8_t *__restrict__ h1,
                               int32_t *__restrict__ block) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        int c = comp[u];
        if (c < 0) { h1[u] = -1; block[u] = -1; continue; }
        int smin = plus[c] < minus[c] ? 1 : -1;   // equal sizes: the s = -1 subset swaps
        int C = spins[u] == smin ? 1 : 0;
        h1[u] = (int8_t)((C & 1) ? 1 - init_h1[u] : init_h1[u]);
        block[u] = c;
    }
}

static int grid_for(int64_t n) {
    int64_t g = ceil_div(n, 256);
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

__global__ void k_zero_counts(int64_t n, int32_t *__restrict__ p) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Device address of `scratch` on device `dev`, looked up once per device with that device
// current (the symbol's host-side name is not a device address).
static int32_t *scratch_on(int dev) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static int32_t *addr[kMaxDevices] = {nullptr};
    if (dev < 0 || dev >= kMaxDevices) fail(QH_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        QH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        addr[dev] = (int32_t *)p;
    }
    return addr[dev];
}

void phase_noalloc(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block, hipStream_t st) {
    if (g->kind != QH_SNP_LLR) {   // the vote uses no scratch memory
        phase(g, spins, h1, block, st);
        return;
    }
    if (g->n_comp > kNoAllocMaxComp)
        fail(QH_EINVAL, "qh_phase_noalloc holds counters for at most %lld components, the graph has %lld",
             (long long)kNoAllocMaxComp, (long long)g->n_comp);
    int dev = 0;
    QH_HIP(hipGetDevice(&dev));
    if (dev != g->device) fail(QH_EINVAL, "graph lives on device %d, current device is %d", g->device, dev);
    int32_t *cnt = scratch_on(dev);
    if (!g->n) return;
    const int64_t nc = std::max<int64_t>(g->n_comp, 1);
    // the counters keep the previous call's values: clear them (a kernel, so that a captured
    // stream records no memset node)
    hipLaunchKernelGGL(k_zero_counts, dim3(grid_for(2 * nc)), dim3(256), 0, st, 2 * nc, cnt);
    hipLaunchKernelGGL(k_comp_sizes, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->comp.p, spins, cnt, cnt + nc);
    hipLaunchKernelGGL(k_phase_parity, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->comp.p, spins, cnt, cnt + nc,
                       g->init_h1.p, h1, block);
    QH_CHECK_LAUNCH();
}

void phase(const qh_graph *g, const int8_t *spins, int8_t *h1, int32_t *block, hipStream_t st) {
    if (g->kind != QH_SNP_LLR) {
        if (!g->n_snp) return;
        hipLaunchKernelGGL(k_phase_vote, dim3(grid_for(g->n_snp)), dim3(256), 0, st, g->n_snp, g->cov_ptr.p,
                           g->cov_frag.p, g->cov_M.p, g->comp.p, spins, g->init_h1.p, h1, block);
        QH_CHECK_LAUNCH();
        return;
    }
    if (!g->n) return;
    DevBuf<int32_t> cnt(2 * std::max<int64_t>(g->n_comp, 1));
    cnt.zero(st);
    hipLaunchKernelGGL(k_comp_sizes, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->comp.p, spins, cnt.p,
                       cnt.p + std::max<int64_t>(g->n_comp, 1));
    hipLaunchKernelGGL(k_phase_parity, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, g->comp.p, spins, cnt.p,
                       cnt.p + std::max<int64_t>(g->n_comp, 1), g->init_h1.p, h1, block);
    QH_CHECK_LAUNCH();
    QH_HIP(hipStreamSynchronize(st));  // cnt is released on return
}

}  // namespace qh

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

// ---------------------------------------------------------------------------
// many graphs in one call: the spins of a batched solve in, every block's haplotype out
// ---------------------------------------------------------------------------

struct PhaseDesc {
    int kind;                 // 0: read graph (vote), 1: SNP graph (parity)
    int64_t n, n_snp;
    const int64_t *cov_ptr;
    const int32_t *cov_frag;
    const int8_t *cov_M;
    const int32_t *comp;
    const uint8_t *init_h1;
    int64_t spin_off, snp_off, cnt_off, n_cnt;   // packed offsets of spins, outputs and counters
};

// work item = (block, first index): 256 SNPs (vote) or vertices (counts, parity) of one block
__global__ void k_phase_vote_batched(const PhaseDesc *__restrict__ D, const int2 *__restrict__ items,
                                     const int8_t *__restrict__ spins, int8_t *__restrict__ h1,
                                     int32_t *__restrict__ block) {
    const int2 it = items[blockIdx.x];
    const PhaseDesc &d = D[it.x];
    const int64_t j = (int64_t)it.y + threadIdx.x;
    if (j >= d.n_snp) return;
    // the same rule as k_phase_vote, on the block's own arrays
    int d1 = 0, d2 = 0, blk = -1;
    const int8_t *sp = spins + d.spin_off;
    for (int64_t p = d.cov_ptr[j]; p < d.cov_ptr[j + 1]; ++p) {
        const int f = d.cov_frag[p];
        const int c = d.comp[f];
        if (c < 0) continue;
        blk = c;
        const int m = d.cov_M[p];
        if (sp[f] > 0) d1 += m; else d2 += m;
    }
    block[d.snp_off + j] = blk;
    const int H1 = d.init_h1[j], H2 = 1 - H1;
    int8_t out;
    if (d1 == 0 && d2 == 0) {
        out = -1;
    } else {
        const int a1 = d1 < 0 ? -d1 : d1, a2 = d2 < 0 ? -d2 : d2;
        if (a1 >= a2) out = (int8_t)(d1 > 0 ? H1 : H2);
        else out = (int8_t)(d2 > 0 ? H2 : H1);
    }
    h1[d.snp_off + j] = out;
}

__global__ void k_comp_sizes_batched(const PhaseDesc *__restrict__ D, const int2 *__restrict__ items,
                                     const int8_t *__restrict__ spins, int32_t *__restrict__ cnt) {
    const int2 it = items[blockIdx.x];
    const PhaseDesc &d = D[it.x];
    const int64_t u = (int64_t)it.y + threadIdx.x;
    if (u >= d.n) return;
    const int c = d.comp[u];
    if (c < 0) return;
    int32_t *plus = cnt + d.cnt_off, *minus = plus + d.n_cnt;
    if (spins[d.spin_off + u] > 0) atomicAdd(&plus[c], 1); else atomicAdd(&minus[c], 1);
}

__global__ void k_phase_parity_batched(const PhaseDesc *__restrict__ D, const int2 *__restrict__ items,
                                       const int8_t *__restrict__ spins, const int32_t *__restrict__ cnt,
                                       int8_t *__restrict__ h1, int32_t *__restrict__ block) {
    const int2 it = items[blockIdx.x];
    const PhaseDesc &d = D[it.x];
    const int64_t u = (int64_t)it.y + threadIdx.x;
    if (u >= d.n) return;
    const int c = d.comp[u];
    const int64_t o = d.snp_off + u;
    if (c < 0) { h1[o] = -1; block[o] = -1; return; }
    const int32_t *plus = cnt + d.cnt_off, *minus = plus + d.n_cnt;
    const int smin = plus[c] < minus[c] ? 1 : -1;   // equal sizes: the s = -1 subset swaps
    const int C = spins[d.spin_off + u] == smin ? 1 : 0;
    h1[o] = (int8_t)((C & 1) ? 1 - d.init_h1[u] : d.init_h1[u]);
    block[o] = c;
}

void phase_batched(const qh_graph *const *gs, int nb, const int8_t *spins, int8_t *h1, int32_t *block,
                   hipStream_t st) {
    int dev = 0;
    QH_HIP(hipGetDevice(&dev));
    std::vector<PhaseDesc> desc(nb);
    std::vector<int2> vote, verts;
    int64_t spin_off = 0, snp_off = 0, cnt_off = 0;
    for (int b = 0; b < nb; ++b) {
        const qh_graph *g = gs[b];
        if (!g) fail(QH_EINVAL, "graph %d is null", b);
        if (g->device != dev) fail(QH_EINVAL, "graph %d lives on device %d, current device is %d", b, g->device, dev);
        PhaseDesc &d = desc[b];
        d.kind = g->kind == QH_SNP_LLR ? 1 : 0;
        d.n = g->n;
        d.n_snp = g->n_snp;
        d.cov_ptr = g->cov_ptr.p;
        d.cov_frag = g->cov_frag.p;
        d.cov_M = g->cov_M.p;
        d.comp = g->comp.p;
        d.init_h1 = g->init_h1.p;
        d.spin_off = spin_off;
        d.snp_off = snp_off;
        d.n_cnt = std::max<int64_t>(g->n_comp, 1);
        d.cnt_off = d.kind ? cnt_off : 0;
        if (d.kind) {
            cnt_off += 2 * d.n_cnt;
            for (int64_t u = 0; u < g->n; u += 256) verts.push_back(make_int2(b, (int)u));
        } else {
            for (int64_t j = 0; j < g->n_snp; j += 256) vote.push_back(make_int2(b, (int)j));
        }
        spin_off += g->n;
        snp_off += g->n_snp;
    }
    if (vote.size() > (size_t)INT32_MAX || verts.size() > (size_t)INT32_MAX)
        fail(QH_EUNSUPPORTED, "too many phasing work items in one call");
    DevBuf<PhaseDesc> d_desc(nb);
    d_desc.upload(desc.data(), nb, st);
    DevBuf<int2> d_vote(std::max<size_t>(vote.size(), 1)), d_verts(std::max<size_t>(verts.size(), 1));
    d_vote.upload(vote.data(), vote.size(), st);
    d_verts.upload(verts.data(), verts.size(), st);
    DevBuf<int32_t> cnt(std::max<int64_t>(cnt_off, 1));
    if (cnt_off) hipLaunchKernelGGL(k_zero_counts, dim3(grid_for(cnt_off)), dim3(256), 0, st, cnt_off, cnt.p);
    if (!vote.empty())
        hipLaunchKernelGGL(k_phase_vote_batched, dim3((unsigned)vote.size()), dim3(256), 0, st, d_desc.p, d_vote.p,
                           spins, h1, block);
    if (!verts.empty()) {
        hipLaunchKernelGGL(k_comp_sizes_batched, dim3((unsigned)verts.size()), dim3(256), 0, st, d_desc.p,
                           d_verts.p, spins, cnt.p);
        hipLaunchKernelGGL(k_phase_parity_batched, dim3((unsigned)verts.size()), dim3(256), 0, st, d_desc.p,
                           d_verts.p, spins, cnt.p, h1, block);
    }
    QH_CHECK_LAUNCH();
    QH_HIP(hipStreamSynchronize(st));   // the tables and counters are released on return
}

}  // namespace qh

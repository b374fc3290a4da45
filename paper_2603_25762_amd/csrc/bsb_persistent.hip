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
//
// The kernel template is in persistent_kernel.h; this file holds the plan builder and
// the launches without a field, bsb_persistent_field.hip the launches with one.
#include <algorithm>
#include <cstring>
#include <vector>

#include "formats.h"
#include "internal.h"
#include "persistent.h"
#include "persistent_kernel.h"
#include "partition.h"

namespace qh {
// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

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
    if (n_rt * 8 * (int64_t)R >= ((int64_t)1 << 32)) return false;   // 16-byte piece offsets are 32-bit
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
        // contiguous partition whose busiest workgroup has the least work (two units per
        // stored tile for its loads and MFMAs, one per row tile for the update and publish:
        // the weighting measured fastest on the read graphs, against 1:1 and 1:0); the
        // fewest row tiles per workgroup on a tie, which selects the kernel with the smaller
        // register budget
        std::vector<int64_t> work(n_rt + 1, 0);
        for (int64_t rt = 0; rt < n_rt; ++rt) work[rt + 1] = work[rt] + 2 * (tptr[rt + 1] - tptr[rt]) + 1;
        std::vector<int32_t> wg_rt;
        int64_t best_b = -1;
        for (int L : {2, 4, kMaxT}) {
            std::vector<int32_t> cut = partition_rows(work, n_rt, wpg, L);
            if (cut.empty()) continue;
            int64_t b = 0;
            for (int w = 0; w < wpg; ++w) b = std::max(b, work[cut[w + 1]] - work[cut[w]]);
            if (best_b < 0 || b < best_b) { best_b = b; wg_rt = cut; }
        }
        if (wg_rt.empty()) continue;
        bool ok = true;
        std::vector<int32_t> owner(n_rt);
        for (int w = 0; w < wpg; ++w)
            for (int32_t rt = wg_rt[w]; rt < wg_rt[w + 1]; ++rt) owner[rt] = w;
        std::vector<int32_t> ct_ptr(wpg + 1, 0), cts, slot(g->n_tiles), nbr_ptr(wpg + 1, 0), nbrs;
        int64_t lds_max_j = 0, lds_max_h = 0, max_tiles = 0, max_ct = 0;
        int max_t = 0;
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
            max_tiles = std::max<int64_t>(max_tiles, tptr[wg_rt[w + 1]] - tptr[wg_rt[w]]);
            max_ct = std::max<int64_t>(max_ct, (int64_t)u.size());
            max_t = std::max(max_t, wg_rt[w + 1] - wg_rt[w]);
            lds_max_j = std::max(lds_max_j, jb);
            lds_max_h = std::max(lds_max_h, (int64_t)u.size() * ct_bytes);
        }
        ct_ptr[wpg] = (int32_t)cts.size();
        nbr_ptr[wpg] = (int32_t)nbrs.size();
        lds_max_j = ceil_div(lds_max_j, 16) * 16;
        const int64_t lds_tab = ceil_div((max_tiles + 2 * max_ct) * 4, 16) * 16;   // slot and column-tile tables
        if (!ok || lds_max_j + lds_max_h + lds_tab > kLdsLimit) continue;
        // upload
        pp.RT = RT;
        pp.ng = ng;
        pp.wpg = wpg;
        pp.lds_j_bytes = lds_max_j;
        pp.lds_tab_off = lds_max_j + lds_max_h;
        pp.lds_bytes = lds_max_j + lds_max_h + lds_tab;
        pp.max_wg_tiles = (int32_t)max_tiles;
        pp.max_ct = (int32_t)max_ct;
        pp.max_t = max_t;
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

void launch_persistent(const qh_graph *g, const PersistPlan &pp, const PersistArgs &args, int coherent,
                       hipStream_t st) {
    if (args.field) launch_persistent_field(g, pp, args, coherent, st);
    else launch_persistent_fld<0>(g, pp, args, coherent, st);
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

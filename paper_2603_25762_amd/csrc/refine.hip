// Iterative refinement of the SNP-based method (Eqs. 15-17).
//
// Round t solves the current graph with seed + t and reads the per-component cut of the
// selected spins s (after greedy).  A component is finished for good when that cut is not
// positive or s puts all of its vertices on one side; in every other component the
// vertices of the smaller subset (the s = -1 subset on a tie) add one to their flip
// counter C, and every edge crossing the partition changes sign (Eq. 15).  Haplotype 1
// takes H1 where C is even and H2 where C is odd (Eqs. 16-17).
//
// Adaptive deformation (Methods, SNP-based solution): while a component that is still
// being refined has a negative cut in round t, the round is solved again (up to
// deform_tries times, same seed) with a deformation field h_i = (deform / c0) (2 u_i - 1),
// u_i uniform on [0, 1) from SplitMix64 with the round's seed at draw 2 n R + (a - 1) n + i
// for attempt a (the draws after those of the initial state).  The force c0 h_i it adds to
// y' is at most deform in magnitude, against a0 = 1 for the pump terms.  A component with
// a negative cut takes the attempt's spins when their cut is higher; the other components
// keep the plain solve.
//
// The sign flips compose: after rounds with effective partitions s_1 .. s_T the weights
// are w_uv * S_u * S_v with S = s_1 * .. * s_T (elementwise), so the original graph is
// restored exactly by one more flip with S.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace qh {

__global__ void k_ref_counts(int64_t n, const int32_t *__restrict__ comp, const int8_t *__restrict__ s,
                             int32_t *__restrict__ plus, int32_t *__restrict__ minus) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int c = comp[u];
        if (c < 0) continue;
        if (s[u] > 0) atomicAdd(&plus[c], 1);
        else atomicAdd(&minus[c], 1);
    }
}

// active[c]: 0 = component left alone this round, else the spin value of its S_min
__global__ void k_ref_apply(int64_t n, const int32_t *__restrict__ comp, const int8_t *__restrict__ s,
                            const int8_t *__restrict__ active, int32_t *__restrict__ C, int8_t *__restrict__ s_eff,
                            int8_t *__restrict__ s_tot) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int c = comp[u];
        const int a = c < 0 ? 0 : active[c];
        if (a == 0) {
            s_eff[u] = 1;
            continue;
        }
        s_eff[u] = s[u];
        if (s[u] == a) C[u] += 1;
        s_tot[u] = (int8_t)(s_tot[u] * s[u]);
    }
}

__global__ void k_ref_phase(int64_t n, const int32_t *__restrict__ comp, const int32_t *__restrict__ C,
                            const uint8_t *__restrict__ init_h1, int8_t *__restrict__ h1, int32_t *__restrict__ block) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int c = comp[u];
        if (c < 0) {
            h1[u] = -1;
            block[u] = -1;
            continue;
        }
        h1[u] = (int8_t)((C[u] & 1) ? 1 - init_h1[u] : init_h1[u]);
        block[u] = c;
    }
}

// deformation field of attempt a: h_i = scale (2 u_i - 1), u_i from draw k0 + i
__global__ void k_ref_field(int64_t n, uint64_t seed, uint64_t k0, double scale, float *__restrict__ h) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)(sm64_draw(seed, k0 + (uint64_t)u) >> 11) * 0x1.0p-53;
        h[u] = (float)(scale * (2.0 * v - 1.0));
    }
}

// dst[u] = src[u] for the vertices of components with take[c] set
__global__ void k_ref_take(int64_t n, const int32_t *__restrict__ comp, const int8_t *__restrict__ take,
                           const int8_t *__restrict__ src, int8_t *__restrict__ dst) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int c = comp[u];
        if (c >= 0 && take[c]) dst[u] = src[u];
    }
}

__global__ void k_fill_i8(int64_t n, int8_t v, int8_t *__restrict__ p) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        p[u] = v;
}

static int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 65536)); }

void refine(qh_graph *g, const qh_bsb_opts *o, int max_rounds, float deform, int deform_tries, int8_t *h1,
            int32_t *block, int32_t *flips, double *round_cuts, int32_t *rounds_out, int32_t *deformed_out,
            hipStream_t st) {
    if (g->kind != QH_SNP_LLR) fail(QH_EUNSUPPORTED, "refinement applies to SNP graphs");
    if (max_rounds < 1) fail(QH_EINVAL, "max_rounds must be >= 1");
    if (!(deform >= 0.0f) || deform_tries < 0) fail(QH_EINVAL, "deform and deform_tries must be >= 0");
    if (!o->init) fail(QH_EINVAL, "every refinement round starts from the seeded state (init = 1)");
    const int64_t n = g->n, nc = g->n_comp;
    const int R = o->replicas;
    const bool deforming = deform > 0.0f && deform_tries > 0;
    DevBuf<int8_t> best(n), s_eff(n), s_tot(n), active(nc), best2(deforming ? n : 0), take(deforming ? nc : 0);
    DevBuf<float> field(deforming ? n : 0);
    DevBuf<int32_t> C(n), cnt(2 * std::max<int64_t>(nc, 1));
    const double c0 = o->c0 > 0.0 ? o->c0 : g->c0_auto;
    DevBuf<double> cuts(R), best_cut(1), sel_cut(1);
    C.zero(st);
    hipLaunchKernelGGL(k_fill_i8, dim3(grid_of(n)), dim3(256), 0, st, n, (int8_t)1, s_tot.p);
    QH_CHECK_LAUNCH();
    std::vector<char> done(nc, 0);
    std::vector<double> cut_c(nc);
    std::vector<int32_t> pm(2 * nc);
    std::vector<int8_t> act(nc), tk(nc);
    std::vector<double> cut2(nc);
    int rounds = 0, deformed = 0;
    try {
        for (int t = 0; t < max_rounds; ++t) {
            if (std::all_of(done.begin(), done.end(), [](char d) { return d != 0; })) break;
            qh_bsb_opts ot = *o;
            ot.seed = o->seed + (uint64_t)t;
            ot.readout = 1;
            ot.step_begin = 0;
            ot.step_end = 0;
            qh_result r{};
            r.best_spins = best.p;
            r.cuts = cuts.p;
            r.best_cut = best_cut.p;
            r.selected_cut = sel_cut.p;
            bsb_solve(g, &ot, &r, st);
            if (!nc) break;
            // per-component cut of the selected spins on the current graph, and subset sizes
            SolvePlan &p = solve_plan(g, R, st);
            QH_HIP(hipMemcpyAsync(cut_c.data(), p.cut1.p, nc * sizeof(double), hipMemcpyDeviceToHost, st));
            QH_HIP(hipStreamSynchronize(st));
            // adaptive deformation: solve the round again under a field while a component
            // being refined has a negative cut
            for (int a = 1; deforming && a <= deform_tries; ++a) {
                bool neg = false;
                for (int64_t c = 0; c < nc; ++c) neg |= !done[c] && cut_c[c] < 0.0;
                if (!neg) break;
                hipLaunchKernelGGL(k_ref_field, dim3(grid_of(n)), dim3(256), 0, st, n, ot.seed,
                                   2ull * (uint64_t)n * (uint64_t)R + (uint64_t)(a - 1) * (uint64_t)n,
                                   (double)deform / c0, field.p);
                QH_CHECK_LAUNCH();
                qh_bsb_opts od = ot;
                od.field = field.p;
                qh_result r2{};
                r2.best_spins = best2.p;
                r2.cuts = cuts.p;
                r2.best_cut = best_cut.p;
                r2.selected_cut = sel_cut.p;
                bsb_solve(g, &od, &r2, st);
                ++deformed;
                QH_HIP(hipMemcpyAsync(cut2.data(), p.cut1.p, nc * sizeof(double), hipMemcpyDeviceToHost, st));
                QH_HIP(hipStreamSynchronize(st));
                bool any_take = false;
                for (int64_t c = 0; c < nc; ++c) {
                    tk[c] = !done[c] && cut_c[c] < 0.0 && cut2[c] > cut_c[c];
                    if (tk[c]) { cut_c[c] = cut2[c]; any_take = true; }
                }
                if (!any_take) continue;
                QH_HIP(hipMemcpyAsync(take.p, tk.data(), nc, hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_ref_take, dim3(grid_of(n)), dim3(256), 0, st, n, g->comp.p, take.p, best2.p,
                                   best.p);
                QH_CHECK_LAUNCH();
                QH_HIP(hipStreamSynchronize(st));   // tk is reused by the next attempt
            }
            cnt.zero(st);
            hipLaunchKernelGGL(k_ref_counts, dim3(grid_of(n)), dim3(256), 0, st, n, g->comp.p, best.p, cnt.p,
                               cnt.p + nc);
            QH_CHECK_LAUNCH();
            QH_HIP(hipMemcpyAsync(pm.data(), cnt.p, 2 * nc * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            QH_HIP(hipStreamSynchronize(st));
            double applied = 0.0;
            bool any = false;
            for (int64_t c = 0; c < nc; ++c) {
                act[c] = 0;
                if (done[c]) continue;
                const int32_t plus = pm[c], minus = pm[nc + c];
                if (cut_c[c] <= 0.0 || plus == 0 || minus == 0) {
                    done[c] = 1;
                    continue;
                }
                act[c] = plus < minus ? 1 : -1;
                applied += cut_c[c];
                any = true;
            }
            if (!any) break;
            QH_HIP(hipMemcpyAsync(active.p, act.data(), nc, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_ref_apply, dim3(grid_of(n)), dim3(256), 0, st, n, g->comp.p, best.p, active.p, C.p,
                               s_eff.p, s_tot.p);
            QH_CHECK_LAUNCH();
            flip_crossing(g, s_eff.p, st);
            if (round_cuts) round_cuts[rounds] = applied;
            ++rounds;
        }
    } catch (...) {
        if (rounds) {
            try { flip_crossing(g, s_tot.p, st); } catch (...) {}
        }
        throw;
    }
    if (rounds) flip_crossing(g, s_tot.p, st);   // back to the caller's weights
    if (n) {
        hipLaunchKernelGGL(k_ref_phase, dim3(grid_of(n)), dim3(256), 0, st, n, g->comp.p, C.p, g->init_h1.p, h1,
                           block);
        QH_CHECK_LAUNCH();
        if (flips) QH_HIP(hipMemcpyAsync(flips, C.p, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
    if (rounds_out) *rounds_out = rounds;
    if (deformed_out) *deformed_out = deformed;
    QH_HIP(hipStreamSynchronize(st));   // scratch buffers are released on return
}

}  // namespace qh

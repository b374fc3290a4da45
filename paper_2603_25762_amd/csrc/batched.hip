// Many independent phasing blocks (connected components / regions) solved with
// one schedule.  Each block keeps its own couplings, c0 and readout.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace qh {

void bsb_solve_batched(const qh_graph *const *gs, int nb, const qh_bsb_opts *o, qh_batched_result *res,
                       hipStream_t st) {
    const int R = o->replicas;
    int64_t voff = 0;
    for (int b = 0; b < nb; ++b) {
        const qh_graph *g = gs[b];
        qh_result r{};
        r.best_spins = res->best_spins + voff;
        r.cuts = res->cuts + (int64_t)b * R;
        r.best_cut = res->best_cut + b;
        r.selected_cut = res->selected_cut ? res->selected_cut + b : nullptr;
        r.x = res->x ? res->x + voff * R : nullptr;
        r.y = res->y ? res->y + voff * R : nullptr;
        qh_bsb_opts ob = *o;
        ob.readout = 1;
        bsb_solve(g, &ob, &r, st);
        voff += g->n;
    }
}

}  // namespace qh

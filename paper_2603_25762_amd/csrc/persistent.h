// Persistent dense bSB plan (tables built once per graph and replica count).
#pragma once

#include "internal.h"

namespace qh {

struct PersistArgs {
    int64_t n;
    int R, kb, ke, ng, wpg;
    const int32_t *wg_rt;       // [wpg + 1] first row tile of each workgroup
    const int32_t *t_ptr;       // tile CSR of the graph
    const uint8_t *t_val;
    const float *row_scale;     // FP8 decode scales (256 s_i)
    const int32_t *wg_ct_ptr;   // [wpg + 1] column tiles referenced by each workgroup
    const int32_t *wg_ct;
    const int32_t *tile_slot;   // [n_tiles] slot of each tile's column tile in its workgroup's list
    const int32_t *nbr_ptr;     // [wpg + 1] neighbour workgroups (other owners of those column tiles)
    const int32_t *nbr;
    float *x, *y;               // [n][R] state in / out
    uint16_t *h0, *h1;          // double-buffered 16-bit copy of x, layout [n_pad/8][R][8]
    int *flags;                 // [ng][wpg] steps published
    int *err;                   // nonzero when a wait gave up
    float c0, dt, a0;
    const float *pump;
    int discrete;               // 1: the 16-bit copy holds sgn(x) (discrete variant)
    const float *field;         // deformation field h [n] added to the coupling sum (nullptr: none)
    int64_t lds_j_bytes;
    int64_t lds_tab_off;        // LDS offset of the tables: slots of the own stored tiles [max_wg_tiles],
                                // then the column tiles staged from memory and their slots [max_ct] each
    int32_t max_wg_tiles;       // most stored tiles of one workgroup
    int32_t max_ct;             // most column tiles of one workgroup
    int64_t max_polls;
};

struct PersistPlan {
    bool ok = false;
    int RT = 0, ng = 0, wpg = 0;
    int max_t = 0;              // most row tiles of one workgroup (selects the kernel's register budget)
    int32_t max_wg_tiles = 0, max_ct = 0;
    int64_t lds_j_bytes = 0, lds_tab_off = 0, lds_bytes = 0;
    DevBuf<int32_t> wg_rt, wg_ct_ptr, wg_ct, tile_slot, nbr_ptr, nbr;
    DevBuf<int> flags;          // ng * wpg flags followed by the error word
};

bool build_persistent_plan(const qh_graph *g, int R, PersistPlan &pp, hipStream_t st);
// coherent = 1 selects the variant whose copy-of-x traffic uses device-coherent accesses
// instead of cache-wide fences (both give identical results)
void launch_persistent(const qh_graph *g, const PersistPlan &pp, const PersistArgs &args, int coherent,
                       hipStream_t st);
// the same with args.field set (the kernels that add the deformation field)
void launch_persistent_field(const qh_graph *g, const PersistPlan &pp, const PersistArgs &args, int coherent,
                             hipStream_t st);

}  // namespace qh

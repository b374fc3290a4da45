// The persistent dense bSB kernel with a deformation field (instantiations only).
#include "persistent_kernel.h"

namespace qh {

void launch_persistent_field(const qh_graph *g, const PersistPlan &pp, const PersistArgs &args, int coherent,
                             hipStream_t st) {
    launch_persistent_fld<1>(g, pp, args, coherent, st);
}

}  // namespace qh

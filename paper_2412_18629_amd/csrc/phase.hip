// phase.hip -- hierarchical 6D phase-space FoF (placeholder until the
// device pipeline lands).
#include <stdlib.h>

#include "common.h"

namespace rs {

int phase_run(const float*, const float*, const float*, const float*, const float*,
              const float*, int64_t, float, const int32_t*, int32_t, int32_t, double, uint32_t,
              const void*, rs_tree**, hipStream_t) {
    return RS_ENOTIMPL;
}

void tree_release(rs_tree* t) {
    if (!t) return;
    free(t);
}

}  // namespace rs

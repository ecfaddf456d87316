// blocked.hip -- Level-2 blocked sweeps (Section 6.4) and the FP32 warm-up.
#include "solver.hpp"

namespace ghsvd {

void carve_blocked(Carver &c, const Plan &pl, PencilWs &w) {
    (void)c;
    (void)pl;
    w.blk = nullptr;
    w.blk_bytes = 0;
}

int run_fp32_stage(const Plan &, const PencilWs &, int, const ghsvd_options &, ghsvd_info &,
                   hipStream_t) {
    return GHSVD_EINVAL;
}

int run_blocked_fp64(const Plan &, const PencilWs &, int, const ghsvd_options &, ghsvd_info &,
                     hipStream_t) {
    return GHSVD_EINVAL;
}

}  // namespace ghsvd

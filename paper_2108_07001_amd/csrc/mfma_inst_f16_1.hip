// mfma_inst_f16_1.hip -- instances of the matrix-core demapping kernels
// (half-precision splits, D = 5..8); split across files so that hipcc runs in parallel.
#include "mfma_wide.h"

namespace air {
#define AIR_MFMA_INST(D) \
  hipError_t launch_mfma_f16_d##D(const DemapArgs& a, const void* rec, int g, const Launch& l, int part) { \
    return launch_mfma_wide_td<D, false>(a, rec, g, l, part); \
  }
AIR_MFMA_INST(5)
AIR_MFMA_INST(6)
AIR_MFMA_INST(7)
AIR_MFMA_INST(8)
#undef AIR_MFMA_INST
}  // namespace air

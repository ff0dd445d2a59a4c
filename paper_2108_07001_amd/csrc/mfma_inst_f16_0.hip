// mfma_inst_f16_0.hip -- instances of the matrix-core demapping kernels
// (half-precision splits, D = 1..4); split across files so that hipcc runs in parallel.
#include "mfma_wide.h"

namespace air {
#define AIR_MFMA_INST(D) \
  hipError_t launch_mfma_f16_d##D(const DemapArgs& a, const void* rec, int g, const Launch& l, int part) { \
    return launch_mfma_wide_td<D, false>(a, rec, g, l, part); \
  }
AIR_MFMA_INST(1)
AIR_MFMA_INST(2)
AIR_MFMA_INST(3)
AIR_MFMA_INST(4)
#undef AIR_MFMA_INST
}  // namespace air

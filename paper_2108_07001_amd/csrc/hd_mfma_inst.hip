// hd_mfma_inst.hip -- instances of the matrix-core hard-decision kernel (D = 1..16).
#include "hd_mfma.h"

namespace air {
#define AIR_HD_MFMA_INST(D)                                                                        \
  hipError_t launch_hd_mfma_d##D(const HdArgs& a, const void* rec, float r2, int g, hipStream_t s) { \
    return launch_hd_mfma_d<D>(a, rec, r2, g, s);                                                  \
  }
AIR_HD_MFMA_INST(1)
AIR_HD_MFMA_INST(2)
AIR_HD_MFMA_INST(3)
AIR_HD_MFMA_INST(4)
AIR_HD_MFMA_INST(5)
AIR_HD_MFMA_INST(6)
AIR_HD_MFMA_INST(7)
AIR_HD_MFMA_INST(8)
AIR_HD_MFMA_INST(9)
AIR_HD_MFMA_INST(10)
AIR_HD_MFMA_INST(11)
AIR_HD_MFMA_INST(12)
AIR_HD_MFMA_INST(13)
AIR_HD_MFMA_INST(14)
AIR_HD_MFMA_INST(15)
AIR_HD_MFMA_INST(16)
#undef AIR_HD_MFMA_INST
}  // namespace air

// hd_inst.hip -- instances of the hard-decision kernel (D = 1..16).
#include "hd_kernels.h"

namespace air {
#define AIR_HD_INST(D) \
  hipError_t launch_hd_d##D(const HdArgs& a, int g, hipStream_t s) { return launch_hd_d<D>(a, g, s); }
AIR_HD_INST(1)
AIR_HD_INST(2)
AIR_HD_INST(3)
AIR_HD_INST(4)
AIR_HD_INST(5)
AIR_HD_INST(6)
AIR_HD_INST(7)
AIR_HD_INST(8)
AIR_HD_INST(9)
AIR_HD_INST(10)
AIR_HD_INST(11)
AIR_HD_INST(12)
AIR_HD_INST(13)
AIR_HD_INST(14)
AIR_HD_INST(15)
AIR_HD_INST(16)
#undef AIR_HD_INST
}  // namespace air

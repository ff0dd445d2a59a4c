// vec_inst_f64_3.hip -- instances of the vector demapping kernels
// (double, D = 13..16); split across files so that hipcc runs in parallel.
#include "vec_kernels.h"

namespace air {
#define AIR_VEC_INST(D) \
  hipError_t launch_vec_f64_d##D(const DemapArgs& a, int g, const Launch& l, bool ml, int part) { \
    return launch_vec_td<double, D>(a, g, l, ml, part); \
  }
AIR_VEC_INST(13)
AIR_VEC_INST(14)
AIR_VEC_INST(15)
AIR_VEC_INST(16)
#undef AIR_VEC_INST
}  // namespace air

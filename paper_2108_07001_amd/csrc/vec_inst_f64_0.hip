// vec_inst_f64_0.hip -- instances of the vector demapping kernels
// (double, D = 1..4); split across files so that hipcc runs in parallel.
#include "vec_kernels.h"

namespace air {
#define AIR_VEC_INST(D) \
  hipError_t launch_vec_f64_d##D(const DemapArgs& a, int g, const Launch& l, bool ml, int part) { \
    return launch_vec_td<double, D>(a, g, l, ml, part); \
  }
AIR_VEC_INST(1)
AIR_VEC_INST(2)
AIR_VEC_INST(3)
AIR_VEC_INST(4)
#undef AIR_VEC_INST
}  // namespace air

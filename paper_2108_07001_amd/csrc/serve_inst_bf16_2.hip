// serve_inst_bf16_2.hip -- instances of the batched serving kernels
// (bfloat16 splits, D = 9..12); split across files so that hipcc runs in parallel.
#include "serve_kernels.h"

namespace air {
#define AIR_SERVE_INST(D)                                                                       \
  hipError_t launch_serve_bf16_d##D(const JobDesc* j, int n, int64_t items, bool half, int g, \
                                   hipStream_t s) {                                            \
    return launch_serve_td<D, true>(j, n, items, half, g, s);                                  \
  }
AIR_SERVE_INST(9)
AIR_SERVE_INST(10)
AIR_SERVE_INST(11)
AIR_SERVE_INST(12)
#undef AIR_SERVE_INST
}  // namespace air

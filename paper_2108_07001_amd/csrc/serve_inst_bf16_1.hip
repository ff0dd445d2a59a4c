// serve_inst_bf16_1.hip -- instances of the batched serving kernels
// (bfloat16 splits, D = 5..8); split across files so that hipcc runs in parallel.
#include "serve_kernels.h"

namespace air {
#define AIR_SERVE_INST(D)                                                                       \
  hipError_t launch_serve_bf16_d##D(const JobDesc* j, int n, int64_t items, bool half, int g, \
                                   hipStream_t s) {                                            \
    return launch_serve_td<D, true>(j, n, items, half, g, s);                                  \
  }
AIR_SERVE_INST(5)
AIR_SERVE_INST(6)
AIR_SERVE_INST(7)
AIR_SERVE_INST(8)
#undef AIR_SERVE_INST
}  // namespace air

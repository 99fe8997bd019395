// The step kernel with FP32 population storage (every template variant).
#include "lbm_step.h"

namespace lbm {

template int step_grid<0>(bool, bool, bool, bool, bool, int);
template hipError_t step_launch<0>(const Params *, const Buffers *, const uint32_t *, int, uint32_t *, int, bool, bool,
                                    bool, bool, bool, int, int, hipStream_t);

}  // namespace lbm

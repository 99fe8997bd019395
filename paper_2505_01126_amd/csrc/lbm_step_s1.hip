// The step kernel with FP16 population storage (every template variant).
#include "lbm_step.h"

namespace lbm {

template int step_grid<1>(bool, bool, bool, bool, bool, int);
template hipError_t step_launch<1>(const Params *, const Buffers *, const uint32_t *, int, uint32_t *, int, bool, bool,
                                    bool, bool, bool, int, int, hipStream_t);

}  // namespace lbm

// Step and batch kernels of the PF32S policy (FP32 shifted, velocity-shift forcing, one relaxation time).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF32S>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF32S>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

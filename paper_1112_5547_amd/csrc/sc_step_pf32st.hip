// Step and batch kernels of the PF32ST policy (FP32 shifted, velocity-shift forcing, two relaxation times).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF32ST>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF32ST>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

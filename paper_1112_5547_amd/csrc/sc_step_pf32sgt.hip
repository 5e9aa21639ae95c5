// Step and batch kernels of the PF32SGT policy (FP32 shifted, Guo forcing, two relaxation times).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF32SGT>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF32SGT>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

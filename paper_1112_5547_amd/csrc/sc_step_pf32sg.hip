// Step and batch kernels of the PF32SG policy (FP32 shifted, Guo forcing, one relaxation time).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF32SG>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF32SG>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

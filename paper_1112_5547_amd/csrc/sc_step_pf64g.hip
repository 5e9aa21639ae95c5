// Step and batch kernels of the PF64G policy (FP64, Guo forcing, one relaxation time).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF64G>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF64G>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

// Step and batch kernels of the PF64 policy (FP64, velocity-shift forcing, one relaxation time).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF64>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF64>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

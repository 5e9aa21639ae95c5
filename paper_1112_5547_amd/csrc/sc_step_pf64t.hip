// Step and batch kernels of the PF64T policy (FP64, velocity-shift forcing, two relaxation times).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF64T>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF64T>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

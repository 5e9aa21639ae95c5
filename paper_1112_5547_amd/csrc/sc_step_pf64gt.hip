// Step and batch kernels of the PF64GT policy (FP64, Guo forcing, two relaxation times).
#include "sc_batch_kernels.h"

namespace sc {
template hipError_t step_launch<PF64GT>(int, int, int, int, const StepParams&, void*, hipStream_t);
template bool batch_fns<PF64GT>(int, int, int, BatchStepFn*, BatchPersFn*);
}  // namespace sc

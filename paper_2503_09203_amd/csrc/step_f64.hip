// Step kernels, double instantiations.
#include "step_kernel.hpp"

namespace mgx {
template hipError_t launch_step<double>(const StepLaunch<double>&, int, int, hipStream_t);
}  // namespace mgx

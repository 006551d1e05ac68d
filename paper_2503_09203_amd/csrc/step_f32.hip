// Step kernels, float instantiations (and the diagnostic read-back of their per-wave phase
// times: every translation unit has its own copy of the timestamp array).
#include "runtime_internal.hpp"
#include "step_kernel.hpp"

namespace mgx {
template hipError_t launch_step<float>(const StepLaunch<float>&, int, int, hipStream_t);
}  // namespace mgx

// Per-wave phase times of the last step launch (diagnostic builds; see g_wave_ts).
extern "C" mgx_status mgx_diag_wave_times(uint64_t* out, int64_t n_waves) {
#ifdef MGX_WAVE_TIMESTAMPS
    if (!out || n_waves < 1 || n_waves > mgx::kWaveTsMax) return mgx::fail(MGX_E_INVALID, "n_waves outside [1, 65536]");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpyFromSymbol(out, HIP_SYMBOL(mgx::g_wave_ts), sizeof(uint64_t) * 4 * n_waves);
    if (e != hipSuccess) return mgx::fail(MGX_E_DEVICE, "wave times: %s", hipGetErrorString(e));
    return MGX_OK;
#else
    (void)out;
    (void)n_waves;
    return mgx::fail(MGX_E_STATE, "built without MGX_WAVE_TIMESTAMPS");
#endif
}

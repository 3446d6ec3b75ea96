// Step kernels with age-dependent shedding (Eq. (infectivity) with a
// profile s(tau) other than 1; Table "agedep_overhead" measures its cost),
// without rate recording and compaction; compiled apart from the other
// step kernels so they all build in parallel.
#include <hip/hip_runtime.h>

#include "fs_kernels.hpp"
#include "fs_step.hpp"

namespace fsk {

const void* step_kernel_fn_shed(int storage, bool weighted, int mode, int udeg)
{
    return step_kernel_pick<true, false>(storage, weighted, mode, udeg);
}

const void* heavy_kernel_fn_shed(bool weighted, bool resident)
{
    if (resident)
        return weighted ? (const void*)&heavy_resident_kernel<true, true> : (const void*)&heavy_resident_kernel<false, true>;
    return weighted ? (const void*)&heavy_pressure_kernel<true, true> : (const void*)&heavy_pressure_kernel<false, true>;
}

} // namespace fsk

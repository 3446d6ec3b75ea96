// Plain step kernels of unit-weight sims with 16 replicas (compiled apart
// from the others so the instantiations build in parallel).
#include <hip/hip_runtime.h>

#include "fs_kernels.hpp"
#include "fs_step.hpp"

namespace fsk {

const void* step_kernel_fn_r16(int storage, int mode, int udeg)
{
    return storage == 0 ? step_kernel_r16_depth<0>(mode, udeg) : step_kernel_r16_depth<1>(mode, udeg);
}

} // namespace fsk

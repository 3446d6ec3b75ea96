// Plain step kernels of sims with one replica (compiled apart from the others
// so the instantiations build in parallel).
#include <hip/hip_runtime.h>

#include "fs_kernels.hpp"
#include "fs_step.hpp"

namespace fsk {

const void* step_kernel_fn_r1(int storage, bool weighted, int mode, int udeg)
{
    if (storage == 0) return weighted ? step_kernel_r1_depth<0, true>(mode, udeg) : step_kernel_r1_depth<0, false>(mode, udeg);
    return weighted ? step_kernel_r1_depth<1, true>(mode, udeg) : step_kernel_r1_depth<1, false>(mode, udeg);
}

} // namespace fsk

// Step kernels with age-dependent shedding that record rates and/or walk
// the active-chunk list of compaction.
#include <hip/hip_runtime.h>

#include "fs_kernels.hpp"
#include "fs_step.hpp"

namespace fsk {

const void* step_kernel_fn_shed_extra(int storage, bool weighted, int mode, int udeg)
{
    return step_kernel_pick<true, true>(storage, weighted, mode, udeg);
}

} // namespace fsk

// Constant-shedding step kernels that record rates and/or walk the
// active-chunk list of compaction (the plain ones compile neither check in).
#include <hip/hip_runtime.h>

#include "fs_kernels.hpp"
#include "fs_step.hpp"

namespace fsk {

const void* step_kernel_fn_extra(int storage, bool weighted, int mode, int udeg)
{
    return step_kernel_pick<false, true>(storage, weighted, mode, udeg);
}

} // namespace fsk

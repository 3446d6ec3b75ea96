// Plain step kernels of uniform layouts with one replica and columns packed
// at 20 bits (compiled apart from the others so the instantiations build in
// parallel).
#include <hip/hip_runtime.h>

#include "fs_kernels.hpp"
#include "fs_step.hpp"

namespace fsk {

const void* step_kernel_fn_r1p20(int storage, int mode, int udeg)
{
    return storage == 0 ? step_kernel_r1p_depth<0, 20, false, false>(mode, udeg) : step_kernel_r1p_depth<1, 20, false, false>(mode, udeg);
}

} // namespace fsk

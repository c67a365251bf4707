// Period-blocked plain-path kernel, float32 series (template in periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    if (a.y_dtype != BFM_Y_F32) return launch_periodic_16(a, order, F, stream);
    return launch_t<float>(a, order, F, stream);
}

}  // namespace bfm

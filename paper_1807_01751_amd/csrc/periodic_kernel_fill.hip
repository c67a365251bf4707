// Period-blocked plain-path kernel with filling of missing observations,
// float32 series (template in periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_fill(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return launch_t<float, true>(a, order, F, stream);
}

}  // namespace bfm

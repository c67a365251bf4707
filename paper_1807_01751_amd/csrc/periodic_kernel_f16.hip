// Period-blocked plain-path kernel, FP16-stored series (template in periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_f16(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return launch_t<dev::f16_t>(a, order, F, stream);
}

}  // namespace bfm

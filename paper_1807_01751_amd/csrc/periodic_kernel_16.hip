// Period-blocked plain-path kernel, series stored in 16 bits: BF16 or FP16
// (template in periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_16(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return a.y_dtype == BFM_Y_F16 ? launch_t<dev::f16_t>(a, order, F, stream)
                                  : launch_t<dev::bf16_t>(a, order, F, stream);
}

}  // namespace bfm

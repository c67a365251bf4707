// Period-blocked masked kernel, series stored in 16 bits: BF16 or FP16
// (template in masked_periodic_kernel.hpp).
#include "masked_periodic_kernel.hpp"

namespace bfm {

hipError_t launch_masked_periodic_16(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    return a.y_dtype == BFM_Y_F16 ? launch_t<dev::f16_t>(a, order, mask_mode, stream)
                                  : launch_t<dev::bf16_t>(a, order, mask_mode, stream);
}

}  // namespace bfm

// Period-blocked masked kernel with the MOSUM in FP32 (BFM_PREC_FP32), float32
// series (template in masked_periodic_kernel.hpp).
#include "masked_periodic_kernel.hpp"

namespace bfm {

hipError_t launch_masked_periodic_m32(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    if (a.y_dtype == BFM_Y_F16) return launch_masked_periodic_m32_f16(a, order, mask_mode, stream);
    if (a.y_dtype != BFM_Y_F32) return hipErrorInvalidValue;
    return launch_t<float, true>(a, order, mask_mode, stream);
}

}  // namespace bfm

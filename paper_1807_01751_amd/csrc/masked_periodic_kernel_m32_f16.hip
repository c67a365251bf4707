// Period-blocked masked kernel with the MOSUM in FP32 (BFM_PREC_FP32),
// FP16-stored series (template in masked_periodic_kernel.hpp).
#include "masked_periodic_kernel.hpp"

namespace bfm {

hipError_t launch_masked_periodic_m32_f16(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    return launch_t<dev::f16_t, true>(a, order, mask_mode, stream);
}

}  // namespace bfm

// Period-blocked masked kernel, float32 series (template in masked_periodic_kernel.hpp).
#include "masked_periodic_kernel.hpp"

namespace bfm {

size_t masked_periodic_lds_bytes(int cap) { return (size_t)ring_slots(cap) * kBlock * 6; }

hipError_t launch_masked_periodic(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    if (a.m32 && a.y_dtype != BFM_Y_BF16) return launch_masked_periodic_m32(a, order, mask_mode, stream);
    if (a.y_dtype == BFM_Y_BF16) return launch_masked_periodic_bf16(a, order, mask_mode, stream);
    if (a.y_dtype == BFM_Y_F16) return launch_masked_periodic_f16(a, order, mask_mode, stream);
    return launch_t<float>(a, order, mask_mode, stream);
}

}  // namespace bfm

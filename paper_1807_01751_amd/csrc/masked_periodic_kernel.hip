// Period-blocked masked kernel, float32 series (template in masked_periodic_kernel.hpp).
#include "masked_periodic_kernel.hpp"

namespace bfm {

// Rings of every wave (6 bytes per slot and lane) and, with a history split,
// the staging of the partial sums (A[F], yy, Bd; acc[F], cnt, zs, ymax, bad)
// and each wave's (count, next slot).
size_t masked_periodic_lds_bytes(int cap, int F, int split)
{
    const size_t rings = (size_t)split * ring_slots(cap) * kBlock * 6;
    const size_t staging = split > 1 ? (size_t)kBlock * (8 * (F + 2) + 4 * (F + 4) + 8 * split) : 0;
    return rings + staging;
}

hipError_t launch_masked_periodic(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    if (a.m32 && a.y_dtype != BFM_Y_BF16) return launch_masked_periodic_m32(a, order, mask_mode, stream);
    if (a.y_dtype == BFM_Y_BF16) return launch_masked_periodic_bf16(a, order, mask_mode, stream);
    if (a.y_dtype == BFM_Y_F16) return launch_masked_periodic_f16(a, order, mask_mode, stream);
    return launch_t<float>(a, order, mask_mode, stream);
}

}  // namespace bfm

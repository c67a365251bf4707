// Period-blocked plain-path kernel, float32 series (template in periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_split(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    switch (a.split) {
    case 2: return launch_periodic_split2(a, order, F, stream);
    case 4: return launch_periodic_split4(a, order, F, stream);
    case 8: return launch_periodic_split8(a, order, F, stream);
    default: return hipErrorInvalidValue;
    }
}

size_t periodic_split_lds(int order, int F, int split, int H)
{
    if (split == 1) return (size_t)H * kPeriodicBlock * sizeof(float);
    if (split != 2 && split != 4 && split != 8) return 0;
    return split_lds_bytes(F, 2 + 2 * order, split, H);
}

hipError_t launch_periodic(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    if (a.y_dtype == BFM_Y_BF16) return launch_periodic_bf16(a, order, F, stream);
    if (a.y_dtype == BFM_Y_F16) return launch_periodic_f16(a, order, F, stream);
    if (a.fill) return launch_periodic_fill(a, order, F, stream);
    if (a.split > 1 && !a.resid && !a.mosum) return launch_periodic_split(a, order, F, stream);
    return launch_t<float>(a, order, F, stream);
}

}  // namespace bfm

// Period-blocked plain-path kernel, BF16-stored series (template in periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_bf16(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return launch_t<dev::bf16_t>(a, order, F, stream);
}

}  // namespace bfm

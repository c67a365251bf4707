// Time-split period-blocked plain kernel, 8 waves per 64 pixels (template in
// periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_split8(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return launch_split_ns<8>(a, order, F, stream);
}

}  // namespace bfm

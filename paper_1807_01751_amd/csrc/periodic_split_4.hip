// Time-split period-blocked plain kernel, 4 waves per 64 pixels (template in
// periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_split4(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return launch_split_ns<4>(a, order, F, stream);
}

}  // namespace bfm

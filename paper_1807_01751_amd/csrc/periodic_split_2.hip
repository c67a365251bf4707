// Time-split period-blocked plain kernel, 2 waves per 64 pixels (template in
// periodic_kernel.hpp).
#include "periodic_kernel.hpp"

namespace bfm {

hipError_t launch_periodic_split2(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    return launch_split_ns<2>(a, order, F, stream);
}

}  // namespace bfm

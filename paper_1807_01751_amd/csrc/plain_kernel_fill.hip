// Table-driven plain-path kernel with filling of missing observations
// (template in plain_kernel.hpp).
#include "plain_kernel.hpp"

namespace bfm {

hipError_t launch_plain_fill(const PlainArgs& a, int p, hipStream_t stream)
{
    return launch_plain_t<false, true>(a, p, stream);
}

}  // namespace bfm

// Table-driven plain-path kernel with per-row exports (resid, mosum), series
// used as read (template in plain_kernel.hpp).
#include "plain_kernel.hpp"

namespace bfm {

hipError_t launch_plain_export(const PlainArgs& a, int p, hipStream_t stream)
{
    return launch_plain_t<true, false>(a, p, stream);
}

}  // namespace bfm

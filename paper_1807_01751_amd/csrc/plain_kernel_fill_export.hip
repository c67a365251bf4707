// Table-driven plain-path kernel with filling and per-row exports (resid,
// mosum) (template in plain_kernel.hpp).
#include "plain_kernel.hpp"

namespace bfm {

hipError_t launch_plain_fill_export(const PlainArgs& a, int p, hipStream_t stream)
{
    return launch_plain_t<true, true>(a, p, stream);
}

}  // namespace bfm

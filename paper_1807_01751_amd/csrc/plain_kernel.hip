// Table-driven plain-path kernel, series used as read (template in
// plain_kernel.hpp), and the status-only kernel for degenerate parameter sets.
#include "plain_kernel.hpp"

namespace bfm {
namespace {

// Pixels whose parameters leave nothing to fit.
template <typename T>
__global__ __launch_bounds__(256) void fill_status_kernel(const T* __restrict__ Y, int64_t ld,
                                                          int64_t P, int N, int n, int p,
                                                          uint8_t st0, bfm_outputs out,
                                                          int mask_mode,
                                                          const uint8_t* __restrict__ valid,
                                                          int64_t ldv)
{
    const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= P) return;
    bool bad = false;
    uint8_t st = st0;
    if (mask_mode == BFM_MASK_FILL) {
        // Filling leaves a series non-finite only when it has no finite value.
        bool any = false;
        for (int t = 0; t < N && !any; ++t) any = isfinite(to_float(Y[(int64_t)t * ld + pix]));
        if (!any) st = BFM_ST_INSUFFICIENT;
    } else if (mask_mode != BFM_MASK_NAN) {
        for (int t = 0; t < N; ++t) {
            bool used = mask_mode == BFM_MASK_NONE || valid[(int64_t)t * ldv + pix] != 0;
            bad |= used && !isfinite(to_float(Y[(int64_t)t * ld + pix]));
        }
        if (bad) st = BFM_ST_NONFINITE;
    }
    const double qnan = __builtin_nan("");
    const int f64 = out.out_dtype == BFM_OUT_F64;
    out.brk[pix] = -1;
    if (out.status) out.status[pix] = st;
    if (out.mag) put_out(out.mag, pix, qnan, f64);
    if (out.sigma) put_out(out.sigma, pix, qnan, f64);
    if (out.beta)
        for (int j = 0; j < p; ++j) put_out(out.beta, (int64_t)j * P + pix, qnan, f64);
    if (out.resid)
        for (int t = 0; t < N; ++t) put_out(out.resid, (int64_t)t * P + pix, qnan, f64);
    if (out.mosum)
        for (int m = 0; m < N - n; ++m) put_out(out.mosum, (int64_t)m * P + pix, qnan, f64);
}

}  // namespace

hipError_t launch_plain(const PlainArgs& a, int p, hipStream_t stream)
{
    const bool exp = a.resid || a.mosum;
    if (a.fill) return exp ? launch_plain_fill_export(a, p, stream) : launch_plain_fill(a, p, stream);
    return exp ? launch_plain_export(a, p, stream) : launch_plain_t<false, false>(a, p, stream);
}

hipError_t launch_fill_status(const void* Y, int y_dtype, int64_t ld, int64_t P, int N, int n, int p,
                              uint8_t st, const bfm_outputs& out, int mask_mode,
                              const uint8_t* valid, int64_t ldv, hipStream_t stream)
{
    const dim3 grid((unsigned)((P + 255) / 256));
    if (y_dtype == BFM_Y_BF16)
        hipLaunchKernelGGL(fill_status_kernel<bf16_t>, grid, dim3(256), 0, stream,
                           static_cast<const bf16_t*>(Y), ld, P, N, n, p, st, out, mask_mode, valid, ldv);
    else if (y_dtype == BFM_Y_F16)
        hipLaunchKernelGGL(fill_status_kernel<f16_t>, grid, dim3(256), 0, stream,
                           static_cast<const f16_t*>(Y), ld, P, N, n, p, st, out, mask_mode, valid, ldv);
    else
        hipLaunchKernelGGL(fill_status_kernel<float>, grid, dim3(256), 0, stream,
                           static_cast<const float*>(Y), ld, P, N, n, p, st, out, mask_mode, valid, ldv);
    return hipGetLastError();
}

}  // namespace bfm

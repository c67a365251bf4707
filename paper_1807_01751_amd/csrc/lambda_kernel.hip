// Critical value lambda of the boundary (Eq. 4) by simulation, on the GPU.
//
// Section 2.1 fixes lambda so that, when nothing changes, the MOSUM crosses
// lambda sqrt(log+(t/n)) with probability alpha; it depends on alpha, the window
// and the horizon N/n and is found by simulation.  One lane simulates one path
// of the MOSUM under no change at the resolution of the series (i.i.d. standard
// normal errors, intercept-only model; its limit W(t) - W(t-h) - h W(1) is the
// process the cited method takes its critical values from, a convention rather
// than the exact limit for the trend regressor of Eq. 2):
//
//   M_k = (sum of z over the window (k-H, k] - (H/n) sum_{i<=n} z_i) / sqrt(n),
//   S   = max_{k=n+1..N} |M_k| / sqrt(log+(k/n)),
//
// and a path crosses lambda sqrt(log+) iff S > lambda.  lambda is the
// ceil((1 - alpha) paths)-th smallest S, selected on the device by a radix
// select over the bit patterns of S (positive doubles order like their bits).
//
// Normals: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011), key
// (seed, 0), counter (j, path, 0, 0), four 64-bit words per block j, each turned
// into a uniform ((w >> 11) + 1/2) 2^-53 and paired by the Box-Muller transform
// into z_{4j+1..4j+4}.  The generator is counter-based, so the normal leaving
// the window is regenerated from its counter instead of being stored: the
// kernel needs no LDS and takes any window length.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "bfm_internal.hpp"

// Scratch of bfm_critical_value_noalloc: the statistics of up to
// BFM_NOALLOC_MAX_PATHS paths, then the 256 digit counters of the selection.
// Each GPU holds its own copy at its own address; host code reaches it only
// through the address noalloc_scratch_init looked up (the array's name is a
// host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[(size_t)BFM_NOALLOC_MAX_PATHS * 8 + 1024];

namespace bfm {
namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;  // round multipliers
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;  // key increments
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr int kLamBlock = 256;

// Four standard normals of block j of a path.
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t path, uint64_t j, double z[4])
{
    uint64_t c0 = j, c1 = path, c2 = 0, c3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    const double s53 = 0x1p-53;
    const double u0 = ((double)(c0 >> 11) + 0.5) * s53, u1 = ((double)(c1 >> 11) + 0.5) * s53;
    const double u2 = ((double)(c2 >> 11) + 0.5) * s53, u3 = ((double)(c3 >> 11) + 0.5) * s53;
    const double r0 = sqrt(-2.0 * log(u0)), r2 = sqrt(-2.0 * log(u2));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z[0] = r0 * c;
    z[1] = r0 * s;
    sincospi(2.0 * u3, &s, &c);
    z[2] = r2 * c;
    z[3] = r2 * s;
}

// z_k (1-based step k) of a path, through a one-block cache.
struct NormalStream {
    uint64_t seed, path;
    int64_t blk = -1;
    double z[4];
    __device__ __forceinline__ double at(int k)
    {
        const int64_t b = (k - 1) >> 2;
        if (b != blk) {  // uniform across the wave: every lane is at the same k
            normals4(seed, path, (uint64_t)b, z);
            blk = b;
        }
        const int q = (k - 1) & 3;
        return q == 0 ? z[0] : q == 1 ? z[1] : q == 2 ? z[2] : z[3];
    }
};

__global__ __launch_bounds__(kLamBlock) void mosum_null_sup_kernel(int n, int N, int H, uint64_t seed,
                                                                  int64_t path0, int64_t paths,
                                                                  double* __restrict__ sup)
{
    const int64_t i = (int64_t)blockIdx.x * kLamBlock + threadIdx.x;
    if (i >= paths) return;
    NormalStream lead{seed, (uint64_t)(path0 + i)}, trail{seed, (uint64_t)(path0 + i)};
    double hist = 0.0, win = 0.0;
    for (int k = 1; k <= n; ++k) {
        const double z = lead.at(k);
        hist += z;
        if (k > n - H) win += z;
    }
    const double mean_term = (double)H / (double)n * hist;
    const double rn = 1.0 / sqrt((double)n);
    double best = 0.0;
    for (int k = n + 1; k <= N; ++k) {
        win += lead.at(k) - trail.at(k - H);
        const double t = (double)k / (double)n;
        const double b = t <= M_E ? 1.0 : sqrt(log(t));
        best = fmax(best, fabs((win - mean_term) * rn) / b);
    }
    sup[i] = best;
}

// Histogram of the next 8-bit digit (at `shift`) of the values whose higher
// bits equal `prefix` under `pmask`.
__global__ __launch_bounds__(kLamBlock) void select_digit_kernel(const uint64_t* __restrict__ v, int64_t cnt,
                                                                uint64_t prefix, uint64_t pmask, int shift,
                                                                uint32_t* __restrict__ counts)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kLamBlock + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * kLamBlock) {
        const uint64_t x = v[i];
        if ((x & pmask) == prefix) atomicAdd(&h[(x >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(&counts[threadIdx.x], c);
}

__global__ void zero_counts_kernel(uint32_t* counts) { counts[threadIdx.x] = 0; }

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
    return hipSuccess;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

hipError_t launch_mosum_null_sup(int n, int N, int H, uint64_t seed, int64_t path0, int64_t paths,
                                 double* sup, hipStream_t stream)
{
    const dim3 grid((unsigned)((paths + kLamBlock - 1) / kLamBlock));
    hipLaunchKernelGGL(mosum_null_sup_kernel, grid, dim3(kLamBlock), 0, stream, n, N, H, seed, path0,
                       paths, sup);
    return hipGetLastError();
}

hipError_t select_rank(const double* v, int64_t cnt, int64_t rank, uint32_t* counts, double* out,
                       hipStream_t stream)
{
    // Positive doubles order like their bit patterns; eight passes of eight
    // bits, most significant first, each keep the digit where the rank falls.
    uint64_t prefix = 0, pmask = 0;
    int64_t k = rank;  // 1-based rank among the values matching the prefix
    const unsigned blocks = (unsigned)std::min<int64_t>((cnt + kLamBlock - 1) / kLamBlock, 1024);
    uint32_t h[256];
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(256), 0, stream, counts);
        hipLaunchKernelGGL(select_digit_kernel, dim3(blocks), dim3(kLamBlock), 0, stream,
                           reinterpret_cast<const uint64_t*>(v), cnt, prefix, pmask, shift, counts);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h, counts, sizeof h, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        int d = 0;
        while (d < 255 && (int64_t)h[d] < k) k -= h[d++];
        prefix |= (uint64_t)d << shift;
        pmask |= (uint64_t)0xff << shift;
    }
    double r;
    std::memcpy(&r, &prefix, sizeof r);
    *out = r;
    return hipSuccess;
}

}  // namespace bfm

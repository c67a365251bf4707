// Internal declarations shared by the host runtime and the kernel launchers of
// libbfm.  Nothing here is part of the public ABI (include/bfm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bfm.h"

namespace bfm {

constexpr int kMaxOrder = 8;                 // k <= 8, p <= 18
constexpr int kMaxP = 2 + 2 * kMaxOrder;
constexpr double kSigmaRelTol = 1e-6;        // DEGENERATE_SIGMA threshold
constexpr double kRankTol = 1e-6;            // |R_jj| <= tol * sqrt(rows)
constexpr int kPlainBlock = 64;              // threads per block (one wave), plain path

// Shared operators of the plain path, built on the host in FP64 (Section 3:
// the pseudo-inverse M is formed once for all pixels; here its orthonormal
// equivalent).  See bfm_host_operators() in bfm.h for the meaning of each.
struct PlainOps {
    int N = 0, n = 0, p = 0, H = 0;
    int m_flat = 0;  // leading monitoring rows with t/n <= e (boundary = lambda)
    bool rank_ok = false;
    std::vector<double> q;     // N x p
    std::vector<double> w;     // (N-n) x p
    std::vector<double> bnd;   // N-n
    std::vector<double> bmap;  // p x p
};

// Window length H for a history of `count` used observations.
int window_length(const bfm_params& prm, int count);

// Build the plain-path operators.  Returns false if the parameters are invalid.
bool build_plain_ops(const bfm_params& prm, PlainOps* ops);

// Arguments of the plain kernel (by value; every pointer is device memory).
struct PlainArgs {
    const float* Y;
    int64_t ld;
    int64_t P;
    const double* q;     // N x p
    const double* w;     // M x p
    const double* bnd;   // M
    const double* bmap;  // p x p
    int N, n, H;
    int m_flat;          // leading monitoring rows where the boundary equals lambda
    double lambda;
    double sqrt_n;       // sqrt(n): MOSUM normaliser of Eq. 3
    double inv_dof;      // 1 / (n - p): Algorithm 1, step 5
    int32_t* brk;
    void* mag;
    void* sigma;
    uint8_t* status;
    void* beta;
    void* resid;
    void* mosum;
    int out_f64;
};

hipError_t launch_plain(const PlainArgs& a, int p, hipStream_t stream);

// Every pixel gets `st` (or NONFINITE if one of its used observations is not
// finite), brk = -1 and NaN floating outputs: used when the parameters make
// every pixel degenerate (history too short, rank-deficient shared design).
hipError_t launch_fill_status(const float* Y, int64_t ld, int64_t P, int N, int n, int p,
                              uint8_t st, const bfm_outputs& out, int mask_mode,
                              const uint8_t* valid, int64_t ldv, hipStream_t stream);

}  // namespace bfm

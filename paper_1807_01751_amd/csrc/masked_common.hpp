// Per-pixel Gram matrix of the masked path: assembly from masked sums by
// product-to-sum identities and an in-register FP64 Cholesky factorisation.
#pragma once

#include <hip/hip_runtime.h>

namespace bfm {
namespace dev {

// Packed lower-triangular index (i >= j).
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <int K>
struct Gram {
    static constexpr int NP = 2 + 2 * K;
    static constexpr int NG = 2 + 6 * K;
    static constexpr int NL = NP * (NP + 1) / 2;

    // Masked sums of sin(m w t) / cos(m w t) for |m| <= 2k; m = 0 gives the count.
    __device__ static double S(const double* gs, int m)
    {
        return m == 0 ? 0.0 : (m > 0 ? gs[1 + m] : -gs[1 - m]);
    }
    __device__ static double C(const double* gs, double cnt, int m)
    {
        const int am = m < 0 ? -m : m;
        return am == 0 ? cnt : gs[1 + 2 * K + am];
    }

    // Gram matrix sum_t w_t x~_t x~_t' in packed lower storage.  Columns: 0 the
    // constant, 1 the trend tau, 2j sin(j w t), 2j+1 cos(j w t).
    __device__ static void assemble(const double* gs, double cnt, double* G)
    {
        G[tri(0, 0)] = cnt;
        G[tri(1, 0)] = gs[0];
        G[tri(1, 1)] = gs[1];
#pragma unroll
        for (int j = 1; j <= K; ++j) {
            G[tri(2 * j, 0)] = S(gs, j);
            G[tri(2 * j + 1, 0)] = C(gs, cnt, j);
            G[tri(2 * j, 1)] = gs[1 + 4 * K + j];
            G[tri(2 * j + 1, 1)] = gs[1 + 5 * K + j];
#pragma unroll
            for (int l = 1; l <= j; ++l) {
                G[tri(2 * j, 2 * l)] = 0.5 * (C(gs, cnt, j - l) - C(gs, cnt, j + l));
                G[tri(2 * j + 1, 2 * l + 1)] = 0.5 * (C(gs, cnt, j - l) + C(gs, cnt, j + l));
                G[tri(2 * j + 1, 2 * l)] = 0.5 * (S(gs, l + j) + S(gs, l - j));
                if (l < j) G[tri(2 * j, 2 * l + 1)] = 0.5 * (S(gs, j + l) + S(gs, j - l));
            }
        }
    }

    // In-place Cholesky G = L L'.  Returns false when a pivot's square is at
    // most tol2 (the history design is rank deficient at that column).
    __device__ static bool cholesky(double* L, double tol2)
    {
        bool ok = true;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double d = L[tri(j, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) d = fma(-L[tri(j, k)], L[tri(j, k)], d);
            ok = ok && d > tol2;
            const double ljj = sqrt(d > tol2 ? d : 1.0);
            const double inv = 1.0 / ljj;
            L[tri(j, j)] = ljj;
#pragma unroll
            for (int i = j + 1; i < NP; ++i) {
                double s = L[tri(i, j)];
#pragma unroll
                for (int k = 0; k < j; ++k) s = fma(-L[tri(i, k)], L[tri(j, k)], s);
                L[tri(i, j)] = s * inv;
            }
        }
        return ok;
    }

    // One step of iterative refinement with the factor L of the Gram matrix:
    // dz = L^-1 dq, beta += L^-T dz where `take` (dq = X~' r, the design's
    // products with the residuals r at beta).  Returns ||dz||^2, by which the
    // residual sum of squares at the refined beta falls short of sum r^2.
    __device__ static double refine(const double* L, const double* dq, double* beta, bool take)
    {
        double dz[NP], db[NP];
        double dd = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double s = dq[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s = fma(-L[tri(i, k)], dz[k], s);
            dz[i] = s / L[tri(i, i)];
            dd = fma(dz[i], dz[i], dd);
        }
#pragma unroll
        for (int i = NP - 1; i >= 0; --i) {
            double s = dz[i];
#pragma unroll
            for (int k = i + 1; k < NP; ++k) s = fma(-L[tri(k, i)], db[k], s);
            db[i] = s / L[tri(i, i)];
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) beta[i] = take ? beta[i] + db[i] : beta[i];
        return dd;
    }
};

}  // namespace dev
}  // namespace bfm

// Slicing of K-word values for the split (Ozaki) trailing update: the
// per-row (per-column) scale, the slice width and the cut into slices.  Used by the
// slicing kernels, by the panel (rows of L21 as it writes them back) and by
// the look-ahead triangular solve (columns of U12 as it finishes them), so
// that every producer cuts exactly the same way.
#pragma once
#include "common.hpp"

namespace bnc {

// Bits per slice for K-word values cut into s slices.  Slice q of a value
// sits on the grid 2^(E - (q+1) beta) and is below (2^beta + K/2) grid
// steps for q = 0, (K 2^(beta-1) + K/2) for q > 0; the products of group
// d = p + q share one grid, and a depth-64 update adds 64 (d+1) of them.
// The group sums grow with d, so the last group (d = s-1) decides: beta is
// the widest slice (at most 26 bits) that keeps its bound below 2^53 grid
// units, every product and partial sum then being exact.  Bounds are kept
// in half steps so they are integers: 2 b_0 = 2^(beta+1) + K,
// 2 b_q = K 2^beta + K, and 64 (2 b)(2 b') / 4 < 2^53 <=> sum < 2^49.
__host__ __device__ constexpr int oz_beta(int K, int s)
{
    for (int b = 26; b > 1; --b) {
        const unsigned long long b0 = (1ull << (b + 1)) + (unsigned)K;
        const unsigned long long bq = (unsigned long long)K * (1ull << b) + (unsigned)K;
        const unsigned long long g = s <= 1 ? b0 * b0 : 2 * b0 * bq + (unsigned long long)(s - 2) * bq * bq;
        if (g < (1ull << 49))
            return b;
    }
    return 1;
}

// Smallest row (column) scale E for which the split scheme stays exact:
// slice q of a row with scale E sits on the grid 2^(E - (q+1) beta) and a
// product of group d on 2^(E + F - (d+2) beta), so with both scales at
// least this bound every slice grid and every product grid, down to group
// s - 1, is at least 2^-1022 (normal binary64, no flush or rounding).  A
// nonzero row or column below it makes the factorisation report info = -3.
__host__ __device__ constexpr int oz_emin(int K, int s)
{
    const int b = oz_beta(K, s);
    const int x = (s + 1) * b - 1022;                 // E + F must reach this
    const int half = x >= 0 ? (x + 1) / 2 : -((-x) / 2);  // ceil(x / 2)
    const int own = s * b - 1022;
    return half > own ? half : own;
}

// Exponent e with |x| <= mx < 2^e for the largest leading word mx of a row
// (column); 0 for an all-zero row.
__device__ __forceinline__ int oz_scale(double mx)
{
    int e = 0;
    if (mx == 0.0)
        return 0;
    (void)frexp(mx, &e);  // mx = f 2^e, f in [1/2, 1)
    return e;
}

// Cut the K-word value v (it becomes the remainder) into slices 0..s-1 on
// the grids 2^(E - (q+1) beta), beta = oz_beta(K, s), and store slice q at
// out[q * stride].
template <int K>
__device__ __forceinline__ void oz_cut_store(double (&v)[K], int E, int s, int beta, double *out, int64_t stride)
{
    for (int q = 0; q < s; ++q) {
        const int e = E - (q + 1) * beta;
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double rho = ldexp(rint(ldexp(v[t], -e)), e);
            v[t] -= rho;
            acc += rho;
        }
        out[q * stride] = acc;
    }
}

}  // namespace bnc

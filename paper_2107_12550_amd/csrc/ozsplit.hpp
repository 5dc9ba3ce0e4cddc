// Slicing of K-word values for the split (Ozaki) trailing update: the
// per-row (per-column) scale and the cut into BETA-bit slices.  Used by the
// slicing kernels, by the panel (rows of L21 as it writes them back) and by
// the look-ahead triangular solve (columns of U12 as it finishes them), so
// that every producer cuts exactly the same way.
#pragma once
#include "common.hpp"

namespace bnc {

constexpr int OZ_BETA = 20;

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
// the grids 2^(E - (q+1) BETA) and store slice q at out[q * stride].
template <int K>
__device__ __forceinline__ void oz_cut_store(double (&v)[K], int E, int s, double *out, int64_t stride)
{
    for (int q = 0; q < s; ++q) {
        const int e = E - (q + 1) * OZ_BETA;
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

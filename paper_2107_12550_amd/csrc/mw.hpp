// Multi-word floating point on the device: a value is an unevaluated sum of
// K binary64 words, leading word first (K = 1 binary64, 2 double-double,
// 3 triple-double, 4 quad-double; 53/106/159/212 bits as in Kouya 2021,
// Table 1).  The paper names the formats but not the word-level algorithms;
// these are built only from error-free transformations and every operation
// order is fixed, so results are reproducible bit for bit:
//
//   two_sum   Knuth's TwoSum:   s = RN(a+b), e = a+b-s exactly (6 flops)
//   two_prod  FMA TwoProd:      p = RN(a*b), e = a*b-p exactly (mul + fma)
//
//   Level accumulation.  Terms of size ~2^(-53 lv) relative to the result go
//   to level lv.  Levels 0..K-2 are summed left to right with two_sum and
//   every rounding error is appended to level lv+1; level K-1 is summed
//   left to right in plain binary64.
//
//   fms(c, a, b) = c - a*b: level lists start with the words of c; then the
//   partial products a_i b_j are visited for i = 0..K-1, j = 0..K-1-i.  With
//   i+j < K-1 the product is split by two_prod (high part at level i+j, error
//   at level i+j+1); with i+j = K-1 it is one plain product at level K-1;
//   products below that are dropped.  mul(a, b) is the same without c and
//   with positive signs; add(a, b) puts (a_lv, b_lv) on level lv.
//
//   renorm (M words -> K words): two_sum upward from the smallest word (the
//   running sum ends in t_0, errors in t_1..t_{M-1}); then downward, each
//   two_sum emits one word and carries its error on, and after K-1 words the
//   remaining t's are added plainly into the last word.
//
//   recip(a): r = 1/a_0 in binary64, then Newton steps r <- r - (-r)(1 - a r)
//   with fms: 0 steps for K = 1, 1 for K = 2, 2 for K = 3 and 4.
//
// Everything must be compiled with -ffp-contract=off so that no product is
// fused into a neighbouring add; the only fused operation is the explicit fma.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bnc {

__device__ __forceinline__ double two_sum(double a, double b, double &e)
{
    const double s = a + b;
    const double bv = s - a;
    const double av = s - bv;
    e = (a - av) + (b - bv);
    return s;
}

__device__ __forceinline__ double two_prod(double a, double b, double &e)
{
    const double p = a * b;
    e = __builtin_fma(a, b, -p);
    return p;
}

// Number of terms level lv receives in fms/mul (HAS_C: c present).
template <int K, bool HAS_C>
__host__ __device__ constexpr int fms_level_terms(int lv)
{
    int n = HAS_C ? 1 : 0;
    for (int i = 0; i < K; ++i)
        for (int j = 0; i + j < K; ++j) {
            const int l = i + j;
            if (l < K - 1) {
                n += (l == lv) ? 1 : 0;
                n += (l + 1 == lv) ? 1 : 0;
            } else {
                n += (lv == K - 1) ? 1 : 0;
            }
        }
    // errors carried in from level lv-1
    if (lv > 0)
        n += fms_level_terms<K, HAS_C>(lv - 1) - 1;
    return n;
}

template <int K>
__host__ __device__ constexpr int fms_level_cap()
{
    int m = 1;
    for (int lv = 0; lv < K; ++lv) {
        const int t = fms_level_terms<K, true>(lv);
        m = t > m ? t : m;
    }
    return m;
}

// Level lists with compile-time capacity; after full unrolling every index
// is a constant, so the arrays live in registers.
template <int K, int CAP>
struct Levels {
    double v[K][CAP];
    int n[K];

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int lv = 0; lv < K; ++lv)
            n[lv] = 0;
    }
    __device__ __forceinline__ void push(int lv, double x) { v[lv][n[lv]++] = x; }

    // Level accumulation; result words per level in s[0..K-1].
    __device__ __forceinline__ void sum(double (&s)[K])
    {
#pragma unroll
        for (int lv = 0; lv < K - 1; ++lv) {
            double acc = v[lv][0];
#pragma unroll
            for (int t = 1; t < CAP; ++t) {
                if (t < n[lv]) {
                    double e;
                    acc = two_sum(acc, v[lv][t], e);
                    push(lv + 1, e);
                }
            }
            s[lv] = acc;
        }
        double acc = v[K - 1][0];
#pragma unroll
        for (int t = 1; t < CAP; ++t)
            if (t < n[K - 1])
                acc = acc + v[K - 1][t];
        s[K - 1] = acc;
    }
};

// M input words (roughly decreasing) -> K words.
template <int K, int M>
__device__ __forceinline__ void renorm(const double (&c)[M], double (&out)[K])
{
    double t[M];
    double s = c[M - 1];
#pragma unroll
    for (int i = M - 2; i >= 0; --i)
        s = two_sum(c[i], s, t[i + 1]);
    t[0] = s;
    double w = t[0];
    int j = 0;
#pragma unroll
    for (int i = 1; i < M; ++i) {
        if (j < K - 1) {
            double lo;
            out[j] = two_sum(w, t[i], lo);
            w = lo;
            ++j;
        } else {
            w = w + t[i];
        }
    }
    out[j] = w;
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (q > j)
            out[q] = 0.0;
}

template <int K, bool HAS_C>
__device__ __forceinline__ void fms_core(const double (&c)[K], const double (&a)[K], const double (&b)[K],
                                         double (&out)[K])
{
    constexpr int CAP = fms_level_cap<K>();
    Levels<K, CAP> L;
    L.clear();
    const double sg = HAS_C ? -1.0 : 1.0;
    if (HAS_C) {
#pragma unroll
        for (int lv = 0; lv < K; ++lv)
            L.push(lv, c[lv]);
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
#pragma unroll
        for (int j = 0; i + j < K; ++j) {
            const int lv = i + j;
            if (lv < K - 1) {
                double e;
                const double p = two_prod(a[i], b[j], e);
                L.push(lv, sg * p);
                L.push(lv + 1, sg * e);
            } else {
                L.push(K - 1, sg * (a[i] * b[j]));
            }
        }
    }
    double s[K];
    L.sum(s);
    renorm<K, K>(s, out);
}

// c - a*b
template <int K>
__device__ __forceinline__ void fms(const double (&c)[K], const double (&a)[K], const double (&b)[K],
                                    double (&out)[K])
{
    fms_core<K, true>(c, a, b, out);
}

// a*b
template <int K>
__device__ __forceinline__ void mul(const double (&a)[K], const double (&b)[K], double (&out)[K])
{
    fms_core<K, false>(a, a, b, out);
}

// a+b
template <int K>
__device__ __forceinline__ void add(const double (&a)[K], const double (&b)[K], double (&out)[K])
{
    Levels<K, 2 * K> L;
    L.clear();
#pragma unroll
    for (int lv = 0; lv < K; ++lv) {
        L.push(lv, a[lv]);
        L.push(lv, b[lv]);
    }
    double s[K];
    L.sum(s);
    renorm<K, K>(s, out);
}

template <int K>
__device__ __forceinline__ void recip(const double (&a)[K], double (&out)[K])
{
    double r[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        r[w] = 0.0;
    r[0] = 1.0 / a[0];
    constexpr int steps = K == 1 ? 0 : (K == 2 ? 1 : 2);
    double one[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        one[w] = w == 0 ? 1.0 : 0.0;
#pragma unroll
    for (int it = 0; it < steps; ++it) {
        double e[K], nr[K], r2[K];
        fms<K>(one, a, r, e);
#pragma unroll
        for (int w = 0; w < K; ++w)
            nr[w] = -r[w];
        fms<K>(r, nr, e, r2);
#pragma unroll
        for (int w = 0; w < K; ++w)
            r[w] = r2[w];
    }
#pragma unroll
    for (int w = 0; w < K; ++w)
        out[w] = r[w];
}

// Pivot order: |a| word by word, leading word first, each word multiplied by
// the sign of the leading word.  True when key(a) > key(b).
template <int K>
__device__ __forceinline__ bool key_gt(const double (&a)[K], const double (&b)[K])
{
    const double sa = a[0] < 0.0 ? -1.0 : 1.0;
    const double sb = b[0] < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int w = 0; w < K; ++w) {
        const double x = sa * a[w], y = sb * b[w];
        if (x > y)
            return true;
        if (x < y)
            return false;
    }
    return false;
}

template <int K>
__device__ __forceinline__ bool is_zero(const double (&a)[K])
{
    bool z = true;
#pragma unroll
    for (int w = 0; w < K; ++w)
        z = z && (a[w] == 0.0);
    return z;
}

// Word-plane access: word w of element idx lives at p[w * ldp + idx].
template <int K>
__device__ __forceinline__ void load_w(const double *p, int64_t ldp, int64_t idx, double (&v)[K])
{
#pragma unroll
    for (int w = 0; w < K; ++w)
        v[w] = p[w * ldp + idx];
}

template <int K>
__device__ __forceinline__ void store_w(double *p, int64_t ldp, int64_t idx, const double (&v)[K])
{
#pragma unroll
    for (int w = 0; w < K; ++w)
        p[w * ldp + idx] = v[w];
}

// Exact scaling by 2^e (|e| small enough to stay in the normal range).
__device__ __forceinline__ double pow2(int e)
{
    return __longlong_as_double((long long)(1023 + e) << 52);
}

}  // namespace bnc

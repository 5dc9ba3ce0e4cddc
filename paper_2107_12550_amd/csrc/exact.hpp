// Exact accumulation of a residual row and its canonical rounding to the
// long precision (the residual step of Listing 1, Kouya 2021 Sec. 2, read
// as: products split exactly, summed exactly, rounded once).
//
// Terms are binary64 numbers (TwoProd halves of A_ij^(u) x_j^(w), and the
// words of b_i).  Each term is cut into fixed-point digits of W bits (34
// unless a caller sets another width) over up to 40 bins anchored at the
// row's largest possible term: the extraction (sigma + t) - sigma with
// sigma = 1.5 * 2^(52 + e_bin) is exact and rounds t to a multiple of
// 2^e_bin.  The bins a row uses reach down to a bound on the lowest bit of
// any term (smallest exponents of the words of A, x and b).  A digit past
// the first bin is at most 2^(W-1) of its bin's quanta, so every digit sum
// is exact while the row has fewer than 2^(53-W) terms (2^19 at W = 34).
// The bins are then read as one signed integer (32-bit limbs in int64,
// carry-save) and rounded greedily to four (or eight) binary64 words with
// round-to-nearest-even.
#pragma once

#include <stdint.h>

#include "mw.hpp"

namespace bnc {

constexpr int RB_W = 34;
constexpr int RB_NB = 40;  // maximum bins per row

// exponent e with 2^e <= |x| < 2^(e+1) for normal x; -1023 for zero/subnormal
__device__ __forceinline__ int ilogb_bits(double x)
{
    return (int)((__double_as_longlong(x) >> 52) & 0x7ff) - 1023;
}

// frexp-style exponent used for the power-of-two normalisation:
// e = floor(log2 m) for m > 0, and -1 for m == 0 (as frexp(0) = (0, 0)).
__host__ __device__ inline int norm_exp(double m)
{
    if (m == 0.0)
        return -1;
    int e;
    (void)frexp(m, &e);
    return e - 1;
}

struct RowAnchor {
    int e0;   // exponent of bin 0's quantum
    int nb;   // bins in use
    bool any; // the row has a nonzero term
};

// Exponent bounds gathered before the residual: the smallest floor(log2|v|)
// over the nonzero words of A, x and b (2000 when there is none).
struct ExpBounds {
    int a, x, b;
};

// lowest bit any term can have: products of words (each word's lowest bit is
// at least its exponent - 52) and the words of b
__device__ __forceinline__ int lowest_bit(const ExpBounds &eb)
{
    int lo = 100000;
    if (eb.a < 2000 && eb.x < 2000)
        lo = eb.a + eb.x - 104;
    if (eb.b < 2000)
        lo = (eb.b - 52) < lo ? (eb.b - 52) : lo;
    return lo;
}

template <int NBMAX = RB_NB, int W = RB_W>
__device__ __forceinline__ RowAnchor row_anchor(double amax, double xmax, double b0, int h, int elow)
{
    int eT = -100000;
    if (amax > 0.0 && xmax > 0.0)
        eT = ilogb_bits(amax) + ilogb_bits(xmax) + 2;
    if (b0 != 0.0) {
        const int eb = ilogb_bits(fabs(b0)) + 1;
        eT = eT > eb ? eT : eb;
    }
    RowAnchor r;
    r.any = eT > -100000;
    int e0 = eT + h - 53;
    if (e0 < -600)
        e0 = -600;
    if (e0 > 900)
        e0 = 900;
    r.e0 = e0;
    // bins q = 0..nb-1 have quanta 2^(e0 - W q); the last must reach elow
    int nb = (e0 - elow + W - 1) / W + 1;
    if (nb < 1)
        nb = 1;
    if (nb > NBMAX)
        nb = NBMAX;
    if (e0 - W * (nb - 1) < -1074 + 0)  // keep every quantum a normal power of two
        nb = (e0 + 1022) / W + 1;
    r.nb = nb;
    return r;
}

template <int NBMAX>
__device__ __forceinline__ void deposit(double t, const double (&sig)[NBMAX], double (&bins)[NBMAX], int nb,
                                        double lim0, bool &bad)
{
    bad = bad || !(fabs(t) <= lim0);
#pragma unroll
    for (int b = 0; b < NBMAX; ++b) {
        if (b < nb) {
            const double d = (sig[b] + t) - sig[b];
            bins[b] = bins[b] + d;
            t = t - d;
        }
    }
    bad = bad || (t != 0.0);
}

// Deposit NT terms at once, bin by bin, for bins q < nbu, nbu the same for
// every lane of the wave (the largest of their rows' bin counts, so the
// loop has no per-lane branch and the terms' chains interleave): each term
// gives its digit of bin q (extraction constant sg0 2^(-W q), an exact
// scaling while the quanta are normal) and keeps the rest; the digits are
// summed pairwise and added to the bin.  Every partial sum of a bin's
// digits is exact (below 2^53 of its quanta), so the grouping does not
// change the bins.  A row's terms have no bits below its own nb bins, so
// the bins past them receive zero digits; a nonzero digit there, or a term
// with bits left after nbu bins, marks the row as inexact, as a term with
// bits left after nb bins does in deposit.
template <int NBMAX, int NT, int W = RB_W>
__device__ __forceinline__ void deposit_many(double (&tt)[NT], double sg0, double (&bins)[NBMAX], int nb, int nbu,
                                             double lim0, bool &bad)
{
    constexpr double STEP = 1.0 / (double)(1ull << W);
#pragma unroll
    for (int k = 0; k < NT; ++k)
        bad = bad || !(fabs(tt[k]) <= lim0);
    double sg = sg0;
#pragma unroll
    for (int q = 0; q < NBMAX; ++q) {
        if (q < nbu) {
            double d[NT];
            bool nz = false;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                d[k] = (sg + tt[k]) - sg;
                tt[k] = tt[k] - d[k];
                nz = nz | (d[k] != 0.0);
            }
            bad = bad | (nz & (q >= nb));
#pragma unroll
            for (int st = 1; st < NT; st *= 2)
#pragma unroll
                for (int k = 0; k + st < NT; k += 2 * st)
                    d[k] = d[k] + d[k + st];
            bins[q] = bins[q] + d[0];
            sg = sg * STEP;
        }
    }
#pragma unroll
    for (int k = 0; k < NT; ++k)
        bad = bad | (tt[k] != 0.0);
}

// The largest of the wave's bin counts (lanes without a row give 0), as a
// wave-uniform value.
__device__ __forceinline__ int wave_max_nb(int nb)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(nb, off, 64);
        nb = o > nb ? o : nb;
    }
    return __builtin_amdgcn_readfirstlane(nb);
}

// ---- exact signed integer in 32-bit limbs (carry-save in int64) ------------
// Limbs for the integer of NB bins: digits below 2^53 units of their bin, the
// top bin's unit at bit W (NB - 1), plus carry and sign headroom.
template <int NB, int W = RB_W>
struct Big {
    static constexpr int L = (NB * W + 53 + 64 + 31) / 32;
    int64_t l[L];
};

// add v * 2^pos, v signed with |v| < 2^63, pos >= 0
template <int NB, int W>
__device__ __forceinline__ void big_add(Big<NB, W> &B, int64_t v, int pos)
{
    const int L = pos >> 5, sh = pos & 31;
    const uint64_t lo = (uint64_t)(v & 0xffffffffLL);
    const int64_t hi = v >> 32;  // arithmetic: v = lo + hi * 2^32
    const uint64_t los = lo << sh;
#pragma unroll
    for (int q = 0; q < Big<NB, W>::L; ++q) {
        if (q == L)
            B.l[q] += (int64_t)(los & 0xffffffffULL);
        if (q == L + 1)
            B.l[q] += (int64_t)(los >> 32) + hi * ((int64_t)1 << sh);
    }
}

template <int NB, int W>
__device__ __forceinline__ void big_norm(Big<NB, W> &B)
{
#pragma unroll
    for (int q = 0; q < Big<NB, W>::L - 1; ++q) {
        const int64_t c = B.l[q] >> 32;
        B.l[q] -= c * ((int64_t)1 << 32);
        B.l[q + 1] += c;
    }
}

template <int NB, int W>
__device__ __forceinline__ void big_neg(Big<NB, W> &B)
{
#pragma unroll
    for (int q = 0; q < Big<NB, W>::L; ++q)
        B.l[q] = -B.l[q];
}

// Round |B| (B normalised, non-negative) to nearest binary64 mantissa:
// returns mant (0 if B == 0) and the bit position of its least significant
// bit.
template <int NB, int W>
__device__ __forceinline__ uint64_t big_round(const Big<NB, W> &M, int &lsb)
{
    constexpr int BLN = Big<NB, W>::L;
    int hl = -1;
#pragma unroll
    for (int q = BLN - 1; q >= 0; --q)
        if (hl < 0 && M.l[q] != 0)
            hl = q;
    if (hl < 0) {
        lsb = 0;
        return 0;
    }
    uint64_t l2 = 0, l1 = 0, l0 = 0;  // limbs hl, hl-1, hl-2
    bool below = false;               // any bit in limbs < hl-2
#pragma unroll
    for (int q = 0; q < BLN; ++q) {
        const uint64_t v = (uint64_t)M.l[q];
        if (q == hl)
            l2 = v;
        if (q == hl - 1)
            l1 = v;
        if (q == hl - 2)
            l0 = v;
        if (q < hl - 2 && v != 0)
            below = true;
    }
    const int msb = 31 - __clz((unsigned)l2);
    // 64 bits starting at the most significant set bit
    const uint64_t top = (l2 << (63 - msb)) | (l1 << (31 - msb)) | (l0 >> (msb + 1));
    const bool lowbits = (l0 & ((1ULL << (msb + 1)) - 1ULL)) != 0;
    uint64_t mant = top >> 11;
    const bool guard = (top >> 10) & 1ULL;
    const bool sticky = ((top & 0x3ffULL) != 0) || lowbits || below;
    int T = 32 * hl + msb;
    if (guard && (sticky || (mant & 1ULL))) {
        ++mant;
        if (mant == (1ULL << 53)) {
            mant >>= 1;
            ++T;
        }
    }
    lsb = T - 52;
    return mant;
}


// Canonical LW-word form (greedy round-to-nearest: quad-double for LW = 4,
// the 424-bit long precision for LW = 8) of the exact sum held in
// bins[0..nb) (bin q holds a multiple of 2^(e0 - W q)); returns true if a
// word fell outside the binary64 normal range.  The integer is kept as its
// magnitude while a word is rounded off it (negated in place), so one limb
// array suffices.
// Add the digits of bins[0..cnt) = bins q0.. of a row with nb bins (bin q
// holds multiples of 2^(e0 - W q)) into the row's integer, whose unit is the
// last bin's quantum.
template <int NB, int W, int CNT>
__device__ __forceinline__ void bins_into_big(Big<NB, W> &B, const double (&bins)[CNT], int q0, int nb, int e0)
{
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
        const int q = q0 + c;
        if (q < nb) {
            const double dig = ldexp(bins[c], -(e0 - W * q));
            big_add(B, (int64_t)dig, W * (nb - 1 - q));
        }
    }
}

// Canonical LW-word rounding of the row's integer (unit 2^elow); returns
// true if a word fell outside the binary64 normal range.
template <int NB, int W, int LW>
__device__ __forceinline__ bool big_to_words(Big<NB, W> &B, int elow, double (&out)[LW])
{
    bool bad = false;
#pragma unroll
    for (int w = 0; w < LW; ++w)
        out[w] = 0.0;
    for (int w = 0; w < LW; ++w) {
        big_norm(B);
        const bool neg = B.l[Big<NB, W>::L - 1] < 0;
        if (neg) {
            big_neg(B);
            big_norm(B);
        }
        int lsb;
        const uint64_t mant = big_round(B, lsb);
        if (mant == 0)
            break;
        const int e = lsb + elow;
        if (e + 52 > 1023 || e + 52 < -1022)
            bad = true;
        const double v = ldexp((double)mant, e);
        out[w] = neg ? -v : v;
        // |value| -= mant * 2^lsb (lsb may be negative only when the integer
        // is below 2^53, then mant's low bits are zero), then back to the sign
        if (lsb >= 0)
            big_add(B, -(int64_t)mant, lsb);
        else
            big_add(B, -((int64_t)mant >> (-lsb)), 0);
        if (neg)
            big_neg(B);
    }
    return bad;
}

template <int NBMAX, int LW, int W = RB_W>
__device__ __forceinline__ bool bins_to_words(const double (&bins)[NBMAX], int nb, int e0, double (&out)[LW])
{
    Big<NBMAX, W> B;
#pragma unroll
    for (int q = 0; q < Big<NBMAX, W>::L; ++q)
        B.l[q] = 0;
    bins_into_big(B, bins, 0, nb, e0);
    return big_to_words(B, e0 - W * (nb - 1), out);
}

template <int NBMAX, int W = RB_W>
__device__ __forceinline__ bool bins_to_qd(const double (&bins)[NBMAX], int nb, int e0, double (&out)[4])
{
    return bins_to_words<NBMAX, 4, W>(bins, nb, e0, out);
}

}  // namespace bnc

// Mixed-precision iterative refinement (Kouya 2021, Sec. 2, Listing 1) and
// its long-precision pieces: the exact residual, norms, the update.  The
// long precision is LW binary64 words: 4 (quad-double) or 8 (424 bits, the
// long precision of the paper's Table 2).
//
// Residual r = b - A x.  Every product A_ij^(u) x_j^(w) is split exactly by
// TwoProd; every resulting binary64 term is cut into fixed-point digits of
// W = 34 bits over up to 40 bins anchored at the row's largest possible term
// (an extraction (sigma + t) - sigma with sigma = 1.5 * 2^(52 + e_bin) is
// exact and rounds t to a multiple of 2^e_bin).  The number of bins a row
// uses reaches down to a bound on the lowest bit of any term, taken from the
// smallest exponents of the words of A, x and b, so the digit sums are
// exact: they stay below 2^53 units of their bin for up to 2^19 terms per
// row.  The bins are then read as one signed integer and rounded greedily
// to LW binary64 words with round-to-nearest-even: the canonical LW-word
// form of the exact residual.  Only data spanning more than 1360
// bits would leave bits below the window; such a row reports "inexact".
#include <string.h>

#include "common.hpp"
#include "exact.hpp"
#include "mw.hpp"

namespace bnc {

// Kernels of the refinement loop take an optional device flag: when it is
// set they return at once (the device-driven loop of bnc_refine_async skips
// the iterations after its stopping tests have fired).  nullptr: run.
#define BNC_SKIP_IF(skip)     \
    if ((skip) && *(skip))    \
        return;

template <int K>
int getrf_run(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *scr,
              hipStream_t s, int oz, double *oz_buf);
size_t oz_slices_bytes(int64_t n);
template <int K>
int getrs_perm(int64_t n, const double *LU, int64_t lda, int64_t ldp, const int32_t *perm, const double *rd,
               const double *b, int64_t ldb, double *y, int64_t ldy, void *ws, hipStream_t s, int64_t *info,
               const int *skip = nullptr);
size_t trsv_ws_bytes(int64_t n);
size_t features_workspace_bytes(int slots);
int features_run(int64_t count, const int64_t *n, const double *const *A, const double *const *b,
                 const int32_t *order, float *F, void *work, int slots, hipStream_t s);
int mlp_forward_run(int64_t B, const float *X, const float *norm, const float *P, float *O, hipStream_t s);
constexpr int64_t SEL_NMAX = 512;  // orders the features kernel takes
template <int K>
int diag_recip_run(int64_t n, const double *LU, int64_t lda, int64_t ldp, double *rd, hipStream_t s);
int ipiv_to_perm(int64_t n, const int64_t *ipiv, int32_t *perm, hipStream_t s);

constexpr int RES_ROWS = 64;
constexpr int RES_WAVES = 4;
constexpr int RED_BLOCKS = 256;  // partial-sum slots of the deterministic reductions
// partial bins of rows [64*bx, +64); workgroup column split sidx, each wave
// a quarter of it: split index sidx*4 + wave
// the deposits of one row's slice of columns into NB bins (nb <= NB used)
template <int AW, int LW, int NB>
__device__ __forceinline__ void resid_slice(const double *__restrict__ A, int64_t lda, int64_t ldpa,
                                            const double *__restrict__ x, int64_t ldx, const double *__restrict__ b,
                                            int64_t ldb, int64_t i, int64_t q0, int64_t q1, bool with_b,
                                            const RowAnchor &an, double *__restrict__ out, int64_t stride, bool &bad)
{
    const int nb = an.nb;
    double bins[NB], sig[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        bins[q] = 0.0;
        sig[q] = q < nb ? 1.5 * pow2(an.e0 - RB_W * q + 52) : 0.0;
    }
    const double lim0 = pow2(an.e0 + 51);
    // column j's words of x and of A are loaded one column ahead, two
    // register sets taking turns (the loads are unconditional, the next
    // index clamped to the slice), so the deposits of one column run while
    // the next column's loads are in flight
    auto load = [&](int64_t j, double (&xv)[LW], double (&av)[AW]) {
#pragma unroll
        for (int w = 0; w < LW; ++w)
            xv[w] = x[w * ldx + j];
#pragma unroll
        for (int u = 0; u < AW; ++u)
            av[u] = A[u * ldpa + j * lda + i];
    };
    auto col = [&](const double (&xv)[LW], const double (&av)[AW]) {
#pragma unroll
        for (int u = 0; u < AW; ++u)
#pragma unroll
            for (int w = 0; w < LW; ++w) {
                double lo;
                const double hi = two_prod(av[u], xv[w], lo);
                deposit(-hi, sig, bins, nb, lim0, bad);
                deposit(-lo, sig, bins, nb, lim0, bad);
            }
    };
    int64_t j = q0;
    if (NB > 16) {  // the rare wide windows: plain loop (their bins already fill the registers)
        for (; j < q1; ++j) {
            double xv[LW], av[AW];
            load(j, xv, av);
            col(xv, av);
        }
    } else if (j < q1) {
        double x0[LW], a0[AW], x1[LW], a1[AW];
        load(j, x0, a0);
        for (; j + 1 < q1; j += 2) {
            load(j + 1, x1, a1);
            col(x0, a0);
            load(j + 2 < q1 ? j + 2 : q1 - 1, x0, a0);
            col(x1, a1);
        }
        if (j < q1)  // odd count: x0, a0 hold column q1 - 1
            col(x0, a0);
    }
    if (with_b) {
#pragma unroll
        for (int w = 0; w < LW; ++w)
            deposit(b[w * ldb + i], sig, bins, nb, lim0, bad);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q)
        if (q < nb)
            out[q * stride] = bins[q];
}

template <int AW, int LW>
__global__ void __launch_bounds__(RES_ROWS *RES_WAVES)
    k_resid_partial(int64_t n, const double *__restrict__ A, int64_t lda, int64_t ldpa, const double *__restrict__ x,
                    int64_t ldx, const double *__restrict__ b, int64_t ldb, const double *__restrict__ rowmax,
                    const double *__restrict__ xmaxp, const ExpBounds *__restrict__ ebp, int h, int64_t chunk,
                    double *__restrict__ part, int32_t *__restrict__ inexact, const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int lane = threadIdx.x % RES_ROWS, wv = threadIdx.x / RES_ROWS;
    const int64_t i = (int64_t)blockIdx.x * RES_ROWS + lane;
    const int split = blockIdx.y * RES_WAVES + wv;
    if (i >= n)
        return;
    bool bad = false;
    const double xm = *xmaxp;
    const RowAnchor an = row_anchor(rowmax[i], xm, b[i], h, lowest_bit(*ebp));
    if (an.any) {
        const int64_t j0 = (int64_t)blockIdx.y * chunk;
        const int64_t j1 = (j0 + chunk) < n ? (j0 + chunk) : n;
        const int64_t len = j1 > j0 ? j1 - j0 : 0;
        const int64_t q0 = j0 + (len * wv) / RES_WAVES, q1 = j0 + (len * (wv + 1)) / RES_WAVES;
        double *out = part + (int64_t)split * RB_NB * n + i;
        // the window is usually a few bins wide: deposit loops sized to it
        if (an.nb <= 8)
            resid_slice<AW, LW, 8>(A, lda, ldpa, x, ldx, b, ldb, i, q0, q1, split == 0, an, out, n, bad);
        else if (an.nb <= 16)
            resid_slice<AW, LW, 16>(A, lda, ldpa, x, ldx, b, ldb, i, q0, q1, split == 0, an, out, n, bad);
        else
            resid_slice<AW, LW, RB_NB>(A, lda, ldpa, x, ldx, b, ldb, i, q0, q1, split == 0, an, out, n, bad);
    }
    if (bad)
        atomicOr(inexact, 1);
}

// smallest floor(log2|v|) over the nonzero words (2000 if none)
__global__ void k_minexp(int64_t rows, int64_t cols, int64_t ld, int words, int64_t ldp, const double *__restrict__ v,
                         int *__restrict__ out, const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    __shared__ int s[256];
    int m = 2000;
    const int64_t n = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t idx = (e / rows) * ld + e % rows;
        for (int w = 0; w < words; ++w) {
            const double t = v[w * ldp + idx];
            if (t != 0.0) {
                const int ex = ilogb_bits(t);
                m = ex < m ? ex : m;
            }
        }
    }
    s[threadIdx.x] = m;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if (threadIdx.x < t)
            s[threadIdx.x] = s[threadIdx.x + t] < s[threadIdx.x] ? s[threadIdx.x + t] : s[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMin(out, s[0]);
}

__global__ void k_fill_i32(int *p, int64_t n, int v, const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

// Sum of the S partial digit sums of bin q of row i into partial slot 0
// (thread per (row, bin); every partial sum is a sum of a subset of the
// row's digits, so each addition is exact and the order does not matter).
__global__ void __launch_bounds__(256)
    k_resid_sum(int64_t n, int S, double *__restrict__ part, const double *__restrict__ rowmax,
                const double *__restrict__ xmaxp, const ExpBounds *__restrict__ ebp, const double *__restrict__ b,
                int h, const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int q = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    if (i >= n || q >= RB_NB)
        return;
    const RowAnchor an = row_anchor(rowmax[i], *xmaxp, b[i], h, lowest_bit(*ebp));
    if (!an.any || q >= an.nb)
        return;
    double s = 0.0;
    for (int t = 0; t < S; ++t)
        s = s + part[((int64_t)t * RB_NB + q) * n + i];
    part[(int64_t)q * n + i] = s;
}

template <int LW>
__global__ void __launch_bounds__(256)
    k_resid_final(int64_t n, int S, const double *__restrict__ part, const double *__restrict__ rowmax,
                  const double *__restrict__ xmaxp, const ExpBounds *__restrict__ ebp, const double *__restrict__ b,
                  int h, double *__restrict__ r, int64_t ldr, int32_t *__restrict__ inexact,
                  const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const RowAnchor an = row_anchor(rowmax[i], *xmaxp, b[i], h, lowest_bit(*ebp));
    double out[LW];
#pragma unroll
    for (int w = 0; w < LW; ++w)
        out[w] = 0.0;
    bool bad = false;
    if (an.any) {
        double bins[RB_NB];
#pragma unroll
        for (int q = 0; q < RB_NB; ++q) {
            double s = 0.0;
            if (q < an.nb)
                for (int t = 0; t < S; ++t)
                    s = s + part[((int64_t)t * RB_NB + q) * n + i];  // S = number of splits
            bins[q] = s;
        }
        bad = bins_to_words<RB_NB, LW>(bins, an.nb, an.e0, out);
    }
#pragma unroll
    for (int w = 0; w < LW; ++w)
        r[w * ldr + i] = out[w];
    if (bad)
        atomicOr(inexact, 1);
}

// ---- small vector / matrix helpers ------------------------------------------

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v, const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ void k_check_finite(int64_t rows, int64_t cols, int words, const double *__restrict__ p, int64_t ld,
                               int64_t ldp, int32_t *__restrict__ flag)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols)
        return;
    const int64_t i = e % rows, j = e / rows;
    bool bad = false;
    for (int w = 0; w < words; ++w)
        bad = bad || !isfinite(p[w * ldp + j * ld + i]);
    if (bad)
        atomicOr(flag, 1);
}

// K-word copy of an aw-word matrix (renormalised)
template <int K, int AW>
__global__ void k_stage(int64_t n, const double *__restrict__ A, int64_t lda, int64_t ldpa, double *__restrict__ LU,
                        int64_t ldl, int64_t ldpl)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n)
        return;
    const int64_t i = e % n, j = e / n;
    double v[AW], o[K];
#pragma unroll
    for (int u = 0; u < AW; ++u)
        v[u] = A[u * ldpa + j * lda + i];
    renorm<K, AW>(v, o);
#pragma unroll
    for (int w = 0; w < K; ++w)
        LU[w * ldpl + j * ldl + i] = o[w];
}

// rowmax[i] = max_j |A0(i, j)|  (thread per row, coalesced across rows)
// row maxima of |A| (leading words): blockIdx.y takes a slice of the
// columns; slices combine with an integer maximum of the bit patterns
// (non-negative doubles order like their bits), which is exact in any order
constexpr int ROWMAX_SPLIT = 32;
__global__ void k_rowmax(int64_t n, const double *__restrict__ A, int64_t lda,
                         unsigned long long *__restrict__ rowmax_bits)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t j0 = (int64_t)blockIdx.y * n / ROWMAX_SPLIT, j1 = ((int64_t)blockIdx.y + 1) * n / ROWMAX_SPLIT;
    double m = 0.0;
    for (int64_t j = j0; j < j1; ++j)
        m = fmax(m, fabs(A[j * lda + i]));
    atomicMax(rowmax_bits + i, (unsigned long long)__double_as_longlong(m));
}

// max |v(i, j)| over rows x cols entries (leading dimension ld), folded into
// *bits with an integer max (non-negative doubles order like their bits)
__global__ void k_absmax(int64_t rows, int64_t cols, int64_t ld, const double *__restrict__ v,
                         unsigned long long *__restrict__ bits, const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    __shared__ double s[256];
    double m = 0.0;
    const int64_t n = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(v[(e / rows) * ld + e % rows]));
    s[threadIdx.x] = m;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if (threadIdx.x < t)
            s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + t]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(bits, (unsigned long long)__double_as_longlong(s[0]));
}

// deterministic sum of (v_i 2^-e)^2: fixed per-block partials, then one
// block sums the partials in order
__global__ void k_sumsq_part(int64_t rows, int64_t cols, int64_t ld, const double *__restrict__ v,
                             const unsigned long long *__restrict__ maxbits, double *__restrict__ part,
                             const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    __shared__ double s[256];
    const double m = __longlong_as_double((long long)*maxbits);
    const double sc = pow2(-(norm_exp(m) + 1));
    double acc = 0.0;
    const int64_t n = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double t = v[(e / rows) * ld + e % rows] * sc;
        acc = acc + t * t;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int t = 128; t > 0; t >>= 1) {
        if (threadIdx.x < t)
            s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + t];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = s[0];
}

__global__ void k_sumsq_final(int nparts, const double *__restrict__ part, double *__restrict__ out,
                              const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < nparts; ++t)
            s = s + part[t];
        *out = s;
    }
}

// dst (K words) = renorm(src (LW words) * 2^-e), e from the power-of-two max
template <int K, int LW>
__global__ void k_round_scaled(int64_t n, const double *__restrict__ src, int64_t lds_,
                               const unsigned long long *__restrict__ maxbits, double *__restrict__ dst, int64_t ldd,
                               const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double sc = maxbits ? pow2(-norm_exp(__longlong_as_double((long long)*maxbits))) : 1.0;
    double v[LW], o[K];
#pragma unroll
    for (int w = 0; w < LW; ++w)
        v[w] = src[w * lds_ + i] * sc;
    renorm<K, LW>(v, o);
#pragma unroll
    for (int w = 0; w < K; ++w)
        dst[w * ldd + i] = o[w];
}

// x = extend(z), LW words from K words
template <int K, int LW>
__global__ void k_extend(int64_t n, const double *__restrict__ z, int64_t ldz, double *__restrict__ x, int64_t ldx,
                         const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
#pragma unroll
    for (int w = 0; w < LW; ++w)
        x[w * ldx + i] = w < K ? z[w * ldz + i] : 0.0;
}

// z <- z * 2^e in place (e from the residual max), then x <- x + extend(z)
// in LW-word addition
template <int K, int LW>
__global__ void k_scale_update(int64_t n, double *__restrict__ z, int64_t ldz,
                               const unsigned long long *__restrict__ rmaxbits, double *__restrict__ x, int64_t ldx,
                               const int *__restrict__ skip)
{
    BNC_SKIP_IF(skip);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double sc = pow2(norm_exp(__longlong_as_double((long long)*rmaxbits)));
    double zv[LW], xv[LW], o[LW];
#pragma unroll
    for (int w = 0; w < LW; ++w) {
        zv[w] = w < K ? z[w * ldz + i] * sc : 0.0;
        xv[w] = x[w * ldx + i];
    }
    add<LW>(xv, zv, o);
#pragma unroll
    for (int w = 0; w < K; ++w)
        z[w * ldz + i] = zv[w];
#pragma unroll
    for (int w = 0; w < LW; ++w)
        x[w * ldx + i] = o[w];
}

__global__ void k_zero(int64_t n, double *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0.0;
}

// ---- host helpers -------------------------------------------------------------

static inline unsigned grid1(int64_t n, int t = 256) { return (unsigned)ceil_div(n > 0 ? n : 1, t); }

static int64_t residual_terms(int64_t n, int aw, int lw) { return 2 * (int64_t)aw * lw * n + lw; }

static int residual_h(int64_t n, int aw, int lw)
{
    // h with 2^h >= 2 * terms; terms per row = 2 * aw * lw * n + lw
    const int64_t N = residual_terms(n, aw, lw);
    int h = 1;
    while (((int64_t)1 << h) < 2 * N)
        ++h;
    return h;
}

// workgroup column splits (each split into RES_WAVES wave splits): enough
// waves to hide the deposit chains' latency (about four per SIMD at n = 4096)
constexpr int RES_SPLITS_MAX = 16;
static int residual_splits(int64_t n)
{
    int64_t S = n / 256;
    if (S < 1)
        S = 1;
    if (S > RES_SPLITS_MAX)
        S = RES_SPLITS_MAX;
    return (int)S;
}

size_t residual_scratch_bytes(int64_t n)
{
    return (size_t)RES_SPLITS_MAX * RES_WAVES * RB_NB * n * sizeof(double) + 256;
}

// minimum exponents of the words of a rows x cols (ld) matrix with `words`
// planes (ldp apart), folded into *out
int minexp_run(int64_t rows, int64_t cols, int64_t ld, int words, int64_t ldp, const double *v, int *out,
               hipStream_t s, const int *skip = nullptr)
{
    unsigned g = grid1(rows * cols);
    if (g > RED_BLOCKS)
        g = RED_BLOCKS;
    hipLaunchKernelGGL(k_minexp, dim3(g), dim3(256), 0, s, rows, cols, ld, words, ldp, v, out, skip);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

int fill_i32_run(int *p, int64_t n, int v, hipStream_t s, const int *skip = nullptr)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1(n)), dim3(256), 0, s, p, n, v, skip);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// r = b - A x (exact -> canonical lw-word form); rowmax, xmax and the
// exponent bounds precomputed on the device; x, b, r have lw words
int residual_run(int64_t n, int aw, int lw, const double *A, int64_t lda, int64_t ldpa, const double *x, int64_t ldx,
                 const double *b, int64_t ldb, const double *rowmax, const double *xmax, const void *ebounds,
                 double *part, double *r, int64_t ldr, int32_t *inexact, hipStream_t s, const int *skip = nullptr)
{
    if (n == 0)
        return BNC_OK;
    if (residual_terms(n, aw, lw) >= (1LL << 19))
        return fail_arg(BNC_ERR_UNSUPPORTED, "residual: too many terms per row for exact accumulation");
    const int h = residual_h(n, aw, lw);
    const int S = residual_splits(n);
    const int64_t chunk = ceil_div(n, S);
    const ExpBounds *eb = (const ExpBounds *)ebounds;
    dim3 grid((unsigned)ceil_div(n, RES_ROWS), (unsigned)S);
    const dim3 t(RES_ROWS * RES_WAVES);
    if (aw == 1 && lw == 4)
        hipLaunchKernelGGL((k_resid_partial<1, 4>), grid, t, 0, s, n, A, lda, ldpa, x, ldx, b, ldb, rowmax, xmax, eb,
                           h, chunk, part, inexact, skip);
    else if (aw == 4 && lw == 4)
        hipLaunchKernelGGL((k_resid_partial<4, 4>), grid, t, 0, s, n, A, lda, ldpa, x, ldx, b, ldb, rowmax, xmax, eb,
                           h, chunk, part, inexact, skip);
    else if (aw == 1)
        hipLaunchKernelGGL((k_resid_partial<1, 8>), grid, t, 0, s, n, A, lda, ldpa, x, ldx, b, ldb, rowmax, xmax, eb,
                           h, chunk, part, inexact, skip);
    else
        hipLaunchKernelGGL((k_resid_partial<4, 8>), grid, t, 0, s, n, A, lda, ldpa, x, ldx, b, ldb, rowmax, xmax, eb,
                           h, chunk, part, inexact, skip);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_resid_sum, dim3((unsigned)ceil_div(n, 64), (unsigned)ceil_div(RB_NB, 4)), dim3(256), 0, s, n,
                       S * RES_WAVES, part, rowmax, xmax, eb, b, h, skip);
    BNC_LAUNCH_CHECK();
    if (lw == 4)
        hipLaunchKernelGGL(k_resid_final<4>, dim3(grid1(n)), dim3(256), 0, s, n, 1, (const double *)part, rowmax, xmax,
                           eb, b, h, r, ldr, inexact, skip);
    else
        hipLaunchKernelGGL(k_resid_final<8>, dim3(grid1(n)), dim3(256), 0, s, n, 1, (const double *)part, rowmax, xmax,
                           eb, b, h, r, ldr, inexact, skip);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// Stand-alone residual (bnc_residual) in a caller workspace: row maxima,
// the vector maximum and exponent bounds, then the partial bins.
size_t residual_workspace_bytes(int64_t n)
{
    if (n <= 0)
        return 0;
    return align256((size_t)n * sizeof(double)) + 256 + residual_scratch_bytes(n);
}

int rowmax_run(int64_t n, const double *A, int64_t lda, double *rowmax, hipStream_t s);
int absmax_run(int64_t rows, int64_t cols, int64_t ld, const double *v, unsigned long long *bits, hipStream_t s,
               const int *skip = nullptr);

int residual_ws_run(int64_t n, int aw, int lw, const double *A, int64_t lda, int64_t ldpa, const double *x,
                    int64_t ldpx, const double *b, int64_t ldpb, double *r, int64_t ldpr, int32_t *inexact, void *work,
                    hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    char *W = (char *)work;
    double *rowmax = (double *)W;
    unsigned long long *xmax = (unsigned long long *)(W + align256((size_t)n * sizeof(double)));
    int *eb = (int *)((char *)xmax + 64);  // exponent bounds a, x, b
    double *part = (double *)((char *)xmax + 256);
    int rc;
    if ((rc = rowmax_run(n, A, lda, rowmax, s)) || (rc = absmax_run(n, 1, n, x, xmax, s)) ||
        (rc = fill_i32_run(eb, 3, 2000, s)) || (rc = minexp_run(n, n, lda, aw, ldpa, A, eb, s)) ||
        (rc = minexp_run(n, 1, n, lw, ldpx, x, eb + 1, s)) || (rc = minexp_run(n, 1, n, lw, ldpb, b, eb + 2, s)))
        return rc;
    return residual_run(n, aw, lw, A, lda, ldpa, x, ldpx, b, ldpb, rowmax, (const double *)xmax, eb, part, r, ldpr,
                        inexact, s);
}

// rowmax of |A0| and a one-element max of a vector's leading words
int rowmax_run(int64_t n, const double *A, int64_t lda, double *rowmax, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid1(n)), dim3(256), 0, s, (uint64_t *)rowmax, n, (uint64_t)0,
                       (const int *)nullptr);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rowmax, dim3(grid1(n), ROWMAX_SPLIT), dim3(256), 0, s, n, A, lda,
                       (unsigned long long *)rowmax);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

int absmax_run(int64_t rows, int64_t cols, int64_t ld, const double *v, unsigned long long *bits, hipStream_t s,
               const int *skip)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t *)bits, (int64_t)1, (uint64_t)0, skip);
    BNC_LAUNCH_CHECK();
    unsigned g = grid1(rows * cols);
    if (g > RED_BLOCKS)
        g = RED_BLOCKS;
    hipLaunchKernelGGL(k_absmax, dim3(g), dim3(256), 0, s, rows, cols, ld, v, bits, skip);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

int sumsq_run(int64_t rows, int64_t cols, int64_t ld, const double *v, const unsigned long long *maxbits,
              double *part, double *out, hipStream_t s, const int *skip = nullptr)
{
    unsigned g = grid1(rows * cols);
    if (g > RED_BLOCKS)
        g = RED_BLOCKS;
    hipLaunchKernelGGL(k_sumsq_part, dim3(g), dim3(256), 0, s, rows, cols, ld, v, maxbits, part, skip);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(64), 0, s, (int)g, (const double *)part, out, skip);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// ---- the refinement driver -----------------------------------------------------

static inline double bits_to_double(unsigned long long u)
{
    double d;
    memcpy(&d, &u, sizeof d);
    return d;
}

struct Scal {
    unsigned long long amax, xmax, rmax, zmax;
    double asq, xsq, rsq, pad;
    int32_t nonfinite, inexact;
    int64_t info;   // getrf info of the last factorisation (-1: exchange timed out)
    int64_t tinfo;  // -1 once a substitution's bounded wait gave up
    ExpBounds eb;   // a, x, b
    int32_t pad2;
    // the device-driven loop (bnc_refine_async): done is the kernels' skip
    // flag, set once a stopping test or a failure has decided the outcome
    int32_t done, status, iters, nz;
    double zlast, zprev, thresh_c, a_norm, resid_norm, x_norm;
};
static_assert(sizeof(Scal) % 8 == 0, "Scal is cleared as 64-bit words");

struct RefineLayout {
    size_t lu, ipiv, perm, rd, r, v, rowmax, part, red, scal, getrf, oz, flags, sel, total;
};

// the selector's scratch (factor_words = 0): the order and the pointers
// the features kernel reads, 24 features, 5 outputs, a contiguous copy of
// A's leading plane, the features workspace
struct SelScratch {
    int64_t n;
    const double *A;
    const double *b;
    int64_t pad;
    float F[24];
    float O[8];
};
static size_t sel_bytes(int64_t n)
{
    if (n > SEL_NMAX)
        return 0;
    return align256(sizeof(SelScratch)) + align256((size_t)n * n * sizeof(double)) + features_workspace_bytes(1);
}

size_t getrf_scratch_bytes(int K, int64_t n);

static RefineLayout refine_layout(int64_t n, int K, bool sel = false)
{
    RefineLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    L.lu = take((size_t)K * n * n * sizeof(double));
    L.ipiv = take((size_t)n * sizeof(int64_t));
    L.perm = take((size_t)n * sizeof(int32_t));
    L.rd = take((size_t)K * n * sizeof(double));
    L.r = take((size_t)8 * n * sizeof(double));  // up to 8 long words
    L.v = take((size_t)K * n * sizeof(double));
    L.rowmax = take((size_t)n * sizeof(double));
    L.part = take(residual_scratch_bytes(n));
    L.red = take((size_t)RED_BLOCKS * sizeof(double));
    L.scal = take(sizeof(Scal));
    L.getrf = take(getrf_scratch_bytes(K, n));
    L.oz = take(oz_slices_bytes(n));
    L.flags = take(trsv_ws_bytes(n));
    L.sel = take(sel ? sel_bytes(n) : 0);
    L.total = off;
    return L;
}

// K = 0: the selector's choice (any K, plus its scratch)
size_t refine_workspace_bytes(int64_t n, int K) { return refine_layout(n, K ? K : 4, K == 0).total; }

__global__ void k_sel_setup(SelScratch *S, int64_t n, const double *A, const double *b)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->n = n;
        S->A = A;
        S->b = b;
    }
}

// dst (n x n, contiguous) = the leading plane of A (leading dimension lda)
__global__ void k_copy_plane(int64_t n, const double *__restrict__ A, int64_t lda, double *__restrict__ dst)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n * n)
        dst[e] = A[(e / n) * lda + e % n];
}

// Dispatch a K-templated launch on the runtime word count kc (1..4).
#define BNC_KSWITCH(kc, BODY)                     \
    switch (kc) {                                 \
    case 1: {                                     \
        constexpr int KK = 1;                     \
        BODY;                                     \
    } break;                                      \
    case 2: {                                     \
        constexpr int KK = 2;                     \
        BODY;                                     \
    } break;                                      \
    case 3: {                                     \
        constexpr int KK = 3;                     \
        BODY;                                     \
    } break;                                      \
    default: {                                    \
        constexpr int KK = 4;                     \
        BODY;                                     \
    } break;                                      \
    }

// Dispatch on the long precision lw (4 or 8 words).
#define BNC_LSWITCH(lw, BODY)          \
    if ((lw) == 8) {                   \
        constexpr int LL = 8;          \
        BODY;                          \
    } else {                           \
        constexpr int LL = 4;          \
        BODY;                          \
    }

// The refinement loop with the factor precision kc as a run-time value, so
// that a stagnating loop can refactor in more words and go on (escalation).
// The long precision (x, b, r) has lw = opts->long_words words (0: 4).
int refine_drive(int K0, int64_t n, int aw, const double *A, int64_t lda, int64_t ldpa, const double *b,
                 int64_t ldpb, double *x, int64_t ldpx, void *work, const bnc_refine_opts *o, bnc_refine_result *res,
                 hipStream_t s)
{
    const RefineLayout L = refine_layout(n, (o->escalate || K0 == 0) ? 4 : K0, K0 == 0);
    char *W = (char *)work;
    double *LU = (double *)(W + L.lu);
    int64_t *ipiv = (int64_t *)(W + L.ipiv);
    int32_t *perm = (int32_t *)(W + L.perm);
    double *rd = (double *)(W + L.rd);
    double *r = (double *)(W + L.r);
    double *v = (double *)(W + L.v);
    double *rowmax = (double *)(W + L.rowmax);
    double *part = (double *)(W + L.part);
    double *red = (double *)(W + L.red);
    Scal *sc = (Scal *)(W + L.scal);
    void *gscr = W + L.getrf;
    double *ozb = (double *)(W + L.oz);
    void *tsflags = (void *)(W + L.flags);
    const int64_t ldp = n * n;
    const int lw = o->long_words ? o->long_words : 4;

    *res = bnc_refine_result{};
    if (K0 == 0) {
        // the learned choice: features of the system (leading words of A,
        // contiguous copy), the network, the largest logit (ties: fewer
        // words); orders the features kernel does not take start at 2
        K0 = 2;
        if (n <= SEL_NMAX) {
            char *SW = W + L.sel;
            SelScratch *ss = (SelScratch *)SW;
            double *Ac = (double *)(SW + align256(sizeof(SelScratch)));
            void *fws = (void *)((char *)Ac + align256((size_t)n * n * sizeof(double)));
            hipLaunchKernelGGL(k_copy_plane, dim3(grid1(n * n)), dim3(256), 0, s, n, A, lda, Ac);
            BNC_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_sel_setup, dim3(1), dim3(64), 0, s, ss, n, (const double *)Ac, b);
            BNC_LAUNCH_CHECK();
            int rc0;
            if ((rc0 = features_run(1, &ss->n, &ss->A, &ss->b, nullptr, ss->F, fws, 1, s)) ||
                (rc0 = mlp_forward_run(1, ss->F, o->selector_norm, o->selector_params, ss->O, s)))
                return rc0;
            float O[8];
            BNC_HIP(hipMemcpyAsync(O, ss->O, sizeof O, hipMemcpyDeviceToHost, s));
            BNC_HIP(hipStreamSynchronize(s));
            int best = 0;
            for (int c = 1; c < 4; ++c)
                if (O[c] > O[best])
                    best = c;
            K0 = best + 1;
        }
    }
    res->first_words = K0;
    res->final_words = K0;
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t *)sc, (int64_t)(sizeof(Scal) / 8), (uint64_t)0,
                       (const int *)nullptr);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_check_finite, dim3(grid1(n * n)), dim3(256), 0, s, n, n, aw, A, lda, ldpa, &sc->nonfinite);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_check_finite, dim3(grid1(n)), dim3(256), 0, s, n, (int64_t)1, lw, b, ldpb, ldpb,
                       &sc->nonfinite);
    BNC_LAUNCH_CHECK();
    Scal h{};
    BNC_HIP(hipMemcpyAsync(&h, sc, sizeof(Scal), hipMemcpyDeviceToHost, s));
    BNC_HIP(hipStreamSynchronize(s));
    auto zero_x = [&]() -> int {
        for (int w = 0; w < lw; ++w) {
            hipLaunchKernelGGL(k_zero, dim3(grid1(n)), dim3(256), 0, s, n, x + w * ldpx);
            BNC_LAUNCH_CHECK();
        }
        BNC_HIP(hipStreamSynchronize(s));
        return BNC_OK;
    };
    if (h.nonfinite) {
        res->status = BNC_NONFINITE;
        return zero_x();
    }
    // ||A||_F from leading words (scaled), row maxima for the residual anchor
    int rc;
    if ((rc = absmax_run(n, n, lda, A, &sc->amax, s)) || (rc = sumsq_run(n, n, lda, A, &sc->amax, red, &sc->asq, s)) ||
        (rc = rowmax_run(n, A, lda, rowmax, s)) || (rc = fill_i32_run(&sc->eb.a, 3, 2000, s)) ||
        (rc = minexp_run(n, n, lda, aw, ldpa, A, &sc->eb.a, s)) ||
        (rc = minexp_run(n, 1, n, lw, ldpb, b, &sc->eb.b, s)))
        return rc;

    // kc-word copy of A, factorisation, pivots as a permutation, diagonal
    // reciprocals; *info_out gets getrf's info
    int kc = K0;
    auto factor = [&](int oz, int64_t *info_out) -> int {
        int rc2 = BNC_OK;
        BNC_KSWITCH(kc, {
            if (aw == 1)
                hipLaunchKernelGGL((k_stage<KK, 1>), dim3(grid1(n * n)), dim3(256), 0, s, n, A, lda, ldpa, LU, n,
                                   ldp);
            else
                hipLaunchKernelGGL((k_stage<KK, 4>), dim3(grid1(n * n)), dim3(256), 0, s, n, A, lda, ldpa, LU, n,
                                   ldp);
            BNC_LAUNCH_CHECK();
            rc2 = getrf_run<KK>(n, LU, n, ldp, ipiv, &sc->info, gscr, s, oz, ozb);
        });
        if (rc2)
            return rc2;
        BNC_HIP(hipMemcpyAsync(&h, sc, sizeof(Scal), hipMemcpyDeviceToHost, s));
        BNC_HIP(hipStreamSynchronize(s));
        *info_out = h.info;
        if (h.info)
            return BNC_OK;
        if ((rc2 = ipiv_to_perm(n, ipiv, perm, s)))
            return rc2;
        BNC_KSWITCH(kc, rc2 = diag_recip_run<KK>(n, LU, n, ldp, rd, s));
        return rc2;
    };
    // v <- kc-word solve of the kc-word copy of src (scaled by 2^-e when
    // rmax is given)
    auto solve = [&](const double *src, int64_t lds, const unsigned long long *rmaxbits) -> int {
        int rc2 = BNC_OK;
        BNC_KSWITCH(kc, {
            BNC_LSWITCH(lw, hipLaunchKernelGGL((k_round_scaled<KK, LL>), dim3(grid1(n)), dim3(256), 0, s, n, src,
                                               lds, rmaxbits, r, n, (const int *)nullptr));
            BNC_LAUNCH_CHECK();
            rc2 = getrs_perm<KK>(n, LU, n, ldp, perm, rd, r, n, v, n, tsflags, s, &sc->tinfo);
        });
        return rc2;
    };

    const auto timed_out = [&]() { return fail_arg(BNC_ERR_TIMEOUT, "refine: a bounded wait gave up"); };
    int64_t info = 0;
    if ((rc = factor(o->ozaki_slices, &info)))
        return rc;
    // the split scheme left its exact range (a row or column scale too
    // small for its slice products): the same words in the plain form
    if (info == -3 && (rc = factor(0, &info)))
        return rc;
    while (info > 0 && o->escalate && kc < 4) {
        ++kc;
        ++res->escalations;
        if ((rc = factor(0, &info)))
            return rc;
    }
    if (info < 0)
        return timed_out();
    res->final_words = kc;
    res->info = info;
    const double amax = bits_to_double(h.amax);
    res->a_norm = sqrt(h.asq) * ldexp(1.0, norm_exp(amax) + 1);
    if (info) {
        res->status = BNC_SINGULAR;
        return zero_x();
    }
    // first solution in kc words, extended to quad-double
    if ((rc = solve(b, ldpb, nullptr)))
        return rc;
    BNC_KSWITCH(kc, BNC_LSWITCH(lw, hipLaunchKernelGGL((k_extend<KK, LL>), dim3(grid1(n)), dim3(256), 0, s, n,
                                                       (const double *)v, n, x, ldpx, (const int *)nullptr)));
    BNC_LAUNCH_CHECK();

    const double thresh_c = sqrt((double)n) * o->rtol * res->a_norm;
    double zlast = 0.0, zprev = 0.0;
    int nz = 0;  // corrections since the last factorisation
    int iters = 0;
    int status = BNC_MAX_ITER;
    for (int it = 0; it <= o->max_iter; ++it) {
        if ((rc = absmax_run(n, 1, n, x, &sc->xmax, s)) || (rc = fill_i32_run(&sc->eb.x, 1, 2000, s)) ||
            (rc = minexp_run(n, 1, n, lw, ldpx, x, &sc->eb.x, s)))
            return rc;
        if ((rc = residual_run(n, aw, lw, A, lda, ldpa, x, ldpx, b, ldpb, rowmax, (const double *)&sc->xmax, &sc->eb,
                               part, r, n, &sc->inexact, s)))
            return rc;
        if ((rc = absmax_run(n, 1, n, r, &sc->rmax, s)) || (rc = sumsq_run(n, 1, n, r, &sc->rmax, red, &sc->rsq, s)) ||
            (rc = sumsq_run(n, 1, n, x, &sc->xmax, red, &sc->xsq, s)))
            return rc;
        BNC_HIP(hipMemcpyAsync(&h, sc, sizeof(Scal), hipMemcpyDeviceToHost, s));
        BNC_HIP(hipStreamSynchronize(s));
        if (h.tinfo)
            return timed_out();
        const double rmax = bits_to_double(h.rmax), xmax = bits_to_double(h.xmax);
        if (nz > 0) {
            zprev = zlast;
            zlast = bits_to_double(h.zmax);
        }
        const double nr = rmax == 0.0 ? 0.0 : sqrt(h.rsq) * ldexp(1.0, norm_exp(rmax) + 1);
        const double nx = xmax == 0.0 ? 0.0 : sqrt(h.xsq) * ldexp(1.0, norm_exp(xmax) + 1);
        res->resid_norm = nr;
        res->x_norm = nx;
        res->residual_inexact = h.inexact ? 1 : 0;
        if (nr < thresh_c * nx + o->atol || (nz > 0 && zlast <= o->ctol * xmax)) {
            status = BNC_CONVERGED;
            break;
        }
        if (o->stagnation_ratio > 0.0 && nz >= 2 && zlast > o->stagnation_ratio * zprev) {
            if (!o->escalate || kc == 4) {
                status = BNC_STAGNATED;
                break;
            }
            do {
                ++kc;
                ++res->escalations;
                if ((rc = factor(0, &info)))
                    return rc;
            } while (info > 0 && kc < 4);
            if (info < 0)
                return timed_out();
            res->final_words = kc;
            res->info = info;
            if (info) {
                status = BNC_SINGULAR;
                break;
            }
            nz = 0;
        }
        if (iters == o->max_iter)
            break;
        // kc-word copy of r * 2^-e, correction solve, x <- x + 2^e z
        if ((rc = solve(r, n, (const unsigned long long *)&sc->rmax)))
            return rc;
        BNC_KSWITCH(kc, BNC_LSWITCH(lw, hipLaunchKernelGGL((k_scale_update<KK, LL>), dim3(grid1(n)), dim3(256), 0, s,
                                                           n, v, n, (const unsigned long long *)&sc->rmax, x, ldpx,
                                                           (const int *)nullptr)));
        BNC_LAUNCH_CHECK();
        if ((rc = absmax_run(n, 1, n, v, &sc->zmax, s)))
            return rc;
        ++nz;
        ++iters;
    }
    res->status = status;
    res->iters = iters;
    return BNC_OK;
}

// ---- the device-driven loop (bnc_refine_async) ---------------------------------
// The same steps and tests as refine_drive, with every decision taken on the
// device: all max_iter + 1 iterations are launched, and once the tests (or
// a failure) have decided the outcome the flag sc->done makes every later
// kernel of the loop return at once.  No host synchronisation, no
// allocation: the sequence can be captured into a HIP graph and replayed
// (the flags are cleared by a kernel at its start).

__global__ void k_async_checked(Scal *sc)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && sc->nonfinite) {
        sc->done = 1;
        sc->status = BNC_NONFINITE;
    }
}

// ||A||_F from the scaled sum of squares, and the listing's threshold
// sqrt(n) rtol ||A||_F (the host driver's formulas)
__global__ void k_async_anorm(Scal *sc, int64_t n, double rtol)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double amax = __longlong_as_double((long long)sc->amax);
        sc->a_norm = sqrt(sc->asq) * ldexp(1.0, norm_exp(amax) + 1);
        sc->thresh_c = sqrt((double)n) * rtol * sc->a_norm;
    }
}

// after the factorisation: an exactly zero pivot or a timed-out exchange
// ends the loop
__global__ void k_async_factored(Scal *sc)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && !sc->done && sc->info != 0) {
        sc->done = 1;
        sc->status = sc->info > 0 ? BNC_SINGULAR : sc->info == -3 ? BNC_SPLIT_RANGE : BNC_TIMED_OUT;
    }
}

// x = 0 when the loop ended before the first solution
__global__ void k_async_zero_x(int64_t n, int lw, double *__restrict__ x, int64_t ldx, const Scal *__restrict__ sc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && sc->done)
        for (int w = 0; w < lw; ++w)
            x[w * ldx + i] = 0.0;
}

// the stopping tests at the top of an iteration, in the host driver's order
__global__ void k_async_tests(Scal *sc, double atol, double ctol, double stag, int max_iter)
{
    if (blockIdx.x != 0 || threadIdx.x != 0 || sc->done)
        return;
    const double rmax = __longlong_as_double((long long)sc->rmax), xmax = __longlong_as_double((long long)sc->xmax);
    if (sc->nz > 0) {
        sc->zprev = sc->zlast;
        sc->zlast = __longlong_as_double((long long)sc->zmax);
    }
    const double nr = rmax == 0.0 ? 0.0 : sqrt(sc->rsq) * ldexp(1.0, norm_exp(rmax) + 1);
    const double nx = xmax == 0.0 ? 0.0 : sqrt(sc->xsq) * ldexp(1.0, norm_exp(xmax) + 1);
    sc->resid_norm = nr;
    sc->x_norm = nx;
    int st = -1;
    if (sc->tinfo)
        st = BNC_TIMED_OUT;
    else if (nr < sc->thresh_c * nx + atol || (sc->nz > 0 && sc->zlast <= ctol * xmax))
        st = BNC_CONVERGED;
    else if (stag > 0.0 && sc->nz >= 2 && sc->zlast > stag * sc->zprev)
        st = BNC_STAGNATED;
    else if (sc->iters == max_iter)
        st = BNC_MAX_ITER;
    if (st >= 0) {
        sc->status = st;
        sc->done = 1;
    }
}

__global__ void k_async_corrected(Scal *sc)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && !sc->done) {
        ++sc->nz;
        ++sc->iters;
    }
}

__global__ void k_async_finish(const Scal *__restrict__ sc, int K, bnc_refine_result *__restrict__ res)
{
    if (blockIdx.x != 0 || threadIdx.x != 0)
        return;
    bnc_refine_result r{};
    r.status = sc->done ? sc->status : BNC_MAX_ITER;
    const bool rejected = r.status == BNC_NONFINITE;  // nothing was factorised
    r.iters = sc->iters;
    r.info = rejected ? 0 : sc->info;
    r.resid_norm = sc->resid_norm;
    r.x_norm = sc->x_norm;
    r.a_norm = rejected ? 0.0 : sc->a_norm;
    r.residual_inexact = sc->inexact ? 1 : 0;
    r.final_words = K;
    r.escalations = 0;
    r.first_words = K;
    *res = r;
}

template <int K>
int refine_async_run(int64_t n, int aw, const double *A, int64_t lda, int64_t ldpa, const double *b, int64_t ldpb,
                     double *x, int64_t ldpx, void *work, const bnc_refine_opts *o, bnc_refine_result *res,
                     hipStream_t s)
{
    const RefineLayout L = refine_layout(n, K);
    char *W = (char *)work;
    double *LU = (double *)(W + L.lu);
    int64_t *ipiv = (int64_t *)(W + L.ipiv);
    int32_t *perm = (int32_t *)(W + L.perm);
    double *rd = (double *)(W + L.rd);
    double *r = (double *)(W + L.r);
    double *v = (double *)(W + L.v);
    double *rowmax = (double *)(W + L.rowmax);
    double *part = (double *)(W + L.part);
    double *red = (double *)(W + L.red);
    Scal *sc = (Scal *)(W + L.scal);
    void *gscr = W + L.getrf;
    double *ozb = (double *)(W + L.oz);
    void *tsflags = (void *)(W + L.flags);
    const int64_t ldp = n * n;
    const int lw = o->long_words ? o->long_words : 4;
    const int *skip = &sc->done;
    const unsigned long long *rmaxb = &sc->rmax;
    int rc;

    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t *)sc, (int64_t)(sizeof(Scal) / 8), (uint64_t)0,
                       (const int *)nullptr);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_check_finite, dim3(grid1(n * n)), dim3(256), 0, s, n, n, aw, A, lda, ldpa, &sc->nonfinite);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_check_finite, dim3(grid1(n)), dim3(256), 0, s, n, (int64_t)1, lw, b, ldpb, ldpb,
                       &sc->nonfinite);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_async_checked, dim3(1), dim3(64), 0, s, sc);
    BNC_LAUNCH_CHECK();
    if ((rc = absmax_run(n, n, lda, A, &sc->amax, s)) || (rc = sumsq_run(n, n, lda, A, &sc->amax, red, &sc->asq, s)) ||
        (rc = rowmax_run(n, A, lda, rowmax, s)) || (rc = fill_i32_run(&sc->eb.a, 3, 2000, s)) ||
        (rc = minexp_run(n, n, lda, aw, ldpa, A, &sc->eb.a, s)) ||
        (rc = minexp_run(n, 1, n, lw, ldpb, b, &sc->eb.b, s)))
        return rc;
    hipLaunchKernelGGL(k_async_anorm, dim3(1), dim3(64), 0, s, sc, n, o->rtol);
    BNC_LAUNCH_CHECK();
    // K-word copy of A and the factorisation (run unconditionally: on a
    // rejected input its result is simply not used)
    if (aw == 1)
        hipLaunchKernelGGL((k_stage<K, 1>), dim3(grid1(n * n)), dim3(256), 0, s, n, A, lda, ldpa, LU, n, ldp);
    else
        hipLaunchKernelGGL((k_stage<K, 4>), dim3(grid1(n * n)), dim3(256), 0, s, n, A, lda, ldpa, LU, n, ldp);
    BNC_LAUNCH_CHECK();
    if ((rc = getrf_run<K>(n, LU, n, ldp, ipiv, &sc->info, gscr, s, o->ozaki_slices, ozb)))
        return rc;
    hipLaunchKernelGGL(k_async_factored, dim3(1), dim3(64), 0, s, sc);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_async_zero_x, dim3(grid1(n)), dim3(256), 0, s, n, lw, x, ldpx, (const Scal *)sc);
    BNC_LAUNCH_CHECK();
    if ((rc = ipiv_to_perm(n, ipiv, perm, s)) || (rc = diag_recip_run<K>(n, LU, n, ldp, rd, s)))
        return rc;
    // v <- K-word solve of the K-word copy of src (scaled by 2^-e when rmax
    // is given)
    auto solve = [&](const double *src, int64_t lds, const unsigned long long *rmaxbits) -> int {
        BNC_LSWITCH(lw, hipLaunchKernelGGL((k_round_scaled<K, LL>), dim3(grid1(n)), dim3(256), 0, s, n, src, lds,
                                           rmaxbits, r, n, skip));
        BNC_LAUNCH_CHECK();
        return getrs_perm<K>(n, LU, n, ldp, perm, rd, r, n, v, n, tsflags, s, &sc->tinfo, skip);
    };
    if ((rc = solve(b, ldpb, nullptr)))
        return rc;
    BNC_LSWITCH(lw, hipLaunchKernelGGL((k_extend<K, LL>), dim3(grid1(n)), dim3(256), 0, s, n, (const double *)v, n, x,
                                       ldpx, skip));
    BNC_LAUNCH_CHECK();
    for (int it = 0; it <= o->max_iter; ++it) {
        if ((rc = absmax_run(n, 1, n, x, &sc->xmax, s, skip)) || (rc = fill_i32_run(&sc->eb.x, 1, 2000, s, skip)) ||
            (rc = minexp_run(n, 1, n, lw, ldpx, x, &sc->eb.x, s, skip)) ||
            (rc = residual_run(n, aw, lw, A, lda, ldpa, x, ldpx, b, ldpb, rowmax, (const double *)&sc->xmax, &sc->eb,
                               part, r, n, &sc->inexact, s, skip)) ||
            (rc = absmax_run(n, 1, n, r, &sc->rmax, s, skip)) ||
            (rc = sumsq_run(n, 1, n, r, &sc->rmax, red, &sc->rsq, s, skip)) ||
            (rc = sumsq_run(n, 1, n, x, &sc->xmax, red, &sc->xsq, s, skip)))
            return rc;
        hipLaunchKernelGGL(k_async_tests, dim3(1), dim3(64), 0, s, sc, o->atol, o->ctol, o->stagnation_ratio,
                           o->max_iter);
        BNC_LAUNCH_CHECK();
        if (it == o->max_iter)
            break;  // the tests above have ended the loop
        if ((rc = solve(r, n, rmaxb)))
            return rc;
        BNC_LSWITCH(lw, hipLaunchKernelGGL((k_scale_update<K, LL>), dim3(grid1(n)), dim3(256), 0, s, n, v, n, rmaxb,
                                           x, ldpx, skip));
        BNC_LAUNCH_CHECK();
        if ((rc = absmax_run(n, 1, n, v, &sc->zmax, s, skip)))
            return rc;
        hipLaunchKernelGGL(k_async_corrected, dim3(1), dim3(64), 0, s, sc);
        BNC_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_async_finish, dim3(1), dim3(64), 0, s, (const Scal *)sc, K, res);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

template <int K>
int refine_run(int64_t n, int aw, const double *A, int64_t lda, int64_t ldpa, const double *b, int64_t ldpb, double *x,
               int64_t ldpx, void *work, const bnc_refine_opts *o, bnc_refine_result *res, hipStream_t s)
{
    return refine_drive(K, n, aw, A, lda, ldpa, b, ldpb, x, ldpx, work, o, res, s);
}

#define INST(K)                                                                                                    \
    template int refine_run<K>(int64_t, int, const double *, int64_t, int64_t, const double *, int64_t, double *, \
                               int64_t, void *, const bnc_refine_opts *, bnc_refine_result *, hipStream_t);     \
    template int refine_async_run<K>(int64_t, int, const double *, int64_t, int64_t, const double *, int64_t,     \
                                     double *, int64_t, void *, const bnc_refine_opts *, bnc_refine_result *,     \
                                     hipStream_t);
INST(1)
INST(2)
INST(3)
INST(4)
#undef INST

}  // namespace bnc

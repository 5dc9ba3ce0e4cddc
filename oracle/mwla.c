/*
 * ORACLE -- test infrastructure, not part of the product path.
 *
 * A plain, slow CPU reference for what the solver computes: multi-word
 * (K = 1 binary64, 2 double-double, 3 triple-double, 4 quad-double)
 * arithmetic built from error-free transformations, unblocked LU with
 * partial pivoting, forward/backward substitution, and the exact residual
 * b - A x rounded once to quad-double.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg load this library.
 *
 * Paper: T. Kouya, "Accelerated Multiple Precision Direct Method and Mixed
 * Precision Iterative Refinement on Python Programming Environment" (2021).
 *   - Sec. 1 / Sec. 2: DD, TD and QD numbers are unevaluated sums of two,
 *     three and four binary64 words (106, 159 and 212 bits, Table 1).
 *   - Sec. 2: LU decomposition with partial pivoting and forward/backward
 *     substitution carried out in that arithmetic.
 *   - Sec. 2, Listing 1: residual in a longer precision than the factors.
 * The paper does not give the word-level algorithms.  The ones below are
 * this project's reading, built only from the textbook error-free
 * transformations (Knuth's TwoSum, Dekker's Fast2Sum, FMA-based TwoProd);
 * the exact operation order is fixed here and pinned against exact rational
 * arithmetic by the tests.
 *
 * Storage ("K-plane"): a K-word matrix is K binary64 planes; plane w holds
 * word w of every entry, column-major with leading dimension lda, and the
 * planes are ldp doubles apart.  Word 0 is the leading word.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no contraction: every rounding below happens exactly as written).
 *
 * Threads: the loops over independent columns (LU updates, substitution of
 * U12, matrix products) and rows (residual) are shared out with OpenMP.
 * Every entry still receives its operations in the order stated at each
 * routine, so the results do not depend on the number of threads
 * (orc_set_threads(1) gives the serial program).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KMAX 4  /* words of a factor */
#define WMAX 8  /* words of a long-precision value (424 bits) */
#define LVMAX 32

/* Number of OpenMP threads the loops below use (n < 1: the runtime's
 * default); returns the number in effect. */
int orc_set_threads(int n)
{
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
}

int orc_get_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------------- */
/* Error-free transformations                                              */
/* ---------------------------------------------------------------------- */

/* TwoSum (Knuth, TAOCP 4.2.2): s = RN(a+b), e = a+b-s exactly. */
static double two_sum(double a, double b, double *e)
{
    double s = a + b;
    double bb = s - a;
    double aa = s - bb;
    *e = (a - aa) + (b - bb);
    return s;
}

/* TwoProd with a fused multiply-add: p = RN(a*b), e = a*b-p exactly. */
static double two_prod(double a, double b, double *e)
{
    double p = a * b;
    *e = fma(a, b, -p);
    return p;
}

/* ---------------------------------------------------------------------- */
/* K-word primitives                                                       */
/* ---------------------------------------------------------------------- */

/*
 * Renormalise m input words c[0..m-1] (roughly decreasing in magnitude) to
 * K output words.  Pass 1 runs TwoSum from the smallest word upward, so
 * t[0] carries the running sum and t[1..] the exact rounding errors.  Pass 2
 * walks down again: each TwoSum emits one output word and keeps its error as
 * the running remainder; once K-1 words are out the rest is added plainly
 * into the last word.
 */
static void renorm(int K, const double *c, int m, double *out)
{
    double t[LVMAX];
    double s = c[m - 1];
    for (int i = m - 2; i >= 0; --i)
        s = two_sum(c[i], s, &t[i + 1]);
    t[0] = s;
    double w = t[0];
    int j = 0;
    for (int i = 1; i < m; ++i) {
        if (j < K - 1) {
            double lo;
            out[j] = two_sum(w, t[i], &lo);
            w = lo;
            ++j;
        } else {
            w = w + t[i];
        }
    }
    out[j++] = w;
    for (; j < K; ++j)
        out[j] = 0.0;
}

typedef struct {
    double v[LVMAX];
    int n;
} level_t;

static void push(level_t *L, double x) { L->v[L->n++] = x; }

/*
 * Sum per-magnitude levels.  Level lv holds terms of size about
 * 2^(-53 lv) relative to the result.  Levels 0..K-2 are summed left to
 * right with TwoSum; each rounding error is appended to the next level.
 * Level K-1 is summed left to right in plain binary64.
 */
static void level_sum(int K, level_t *L, double *out)
{
    for (int lv = 0; lv < K - 1; ++lv) {
        double s = L[lv].v[0];
        for (int t = 1; t < L[lv].n; ++t) {
            double e;
            s = two_sum(s, L[lv].v[t], &e);
            push(&L[lv + 1], e);
        }
        out[lv] = s;
    }
    double s = L[K - 1].v[0];
    for (int t = 1; t < L[K - 1].n; ++t)
        s = s + L[K - 1].v[t];
    out[K - 1] = s;
}

/*
 * Fused multiply-subtract c - a*b (c == NULL: the product a*b).
 * Level lists are filled in this order: the words of c, then the partial
 * products a_i*b_j for i = 0..K-1, j = 0..K-1-i.  A product with
 * i+j < K-1 is split exactly by TwoProd (high part at level i+j, error at
 * level i+j+1); a product with i+j == K-1 is a plain binary64 product at
 * level K-1.  Products with i+j >= K are dropped.
 */
static void mw_fms(int K, const double *c, const double *a, const double *b, double *out)
{
    level_t L[WMAX];
    for (int lv = 0; lv < K; ++lv)
        L[lv].n = 0;
    double sg = 1.0;
    if (c) {
        sg = -1.0;
        for (int lv = 0; lv < K; ++lv)
            push(&L[lv], c[lv]);
    }
    for (int i = 0; i < K; ++i) {
        for (int j = 0; j + i < K; ++j) {
            int lv = i + j;
            if (lv < K - 1) {
                double e;
                double p = two_prod(a[i], b[j], &e);
                push(&L[lv], sg * p);
                push(&L[lv + 1], sg * e);
            } else {
                push(&L[K - 1], sg * (a[i] * b[j]));
            }
        }
    }
    double lvl[WMAX];
    level_sum(K, L, lvl);
    renorm(K, lvl, K, out);
}

static void mw_mul(int K, const double *a, const double *b, double *out)
{
    mw_fms(K, NULL, a, b, out);
}

/* a + b: level lv gets (a_lv, b_lv); then level_sum and renorm. */
static void mw_add(int K, const double *a, const double *b, double *out)
{
    level_t L[WMAX];
    for (int lv = 0; lv < K; ++lv) {
        L[lv].n = 0;
        push(&L[lv], a[lv]);
        push(&L[lv], b[lv]);
    }
    double lvl[WMAX];
    level_sum(K, L, lvl);
    renorm(K, lvl, K, out);
}

/* Newton steps for 1/a: 0 (K=1), 1 (K=2), 2 (K=3, 4). */
static int recip_steps(int K) { return K == 1 ? 0 : (K == 2 ? 1 : 2); }

/*
 * Reciprocal by Newton's iteration r <- r + r (1 - a r), started from the
 * binary64 quotient 1/a_0; each step doubles the number of correct bits.
 */
static void mw_recip(int K, const double *a, double *out)
{
    double r[WMAX] = {0}, e[WMAX], nr[WMAX], one[WMAX] = {0};
    one[0] = 1.0;
    r[0] = 1.0 / a[0];
    for (int it = 0; it < recip_steps(K); ++it) {
        mw_fms(K, one, a, r, e);          /* e = 1 - a r */
        for (int w = 0; w < K; ++w)
            nr[w] = -r[w];
        mw_fms(K, r, nr, e, r);           /* r = r - (-r) e */
    }
    memcpy(out, r, sizeof(double) * K);
}

/*
 * Pivot key order: |a| compared word by word, leading word first, after
 * multiplying every word by the sign of the leading word.  Returns 1 when
 * key(a) > key(b).
 */
static int key_gt(int K, const double *a, const double *b)
{
    double sa = a[0] < 0.0 ? -1.0 : 1.0;
    double sb = b[0] < 0.0 ? -1.0 : 1.0;
    for (int w = 0; w < K; ++w) {
        double x = sa * a[w], y = sb * b[w];
        if (x > y)
            return 1;
        if (x < y)
            return 0;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Vectorised primitives for the tests (each entry independent)            */
/* Arrays are word-major: word w of entry i at p[w*n + i].                 */
/* ---------------------------------------------------------------------- */

static void gather(int K, const double *p, int64_t n, int64_t i, double *v)
{
    for (int w = 0; w < K; ++w)
        v[w] = p[w * n + i];
}
static void scatter(int K, double *p, int64_t n, int64_t i, const double *v)
{
    for (int w = 0; w < K; ++w)
        p[w * n + i] = v[w];
}

void orc_two_sum(int64_t n, const double *a, const double *b, double *s, double *e)
{
    for (int64_t i = 0; i < n; ++i)
        s[i] = two_sum(a[i], b[i], &e[i]);
}

void orc_two_prod(int64_t n, const double *a, const double *b, double *p, double *e)
{
    for (int64_t i = 0; i < n; ++i)
        p[i] = two_prod(a[i], b[i], &e[i]);
}

void orc_fms_vec(int K, int64_t n, const double *c, const double *a, const double *b, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double cv[WMAX], av[WMAX], bv[WMAX], o[WMAX];
        gather(K, c, n, i, cv);
        gather(K, a, n, i, av);
        gather(K, b, n, i, bv);
        mw_fms(K, cv, av, bv, o);
        scatter(K, out, n, i, o);
    }
}

/*
 * Multi-word matrix multiply-subtract C <- C - A B (the block matrix
 * multiplication of the multi-word library, Sec. 2 and Fig. 1), as its
 * definition: every entry c_ij <- fms(c_ij, a_il, b_lj) for l = 0..k-1 in
 * increasing l.  K-plane column-major matrices: word w of A(i, l) at
 * A[w*ldpa + l*lda + i], and likewise for B and C.
 */
void orc_gemm(int K, int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
              int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double c[WMAX], a[WMAX], b[WMAX], o[WMAX];
            for (int w = 0; w < K; ++w)
                c[w] = C[w * ldpc + j * ldc + i];
            for (int64_t l = 0; l < k; ++l) {
                for (int w = 0; w < K; ++w) {
                    a[w] = A[w * ldpa + l * lda + i];
                    b[w] = B[w * ldpb + j * ldb + l];
                }
                mw_fms(K, c, a, b, o);
                for (int w = 0; w < K; ++w)
                    c[w] = o[w];
            }
            for (int w = 0; w < K; ++w)
                C[w * ldpc + j * ldc + i] = c[w];
        }
}

void orc_mul_vec(int K, int64_t n, const double *a, const double *b, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double av[WMAX], bv[WMAX], o[WMAX];
        gather(K, a, n, i, av);
        gather(K, b, n, i, bv);
        mw_mul(K, av, bv, o);
        scatter(K, out, n, i, o);
    }
}

void orc_add_vec(int K, int64_t n, const double *a, const double *b, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double av[WMAX], bv[WMAX], o[WMAX];
        gather(K, a, n, i, av);
        gather(K, b, n, i, bv);
        mw_add(K, av, bv, o);
        scatter(K, out, n, i, o);
    }
}

void orc_recip_vec(int K, int64_t n, const double *a, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double av[WMAX], o[WMAX];
        gather(K, a, n, i, av);
        mw_recip(K, av, o);
        scatter(K, out, n, i, o);
    }
}

/* Round m-word values (m <= 8, word-major, stride n) to K <= 8 words. */
void orc_round_vec(int K, int m, int64_t n, const double *src, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double v[WMAX], o[WMAX];
        gather(m, src, n, i, v);
        renorm(K, v, m, o);
        scatter(K, out, n, i, o);
    }
}

/* key(a_i) > key(b_i) for each i. */
void orc_key_gt_vec(int K, int64_t n, const double *a, const double *b, int32_t *gt)
{
    for (int64_t i = 0; i < n; ++i) {
        double av[WMAX], bv[WMAX];
        gather(K, a, n, i, av);
        gather(K, b, n, i, bv);
        gt[i] = key_gt(K, av, bv);
    }
}

/* ---------------------------------------------------------------------- */
/* LU with partial pivoting and the substitutions                         */
/* ---------------------------------------------------------------------- */

#define AT(P, i, j, w) (P)[(int64_t)(w) * ldp + (int64_t)(j) * lda + (i)]

static void load(int K, const double *A, int64_t lda, int64_t ldp, int64_t i, int64_t j, double *v)
{
    for (int w = 0; w < K; ++w)
        v[w] = AT(A, i, j, w);
}
static void store(int K, double *A, int64_t lda, int64_t ldp, int64_t i, int64_t j, const double *v)
{
    for (int w = 0; w < K; ++w)
        AT(A, i, j, w) = v[w];
}

static int is_zero(int K, const double *v)
{
    for (int w = 0; w < K; ++w)
        if (v[w] != 0.0)
            return 0;
    return 1;
}

/*
 * In-place PA = LU, right-looking and unblocked (LAPACK getf2 conventions):
 * at step k the pivot is the first row i >= k whose entry in column k has
 * the largest key; rows k and ipiv[k] are swapped across all n columns; the
 * multipliers are a_ik * (1/a_kk); every trailing entry then gets
 * a_ij <- a_ij - l_ik * u_kj, so each entry sees its updates in increasing
 * k.  ipiv is 0-based swap-sequence.  Returns info: 0, or k+1 for the first
 * exactly-zero pivot (the factorisation continues, LAPACK style).
 */
int64_t orc_getrf(int K, int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv)
{
    int64_t info = 0;
    double best[WMAX], v[WMAX], r[WMAX], o[WMAX];
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        load(K, A, lda, ldp, k, k, best);
        for (int64_t i = k + 1; i < n; ++i) {
            load(K, A, lda, ldp, i, k, v);
            if (key_gt(K, v, best)) {
                p = i;
                memcpy(best, v, sizeof(double) * K);
            }
        }
        ipiv[k] = p;
        if (p != k) {
            for (int64_t j = 0; j < n; ++j)
                for (int w = 0; w < K; ++w) {
                    double tmp = AT(A, k, j, w);
                    AT(A, k, j, w) = AT(A, p, j, w);
                    AT(A, p, j, w) = tmp;
                }
        }
        load(K, A, lda, ldp, k, k, v);
        if (is_zero(K, v)) {
            if (info == 0)
                info = k + 1;
            continue;
        }
        mw_recip(K, v, r);
        for (int64_t i = k + 1; i < n; ++i) {
            load(K, A, lda, ldp, i, k, v);
            mw_mul(K, v, r, o);
            store(K, A, lda, ldp, i, k, o);
        }
#pragma omp parallel for schedule(static) if (n - k > 32)
        for (int64_t j = k + 1; j < n; ++j) {
            double u[WMAX], l[WMAX], w[WMAX], q[WMAX];
            load(K, A, lda, ldp, k, j, u);
            for (int64_t i = k + 1; i < n; ++i) {
                load(K, A, lda, ldp, i, k, l);
                load(K, A, lda, ldp, i, j, w);
                mw_fms(K, w, l, u, q);
                store(K, A, lda, ldp, i, j, q);
            }
        }
    }
    return info;
}

/*
 * Solve A x = b with the factors of orc_getrf, nrhs right-hand sides.
 * B: K planes of ldb x nrhs (column-major), plane stride ldpb; overwritten
 * by X.  Order: apply the swaps k = 0..n-1; forward substitution with the
 * unit lower factor (y_i <- y_i - l_ik y_k for k = 0..i-1, increasing k);
 * backward substitution (x_k = y_k * (1/u_kk), then y_i <- y_i - u_ik x_k
 * for k = n-1..i+1, decreasing k).
 */
void orc_getrs(int K, int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp,
               const int64_t *ipiv, double *B, int64_t ldb, int64_t ldpb)
{
    double yk[WMAX], v[WMAX], l[WMAX], o[WMAX], r[WMAX];
#define BT(i, c, w) B[(int64_t)(w) * ldpb + (int64_t)(c) * ldb + (i)]
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t k = 0; k < n; ++k) {
            int64_t p = ipiv[k];
            if (p != k)
                for (int w = 0; w < K; ++w) {
                    double tmp = BT(k, c, w);
                    BT(k, c, w) = BT(p, c, w);
                    BT(p, c, w) = tmp;
                }
        }
        for (int64_t k = 0; k < n; ++k) {
            for (int w = 0; w < K; ++w)
                yk[w] = BT(k, c, w);
            for (int64_t i = k + 1; i < n; ++i) {
                load(K, LU, lda, ldp, i, k, l);
                for (int w = 0; w < K; ++w)
                    v[w] = BT(i, c, w);
                mw_fms(K, v, l, yk, o);
                for (int w = 0; w < K; ++w)
                    BT(i, c, w) = o[w];
            }
        }
        for (int64_t k = n - 1; k >= 0; --k) {
            load(K, LU, lda, ldp, k, k, v);
            mw_recip(K, v, r);
            for (int w = 0; w < K; ++w)
                v[w] = BT(k, c, w);
            mw_mul(K, v, r, yk);
            for (int w = 0; w < K; ++w)
                BT(k, c, w) = yk[w];
            for (int64_t i = 0; i < k; ++i) {
                load(K, LU, lda, ldp, i, k, l);
                for (int w = 0; w < K; ++w)
                    v[w] = BT(i, c, w);
                mw_fms(K, v, l, yk, o);
                for (int w = 0; w < K; ++w)
                    BT(i, c, w) = o[w];
            }
        }
    }
#undef BT
}

/* ---------------------------------------------------------------------- */
/* Trailing update by error-free splitting (Ozaki scheme)                  */
/* ---------------------------------------------------------------------- */

/*
 * Not in the paper: an alternative form of the blocked LU's trailing update
 * A22 <- A22 - L21 U12 after Ozaki, Ogita, Oishi and Rump (Numer.
 * Algorithms 59, 2012).  Each row of L21 and each column of U12 is cut into
 * s binary64 slices of beta bits on a power-of-two grid fixed by the
 * row's (column's) largest leading word, so that every slice product and
 * every sum of them below is exact in binary64.  For each diagonal
 * d = p + q (p, q slice indices of the row and column operands) the group
 * sum acc_d = sum_{p+q=d} sum_k L_p[i][k] U_q[k][j] is therefore an exact
 * binary64 number, whatever the summation order; pairs with d >= s are
 * dropped (the factor is then slightly less accurate; the refinement
 * recovers the accuracy).  Finally a_ij <- (((a_ij - acc_0) - acc_1) ...)
 * - acc_{s-1} in K-word arithmetic, in that order.
 *
 * Exactness: with a row scale E (|x| < 2^E for every entry x of the row),
 * slice q lies on the grid g_q = 2^(E - (q+1) beta).  Slice q is the sum
 * over the words of the remaining value of each word rounded to the nearest
 * multiple of g_q (ties to even), so |slice_0| <= (2^beta + K/2) g_0 and
 * |slice_q| <= (K 2^(beta-1) + K/2) g_q for q >= 1.  All products of one
 * group d share the grid g_p g_(d-p), and the group has kb (d+1) of them,
 * kb <= 64.  The slice width beta therefore depends on K and s: it is the
 * largest width (at most 26) for which the bound on every group sum,
 * 64 * sum_p |slice_p| |slice_(d-p)| over d < s, stays below 2^53 units of
 * the group's grid; then every product and every partial sum is an exact
 * binary64 number as long as the grids stay in the normal range.  For
 * s = 16 and K >= 3 this gives 20 bits; a double-double factor with 5
 * slices gets 22 (110 bits, more than the factor's 106).
 */
#define OZ_SMAX 16
#define OZ_KBMAX 64

static int oz_beta(int K, int s)
{
    for (int beta = 26; beta > 1; --beta) {
        /* bounds in half units of the grid, so that they are integers */
        unsigned __int128 b[OZ_SMAX];
        for (int q = 0; q < s; ++q)
            b[q] = q == 0 ? ((unsigned __int128)1 << (beta + 1)) + (unsigned)K
                          : (unsigned __int128)K * ((unsigned __int128)1 << beta) + (unsigned)K;
        int ok = 1;
        for (int d = 0; d < s && ok; ++d) {
            unsigned __int128 g = 0;
            for (int p = 0; p <= d; ++p)
                g += b[p] * b[d - p];
            /* OZ_KBMAX * g / 4 < 2^53 */
            ok = OZ_KBMAX * g < ((unsigned __int128)1 << 55);
        }
        if (ok)
            return beta;
    }
    return 1;
}

int orc_oz_beta(int K, int s) { return (K < 1 || K > KMAX || s < 1 || s > OZ_SMAX) ? -1 : oz_beta(K, s); }

/* Smallest row/column scale for which every slice (grid 2^(E - (q+1)
 * beta), q < s) and every kept product (grid 2^(E + F - (d+2) beta), d < s)
 * stays on a grid of 2^-1022 or above when both scales reach it: the
 * larger of ceil(((s+1) beta - 1022) / 2) and s beta - 1022.  Below it a
 * product could round or flush, so the scheme would not be exact. */
static int oz_emin(int K, int s)
{
    int b = oz_beta(K, s);
    int x = (s + 1) * b - 1022;
    int half = x >= 0 ? (x + 1) / 2 : -((-x) / 2);
    int own = s * b - 1022;
    return half > own ? half : own;
}

int orc_oz_emin(int K, int s) { return (K < 1 || K > KMAX || s < 1 || s > OZ_SMAX) ? -100000 : oz_emin(K, s); }


/* Row/column scale: smallest E with |x_0| < 2^E for every leading word
 * x_0 of the m entries (stride inc); 0 when all are zero. */
static int oz_scale(const double *x0, int64_t m, int64_t inc)
{
    double mx = 0.0;
    for (int64_t k = 0; k < m; ++k)
        mx = fmax(mx, fabs(x0[k * inc]));
    return mx == 0.0 ? 0 : ilogb(mx) + 1;
}

/* Cut one K-word value v (consumed: it becomes the remainder) into s
 * slices on the grids 2^(E - (q+1) beta), beta = oz_beta(K, s). */
static void oz_cut(int K, int s, int E, double *v, double *sl)
{
    const int beta = oz_beta(K, s);
    for (int q = 0; q < s; ++q) {
        int e = E - (q + 1) * beta;
        double acc = 0.0;
        for (int t = 0; t < K; ++t) {
            double rho = ldexp(nearbyint(ldexp(v[t], -e)), e);
            v[t] -= rho;
            acc += rho;
        }
        sl[q] = acc;
    }
}

/* Vectorised for the tests: m K-word values x (word-major, word w of
 * entry i at x[w*m + i]) -> slices sl[q*m + i] and remainders rem (same
 * layout as x; may be NULL), all with the one scale E. */
void orc_oz_slices(int K, int s, int64_t m, const double *x, int32_t E, double *sl, double *rem)
{
    double v[WMAX], o[OZ_SMAX];
    for (int64_t i = 0; i < m; ++i) {
        gather(K, x, m, i, v);
        oz_cut(K, s, E, v, o);
        for (int q = 0; q < s; ++q)
            sl[q * m + i] = o[q];
        if (rem)
            scatter(K, rem, m, i, v);
    }
}

int32_t orc_oz_scale(int64_t m, const double *x0) { return oz_scale(x0, m, 1); }

/*
 * C <- C - L U by the scheme above.  L: K planes m x kb (column-major,
 * leading dimension ldl, plane stride ldpl); U: K planes kb x nc (ldu,
 * ldpu); C: K planes m x nc (ldc, ldpc).  acc (may be NULL) receives the
 * group sums, acc[(d*nc + j)*m + i].  Returns -1 when kb or s is out of
 * range, 1 when a nonzero row of L or column of U has its scale below
 * oz_emin (the sums are then not guaranteed exact), else 0.
 */
int orc_oz_update(int K, int s, int64_t m, int64_t nc, int64_t kb, const double *L, int64_t ldl, int64_t ldpl,
                  const double *U, int64_t ldu, int64_t ldpu, double *C, int64_t ldc, int64_t ldpc, double *acc)
{
    if (kb < 0 || kb > OZ_KBMAX || s < 1 || s > OZ_SMAX)
        return -1;
    if (m <= 0 || nc <= 0)
        return 0;
    double *Ls = malloc(sizeof(double) * (size_t)(s * m * (kb ? kb : 1)));
    double *Us = malloc(sizeof(double) * (size_t)(s * nc * (kb ? kb : 1)));
    const int emin = oz_emin(K, s);
    int low = 0; /* a scale below emin (a zero row or column has scale 0) */
    /* slices of the rows of L: Ls[(q*kb + k)*m + i] */
#pragma omp parallel for schedule(static) reduction(| : low)
    for (int64_t i = 0; i < m; ++i) {
        double v[WMAX], o[OZ_SMAX];
        int E = oz_scale(L + i, kb, ldl);
        low |= E < emin;
        for (int64_t k = 0; k < kb; ++k) {
            for (int w = 0; w < K; ++w)
                v[w] = L[w * ldpl + k * ldl + i];
            oz_cut(K, s, E, v, o);
            for (int q = 0; q < s; ++q)
                Ls[(q * kb + k) * m + i] = o[q];
        }
    }
    /* slices of the columns of U: Us[(q*nc + j)*kb + k] */
#pragma omp parallel for schedule(static) reduction(| : low)
    for (int64_t j = 0; j < nc; ++j) {
        double v[WMAX], o[OZ_SMAX];
        int F = oz_scale(U + j * ldu, kb, 1);
        low |= F < emin;
        for (int64_t k = 0; k < kb; ++k) {
            for (int w = 0; w < K; ++w)
                v[w] = U[w * ldpu + j * ldu + k];
            oz_cut(K, s, F, v, o);
            for (int q = 0; q < s; ++q)
                Us[(q * nc + j) * kb + k] = o[q];
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nc; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double c[WMAX], a[WMAX], t[WMAX];
            for (int w = 0; w < K; ++w)
                c[w] = C[w * ldpc + j * ldc + i];
            for (int d = 0; d < s; ++d) {
                double g = 0.0; /* exact */
                for (int p = 0; p <= d; ++p)
                    for (int64_t k = 0; k < kb; ++k)
                        g += Ls[(p * kb + k) * m + i] * Us[((d - p) * nc + j) * kb + k];
                if (acc)
                    acc[(d * nc + j) * m + i] = g;
                memset(a, 0, sizeof(a));
                a[0] = -g;
                mw_add(K, c, a, t);
                memcpy(c, t, sizeof(double) * K);
            }
            for (int w = 0; w < K; ++w)
                C[w * ldpc + j * ldc + i] = c[w];
        }
    free(Ls);
    free(Us);
    return low ? 1 : 0;
}

/*
 * Blocked right-looking PA = LU with panel width nb (1..64) whose trailing
 * update is orc_oz_update with s slices.  Per panel: the unblocked LU of
 * the panel columns (pivot search, row swaps over all n columns,
 * multipliers, rank-1 updates inside the panel, each entry's updates in
 * increasing k), then U12 <- L11^-1 A12 by column-oriented forward
 * substitution (increasing k), then the split update of A22.  Pivot rule,
 * ipiv and info as orc_getrf, except that a factorisation with no zero
 * pivot whose split updates met a row or column scale below oz_emin
 * returns -3 (its factors are not those of the exact scheme).  Returns -2
 * on bad nb or s.
 */
int64_t orc_getrf_ozaki(int K, int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t nb, int s)
{
    if (nb < 1 || nb > OZ_KBMAX || s < 1 || s > OZ_SMAX)
        return -2;
    int64_t info = 0;
    int low = 0;
    double best[WMAX], v[WMAX], r[WMAX], o[WMAX];
    for (int64_t j0 = 0; j0 < n; j0 += nb) {
        int64_t jb = n - j0 < nb ? n - j0 : nb;
        int64_t je = j0 + jb;
        for (int64_t k = j0; k < je; ++k) {
            int64_t p = k;
            load(K, A, lda, ldp, k, k, best);
            for (int64_t i = k + 1; i < n; ++i) {
                load(K, A, lda, ldp, i, k, v);
                if (key_gt(K, v, best)) {
                    p = i;
                    memcpy(best, v, sizeof(double) * K);
                }
            }
            ipiv[k] = p;
            if (p != k)
                for (int64_t j = 0; j < n; ++j)
                    for (int w = 0; w < K; ++w) {
                        double tmp = AT(A, k, j, w);
                        AT(A, k, j, w) = AT(A, p, j, w);
                        AT(A, p, j, w) = tmp;
                    }
            load(K, A, lda, ldp, k, k, v);
            if (is_zero(K, v)) {
                if (info == 0)
                    info = k + 1;
                continue;
            }
            mw_recip(K, v, r);
            for (int64_t i = k + 1; i < n; ++i) {
                load(K, A, lda, ldp, i, k, v);
                mw_mul(K, v, r, o);
                store(K, A, lda, ldp, i, k, o);
            }
#pragma omp parallel for schedule(static) if (n - k > 32)
            for (int64_t j = k + 1; j < je; ++j) {
                double u[WMAX], l[WMAX], w[WMAX], q[WMAX];
                load(K, A, lda, ldp, k, j, u);
                for (int64_t i = k + 1; i < n; ++i) {
                    load(K, A, lda, ldp, i, k, l);
                    load(K, A, lda, ldp, i, j, w);
                    mw_fms(K, w, l, u, q);
                    store(K, A, lda, ldp, i, j, q);
                }
            }
        }
        if (je >= n)
            break;
#pragma omp parallel for schedule(static)
        for (int64_t j = je; j < n; ++j)
            for (int64_t k = j0; k < je; ++k) {
                double u[WMAX], l[WMAX], w[WMAX], q[WMAX];
                load(K, A, lda, ldp, k, j, u);
                for (int64_t i = k + 1; i < je; ++i) {
                    load(K, A, lda, ldp, i, k, l);
                    load(K, A, lda, ldp, i, j, w);
                    mw_fms(K, w, l, u, q);
                    store(K, A, lda, ldp, i, j, q);
                }
            }
        low |= orc_oz_update(K, s, n - je, n - je, jb, &AT(A, je, j0, 0), lda, ldp, &AT(A, j0, je, 0), lda, ldp,
                             &AT(A, je, je, 0), lda, ldp, NULL) == 1;
    }
    return (info == 0 && low) ? -3 : info;
}

/* ---------------------------------------------------------------------- */
/* Exact residual                                                          */
/* ---------------------------------------------------------------------- */

/*
 * A fixed-point integer wide enough for every product of two finite
 * binary64 numbers and any sum of up to 2^30 of them: NL limbs of 32 bits
 * (kept in int64 so that signed chunks can be added without carrying),
 * limb i has weight 2^(32 i + BASE).
 */
#define BASE (-2304)
#define NL 144

typedef struct {
    int64_t l[NL];
} bigfix_t;

/* add (v << s) * 2^(32 L + BASE), v a signed 64-bit integer, 0 <= s < 32 */
static void bf_add_i64(bigfix_t *A, int64_t v, int L, int s)
{
    __int128 w = (__int128)v << s;
    A->l[L] += (int64_t)(w & 0xffffffff);
    A->l[L + 1] += (int64_t)((w >> 32) & 0xffffffff);
    A->l[L + 2] += (int64_t)(w >> 64);
}

/* add the exact value m * 2^e, m a signed integer (|m| < 2^106) */
static void bf_add_scaled(bigfix_t *A, __int128 m, int e)
{
    if (m == 0)
        return;
    int pos = e - BASE;
    uint64_t lo = (uint64_t)m;
    int64_t hi = (int64_t)(m >> 64);
    /* m = lo + hi * 2^64 with lo read as unsigned */
    int L = pos >> 5, s = pos & 31;
    bf_add_i64(A, (int64_t)(lo & 0xffffffffULL), L, s);
    bf_add_i64(A, (int64_t)(lo >> 32), L + 1, s);
    bf_add_i64(A, hi, L + 2, s);
}

/* x = m * 2^e with m an integer, |m| < 2^53 */
static void split_double(double x, int64_t *m, int *e)
{
    if (x == 0.0) {
        *m = 0;
        *e = 0;
        return;
    }
    int ex;
    double f = frexp(x, &ex); /* x = f 2^ex, 0.5 <= |f| < 1 */
    *m = (int64_t)ldexp(f, 53);
    *e = ex - 53;
}

static void bf_add_double(bigfix_t *A, double x, int sign)
{
    int64_t m;
    int e;
    split_double(x, &m, &e);
    bf_add_scaled(A, (__int128)(sign * m), e);
}

static void bf_add_product(bigfix_t *A, double x, double y, int sign)
{
    int64_t mx, my;
    int ex, ey;
    split_double(x, &mx, &ex);
    split_double(y, &my, &ey);
    if (mx == 0 || my == 0)
        return;
    bf_add_scaled(A, (__int128)sign * (__int128)mx * (__int128)my, ex + ey);
}

/* carry-propagate so that limbs 0..NL-2 lie in [0, 2^32) */
static void bf_normalize(bigfix_t *A)
{
    for (int i = 0; i < NL - 1; ++i) {
        int64_t c = A->l[i] >> 32; /* floor division by 2^32 */
        A->l[i] -= c * ((int64_t)1 << 32);
        A->l[i + 1] += c;
    }
}

static int bf_bit(const bigfix_t *A, int pos)
{
    if (pos < 0)
        return 0;
    return (int)((A->l[pos >> 5] >> (pos & 31)) & 1);
}

static int bf_any_below(const bigfix_t *A, int pos) /* any bit in [0, pos) */
{
    for (int p = 0; p < pos; ++p)
        if (bf_bit(A, p))
            return 1;
    return 0;
}

/*
 * Round the (normalised, non-negative) value to the nearest binary64, ties
 * to even.  Returns 0 for zero; sets *bad when the result would be
 * subnormal or overflow (not needed by any workload here).
 */
static double bf_round_nonneg(const bigfix_t *A, int *bad)
{
    int top = -1;
    for (int i = NL - 1; i >= 0 && top < 0; --i)
        if (A->l[i])
            for (int b = 31; b >= 0; --b)
                if ((A->l[i] >> b) & 1) {
                    top = 32 * i + b;
                    break;
                }
    if (top < 0)
        return 0.0;
    uint64_t mant = 0;
    for (int p = top; p > top - 53; --p)
        mant = 2 * mant + (uint64_t)bf_bit(A, p);
    int guard = bf_bit(A, top - 53);
    int sticky = bf_any_below(A, top - 53);
    int lsb_pos = top - 52;
    if (guard && (sticky || (mant & 1))) {
        mant += 1;
        if (mant == ((uint64_t)1 << 53)) {
            mant >>= 1;
            lsb_pos += 1;
        }
    }
    int e = lsb_pos + BASE;
    if (e + 52 > 1023 || e + 52 < -1022)
        *bad = 1;
    return ldexp((double)mant, e);
}

/*
 * Round the exact value held in A to the canonical K-word form: w_0 is the
 * nearest binary64 to the value, w_1 the nearest to what is left, and so on
 * (greedy round-to-nearest).  A is consumed.
 */
static int bf_to_words(bigfix_t *A, int K, double *out)
{
    int bad = 0;
    for (int w = 0; w < K; ++w) {
        bf_normalize(A);
        int neg = A->l[NL - 1] < 0;
        bigfix_t mag = *A;
        if (neg) {
            for (int i = 0; i < NL; ++i)
                mag.l[i] = -mag.l[i];
            bf_normalize(&mag);
        }
        double v = bf_round_nonneg(&mag, &bad);
        if (neg)
            v = -v;
        out[w] = v;
        bf_add_double(A, v, -1);
    }
    bf_normalize(A);
    return bad;
}

/*
 * r = b - A x, computed exactly and rounded once to the canonical lw-word
 * form (lw = 4: quad-double; lw = 8: the 424-bit long precision of the
 * paper's Table 2).  A has aw words (1: binary64 entries, 4: quad-double
 * entries), column-major n x n per plane (lda, ldpa); x, b, r are lw-plane
 * vectors (plane strides ldx, ldb, ldr).  Returns the number of rows whose
 * rounded words fell outside the binary64 normal range (0 for every
 * workload here).
 */
int64_t orc_residual(int64_t n, int aw, int lw, const double *A, int64_t lda, int64_t ldpa, const double *x,
                     int64_t ldx, const double *b, int64_t ldb, double *r, int64_t ldr)
{
    int64_t bad_rows = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad_rows)
    for (int64_t i = 0; i < n; ++i) {
        bigfix_t *acc = (bigfix_t *)malloc(sizeof(bigfix_t));
        memset(acc, 0, sizeof(bigfix_t));
        for (int w = 0; w < lw; ++w)
            bf_add_double(acc, b[w * ldb + i], +1);
        for (int64_t j = 0; j < n; ++j)
            for (int u = 0; u < aw; ++u) {
                double a = A[u * ldpa + j * lda + i];
                for (int w = 0; w < lw; ++w)
                    bf_add_product(acc, a, x[w * ldx + j], -1);
            }
        double o[WMAX];
        if (bf_to_words(acc, lw, o))
            ++bad_rows;
        for (int w = 0; w < lw; ++w)
            r[w * ldr + i] = o[w];
        free(acc);
    }
    return bad_rows;
}

/*
 * Exact value of sum_t s_t * p_t * q_t (s = +-1 signs; q may be NULL for
 * plain sums) rounded to K canonical words.  Used by the tests to check
 * the K-word primitives against exact arithmetic without rational numbers.
 */
int orc_exact_dot(int K, int64_t m, const double *p, const double *q, const int32_t *s, double *out)
{
    bigfix_t *acc = (bigfix_t *)malloc(sizeof(bigfix_t));
    memset(acc, 0, sizeof(bigfix_t));
    for (int64_t t = 0; t < m; ++t) {
        if (q)
            bf_add_product(acc, p[t], q[t], s[t]);
        else
            bf_add_double(acc, p[t], s[t]);
    }
    int bad = bf_to_words(acc, K, out);
    free(acc);
    return bad;
}

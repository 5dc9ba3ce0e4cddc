/*
 * bnc.h -- multi-word dense linear solves on one AMD Instinct MI355X (gfx950).
 *
 * Method: T. Kouya, "Accelerated Multiple Precision Direct Method and Mixed
 * Precision Iterative Refinement on Python Programming Environment" (2021):
 * LU decomposition with partial pivoting and forward/backward substitution
 * in double-double (DD, 2 words), triple-double (TD, 3 words) and
 * quad-double (QD, 4 words) arithmetic (Sec. 1-2, Table 1), driven by the
 * mixed-precision iterative refinement of Sec. 2, Listing 1 (stopping rule
 * eq. (2) of Sec. 3).
 *
 * Conventions shared by every entry point
 *  - Storage ("K-plane"): a K-word number is an unevaluated sum of K binary64
 *    words, leading word first.  A K-word n x n matrix is K planes of
 *    binary64; plane w holds word w of every entry, column-major with leading
 *    dimension lda >= n; consecutive planes are ldp >= lda*n doubles apart.
 *    Word w of entry (i, j) is at A[w*ldp + j*lda + i].  A K-word vector of
 *    length n is K planes ldv >= n doubles apart.
 *  - Pointers are DEVICE pointers unless marked (host).  The caller owns
 *    every buffer, workspaces included (sized by the *_workspace_size
 *    queries); no call allocates or frees device memory.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are asynchronous on that stream unless marked synchronous.
 *  - Return value: BNC_OK, -i when argument i (1-based) is invalid (nothing
 *    is launched), or a BNC_ERR_* code; bnc_last_error() describes the last
 *    failure.
 *  - ipiv: int64, 0-based, LAPACK swap-sequence semantics (row k was
 *    interchanged with row ipiv[k] >= k, in order k = 0..n-1).
 *  - Pivot choice: the first row (smallest index) whose entry has the
 *    largest magnitude, magnitudes compared word by word after multiplying
 *    each word by the sign of the leading word.
 *  - Results are reproducible bit for bit: every operation order is fixed.
 *  - Limits: n <= 16384 for the factorisation.  The factorisations use one
 *    side stream and four events per device, created on the first call and
 *    released at process exit: factorisations (bnc_getrf_*, and those inside
 *    bnc_refine) must not run concurrently on one device.
 */
#ifndef BNC_H
#define BNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BNC_OK 0
#define BNC_ERR_HIP (-100)         /* a HIP runtime or launch call failed */
#define BNC_ERR_UNSUPPORTED (-101) /* size beyond the documented limits */
#define BNC_ERR_WORKSPACE (-102)   /* workspace smaller than required */
#define BNC_ERR_TIMEOUT (-103)     /* a bounded wait between workgroups gave up
                                      (bnc_refine; the asynchronous calls
                                      report it through their info) */

/* bnc_refine_opts.factor_words: let the learned selector choose. */
#define BNC_AUTO 0

/* Refinement outcome (bnc_refine_result.status). */
#define BNC_CONVERGED 0 /* a stopping test passed */
#define BNC_MAX_ITER 1  /* max_iter corrections applied, no test passed */
#define BNC_SINGULAR 2  /* exactly zero pivot met: no solve was attempted */
#define BNC_NONFINITE 3 /* NaN or Inf in A or b: nothing was factorised */
#define BNC_BAD_SIZE 4  /* batched solve: order outside 1..threads (at most
                           512) or words of A not 1 or 4 */
#define BNC_STAGNATED 5 /* corrections stopped shrinking (stagnation_ratio)
                           and no escalation was left */
#define BNC_TIMED_OUT 6 /* bnc_refine_async: a bounded wait between
                           workgroups gave up (bnc_refine returns
                           BNC_ERR_TIMEOUT instead); x is invalid */
#define BNC_SPLIT_RANGE 7 /* bnc_refine_async with ozaki_slices > 0: a row
                           or column scale fell below the split scheme's
                           exact range (bnc_getrf_ozaki info -3; bnc_refine
                           refactors in the plain form instead); x = 0 */

/*
 * LU decomposition with partial pivoting, in place: P A = L U (Kouya 2021,
 * Sec. 2: the K-word direct method; Listing 1 calls it on the short-precision
 * copy of A).  _d: 1 word (binary64), _dd: 2, _td: 3, _qd: 4.
 *   n     order of A (>= 0)
 *   A     K-plane matrix, overwritten by L (unit lower, strictly below the
 *         diagonal) and U (upper)
 *   lda   leading dimension (>= max(1, n));  ldp  plane stride (>= lda*n)
 *   ipiv  n int64 (device), pivot sequence as above
 *   info  one int64 (device): 0, or k+1 for the first exactly zero pivot
 *         U(k,k); the factorisation still completes (LAPACK getrf).  -1:
 *         the panel's cross-workgroup exchange timed out (it cannot happen
 *         on finite input; an entry holding the exchange's sentinel, the
 *         signalling NaN 0xFFF40000DEADBEEF, can cause it); the factors are
 *         then invalid
 *   work, work_bytes  caller workspace (device), at least
 *         bnc_getrf_workspace_size(K, 0, n) bytes (NULL allowed for n = 0):
 *         the panel exchange buffers; BNC_ERR_WORKSPACE if smaller
 */
int bnc_getrf_d(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                size_t work_bytes, void *stream);
int bnc_getrf_dd(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                 size_t work_bytes, void *stream);
int bnc_getrf_td(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                 size_t work_bytes, void *stream);
int bnc_getrf_qd(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                 size_t work_bytes, void *stream);

/*
 * The same factorisation with the split form of the trailing update (not
 * in the paper; the error-free splitting of Ozaki, Ogita, Oishi and Rump,
 * Numer. Algorithms 59 (2012), run on the FP64 matrix cores).  After each
 * 64-wide panel (pivoting, multipliers and U12 exactly as bnc_getrf_*),
 * every row of L21 and column of U12 is cut into `slices` binary64 slices of
 * bnc_oz_beta(K, slices) bits on a power-of-two grid fixed by its largest
 * leading word; for each d < slices the products of slice pairs (p, d - p)
 * are summed exactly in binary64, and a_ij <- (((a_ij - acc_0) - acc_1) ...)
 * - acc_{slices-1} in K-word addition.  Pairs with p + q >= slices are
 * dropped, so the factor carries about beta * slices bits relative to each
 * row/column scale (5 slices of 22 bits match double-double, 5-6 of 21
 * come near triple-double, 11 of 20 quad-double); bnc_refine recovers full
 * accuracy.
 * Deterministic, and independent of tiling: every slice and every group
 * sum is exact while every nonzero row and column scale (the exponent E
 * with max|leading word| < 2^E) is at least E_min(K, slices) = max(ceil(
 * ((slices + 1) beta - 1022) / 2), slices beta - 1022), which keeps every
 * slice and product grid at 2^-1022 or above (-456 for 2 words and 4
 * slices).  When a row of L21 or a column of U12 falls below it, the
 * factorisation still runs but reports info = -3 (if it is otherwise
 * complete and nonsingular): its factors are not those of the exact scheme.
 * bnc_refine then refactors in the plain form; bnc_refine_async ends with
 * BNC_SPLIT_RANGE.
 *   factor_words  K in 1..4;  slices  1..12
 *   the remaining arguments as bnc_getrf_* (argument errors are numbered
 *   from n = 3); the workspace, bnc_getrf_workspace_size(K, slices, n)
 *   bytes, also holds the slices (3 * 12 * 64 * n doubles).
 */
int bnc_getrf_ozaki(int32_t factor_words, int32_t slices, int64_t n, double *A, int64_t lda, int64_t ldp,
                    int64_t *ipiv, int64_t *info, void *work, size_t work_bytes, void *stream);

/* Workspace bytes of bnc_getrf_* (slices = 0) and bnc_getrf_ozaki (slices
 * 1..12) for K = factor_words and order n (host; 0 for n = 0 or arguments
 * out of range). */
size_t bnc_getrf_workspace_size(int32_t factor_words, int32_t slices, int64_t n);

/*
 * Slice width of the split form: the widest slice (at most 26 bits) for
 * which every group sum of a depth-64 update of K-word values cut into
 * `slices` slices stays below 2^53 steps of its grid, hence exact.  Slice q
 * is below (2^beta + K/2) steps for q = 0 and (K 2^(beta-1) + K/2) for
 * q > 0, and group d adds 64 (d + 1) products.  Host function, no GPU use.
 *   factor_words  K in 1..4;  slices  1..12
 * Returns beta, or -1 for arguments out of range.
 */
int bnc_oz_beta(int32_t factor_words, int32_t slices);

/*
 * Solve A X = B with the factors of bnc_getrf_* (Kouya 2021, Sec. 2:
 * forward and backward substitution; Listing 1 calls it for the first
 * solution and for every correction).  Rows of B are permuted by ipiv, then
 * L y = P b (unit lower, each y_i updated in increasing k), then U x = y
 * (x_k = y_k * (1/u_kk), each y_i updated in decreasing k).
 *   n, nrhs  order and number of right-hand sides (>= 0)
 *   LU, lda, ldp, ipiv   as returned by bnc_getrf_* with the same K
 *   B     K-plane n x nrhs matrix (leading dimension ldb, plane stride ldpb),
 *         overwritten by X
 *   info  one int64 (device, may be NULL): 0, or -1 when a bounded wait of
 *         the streamed substitutions gave up (a right-hand side holding the
 *         signalling NaN 0xFFF40000DEADBEEF can cause it); X is then invalid
 *   work, work_bytes  caller workspace, >= bnc_getrs_workspace_size(K, n)
 *         bytes (NULL allowed when n or nrhs is 0)
 * An ipiv entry outside [k, n) is taken as no interchange.
 * A zero pivot yields Inf/NaN in X; check getrf's info first.
 */
int bnc_getrs_d(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream);
int bnc_getrs_dd(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                 double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream);
int bnc_getrs_td(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                 double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream);
int bnc_getrs_qd(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                 double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream);

/* Workspace bytes of bnc_getrs_* for K = factor_words and order n (host;
 * 0 for n = 0 or arguments out of range). */
size_t bnc_getrs_workspace_size(int32_t factor_words, int64_t n);

/*
 * bnc_getrs_* without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Its scratch is a fixed device
 * array of about 2.1 MB inside the library (the workspace of a quad-double
 * solve of order 16384), one per device, held until the process ends; its
 * device address is looked up on the first call on each device.  The call
 * allocates nothing.  factor_words K in 1..4 comes first; the other
 * arguments, results and errors are those of bnc_getrs_{d,dd,td,qd}
 * (argument errors numbered from n = 2).  n <= 16384, BNC_ERR_UNSUPPORTED
 * above.  Every call on a device shares that device's array (each call
 * writes every word it reads first): calls that overlap on one device, from
 * several streams or host threads, race and give garbage.
 */
int bnc_getrs_noalloc(int32_t factor_words, int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp,
                      const int64_t *ipiv, double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *stream);

/*
 * Multi-word matrix multiply-subtract C <- C - A B (Kouya 2021, Sec. 2 and
 * Fig. 1: the block matrix multiplication of the multi-word library the
 * direct methods are built on; here the LU's K-word trailing-update kernel,
 * exported).  Every entry gets c_ij <- fms(c_ij, a_il, b_lj) for l = 0..k-1
 * in increasing l, one K-word multiply-subtract each, so the result does
 * not depend on tiling and equals the plain triple loop bit for bit.
 * Negating B (exact, word by word) turns it into C + A B; with C = 0 and -B
 * it gives A B.
 *   m, n, k   C is m x n, A m x k, B k x n (>= 0; nothing happens when any
 *             is 0)
 *   A, lda, ldpa   K-plane, column-major, lda >= max(1, m), plane stride
 *                  ldpa >= lda * k (ignored for K = 1)
 *   B, ldb, ldpb   K-plane, ldb >= max(1, k), ldpb >= ldb * n
 *   C, ldc, ldpc   K-plane, ldc >= max(1, m), ldpc >= ldc * n; must not
 *                  overlap A or B
 * Words of A and B need not be normalised; C's words come out as the
 * multiply-subtract leaves them.  No scratch.  Argument errors as above
 * (-i for argument i); BNC_ERR_UNSUPPORTED when n > 1048560, m > 2^31 or
 * k > 2^30.
 */
int bnc_gemm_d(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
               int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream);
int bnc_gemm_dd(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
                int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream);
int bnc_gemm_td(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
                int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream);
int bnc_gemm_qd(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
                int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream);

/* Options of the refinement loop (host struct). */
typedef struct bnc_refine_opts {
    int32_t factor_words; /* K of the factorisation: 1, 2, 3 or 4; 0 (BNC_AUTO,
                             bnc_refine only): chosen by the learned
                             selector, see selector_params */
    int32_t max_iter;     /* maximum number of corrections (>= 0) */
    double rtol;          /* residual test of Listing 1 / eq. (2): stop when
                             ||r||_2 < sqrt(n) rtol ||A||_F ||x||_2 + atol */
    double atol;
    double ctol;          /* forward test: stop when the last correction had
                             ||z||_inf <= ctol ||x||_inf (0 disables) */
    int32_t ozaki_slices; /* 0: K-word trailing updates (bnc_getrf_*);
                             1..12: the split form (bnc_getrf_ozaki) with
                             that many slices for the first factorisation.
                             Batched solves take 0. */
    int32_t escalate;     /* 0 or 1: on stagnation or an exactly zero pivot,
                             refactor with one more word (plain form) and
                             go on from the current x, up to 4 words.
                             Batched solves take 0. */
    double stagnation_ratio; /* > 0: after two corrections since the last
                             factorisation, the loop stagnates when
                             ||z_i||_inf > stagnation_ratio ||z_(i-1)||_inf
                             (checked after the stopping tests); 0 disables.
                             Batched solves report BNC_STAGNATED (they take
                             escalate = 0). */
    int32_t batch_panel;  /* batched solves: LU panel width 4, 8 or 16 (0 = 8;
                             a width whose panel would not fit the LDS of a
                             compute unit, or 16 below 128 threads, runs as
                             the next narrower one) */
    int32_t batch_threads; /* batched solves: threads per workgroup, 64, 128,
                             256 or 512 (0 = 256); systems of order above it get
                             BNC_BAD_SIZE.  Both are tuning knobs that leave
                             every result unchanged; bnc_refine ignores them. */
    int32_t long_words;   /* words of the long precision (x, b and the
                             residual): 4 (quad-double; 0 means 4) or 8
                             (424 bits, the long precision of Table 2).
                             Batched solves take 0 or 4. */
    int32_t reserved;     /* 0 */
    const float *selector_params; /* factor_words = 0: the network's
                             parameters (device, bnc_mlp_param_count()
                             floats) and input normalisation (device, 48
                             floats), as for bnc_mlp_forward.  bnc_refine
                             computes the 24 features of the system
                             (bnc_features; orders 1..512, the leading words
                             of A), runs the network and factors with the
                             predicted number of words; escalation (when
                             enabled) stays the fallback.  For orders above
                             512 it starts at 2 words.  Ignored otherwise. */
    const float *selector_norm;
} bnc_refine_opts;

/* Outcome of the refinement loop (host struct, filled synchronously). */
typedef struct bnc_refine_result {
    int32_t status;            /* BNC_CONVERGED ... BNC_NONFINITE */
    int32_t iters;             /* corrections applied */
    int64_t info;              /* getrf info */
    double resid_norm;         /* ||r||_2 of the last residual (leading words) */
    double x_norm;             /* ||x||_2 (leading words) */
    double a_norm;             /* ||A||_F (leading words) */
    int32_t residual_inexact;  /* 1 if any residual row lost bits below its
                                  exact accumulator (never for sane inputs) */
    int32_t final_words;       /* K of the last factorisation */
    int32_t escalations;       /* refactorisations with more words */
    int32_t first_words;       /* K of the first factorisation (the
                                  requested or, with factor_words = 0, the
                                  selector's choice) */
} bnc_refine_result;

/* Workspace bytes bnc_refine needs for order n and K = factor_words (host);
 * with escalate = 1 it needs the size for factor_words = 4; factor_words = 0
 * (the selector) covers every choice and the features. */
size_t bnc_refine_workspace_size(int64_t n, int32_t factor_words);

/*
 * Mixed-precision iterative refinement (Kouya 2021, Sec. 2, Listing 1):
 * short-precision (K-word) copies of A and b, LU + substitution, x to the
 * long precision; then repeat: r = b - A x, the stopping tests, r scaled by a
 * power of two 2^-e (the listing's normalisation), K-word copy of r,
 * substitution -> z, x <- x + 2^e z.  The long precision is L =
 * opts->long_words binary64 words, quad-double (L = 4) or 424 bits (L = 8,
 * the long precision of Table 2): the residual is accumulated exactly from
 * error-free products and rounded once to its canonical L-word form; x and
 * the update are L-word.
 *   n        order (>= 1)
 *   a_words  words per entry of A: 1 (binary64) or 4 (quad-double)
 *   A, lda, ldpa  a_words-plane matrix (not modified)
 *   b, ldpb  L-plane right-hand side (not modified)
 *   x, ldpx  L-plane solution (output)
 *   work, work_bytes  caller workspace, >= bnc_refine_workspace_size(n, K)
 *   opts     host options; result  host outcome
 * Synchronous: returns after the loop has finished (it reads the stopping
 * quantities back each iteration).  BNC_ERR_TIMEOUT when a bounded wait of
 * a factorisation or substitution gave up (x is then invalid).
 */
int bnc_refine(int64_t n, int32_t a_words, const double *A, int64_t lda, int64_t ldpa, const double *b,
               int64_t ldpb, double *x, int64_t ldpx, void *work, size_t work_bytes, const bnc_refine_opts *opts,
               bnc_refine_result *result, void *stream);

/*
 * bnc_refine with every decision taken on the device, for callers that
 * need an asynchronous call or want to capture the solve into a HIP graph
 * (Kouya 2021, Sec. 2, Listing 1: the same steps, tests and results as
 * bnc_refine).  All max_iter + 1 iterations are enqueued; the stopping
 * tests run in a small kernel after each residual and, once they (or a
 * failure) have decided, a flag in the workspace makes every later kernel
 * of the loop return at once.  Nothing is read back and nothing allocated:
 * the call returns after enqueueing, and the sequence can be captured
 * (replays reset the flags themselves).  Arguments as bnc_refine, except:
 *   opts     factor_words 1..4 (no BNC_AUTO) and escalate = 0; stagnation
 *            ends the loop with BNC_STAGNATED
 *   result   DEVICE bnc_refine_result, valid once the stream has reached
 *            the end of the call; a timed-out bounded wait gives status
 *            BNC_TIMED_OUT, a split factorisation out of its exact range
 *            BNC_SPLIT_RANGE
 * x, status, corrections and norms equal those of bnc_refine bit for bit.
 * The first factorisation on a device creates the library's look-ahead
 * stream: make one call outside a capture first.
 */
int bnc_refine_async(int64_t n, int32_t a_words, const double *A, int64_t lda, int64_t ldpa, const double *b,
                     int64_t ldpb, double *x, int64_t ldpx, void *work, size_t work_bytes,
                     const bnc_refine_opts *opts, bnc_refine_result *result, void *stream);

/* Outcome of one system of a batched solve (device struct). */
typedef struct bnc_batch_result {
    int32_t status;           /* BNC_CONVERGED ... BNC_BAD_SIZE */
    int32_t iters;            /* corrections applied */
    int64_t info;             /* getrf info */
    uint64_t t_start, t_end;  /* device wall-clock ticks (bnc_wall_clock_khz) */
    int32_t residual_inexact;
    int32_t reserved;
    uint64_t t_factored;      /* tick at the end of the factorisation (t_start
                                 when none was made) */
} bnc_batch_result;

/* Workspace bytes of bnc_refine_batched for K = factor_words, `slots`
 * persistent workgroups (0 = the default) of `threads` threads (0 = 256)
 * (host; 0 for invalid arguments). */
size_t bnc_refine_batched_workspace_size(int32_t factor_words, int32_t slots, int32_t threads);

/* The default number of persistent workgroups for K = factor_words, LU
 * panel width `panel` and `threads` per workgroup (0 = defaults) on the
 * current device: resident workgroups per compute unit (from the kernel's
 * LDS and register use) times the compute units.  Negative on bad
 * arguments. */
int32_t bnc_refine_batched_default_slots(int32_t factor_words, int32_t panel, int32_t threads);

/*
 * Batched mixed-precision iterative refinement: bnc_refine (Kouya 2021,
 * Sec. 2, Listing 1) on `count` independent systems of order 1..512 in one
 * persistent launch.  Each system's x, status and corrections equal those of
 * bnc_refine on that system alone, bit for bit, when the residual test is
 * off (rtol = 0, the forward test deciding); with rtol > 0 its 2-norms are
 * summed in another fixed order than bnc_refine's (one workgroup's tree), so
 * a system whose residual norm lies within a rounding of the threshold can
 * stop one correction apart.
 *   count      number of systems
 *   n          device int64[count]: orders
 *   a_words    device int32[count]: words per entry of A[s], 1 (binary64)
 *              or 4 (quad-double words, for matrices whose condition a
 *              binary64 copy cannot hold); NULL: all 1
 *   A, b, x    device arrays of device pointers: A[s] a_words[s] planes of
 *              n x n, column-major (lda = n, plane stride n*n); b[s], x[s]
 *              4-plane vectors (ldv = n)
 *   order      device int32[count] giving the order systems are taken in
 *              (NULL: 0..count-1); largest first balances the load
 *   work       >= bnc_refine_batched_workspace_size(K, slots, threads) bytes
 *   opts       host options (as bnc_refine); opts->batch_threads bounds the
 *              orders one launch takes (0 = 256; 512 for orders above 256)
 *   slots      persistent workgroups (0 = default)
 *   results    device bnc_batch_result[count]
 * Asynchronous on stream.  A system of order outside 1..threads, or with a
 * word count other than 1 or 4, gets BNC_BAD_SIZE.
 */
int bnc_refine_batched(int64_t count, const int64_t *n, const int32_t *a_words, const double *const *A,
                       const double *const *b, double *const *x, const int32_t *order, void *work,
                       size_t work_bytes, const bnc_refine_opts *opts, int32_t slots, bnc_batch_result *results,
                       void *stream);

/*
 * Same launch captured once into a HIP graph and replayed: when *graph_exec
 * is NULL the call captures bnc_refine_batched on `stream` (same arguments),
 * instantiates the graph, stores it in *graph_exec and launches it; later
 * calls with that handle only launch it (the arguments are those captured).
 * Free the handle with bnc_graph_destroy.
 */
int bnc_refine_batched_graph(int64_t count, const int64_t *n, const int32_t *a_words, const double *const *A,
                             const double *const *b, double *const *x, const int32_t *order, void *work,
                             size_t work_bytes, const bnc_refine_opts *opts, int32_t slots,
                             bnc_batch_result *results, void *stream, void **graph_exec);
int bnc_graph_destroy(void *graph_exec);

/* Tick rate of the device wall clock used by bnc_batch_result, in kHz. */
int64_t bnc_wall_clock_khz(void);

/* ------------------------------------------------------------------------
 * Learned choice of the factor precision (not in the paper: a project
 * addition on top of its refinement loop, Sec. 2 / Listing 1).  A small
 * network predicts from cheap binary64 features which factor precision
 * (1..4 words) a system needs and how many corrections it will take; the
 * escalation rule of bnc_refine_opts stays the fallback.
 * ---------------------------------------------------------------------- */
#define BNC_NFEATURES 24

/* Workspace bytes of bnc_features for `slots` workgroups (host). */
size_t bnc_features_workspace_size(int32_t slots);
/* Default number of workgroups of bnc_features (as many as fit on the
 * device at once). */
int32_t bnc_features_default_slots(void);

/*
 * 24 binary32 features per system, features[s * 24 + f] (orders 1..512;
 * others get zeros), each computed in binary64 from the leading words of A
 * and b and rounded:
 *   0 log2 n;  1 log2 ||A||_F;  2-4 log2 of ||A||_1, ||A||_inf, max|a_ij|
 *   relative to ||A||_F;  5-7 diagonal dominance |a_ii| / sum_{j!=i} |a_ij|:
 *   log2 of its minimum and mean, fraction of rows above 1;  8 log2 of the
 *   diagonal's 2-norm relative to ||A||_F;  9-10 log2 of the smallest over
 *   the largest column / row 2-norm;  11 log2 ||A - A^T||_F / ||A||_F;
 *   then a binary64 LU with partial pivoting (the bnc_getrf_d algorithm):
 *   12 log2 max|u_ij| / max|a_ij|;  13 log2 min|u_ii| / max|u_ii|;
 *   14 log2 max|u_ii| / ||A||_F;  15 mean log2|u_ii| - log2 max|u_ii|;
 *   16 fraction of |u_ii| below 2^-26 max|u_ii|;  17-19 log2 of ||A||_1
 *   times Hager's estimate of ||A^-1||_1 after 1, 2, 3 steps (Hager 1984;
 *   Higham 1988; solves with A and A^T; an early stop repeats the last);
 *   20 log2 ||x0||_inf ||A||_inf / ||b0||_inf and 21 log2 of the backward
 *   error ||b0 - A x0||_inf / (||A||_inf ||x0||_inf) of the binary64
 *   solution x0 of A x0 = b0 (b0 = leading words of b);  22 Hager steps
 *   taken;  23 log2 max|a_ii| / max|a_ij|.  log2 of 0 is -1100; an exactly
 *   singular binary64 factor gives 1000 + log2 ||A||_1 in 17-19, 1100 in
 *   20 and 0 in 21-22.  Sums run in index order, so the values do not
 *   depend on `slots`.
 *   count, n, A, b, order   as bnc_refine_batched (A[s]: its leading
 *             plane, lda = n, is read; b 4-plane; order: the order systems
 *             are taken in, NULL = 0..count-1, largest first balances the
 *             load)
 *   features  device float[count * 24]
 *   work      >= bnc_features_workspace_size(slots) bytes;  slots 0 = default
 * Asynchronous on stream.
 */
int bnc_features(int64_t count, const int64_t *n, const double *const *A, const double *const *b,
                 const int32_t *order, float *features, void *work, size_t work_bytes, int32_t slots, void *stream);

/*
 * Multilayer perceptron 24 -> 64 -> 64 -> 5 in binary32 with ReLU hidden
 * layers.  params (device, bnc_mlp_param_count() floats), packed as
 * W1[24][64] b1[64] W2[64][64] b2[64] W3[64][5] b3[5], W[i][j] mapping
 * input i to output j.  norm (device float[48]): inputs are replaced by
 * (x_i - norm[i]) * norm[24 + i] first.  Outputs 0-3 are the logits of the
 * factor precision 1..4 words, output 4 predicts log2(1 + corrections).
 */
int32_t bnc_mlp_param_count(void);
size_t bnc_mlp_workspace_size(int64_t batch);
/* out: device float[batch * 5].  Asynchronous on stream. */
int bnc_mlp_forward(int64_t batch, const float *X, const float *norm, const float *params, float *out, void *stream);
/*
 * Gradient of the mean loss over the batch, cross-entropy of the logits
 * against cls (int32 in 0..3 = words - 1) plus 0.5 Huber (delta 1) of
 * output 4 against target, with respect to params -> grads (device
 * float[param_count]); *loss (device float) gets the mean loss.  Batch sums
 * run in sample order (deterministic).  work >= bnc_mlp_workspace_size.
 */
int bnc_mlp_grad(int64_t batch, const float *X, const float *norm, const int32_t *cls, const float *target,
                 const float *params, float *grads, float *loss, void *work, size_t work_bytes, void *stream);

/* Adam step (Kingma and Ba 2015) with bias correction for step >= 1. */
typedef struct bnc_adam_opts {
    float lr, beta1, beta2, eps;
    int64_t step;
} bnc_adam_opts;
int bnc_mlp_adam(float *params, const float *grads, float *m, float *v, const bnc_adam_opts *opts, void *stream);

/*
 * r = b - A x computed exactly and rounded once to its canonical L-word form
 * (w0 = nearest binary64 to the value, w1 nearest to the remainder, ...):
 * the residual step of Listing 1 in the long precision.  A has a_words
 * planes (1 or 4); x, b, r are L-plane vectors, L = long_words (4 or 8).
 * *inexact (device int32) is set to 1 if a row had bits below its
 * 1360-bit accumulator window (then the row is faithful, not exactly
 * rounded); it is not cleared.  Rows may hold at most 2^19 - 1 terms
 * (2 a_words L n + L), else BNC_ERR_UNSUPPORTED.
 * work, work_bytes: >= bnc_residual_workspace_size(n) bytes (row maxima and
 * the partial bin sums).
 */
int bnc_residual(int64_t n, int32_t a_words, int32_t long_words, const double *A, int64_t lda, int64_t ldpa,
                 const double *x, int64_t ldpx, const double *b, int64_t ldpb, double *r, int64_t ldpr,
                 int32_t *inexact, void *work, size_t work_bytes, void *stream);
size_t bnc_residual_workspace_size(int64_t n);

/*
 * Element-wise K-word primitive on word-major arrays (word w of element i at
 * p[w*n + i]); exposes the device arithmetic every routine above is built
 * from.  op: 0 out = c - a*b, 1 out = a*b, 2 out = a+b, 3 out = 1/a,
 * 4 out = a rounded from m = K_in words (c unused, a has 4 planes; result
 * K words).  K in 1..4.
 */
#define BNC_OP_FMS 0
#define BNC_OP_MUL 1
#define BNC_OP_ADD 2
#define BNC_OP_RECIP 3
#define BNC_OP_ROUND4 4
int bnc_mw_apply(int32_t op, int32_t K, int64_t n, const double *c, const double *a, const double *b, double *out,
                 void *stream);

/*
 * Timing of the trailing-update launches inside bnc_getrf_* and bnc_refine:
 * with profiling on, every big-tile trailing-update launch (the update of
 * the columns right of the look-ahead panel, on the caller's stream) is
 * bracketed by hipEvents on its stream; the thin look-ahead launches are
 * not timed.  bnc_profile_read synchronises on the recorded events and
 * returns the summed milliseconds, the summed algorithmic FP64 operations
 * (m * n * k multiply-subtracts times the per-operation count) and the number
 * of launches since the last read, then clears them (host pointers).
 */
int bnc_profile_enable(int32_t on);
int bnc_profile_read(double *ms, double *flops, int64_t *launches);

/*
 * Test hook for the timeout paths (not for production use): with bit 0 set,
 * every factorisation raises its exchange's abort flag right after clearing
 * it, so every panel poll gives up at once and the factorisation reports
 * info = -1; with bit 1 set, every substitution does the same with its
 * streamed values (getrs info = -1).  Every kernel still runs to its end,
 * reading and writing only in-bounds memory.  0 turns it off.  Host-global.
 */
int bnc_test_force_timeout(int32_t bits);

const char *bnc_status_string(int32_t status);
const char *bnc_last_error(void);
const char *bnc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BNC_H */

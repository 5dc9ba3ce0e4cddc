// C-ABI of the solver library (declarations and contracts in include/bnc.h):
// argument checks, workspace size queries, launch-timing hooks and the
// element-wise primitive kernels.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "mw.hpp"
#include "ozsplit.hpp"

namespace bnc {

template <int K>
int getrf_run(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *scr,
              hipStream_t s, int oz, double *oz_buf);
size_t oz_slices_bytes(int64_t n);
template <int K>
int getrs_run(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv, double *B,
              int64_t ldb, int64_t ldpb, int64_t *info, void *scr, hipStream_t s);
size_t getrf_workspace_bytes(int K, int64_t n, int oz);
template <int K>
int refine_run(int64_t n, int aw, const double *A, int64_t lda, int64_t ldpa, const double *b, int64_t ldpb, double *x,
               int64_t ldpx, void *work, const bnc_refine_opts *o, bnc_refine_result *res, hipStream_t s);
size_t getrs_workspace_bytes(int K, int64_t n);
template <int K>
int batch_run(int64_t count, const int64_t *n, const int32_t *aw, const double *const *A, const double *const *b,
              double *const *x, const int32_t *order, void *work, int slots, const bnc_refine_opts *o,
              bnc_batch_result *res, hipStream_t s);
size_t batch_workspace_bytes(int K, int slots, int threads);
int batch_default_slots(int K, int pw, int nt);
bool batch_panel_ok(int pw);
bool batch_threads_ok(int nt);
size_t features_workspace_bytes(int slots);
int features_default_slots();
int features_run(int64_t count, const int64_t *n, const double *const *A, const double *const *b,
                 const int32_t *order, float *F, void *work, int slots, hipStream_t s);
int mlp_param_count();
size_t mlp_workspace_bytes(int64_t B);
int mlp_forward_run(int64_t B, const float *X, const float *norm, const float *P, float *O, hipStream_t s);
int mlp_grad_run(int64_t B, const float *X, const float *norm, const int32_t *cls, const float *tgt, const float *P,
                 float *G, float *loss, void *work, hipStream_t s);
int mlp_adam_run(float *P, const float *G, float *M, float *V, float lr, float b1, float b2, float eps, int64_t step,
                 hipStream_t s);

size_t refine_workspace_bytes(int64_t n, int K);
int refine_drive(int K0, int64_t n, int aw, const double *A, int64_t lda, int64_t ldpa, const double *b,
                 int64_t ldpb, double *x, int64_t ldpx, void *work, const bnc_refine_opts *o, bnc_refine_result *res,
                 hipStream_t s);
template <int K>
int refine_async_run(int64_t n, int aw, const double *A, int64_t lda, int64_t ldpa, const double *b, int64_t ldpb,
                     double *x, int64_t ldpx, void *work, const bnc_refine_opts *o, bnc_refine_result *res,
                     hipStream_t s);
size_t residual_workspace_bytes(int64_t n);
int residual_ws_run(int64_t n, int aw, int lw, const double *A, int64_t lda, int64_t ldpa, const double *x,
                    int64_t ldpx, const double *b, int64_t ldpb, double *r, int64_t ldpr, int32_t *inexact, void *work,
                    hipStream_t s);

// ---- errors -------------------------------------------------------------------
static thread_local std::string g_last_error;

int fail_hip(hipError_t e, const char *what, const char *file, int line)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    g_last_error = buf;
    return BNC_ERR_HIP;
}

int fail_arg(int code, const char *msg)
{
    g_last_error = msg;
    return code;
}

// ---- timeout test hook -------------------------------------------------------------
namespace {
int g_force_timeout = 0;
}  // namespace

int force_timeout_bits() { return g_force_timeout; }

// ---- trailing-update timing ------------------------------------------------------
namespace {
struct Ev {
    hipEvent_t a, b;
    double flops;
};
bool g_prof = false;
std::vector<Ev> g_events;
std::mutex g_prof_mu;
}  // namespace

bool UpdateTimer::enabled() { return g_prof; }

int UpdateTimer::begin(hipStream_t s)
{
    if (!g_prof)
        return -1;
    Ev e{};
    if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess)
        return -1;
    (void)hipEventRecord(e.a, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_events.push_back(e);
    return (int)g_events.size() - 1;
}

void UpdateTimer::end(int idx, hipStream_t s, double flops)
{
    if (idx < 0)
        return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_events[idx].flops = flops;
    (void)hipEventRecord(g_events[idx].b, s);
}

// ---- element-wise primitives -------------------------------------------------------
template <int K>
__global__ void k_apply(int op, int64_t n, const double *__restrict__ c, const double *__restrict__ a,
                        const double *__restrict__ b, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double av[K], bv[K], cv[K], o[K];
    if (op == BNC_OP_ROUND4) {
        double v[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            v[w] = a[w * n + i];
        renorm<K, 4>(v, o);
    } else {
        load_w<K>(a, n, i, av);
        if (op != BNC_OP_RECIP)
            load_w<K>(b, n, i, bv);
        if (op == BNC_OP_FMS) {
            load_w<K>(c, n, i, cv);
            fms<K>(cv, av, bv, o);
        } else if (op == BNC_OP_MUL) {
            mul<K>(av, bv, o);
        } else if (op == BNC_OP_ADD) {
            add<K>(av, bv, o);
        } else {
            recip<K>(av, o);
        }
    }
    store_w<K>(out, n, i, o);
}

}  // namespace bnc

using namespace bnc;

static hipStream_t S(void *s) { return (hipStream_t)s; }

template <int K>
static int getrf_entry(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                       size_t work_bytes, void *stream, int oz = 0, int argoff = 0)
{
    if (n < 0)
        return fail_arg(-(1 + argoff), "getrf: n < 0");
    if (n > 0 && !A)
        return fail_arg(-(2 + argoff), "getrf: A is NULL");
    if (lda < (n > 1 ? n : 1))
        return fail_arg(-(3 + argoff), "getrf: lda < max(1, n)");
    if (K > 1 && ldp < lda * n)
        return fail_arg(-(4 + argoff), "getrf: ldp < lda * n");
    if (n > 0 && !ipiv)
        return fail_arg(-(5 + argoff), "getrf: ipiv is NULL");
    if (!info)
        return fail_arg(-(6 + argoff), "getrf: info is NULL");
    if (n > 16384)
        return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: n > 16384");
    if (n > 0 && !work)
        return fail_arg(-(7 + argoff), "getrf: work is NULL");
    if (work_bytes < getrf_workspace_bytes(K, n, oz))
        return fail_arg(BNC_ERR_WORKSPACE, "getrf: workspace smaller than bnc_getrf_workspace_size");
    double *ozb = oz && n > 0 ? (double *)((char *)work + align256(getrf_scratch_bytes(K, n))) : nullptr;
    return getrf_run<K>(n, A, lda, ldp, ipiv, info, work, S(stream), oz, ozb);
}

template <int K>
static int getrs_entry(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                       double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes,
                       void *stream, int argoff = 0)
{
    if (n < 0)
        return fail_arg(-(1 + argoff), "getrs: n < 0");
    if (nrhs < 0)
        return fail_arg(-(2 + argoff), "getrs: nrhs < 0");
    if (n > 0 && !LU)
        return fail_arg(-(3 + argoff), "getrs: LU is NULL");
    if (lda < (n > 1 ? n : 1))
        return fail_arg(-(4 + argoff), "getrs: lda < max(1, n)");
    if (K > 1 && ldp < lda * n)
        return fail_arg(-(5 + argoff), "getrs: ldp < lda * n");
    if (n > 0 && !ipiv)
        return fail_arg(-(6 + argoff), "getrs: ipiv is NULL");
    if (n > 0 && nrhs > 0 && !B)
        return fail_arg(-(7 + argoff), "getrs: B is NULL");
    if (ldb < (n > 1 ? n : 1))
        return fail_arg(-(8 + argoff), "getrs: ldb < max(1, n)");
    if (K > 1 && ldpb < ldb * nrhs)
        return fail_arg(-(9 + argoff), "getrs: ldpb < ldb * nrhs");
    if (n > 16384)
        return fail_arg(BNC_ERR_UNSUPPORTED, "getrs: n > 16384");
    if (n > 0 && nrhs > 0 && !work)
        return fail_arg(-11, "getrs: work is NULL");
    if (work_bytes < getrs_workspace_bytes(K, n))
        return fail_arg(BNC_ERR_WORKSPACE, "getrs: workspace smaller than bnc_getrs_workspace_size");
    return getrs_run<K>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, work, S(stream));
}

template <int K>
static int gemm_entry(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
                      int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream)
{
    if (m < 0)
        return fail_arg(-1, "gemm: m < 0");
    if (n < 0)
        return fail_arg(-2, "gemm: n < 0");
    if (k < 0)
        return fail_arg(-3, "gemm: k < 0");
    if (m > 0 && k > 0 && !A)
        return fail_arg(-4, "gemm: A is NULL");
    if (lda < (m > 1 ? m : 1))
        return fail_arg(-5, "gemm: lda < max(1, m)");
    if (K > 1 && ldpa < lda * k)
        return fail_arg(-6, "gemm: ldpa < lda * k");
    if (k > 0 && n > 0 && !B)
        return fail_arg(-7, "gemm: B is NULL");
    if (ldb < (k > 1 ? k : 1))
        return fail_arg(-8, "gemm: ldb < max(1, k)");
    if (K > 1 && ldpb < ldb * n)
        return fail_arg(-9, "gemm: ldpb < ldb * n");
    if (m > 0 && n > 0 && !C)
        return fail_arg(-10, "gemm: C is NULL");
    if (ldc < (m > 1 ? m : 1))
        return fail_arg(-11, "gemm: ldc < max(1, m)");
    if (K > 1 && ldpc < ldc * n)
        return fail_arg(-12, "gemm: ldpc < ldc * n");
    if (n > 65535LL * 16 || m > ((int64_t)1 << 31) || k > ((int64_t)1 << 30))
        return fail_arg(BNC_ERR_UNSUPPORTED, "gemm: m, n or k too large for one launch");
    return gemm_run<K>(m, n, k, A, lda, ldpa, B, ldb, ldpb, C, ldc, ldpc, S(stream));
}

extern "C" {

int bnc_getrf_d(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                size_t work_bytes, void *stream)
{
    return getrf_entry<1>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream);
}
int bnc_getrf_dd(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                 size_t work_bytes, void *stream)
{
    return getrf_entry<2>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream);
}
int bnc_getrf_td(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                 size_t work_bytes, void *stream)
{
    return getrf_entry<3>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream);
}
int bnc_getrf_qd(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *work,
                 size_t work_bytes, void *stream)
{
    return getrf_entry<4>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream);
}

int bnc_gemm_d(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
              int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream)
{
    return gemm_entry<1>(m, n, k, A, lda, ldpa, B, ldb, ldpb, C, ldc, ldpc, stream);
}
int bnc_gemm_dd(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
               int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream)
{
    return gemm_entry<2>(m, n, k, A, lda, ldpa, B, ldb, ldpb, C, ldc, ldpc, stream);
}
int bnc_gemm_td(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
               int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream)
{
    return gemm_entry<3>(m, n, k, A, lda, ldpa, B, ldb, ldpb, C, ldc, ldpc, stream);
}
int bnc_gemm_qd(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
               int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, void *stream)
{
    return gemm_entry<4>(m, n, k, A, lda, ldpa, B, ldb, ldpb, C, ldc, ldpc, stream);
}

int bnc_oz_beta(int32_t factor_words, int32_t slices)
{
    if (factor_words < 1 || factor_words > 4 || slices < 1 || slices > OZ_SMAX)
        return -1;
    return oz_beta(factor_words, slices);
}

int bnc_getrs_noalloc(int32_t factor_words, int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp,
                      const int64_t *ipiv, double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *stream)
{
    if (factor_words < 1 || factor_words > 4)
        return fail_arg(-1, "getrs_noalloc: factor_words outside 1..4");
    if (n > GETRS_NOALLOC_NMAX)
        return fail_arg(BNC_ERR_UNSUPPORTED, "getrs_noalloc: n above 16384, the order its fixed scratch holds");
    void *p = nullptr;
    size_t bytes = 0;
    const int rc = noalloc_scratch(&p, &bytes);
    if (rc)
        return rc;
    switch (factor_words) {
    case 1:
        return getrs_entry<1>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, p, bytes, stream, 1);
    case 2:
        return getrs_entry<2>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, p, bytes, stream, 1);
    case 3:
        return getrs_entry<3>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, p, bytes, stream, 1);
    default:
        return getrs_entry<4>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, p, bytes, stream, 1);
    }
}

size_t bnc_getrf_workspace_size(int32_t factor_words, int32_t slices, int64_t n)
{
    if (factor_words < 1 || factor_words > 4 || slices < 0 || slices > OZ_SMAX || n < 0 || n > 16384)
        return 0;
    return getrf_workspace_bytes(factor_words, n, slices);
}

size_t bnc_getrs_workspace_size(int32_t factor_words, int64_t n)
{
    if (factor_words < 1 || factor_words > 4 || n < 0 || n > 16384)
        return 0;
    return getrs_workspace_bytes(factor_words, n);
}

size_t bnc_residual_workspace_size(int64_t n)
{
    if (n < 0)
        return 0;
    return residual_workspace_bytes(n);
}

int bnc_test_force_timeout(int32_t bits)
{
    if (bits < 0 || bits > 3)
        return fail_arg(-1, "test_force_timeout: bits outside 0..3");
    g_force_timeout = bits;
    return BNC_OK;
}

int bnc_getrf_ozaki(int32_t factor_words, int32_t slices, int64_t n, double *A, int64_t lda, int64_t ldp,
                    int64_t *ipiv, int64_t *info, void *work, size_t work_bytes, void *stream)
{
    if (factor_words < 1 || factor_words > 4)
        return fail_arg(-1, "getrf_ozaki: factor_words outside 1..4");
    if (slices < 1 || slices > OZ_SMAX)
        return fail_arg(-2, "getrf_ozaki: slices outside 1..12");
    switch (factor_words) {
    case 1:
        return getrf_entry<1>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream, slices, 2);
    case 2:
        return getrf_entry<2>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream, slices, 2);
    case 3:
        return getrf_entry<3>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream, slices, 2);
    default:
        return getrf_entry<4>(n, A, lda, ldp, ipiv, info, work, work_bytes, stream, slices, 2);
    }
}

int bnc_getrs_d(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream)
{
    return getrs_entry<1>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, work, work_bytes, stream);
}
int bnc_getrs_dd(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                 double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream)
{
    return getrs_entry<2>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, work, work_bytes, stream);
}
int bnc_getrs_td(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                 double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream)
{
    return getrs_entry<3>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, work, work_bytes, stream);
}
int bnc_getrs_qd(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv,
                 double *B, int64_t ldb, int64_t ldpb, int64_t *info, void *work, size_t work_bytes, void *stream)
{
    return getrs_entry<4>(n, nrhs, LU, lda, ldp, ipiv, B, ldb, ldpb, info, work, work_bytes, stream);
}

size_t bnc_refine_workspace_size(int64_t n, int32_t factor_words)
{
    if (n < 1 || factor_words < 0 || factor_words > 4)
        return 0;
    return refine_workspace_bytes(n, factor_words);
}

int bnc_refine(int64_t n, int32_t a_words, const double *A, int64_t lda, int64_t ldpa, const double *b, int64_t ldpb,
               double *x, int64_t ldpx, void *work, size_t work_bytes, const bnc_refine_opts *opts,
               bnc_refine_result *result, void *stream)
{
    if (n < 1)
        return fail_arg(-1, "refine: n < 1");
    if (a_words != 1 && a_words != 4)
        return fail_arg(-2, "refine: a_words must be 1 or 4");
    if (!A)
        return fail_arg(-3, "refine: A is NULL");
    if (lda < n)
        return fail_arg(-4, "refine: lda < n");
    if (a_words > 1 && ldpa < lda * n)
        return fail_arg(-5, "refine: ldpa < lda * n");
    if (!b)
        return fail_arg(-6, "refine: b is NULL");
    if (ldpb < n)
        return fail_arg(-7, "refine: ldpb < n");
    if (!x)
        return fail_arg(-8, "refine: x is NULL");
    if (ldpx < n)
        return fail_arg(-9, "refine: ldpx < n");
    if (!work)
        return fail_arg(-10, "refine: work is NULL");
    if (!opts)
        return fail_arg(-12, "refine: opts is NULL");
    const bool autok = opts->factor_words == BNC_AUTO;
    if (autok && (!opts->selector_params || !opts->selector_norm))
        return fail_arg(-12, "refine: factor_words = 0 needs the selector's parameters and normalisation");
    if ((!autok && (opts->factor_words < 1 || opts->factor_words > 4)) || opts->max_iter < 0 || !(opts->rtol >= 0) ||
        opts->ozaki_slices < 0 || opts->ozaki_slices > OZ_SMAX || (opts->escalate != 0 && opts->escalate != 1) ||
        !batch_panel_ok(opts->batch_panel) || !batch_threads_ok(opts->batch_threads) ||
        !(opts->stagnation_ratio >= 0) || (opts->long_words != 0 && opts->long_words != 4 && opts->long_words != 8) ||
        !(opts->atol >= 0) || !(opts->ctol >= 0))
        return fail_arg(-12, "refine: invalid options");
    if (!result)
        return fail_arg(-13, "refine: result is NULL");
    if (n > 16384)
        return fail_arg(BNC_ERR_UNSUPPORTED, "refine: n > 16384");
    if (work_bytes < refine_workspace_bytes(n, autok ? 0 : (opts->escalate ? 4 : opts->factor_words)))
        return fail_arg(-11, "refine: workspace too small");
    if (autok)
        return refine_drive(0, n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    switch (opts->factor_words) {
    case 1:
        return refine_run<1>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    case 2:
        return refine_run<2>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    case 3:
        return refine_run<3>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    default:
        return refine_run<4>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    }
}

int bnc_refine_async(int64_t n, int32_t a_words, const double *A, int64_t lda, int64_t ldpa, const double *b,
                     int64_t ldpb, double *x, int64_t ldpx, void *work, size_t work_bytes,
                     const bnc_refine_opts *opts, bnc_refine_result *result, void *stream)
{
    if (n < 1)
        return fail_arg(-1, "refine_async: n < 1");
    if (a_words != 1 && a_words != 4)
        return fail_arg(-2, "refine_async: a_words must be 1 or 4");
    if (!A)
        return fail_arg(-3, "refine_async: A is NULL");
    if (lda < n)
        return fail_arg(-4, "refine_async: lda < n");
    if (a_words > 1 && ldpa < lda * n)
        return fail_arg(-5, "refine_async: ldpa < lda * n");
    if (!b)
        return fail_arg(-6, "refine_async: b is NULL");
    if (ldpb < n)
        return fail_arg(-7, "refine_async: ldpb < n");
    if (!x)
        return fail_arg(-8, "refine_async: x is NULL");
    if (ldpx < n)
        return fail_arg(-9, "refine_async: ldpx < n");
    if (!work)
        return fail_arg(-10, "refine_async: work is NULL");
    if (!opts || opts->factor_words < 1 || opts->factor_words > 4 || opts->escalate != 0 || opts->max_iter < 0 ||
        !(opts->rtol >= 0) || !(opts->atol >= 0) || !(opts->ctol >= 0) || !(opts->stagnation_ratio >= 0) ||
        opts->ozaki_slices < 0 || opts->ozaki_slices > OZ_SMAX ||
        (opts->long_words != 0 && opts->long_words != 4 && opts->long_words != 8))
        return fail_arg(-12, "refine_async: invalid options (factor_words 1..4, escalate 0)");
    if (!result)
        return fail_arg(-13, "refine_async: result is NULL");
    if (n > 16384)
        return fail_arg(BNC_ERR_UNSUPPORTED, "refine_async: n > 16384");
    if (work_bytes < refine_workspace_bytes(n, opts->factor_words))
        return fail_arg(-11, "refine_async: workspace too small");
    switch (opts->factor_words) {
    case 1:
        return refine_async_run<1>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    case 2:
        return refine_async_run<2>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    case 3:
        return refine_async_run<3>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    default:
        return refine_async_run<4>(n, a_words, A, lda, ldpa, b, ldpb, x, ldpx, work, opts, result, S(stream));
    }
}

size_t bnc_refine_batched_workspace_size(int32_t factor_words, int32_t slots, int32_t threads)
{
    if (factor_words < 1 || factor_words > 4 || slots < 0 || !batch_threads_ok(threads))
        return 0;
    return batch_workspace_bytes(factor_words, slots ? slots : batch_default_slots(factor_words, 0, threads),
                                 threads);
}

int32_t bnc_refine_batched_default_slots(int32_t factor_words, int32_t panel, int32_t threads)
{
    if (factor_words < 1 || factor_words > 4)
        return fail_arg(-1, "refine_batched_default_slots: factor_words outside 1..4");
    if (!batch_panel_ok(panel))
        return fail_arg(-2, "refine_batched_default_slots: panel not 0, 4, 8 or 16");
    if (!batch_threads_ok(threads))
        return fail_arg(-3, "refine_batched_default_slots: threads not 0, 64, 128, 256 or 512");
    return batch_default_slots(factor_words, panel, threads);
}

int bnc_refine_batched(int64_t count, const int64_t *n, const int32_t *a_words, const double *const *A,
                       const double *const *b, double *const *x, const int32_t *order, void *work,
                       size_t work_bytes, const bnc_refine_opts *opts, int32_t slots, bnc_batch_result *results,
                       void *stream)
{
    if (count < 0)
        return fail_arg(-1, "refine_batched: count < 0");
    if (count > 0 && !n)
        return fail_arg(-2, "refine_batched: n is NULL");
    if (count > 0 && !A)
        return fail_arg(-4, "refine_batched: A is NULL");
    if (count > 0 && !b)
        return fail_arg(-5, "refine_batched: b is NULL");
    if (count > 0 && !x)
        return fail_arg(-6, "refine_batched: x is NULL");
    if (!work)
        return fail_arg(-8, "refine_batched: work is NULL");
    if (!opts || opts->factor_words < 1 || opts->factor_words > 4 || opts->max_iter < 0 || !(opts->rtol >= 0) ||
        opts->ozaki_slices != 0 || opts->escalate != 0 || !(opts->stagnation_ratio >= 0) ||
        (opts->long_words != 0 && opts->long_words != 4) ||
        !batch_panel_ok(opts->batch_panel) || !batch_threads_ok(opts->batch_threads) ||
        !(opts->atol >= 0) || !(opts->ctol >= 0))
        return fail_arg(-10, "refine_batched: invalid options");
    if (slots < 0)
        return fail_arg(-11, "refine_batched: slots < 0");
    if (count > 0 && !results)
        return fail_arg(-12, "refine_batched: results is NULL");
    const int sl = slots ? slots : batch_default_slots(opts->factor_words, opts->batch_panel, opts->batch_threads);
    if (work_bytes < batch_workspace_bytes(opts->factor_words, sl, opts->batch_threads))
        return fail_arg(-9, "refine_batched: workspace too small");
    switch (opts->factor_words) {
    case 1:
        return batch_run<1>(count, n, a_words, A, b, x, order, work, sl, opts, results, S(stream));
    case 2:
        return batch_run<2>(count, n, a_words, A, b, x, order, work, sl, opts, results, S(stream));
    case 3:
        return batch_run<3>(count, n, a_words, A, b, x, order, work, sl, opts, results, S(stream));
    default:
        return batch_run<4>(count, n, a_words, A, b, x, order, work, sl, opts, results, S(stream));
    }
}

int bnc_refine_batched_graph(int64_t count, const int64_t *n, const int32_t *a_words, const double *const *A,
                             const double *const *b, double *const *x, const int32_t *order, void *work,
                             size_t work_bytes, const bnc_refine_opts *opts, int32_t slots,
                             bnc_batch_result *results, void *stream, void **graph_exec)
{
    if (!graph_exec)
        return fail_arg(-14, "refine_batched_graph: graph_exec is NULL");
    hipStream_t s = S(stream);
    if (!*graph_exec) {
        if (!s)
            return fail_arg(-13, "refine_batched_graph: capture needs a non-null stream");
        BNC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int rc =
            bnc_refine_batched(count, n, a_words, A, b, x, order, work, work_bytes, opts, slots, results, stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &g);
        if (rc)
            return rc;
        if (e != hipSuccess)
            return fail_hip(e, "hipStreamEndCapture", __FILE__, __LINE__);
        hipGraphExec_t ge = nullptr;
        BNC_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        BNC_HIP(hipGraphDestroy(g));
        *graph_exec = (void *)ge;
    }
    BNC_HIP(hipGraphLaunch((hipGraphExec_t)*graph_exec, s));
    return BNC_OK;
}

int bnc_graph_destroy(void *graph_exec)
{
    if (graph_exec)
        BNC_HIP(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
    return BNC_OK;
}

int64_t bnc_wall_clock_khz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return 0;
    return khz;
}

int bnc_residual(int64_t n, int32_t a_words, int32_t long_words, const double *A, int64_t lda, int64_t ldpa,
                 const double *x, int64_t ldpx, const double *b, int64_t ldpb, double *r, int64_t ldpr,
                 int32_t *inexact, void *work, size_t work_bytes, void *stream)
{
    if (n < 0)
        return fail_arg(-1, "residual: n < 0");
    if (a_words != 1 && a_words != 4)
        return fail_arg(-2, "residual: a_words must be 1 or 4");
    if (long_words != 4 && long_words != 8)
        return fail_arg(-3, "residual: long_words must be 4 or 8");
    if (n == 0)
        return BNC_OK;
    if (!A)
        return fail_arg(-4, "residual: A is NULL");
    if (lda < n)
        return fail_arg(-5, "residual: lda < n");
    if (a_words > 1 && ldpa < lda * n)
        return fail_arg(-6, "residual: ldpa < lda * n");
    if (!x)
        return fail_arg(-7, "residual: x is NULL");
    if (ldpx < n)
        return fail_arg(-8, "residual: ldpx < n");
    if (!b)
        return fail_arg(-9, "residual: b is NULL");
    if (ldpb < n)
        return fail_arg(-10, "residual: ldpb < n");
    if (!r)
        return fail_arg(-11, "residual: r is NULL");
    if (ldpr < n)
        return fail_arg(-12, "residual: ldpr < n");
    if (!inexact)
        return fail_arg(-13, "residual: inexact is NULL");
    if (!work)
        return fail_arg(-14, "residual: work is NULL");
    if (work_bytes < residual_workspace_bytes(n))
        return fail_arg(BNC_ERR_WORKSPACE, "residual: workspace smaller than bnc_residual_workspace_size");
    return residual_ws_run(n, a_words, long_words, A, lda, ldpa, x, ldpx, b, ldpb, r, ldpr, inexact, work,
                           S(stream));
}

int bnc_mw_apply(int32_t op, int32_t K, int64_t n, const double *c, const double *a, const double *b, double *out,
                 void *stream)
{
    if (op < 0 || op > 4)
        return fail_arg(-1, "mw_apply: unknown op");
    if (K < 1 || K > 4)
        return fail_arg(-2, "mw_apply: K must be 1..4");
    if (n < 0)
        return fail_arg(-3, "mw_apply: n < 0");
    if (n == 0)
        return BNC_OK;
    if (op == BNC_OP_FMS && !c)
        return fail_arg(-4, "mw_apply: c is NULL");
    if (!a)
        return fail_arg(-5, "mw_apply: a is NULL");
    if ((op == BNC_OP_FMS || op == BNC_OP_MUL || op == BNC_OP_ADD) && !b)
        return fail_arg(-6, "mw_apply: b is NULL");
    if (!out)
        return fail_arg(-7, "mw_apply: out is NULL");
    const dim3 g((unsigned)ceil_div(n, 256)), t(256);
    hipStream_t s = S(stream);
    switch (K) {
    case 1:
        hipLaunchKernelGGL(k_apply<1>, g, t, 0, s, op, n, c, a, b, out);
        break;
    case 2:
        hipLaunchKernelGGL(k_apply<2>, g, t, 0, s, op, n, c, a, b, out);
        break;
    case 3:
        hipLaunchKernelGGL(k_apply<3>, g, t, 0, s, op, n, c, a, b, out);
        break;
    default:
        hipLaunchKernelGGL(k_apply<4>, g, t, 0, s, op, n, c, a, b, out);
        break;
    }
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

int bnc_profile_enable(int32_t on)
{
    g_prof = on != 0;
    return BNC_OK;
}

int bnc_profile_read(double *ms, double *flops, int64_t *launches)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double tms = 0.0, tf = 0.0;
    for (auto &e : g_events) {
        float m = 0.f;
        BNC_HIP(hipEventSynchronize(e.b));
        BNC_HIP(hipEventElapsedTime(&m, e.a, e.b));
        tms += m;
        tf += e.flops;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    if (launches)
        *launches = (int64_t)g_events.size();
    g_events.clear();
    if (ms)
        *ms = tms;
    if (flops)
        *flops = tf;
    return BNC_OK;
}

size_t bnc_features_workspace_size(int32_t slots)
{
    if (slots < 0)
        return 0;
    return features_workspace_bytes(slots ? slots : features_default_slots());
}

int32_t bnc_features_default_slots(void) { return features_default_slots(); }

int bnc_features(int64_t count, const int64_t *n, const double *const *A, const double *const *b,
                 const int32_t *order, float *features, void *work, size_t work_bytes, int32_t slots, void *stream)
{
    if (count < 0)
        return fail_arg(-1, "features: count < 0");
    if (count > 0 && (!n || !A || !b || !features))
        return fail_arg(!n ? -2 : !A ? -3 : !b ? -4 : -6, "features: NULL pointer");
    if (slots < 0)
        return fail_arg(-9, "features: slots < 0");
    const int sl = slots ? slots : features_default_slots();
    if (!work || work_bytes < features_workspace_bytes(sl))
        return fail_arg(-7, "features: workspace too small");
    return features_run(count, n, A, b, order, features, work, sl, S(stream));
}

int32_t bnc_mlp_param_count(void) { return mlp_param_count(); }

size_t bnc_mlp_workspace_size(int64_t batch) { return batch < 0 ? 0 : mlp_workspace_bytes(batch); }

int bnc_mlp_forward(int64_t batch, const float *X, const float *norm, const float *params, float *out, void *stream)
{
    if (batch < 0)
        return fail_arg(-1, "mlp_forward: batch < 0");
    if (batch > 0 && (!X || !norm || !params || !out))
        return fail_arg(!X ? -2 : !norm ? -3 : !params ? -4 : -5, "mlp_forward: NULL pointer");
    return mlp_forward_run(batch, X, norm, params, out, S(stream));
}

int bnc_mlp_grad(int64_t batch, const float *X, const float *norm, const int32_t *cls, const float *target,
                 const float *params, float *grads, float *loss, void *work, size_t work_bytes, void *stream)
{
    if (batch < 1)
        return fail_arg(-1, "mlp_grad: batch < 1");
    if (!X || !norm || !cls || !target || !params || !grads || !loss)
        return fail_arg(!X ? -2 : !norm ? -3 : !cls ? -4 : !target ? -5 : !params ? -6 : !grads ? -7 : -8,
                        "mlp_grad: NULL pointer");
    if (!work || work_bytes < mlp_workspace_bytes(batch))
        return fail_arg(-9, "mlp_grad: workspace too small");
    return mlp_grad_run(batch, X, norm, cls, target, params, grads, loss, work, S(stream));
}

int bnc_mlp_adam(float *params, const float *grads, float *m, float *v, const bnc_adam_opts *opts, void *stream)
{
    if (!params || !grads || !m || !v)
        return fail_arg(!params ? -1 : !grads ? -2 : !m ? -3 : -4, "mlp_adam: NULL pointer");
    if (!opts || opts->step < 1 || !(opts->lr >= 0) || !(opts->beta1 >= 0 && opts->beta1 < 1) ||
        !(opts->beta2 >= 0 && opts->beta2 < 1) || !(opts->eps > 0))
        return fail_arg(-5, "mlp_adam: invalid options");
    return mlp_adam_run(params, grads, m, v, opts->lr, opts->beta1, opts->beta2, opts->eps, opts->step, S(stream));
}

const char *bnc_status_string(int32_t status)
{
    switch (status) {
    case BNC_CONVERGED:
        return "converged";
    case BNC_MAX_ITER:
        return "max_iter";
    case BNC_SINGULAR:
        return "singular";
    case BNC_NONFINITE:
        return "nonfinite";
    case BNC_BAD_SIZE:
        return "bad_size";
    case BNC_STAGNATED:
        return "stagnated";
    case BNC_TIMED_OUT:
        return "timed_out";
    case BNC_SPLIT_RANGE:
        return "split_range";
    default:
        return "unknown";
    }
}

const char *bnc_last_error(void) { return g_last_error.c_str(); }

const char *bnc_version(void) { return "bnc 0.1 (gfx950)"; }

}  // extern "C"

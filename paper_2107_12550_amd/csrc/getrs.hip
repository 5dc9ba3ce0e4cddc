// Forward/backward substitution with K-word LU factors (Kouya 2021, Sec. 2:
// the substitution step used for the first solution and every correction of
// Listing 1).
//
// The right-hand side is first gathered through the row permutation that
// the pivot sequence composes to (y = P b).  Each triangle is then solved
// by one persistent launch with a workgroup per 64-row block (see
// k_trsv_lower / k_trsv_upper).  Per row the updates arrive in increasing k
// for L and in decreasing k for U, exactly as in the unblocked
// column-oriented solve.
#include "common.hpp"
#include "mw.hpp"

namespace bnc {

constexpr int TS_BS = 64;  // block rows; equals the workgroup size

// perm[i] = original index of the row that ends at position i after the
// swaps k = 0..n-1 (one thread walks the sequence in LDS).
__global__ void __launch_bounds__(256) k_ipiv_to_perm(int64_t n, const int64_t *__restrict__ ipiv,
                                                      int32_t *__restrict__ perm)
{
    extern __shared__ int32_t sp[];
    int32_t *p = sp;          // n
    int32_t *iv = sp + n;     // n
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        p[i] = (int32_t)i;
        iv[i] = (int32_t)ipiv[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int64_t k = 0; k < n; ++k) {
            const int32_t q = iv[k];
            const int32_t t = p[k];
            p[k] = p[q];
            p[q] = t;
        }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        perm[i] = p[i];
}

template <int K>
__global__ void k_gather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ src, int64_t lds_,
                         double *__restrict__ dst, int64_t ldd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t s = perm[i];
#pragma unroll
    for (int w = 0; w < K; ++w)
        dst[w * ldd + i] = src[w * lds_ + s];
}

template <int K>
__global__ void k_copy_vec(int64_t n, const double *__restrict__ src, int64_t lds_, double *__restrict__ dst,
                           int64_t ldd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
#pragma unroll
    for (int w = 0; w < K; ++w)
        dst[w * ldd + i] = src[w * lds_ + i];
}

// Reciprocals of U's diagonal, r_k = 1 / u_kk, computed once per
// factorisation with the same K-word recip the unblocked solve uses.
template <int K>
__global__ void k_diag_recip(int64_t n, const double *__restrict__ LU, int64_t lda, int64_t ldp,
                             double *__restrict__ rd)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    double d[K], r[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        d[w] = LU[w * ldp + k * lda + k];
    recip<K>(d, r);
#pragma unroll
    for (int w = 0; w < K; ++w)
        rd[w * n + k] = r[w];
}

// Stage the square block rows/cols [b0, b0+bsz) of one triangle into LDS:
// blk[(w*TS_BS + c)*TS_BS + r] = word w of entry (b0+r, b0+c).
// ---- one persistent launch per triangle ---------------------------------
// Workgroup (one wave) per 64-row block.  A block takes every earlier
// block's finished values as soon as that block's flag is set (columns in
// solve order, so each row still sees its updates in the unblocked order),
// then solves its own diagonal block with wave shuffles, publishes its
// values through coherent device-scope atomics and sets its flag.  Blocks
// wait only on blocks that were dispatched before them, and every spin is
// bounded (on timeout the abort flag releases all waits).
constexpr int TS_G = 16;  // columns whose factor entries are fetched together
constexpr unsigned TS_SPIN = 1u << 22;

__device__ __forceinline__ void ts_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ts_load(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ts_wait(int *flag, int *abort_flag)
{
    if (threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > TS_SPIN) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void ts_publish_flag(int *flag)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_ts_flags_reset(int *flags, int count)
{
    for (int e = threadIdx.x; e < count; e += blockDim.x)
        flags[e] = 0;
}

// y <- L^-1 y (unit lower), y already permuted
template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_trsv_lower(const double *__restrict__ LU, int64_t lda, int64_t ldp, double *__restrict__ y, int64_t ldy,
                 int64_t n, int *__restrict__ flags, int *__restrict__ abort_flag)
{
    extern __shared__ double dblk[];  // own diagonal block [w][c][r]
    __shared__ double yb[TS_BS][K];
    const int b = blockIdx.x, lane = threadIdx.x;
    const int64_t r0 = (int64_t)b * TS_BS;
    const int bsz = (int)((n - r0) < TS_BS ? (n - r0) : TS_BS);
    const int64_t i = r0 + lane;
    const bool act = lane < bsz;
    for (int c = 0; c < bsz; ++c)
        if (act)
#pragma unroll
            for (int w = 0; w < K; ++w)
                dblk[(w * TS_BS + c) * TS_BS + lane] = LU[w * ldp + (r0 + c) * lda + i];
    double v[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        v[w] = act ? y[w * ldy + i] : 0.0;
    for (int c = 0; c < b; ++c) {  // earlier blocks are full
        const int64_t k0 = (int64_t)c * TS_BS;
        double t[TS_G][K];
#pragma unroll
        for (int q = 0; q < TS_G; ++q)
#pragma unroll
            for (int w = 0; w < K; ++w)
                t[q][w] = act ? LU[w * ldp + (k0 + q) * lda + i] : 0.0;
        ts_wait(flags + c, abort_flag);
#pragma unroll
        for (int w = 0; w < K; ++w)
            yb[lane][w] = ts_load(y + w * ldy + k0 + lane);
        __syncthreads();
        for (int g0 = 0; g0 < TS_BS; g0 += TS_G) {
            double tn[TS_G][K];
            const bool more = g0 + TS_G < TS_BS;
            if (more)
#pragma unroll
                for (int q = 0; q < TS_G; ++q)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        tn[q][w] = act ? LU[w * ldp + (k0 + g0 + TS_G + q) * lda + i] : 0.0;
#pragma unroll
            for (int q = 0; q < TS_G; ++q) {
                double yk[K], o[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    yk[w] = yb[g0 + q][w];
                fms<K>(v, t[q], yk, o);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    v[w] = o[w];
            }
            if (more)
#pragma unroll
                for (int q = 0; q < TS_G; ++q)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        t[q][w] = tn[q][w];
        }
        __syncthreads();
    }
    __syncthreads();
    for (int kk = 0; kk < bsz; ++kk) {
        double yk[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            yk[w] = __shfl(v[w], kk, 64);
        if (act && lane > kk) {
            double l[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                l[w] = dblk[(w * TS_BS + kk) * TS_BS + lane];
            fms<K>(v, l, yk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = o[w];
        }
    }
    if (act)
#pragma unroll
        for (int w = 0; w < K; ++w)
            ts_store(y + w * ldy + i, v[w]);
    ts_publish_flag(flags + b);
}

// y <- U^-1 y with rd = 1/u_kk; workgroup g solves block nblk-1-g
template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_trsv_upper(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ rd, double *__restrict__ y,
                 int64_t ldy, int64_t n, int *__restrict__ flags, int *__restrict__ abort_flag)
{
    extern __shared__ double dblk[];
    __shared__ double xb[TS_BS][K];
    const int nblk = gridDim.x, lane = threadIdx.x;
    const int b = nblk - 1 - (int)blockIdx.x;
    const int64_t r0 = (int64_t)b * TS_BS;
    const int bsz = (int)((n - r0) < TS_BS ? (n - r0) : TS_BS);
    const int64_t i = r0 + lane;
    const bool act = lane < bsz;
    for (int c = 0; c < bsz; ++c)
        if (act)
#pragma unroll
            for (int w = 0; w < K; ++w)
                dblk[(w * TS_BS + c) * TS_BS + lane] = LU[w * ldp + (r0 + c) * lda + i];
    double v[K], rk[K];
#pragma unroll
    for (int w = 0; w < K; ++w) {
        v[w] = act ? y[w * ldy + i] : 0.0;
        rk[w] = act ? rd[w * n + i] : 0.0;
    }
    for (int c = nblk - 1; c > b; --c) {
        const int64_t k0 = (int64_t)c * TS_BS;
        const int bc = (int)((n - k0) < TS_BS ? (n - k0) : TS_BS);
        double t[TS_G][K];
#pragma unroll
        for (int q = 0; q < TS_G; ++q)
#pragma unroll
            for (int w = 0; w < K; ++w)
                t[q][w] = (act && q < bc) ? LU[w * ldp + (k0 + bc - 1 - q) * lda + i] : 0.0;
        ts_wait(flags + c, abort_flag);
#pragma unroll
        for (int w = 0; w < K; ++w)
            xb[lane][w] = lane < bc ? ts_load(y + w * ldy + k0 + lane) : 0.0;
        __syncthreads();
        for (int g0 = 0; g0 < bc; g0 += TS_G) {
            double tn[TS_G][K];
            const bool more = g0 + TS_G < bc;
            if (more)
#pragma unroll
                for (int q = 0; q < TS_G; ++q)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        tn[q][w] = (act && g0 + TS_G + q < bc)
                                       ? LU[w * ldp + (k0 + bc - 1 - (g0 + TS_G + q)) * lda + i]
                                       : 0.0;
#pragma unroll
            for (int q = 0; q < TS_G; ++q) {
                if (g0 + q < bc) {
                    double xk[K], o[K];
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        xk[w] = xb[bc - 1 - (g0 + q)][w];
                    fms<K>(v, t[q], xk, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        v[w] = o[w];
                }
            }
            if (more)
#pragma unroll
                for (int q = 0; q < TS_G; ++q)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        t[q][w] = tn[q][w];
        }
        __syncthreads();
    }
    __syncthreads();
    for (int kk = bsz - 1; kk >= 0; --kk) {
        if (lane == kk) {
            double xk[K];
            mul<K>(v, rk, xk);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = xk[w];
        }
        double xk[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            xk[w] = __shfl(v[w], kk, 64);
        if (act && lane < kk) {
            double u[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                u[w] = dblk[(w * TS_BS + kk) * TS_BS + lane];
            fms<K>(v, u, xk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = o[w];
        }
    }
    if (act)
#pragma unroll
        for (int w = 0; w < K; ++w)
            ts_store(y + w * ldy + i, v[w]);
    ts_publish_flag(flags + b);
}

template <int K>
static size_t block_lds() { return (size_t)K * TS_BS * TS_BS * sizeof(double); }

template <int K>
static void allow_lds()
{
    static bool done = false;
    if (done)
        return;
    const int b = (int)block_lds<K>();
    if (hipFuncSetAttribute((const void *)k_trsv_lower<K>, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_trsv_upper<K>, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess)
        (void)hipGetLastError();
    done = true;
}

template <int K>
int diag_recip_run(int64_t n, const double *LU, int64_t lda, int64_t ldp, double *rd, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    hipLaunchKernelGGL((k_diag_recip<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, LU, lda, ldp, rd);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// Solve in place on y (already permuted), one right-hand side; rd = 1/u_kk.
// flags: 2 * ceil(n/64) + 1 ints of scratch for the persistent launches.
template <int K>
int trsv_pair(int64_t n, const double *LU, int64_t lda, int64_t ldp, const double *rd, double *y, int64_t ldy,
              int *flags, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    allow_lds<K>();
    const size_t lds = block_lds<K>();
    const int64_t nblk = ceil_div(n, TS_BS);
    const int nf = (int)(2 * nblk + 1);
    int *abort_flag = flags + 2 * nblk;
    hipLaunchKernelGGL(k_ts_flags_reset, dim3(1), dim3(256), 0, s, flags, nf);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_trsv_lower<K>), dim3((unsigned)nblk), dim3(TS_BS), lds, s, LU, lda, ldp, y, ldy, n, flags,
                       abort_flag);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_trsv_upper<K>), dim3((unsigned)nblk), dim3(TS_BS), lds, s, LU, lda, ldp, rd, y, ldy, n,
                       flags + nblk, abort_flag);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

size_t trsv_flags_bytes(int64_t n) { return (size_t)(2 * ceil_div(n, TS_BS) + 1) * sizeof(int); }

size_t getrs_scratch_bytes(int K, int64_t n)
{
    return (size_t)n * sizeof(int32_t) + 2 * (size_t)K * n * sizeof(double) + trsv_flags_bytes(n) + 1024;
}

int ipiv_to_perm(int64_t n, const int64_t *ipiv, int32_t *perm, hipStream_t s)
{
    const size_t lds = 2 * (size_t)n * sizeof(int32_t);
    hipLaunchKernelGGL(k_ipiv_to_perm, dim3(1), dim3(256), lds, s, n, ipiv, perm);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// y = P b, solve, with caller-provided perm, diagonal reciprocals rd
// (K planes, stride n) and y buffer
template <int K>
int getrs_perm(int64_t n, const double *LU, int64_t lda, int64_t ldp, const int32_t *perm, const double *rd,
               const double *b, int64_t ldb, double *y, int64_t ldy, int *flags, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    hipLaunchKernelGGL((k_gather<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, perm, b, ldb, y, ldy);
    BNC_LAUNCH_CHECK();
    return trsv_pair<K>(n, LU, lda, ldp, rd, y, ldy, flags, s);
}

template <int K>
int getrs_run(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv, double *B,
              int64_t ldb, int64_t ldpb, void *scr, hipStream_t s)
{
    if (n == 0 || nrhs == 0)
        return BNC_OK;
    int32_t *perm = (int32_t *)scr;
    double *y = (double *)((char *)scr + ((n * sizeof(int32_t) + 255) / 256) * 256);
    double *rd = y + (size_t)K * n;
    int *flags = (int *)(rd + (size_t)K * n);
    int rc = ipiv_to_perm(n, ipiv, perm, s);
    if (rc)
        return rc;
    if ((rc = diag_recip_run<K>(n, LU, lda, ldp, rd, s)))
        return rc;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *bc = B + c * ldb;
        rc = getrs_perm<K>(n, LU, lda, ldp, perm, rd, bc, ldpb, y, n, flags, s);
        if (rc)
            return rc;
        hipLaunchKernelGGL((k_copy_vec<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, y, n, bc, ldpb);
        BNC_LAUNCH_CHECK();
    }
    return BNC_OK;
}

#define INST(K)                                                                                                     \
    template int getrs_perm<K>(int64_t, const double *, int64_t, int64_t, const int32_t *, const double *,          \
                               const double *, int64_t, double *, int64_t, int *, hipStream_t);                     \
    template int diag_recip_run<K>(int64_t, const double *, int64_t, int64_t, double *, hipStream_t);               \
    template int getrs_run<K>(int64_t, int64_t, const double *, int64_t, int64_t, const int64_t *, double *,        \
                              int64_t, int64_t, void *, hipStream_t);
INST(1)
INST(2)
INST(3)
INST(4)
#undef INST

}  // namespace bnc

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
// swaps k = 0..n-1.  Each thread follows one original row through the whole
// sequence (the swap k moves the row at position k to ipiv[k] and the row
// at ipiv[k] to k), then writes its index at its final position.  The
// pivots pass through LDS in chunks, read four at a time one group ahead of
// their use.  An entry outside [k, n) is taken as no interchange, so the
// result is always a permutation of 0..n-1 and every write stays in perm.
constexpr int PERM_CHUNK = 4096;
__global__ void __launch_bounds__(256) k_ipiv_to_perm(int64_t n, const int64_t *__restrict__ ipiv,
                                                      int32_t *__restrict__ perm)
{
    __shared__ int4 sp4[PERM_CHUNK / 4];
    int32_t *sp = (int32_t *)sp4;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t pos = (int32_t)(r < n ? r : 0);
    for (int64_t c0 = 0; c0 < n; c0 += PERM_CHUNK) {
        const int len = (int)((n - c0) < PERM_CHUNK ? (n - c0) : PERM_CHUNK);
        __syncthreads();
        for (int e = threadIdx.x; e < PERM_CHUNK; e += blockDim.x) {
            const int64_t k = c0 + e;
            int32_t p = (int32_t)k;  // padding past n: no interchange
            if (e < len) {
                const int64_t q = ipiv[k];
                if (q >= k && q < n)
                    p = (int32_t)q;
            }
            sp[e] = p;
        }
        __syncthreads();
        const int ng = (len + 3) / 4;
        int4 cur = sp4[0];
        for (int g = 0; g < ng; ++g) {
            const int4 nxt = sp4[g + 1 < ng ? g + 1 : g];
            const int32_t k = (int32_t)c0 + 4 * g;
            pos = pos == k ? cur.x : (pos == cur.x ? k : pos);
            pos = pos == k + 1 ? cur.y : (pos == cur.y ? k + 1 : pos);
            pos = pos == k + 2 ? cur.z : (pos == cur.z ? k + 2 : pos);
            pos = pos == k + 3 ? cur.w : (pos == cur.w ? k + 3 : pos);
            cur = nxt;
        }
    }
    if (r < n)
        perm[pos] = (int32_t)r;
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
// Workgroup (one wave) per 64-row block.  Solved values are streamed: the
// output planes start as XSENT (a signalling NaN that no arithmetic
// produces) and every value is written once, by its lane, the moment it is
// final (during the block's own diagonal solve).  A block consumes an
// earlier block's values TS_G at a time, polling the words themselves, in
// solve order, so each row still sees its updates in the unblocked order;
// blocks wait only on blocks that were dispatched before them, and every
// poll is bounded (on timeout the abort flag releases all waits and the
// result is garbage).  A right-hand side that holds the XSENT bit pattern
// can stall a poll in the same way.
constexpr int TS_G = 8;  // columns fetched and consumed together
constexpr unsigned TS_SPIN = 1u << 22;
constexpr int64_t TS_SENT = (int64_t)0xFFF40000DEADBEEFull;

__device__ __forceinline__ void ts_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ts_load(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool ts_sent(double v) { return __double_as_longlong(v) == (long long)TS_SENT; }

// lane l's double (l wave-uniform) to every lane, through scalar registers
__device__ __forceinline__ double ts_bcast(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Wait until the lanes in `need` of the 64-value block at src (K planes,
// stride n) are final; lanes that have their value put it in vb[lane].
// `have` (per lane; set beforehand for lanes past the end of a short block,
// which then never load) and the returned mask carry over between calls.
template <int K>
__device__ __forceinline__ unsigned long long ts_poll(const double *src, int64_t n, unsigned long long need,
                                                     unsigned long long fin, bool &have, double (&vb)[TS_BS][K],
                                                     int *abort_flag, unsigned &spins)
{
    const int lane = threadIdx.x;
    while ((fin & need) != need) {
        if (!have) {
            double q[K];
            bool ok = true;
#pragma unroll
            for (int w = 0; w < K; ++w) {
                q[w] = ts_load(src + w * n + lane);
                ok = ok && !ts_sent(q[w]);
            }
            if (ok) {
#pragma unroll
                for (int w = 0; w < K; ++w)
                    vb[lane][w] = q[w];
                have = true;
            }
        }
        fin = __ballot(have);
        if ((fin & need) != need) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > TS_SPIN ||
                ((spins & 1023u) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                spins = TS_SPIN;
                return ~0ull;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    return fin;
}

// both output planes to XSENT, abort flag cleared
__global__ void k_ts_reset(uint64_t *xs, int64_t nw, int *abort_flag)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += stride)
        xs[e] = (uint64_t)TS_SENT;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *abort_flag = 0;
}

// x = L^-1 y (unit lower), y already permuted; x: K planes of stride n
template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_trsv_lower(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ y, int64_t ldy,
                 int64_t n, double *__restrict__ x, int *__restrict__ abort_flag)
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
    unsigned spins = 0;
    for (int c = 0; c < b; ++c) {  // earlier blocks are full
        const int64_t k0 = (int64_t)c * TS_BS;
        double t[TS_G][K];
#pragma unroll
        for (int q = 0; q < TS_G; ++q)
#pragma unroll
            for (int w = 0; w < K; ++w)
                t[q][w] = act ? LU[w * ldp + (k0 + q) * lda + i] : 0.0;
        unsigned long long fin = 0;
        bool have = false;
        for (int g0 = 0; g0 < TS_BS; g0 += TS_G) {
            fin = ts_poll<K>(x + k0, n, ((1ull << TS_G) - 1) << g0, fin, have, yb, abort_flag, spins);
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
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // own diagonal block: lane kk is final when its turn comes; it
    // publishes its value before the others use it.  The block's next
    // column is read from LDS one step ahead (all 64 columns are there).
    double l[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        l[w] = dblk[(w * TS_BS) * TS_BS + lane];
    for (int kk = 0; kk < bsz; ++kk) {
        double yk[K], ln[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            yk[w] = ts_bcast(v[w], kk);
        if (lane == kk)
#pragma unroll
            for (int w = 0; w < K; ++w)
                ts_store(x + w * n + i, v[w]);
        const int kn = kk + 1 < TS_BS ? kk + 1 : kk;
#pragma unroll
        for (int w = 0; w < K; ++w)
            ln[w] = dblk[(w * TS_BS + kn) * TS_BS + lane];
        if (act && lane > kk) {
            double o[K];
            fms<K>(v, l, yk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = o[w];
        }
#pragma unroll
        for (int w = 0; w < K; ++w)
            l[w] = ln[w];
    }
}

// y = U^-1 x with rd = 1/u_kk; the values go to xo (streamed, K planes of
// stride n) and to y; workgroup g solves block nblk-1-g
template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_trsv_upper(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ rd,
                 const double *__restrict__ x, double *__restrict__ xo, double *__restrict__ y, int64_t ldy, int64_t n,
                 int *__restrict__ abort_flag)
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
        v[w] = act ? x[w * n + i] : 0.0;
        rk[w] = act ? rd[w * n + i] : 0.0;
    }
    unsigned spins = 0;
    for (int c = nblk - 1; c > b; --c) {
        const int64_t k0 = (int64_t)c * TS_BS;
        const int bc = (int)((n - k0) < TS_BS ? (n - k0) : TS_BS);
        // columns in decreasing order: position q of the sweep is column
        // bc-1-q of the block
        double t[TS_G][K];
#pragma unroll
        for (int q = 0; q < TS_G; ++q)
#pragma unroll
            for (int w = 0; w < K; ++w)
                t[q][w] = (act && q < bc) ? LU[w * ldp + (k0 + bc - 1 - q) * lda + i] : 0.0;
        unsigned long long fin = 0;
        bool have = lane >= bc;  // lanes beyond a short last block never load
        for (int g0 = 0; g0 < bc; g0 += TS_G) {
            // the block's lanes bc-1-g0-q for q < TS_G (those >= 0)
            const int hi = bc - 1 - g0, lo = (hi - TS_G + 1) > 0 ? (hi - TS_G + 1) : 0;
            const unsigned long long need = (hi - lo + 1 == 64 ? ~0ull : ((1ull << (hi - lo + 1)) - 1)) << lo;
            fin = ts_poll<K>(xo + k0, n, need, fin, have, xb, abort_flag, spins);
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
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // the loads of v and rd are complete here; waiting for them explicitly
    // keeps the compiler from placing a full vector-memory wait at the head
    // of the loop below, where it would also wait for each published store
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // own diagonal block in decreasing order; the next column is read
    // from LDS one step ahead
    double u[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        u[w] = dblk[(w * TS_BS + (bsz > 0 ? bsz - 1 : 0)) * TS_BS + lane];
    for (int kk = bsz - 1; kk >= 0; --kk) {
        if (lane == kk) {
            double xk[K];
            mul<K>(v, rk, xk);
#pragma unroll
            for (int w = 0; w < K; ++w) {
                v[w] = xk[w];
                ts_store(xo + w * n + i, xk[w]);
            }
        }
        double xk[K], un[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            xk[w] = ts_bcast(v[w], kk);
        const int kn = kk > 0 ? kk - 1 : 0;
#pragma unroll
        for (int w = 0; w < K; ++w)
            un[w] = dblk[(w * TS_BS + kn) * TS_BS + lane];
        if (act && lane < kk) {
            double o[K];
            fms<K>(v, u, xk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = o[w];
        }
#pragma unroll
        for (int w = 0; w < K; ++w)
            u[w] = un[w];
    }
    if (act)
#pragma unroll
        for (int w = 0; w < K; ++w)
            y[w * ldy + i] = v[w];
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
// ws: trsv_ws_bytes(n) bytes of scratch (the two streamed planes sets and
// the abort flag of the persistent launches).
template <int K>
int trsv_pair(int64_t n, const double *LU, int64_t lda, int64_t ldp, const double *rd, double *y, int64_t ldy,
              void *ws, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    allow_lds<K>();
    const size_t lds = block_lds<K>();
    const int64_t nblk = ceil_div(n, TS_BS);
    double *x1 = (double *)ws, *x2 = x1 + (size_t)K * n;
    int *abort_flag = (int *)(x2 + (size_t)K * n);
    hipLaunchKernelGGL(k_ts_reset, dim3((unsigned)(ceil_div(2 * K * n, 256) < 64 ? ceil_div(2 * K * n, 256) : 64)),
                       dim3(256), 0, s, (uint64_t *)x1, (int64_t)(2 * K * n), abort_flag);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_trsv_lower<K>), dim3((unsigned)nblk), dim3(TS_BS), lds, s, LU, lda, ldp, y, ldy, n, x1,
                       abort_flag);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_trsv_upper<K>), dim3((unsigned)nblk), dim3(TS_BS), lds, s, LU, lda, ldp, rd, x1, x2, y, ldy,
                       n, abort_flag);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// up to four words per value
size_t trsv_ws_bytes(int64_t n) { return 2 * 4 * (size_t)(n > 0 ? n : 1) * sizeof(double) + 256; }

size_t getrs_scratch_bytes(int K, int64_t n)
{
    return (size_t)n * sizeof(int32_t) + 2 * (size_t)K * n * sizeof(double) + trsv_ws_bytes(n) + 1024;
}

int ipiv_to_perm(int64_t n, const int64_t *ipiv, int32_t *perm, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    hipLaunchKernelGGL(k_ipiv_to_perm, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, ipiv, perm);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// y = P b, solve, with caller-provided perm, diagonal reciprocals rd
// (K planes, stride n) and y buffer
template <int K>
int getrs_perm(int64_t n, const double *LU, int64_t lda, int64_t ldp, const int32_t *perm, const double *rd,
               const double *b, int64_t ldb, double *y, int64_t ldy, void *ws, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    hipLaunchKernelGGL((k_gather<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, perm, b, ldb, y, ldy);
    BNC_LAUNCH_CHECK();
    return trsv_pair<K>(n, LU, lda, ldp, rd, y, ldy, ws, s);
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
    void *ws = (void *)(rd + (size_t)K * n);
    int rc = ipiv_to_perm(n, ipiv, perm, s);
    if (rc)
        return rc;
    if ((rc = diag_recip_run<K>(n, LU, lda, ldp, rd, s)))
        return rc;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *bc = B + c * ldb;
        rc = getrs_perm<K>(n, LU, lda, ldp, perm, rd, bc, ldpb, y, n, ws, s);
        if (rc)
            return rc;
        hipLaunchKernelGGL((k_copy_vec<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, y, n, bc, ldpb);
        BNC_LAUNCH_CHECK();
    }
    return BNC_OK;
}

#define INST(K)                                                                                                     \
    template int getrs_perm<K>(int64_t, const double *, int64_t, int64_t, const int32_t *, const double *,          \
                               const double *, int64_t, double *, int64_t, void *, hipStream_t);                    \
    template int diag_recip_run<K>(int64_t, const double *, int64_t, int64_t, double *, hipStream_t);               \
    template int getrs_run<K>(int64_t, int64_t, const double *, int64_t, int64_t, const int64_t *, double *,        \
                              int64_t, int64_t, void *, hipStream_t);
INST(1)
INST(2)
INST(3)
INST(4)
#undef INST

}  // namespace bnc

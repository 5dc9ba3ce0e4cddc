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
#include <mutex>

#include "common.hpp"
#include "mw.hpp"

namespace bnc {

// skip flag of the device-driven refinement loop (nullptr: run)
#define TS_SKIP_IF(skip)      \
    if ((skip) && *(skip))    \
        return;

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
                         double *__restrict__ dst, int64_t ldd, const int *__restrict__ skip)
{
    TS_SKIP_IF(skip);
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
// Workgroup per 64-row block, two waves.  Solved values are streamed: the
// output planes start as XSENT (a signalling NaN that no arithmetic
// produces) and every value is written once, by its lane, the moment it is
// final (during the block's own diagonal solve).  Wave 1 fetches the
// earlier blocks' values in solve order, polling the words themselves,
// into a two-slot LDS ring; each lane stamps its entry with the block's
// tag once its words are there.  Wave 0 consumes them TS_G columns at a
// time, waiting on the stamps in LDS, so each row still sees its updates
// in the unblocked order, then solves its own diagonal block.  Keeping the
// polls in their own wave keeps their memory waits away from wave 0, whose
// loads of the triangle's entries stay TS_PF groups ahead of their use.
// Blocks wait only on blocks dispatched before them, and every wait is
// bounded (on timeout the abort flag releases all waits and the result is
// garbage).  A right-hand side that holds the XSENT bit pattern can stall
// a poll in the same way.
// Columns consumed together, a divisor of 64 below it, by word count (the
// faster of 4 and 8 for each K at n = 4096; the solution does not depend on
// it).  Each kernel names it TS_G and its groups per block TS_NG.
template <int K>
constexpr int ts_group()
{
    return (K == 2 || K == 4) ? 4 : 8;
}
constexpr int TS_PF = 4;  // groups of entries in flight (wave 0)
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

// One more round of a bounded wait: false once the spin budget is spent or
// another wave has raised the abort flag (then it is raised here too and
// every later wait of this wave gives up at once).
__device__ __forceinline__ bool ts_again(unsigned &spins, int *abort_flag)
{
    __builtin_amdgcn_s_sleep(1);
    if (++spins > TS_SPIN ||
        ((spins & 1023u) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        spins = TS_SPIN;
        return false;
    }
    return true;
}

// Wave 1: lanes [0, cnt) of the 64-value block at src (K planes, stride n)
// into slot[lane] as soon as their words are final, each entry stamped
// with tag after its words are in LDS.
template <int K>
__device__ __forceinline__ void ts_fetch(const double *src, int64_t n, int cnt, int tag, double (*slot)[K],
                                         int *stamp, unsigned &spins, int *abort_flag)
{
    const int lane = threadIdx.x & 63;
    bool have = lane >= cnt;
    for (;;) {
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
                    slot[lane][w] = q[w];
                __hip_atomic_store(&stamp[lane], tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                have = true;
            }
        }
        if (__ballot(!have) == 0ull || !ts_again(spins, abort_flag))
            break;
    }
}

// Wave 0: until the entries of the lanes in `need` carry tag.
__device__ __forceinline__ void ts_wait(const int *stamp, unsigned long long need, int tag, unsigned &spins,
                                        int *abort_flag)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        const bool ok = __hip_atomic_load(const_cast<int *>(&stamp[lane]), __ATOMIC_ACQUIRE,
                                          __HIP_MEMORY_SCOPE_WORKGROUP) == tag;
        if ((__ballot(ok) & need) == need || !ts_again(spins, abort_flag))
            break;
    }
}

// Wave 1: until wave 0 has finished `want` blocks (a slot is reused two
// blocks later).
__device__ __forceinline__ void ts_wait_done(const int *done, int want, unsigned &spins, int *abort_flag)
{
    while (__hip_atomic_load(const_cast<int *>(done), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < want)
        if (!ts_again(spins, abort_flag))
            break;
}

// both output planes to XSENT, abort flag cleared
__global__ void k_ts_reset(uint64_t *xs, int64_t nw, int *abort_flag, const int *__restrict__ skip)
{
    TS_SKIP_IF(skip);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += stride)
        xs[e] = (uint64_t)TS_SENT;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *abort_flag = 0;
}

// raise the abort flag (the timeout test hook) / report it: info = -1
__global__ void k_ts_raise(int *abort_flag)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *abort_flag = 1;
}

__global__ void k_ts_info(const int *abort_flag, int64_t *info, const int *__restrict__ skip)
{
    TS_SKIP_IF(skip);
    if (blockIdx.x == 0 && threadIdx.x == 0 && *abort_flag)
        *info = -1;
}

__global__ void k_ts_zero(int64_t *info)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *info = 0;
}

// x = L^-1 y (unit lower), y already permuted; x: K planes of stride n
template <int K>
__global__ void __launch_bounds__(2 * TS_BS)
    k_trsv_lower(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ y, int64_t ldy,
                 int64_t n, double *__restrict__ x, int *__restrict__ abort_flag, const int *__restrict__ skip)
{
    constexpr int TS_G = ts_group<K>(), TS_NG = TS_BS / TS_G;
    static_assert(TS_G < 64 && TS_BS % TS_G == 0 && TS_NG % TS_PF == 0, "group size must tile the block");
    TS_SKIP_IF(skip);  // every thread of the grid reads the same flag
    extern __shared__ double dblk[];  // own diagonal block [w][c][r]
    __shared__ double yb[2][TS_BS][K];
    __shared__ int stamp[2][TS_BS];
    __shared__ int done;
    const int b = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)b * TS_BS;
    const int bsz = (int)((n - r0) < TS_BS ? (n - r0) : TS_BS);
    const int64_t i = r0 + lane;
    const bool act = lane < bsz;
#pragma unroll 2
    for (int c = wave; c < bsz; c += 2)
        if (act)
#pragma unroll
            for (int w = 0; w < K; ++w)
                dblk[(w * TS_BS + c) * TS_BS + lane] = LU[w * ldp + (r0 + c) * lda + i];
    stamp[wave][lane] = 0;
    if (threadIdx.x == 0)
        done = 0;
    __syncthreads();
    unsigned spins = 0;
    if (wave == 1) {  // earlier blocks are full
        for (int c = 0; c < b; ++c) {
            if (c >= 2)
                ts_wait_done(&done, c - 1, spins, abort_flag);
            ts_fetch<K>(x + (int64_t)c * TS_BS, n, TS_BS, c + 1, yb[c & 1], stamp[c & 1], spins, abort_flag);
        }
        return;
    }
    double v[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        v[w] = act ? y[w * ldy + i] : 0.0;
    // group G = columns G*TS_G.. of the earlier blocks; its L entries are
    // loaded TS_PF groups ahead, unconditionally from in-bounds addresses
    // (lanes past a short block read its last row, groups past the end
    // re-read the last one), so the loads in flight can be counted; those
    // lanes' values are never stored
    const int64_t ic = r0 + (act ? lane : bsz - 1);
    const int NG = b * TS_NG;
    double tr[TS_PF][TS_G][K];
    auto fetch = [&](int G, double (&t)[TS_G][K]) {
        const int64_t k = (int64_t)(G < NG ? G : NG - 1) * TS_G;
#pragma unroll
        for (int q = 0; q < TS_G; ++q)
#pragma unroll
            for (int w = 0; w < K; ++w)
                t[q][w] = LU[w * ldp + (k + q) * lda + ic];
    };
    if (NG > 0)
#pragma unroll
        for (int p = 0; p < TS_PF; ++p)
            fetch(p, tr[p]);
    for (int G0 = 0; G0 < NG; G0 += TS_PF) {  // NG is a multiple of TS_PF
#pragma unroll
        for (int p = 0; p < TS_PF; ++p) {
            const int G = G0 + p;
            const int c = G / TS_NG, g0 = (G % TS_NG) * TS_G;
            ts_wait(stamp[c & 1], ((1ull << TS_G) - 1) << g0, c + 1, spins, abort_flag);
#pragma unroll
            for (int q = 0; q < TS_G; ++q) {
                double yk[K], o[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    yk[w] = yb[c & 1][g0 + q][w];
                fms<K>(v, tr[p][q], yk, o);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    v[w] = o[w];
            }
            // the group's arithmetic is done here, before the next wait (it
            // would otherwise sink past it, to where v is next used)
#pragma unroll
            for (int w = 0; w < K; ++w)
                __asm__ volatile("" ::"v"(v[w]) : "memory");
            if (g0 + TS_G == TS_BS && lane == 0)
                __hip_atomic_store(&done, c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            // the refill stays after the group's arithmetic, so that it
            // reuses the group's registers instead of doubling them
            __builtin_amdgcn_sched_barrier(0);
            fetch(G + TS_PF, tr[p]);
        }
    }
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
__global__ void __launch_bounds__(2 * TS_BS)
    k_trsv_upper(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ rd,
                 const double *__restrict__ x, double *__restrict__ xo, double *__restrict__ y, int64_t ldy, int64_t n,
                 int *__restrict__ abort_flag, const int *__restrict__ skip)
{
    constexpr int TS_G = ts_group<K>(), TS_NG = TS_BS / TS_G;
    static_assert(TS_G < 64 && TS_BS % TS_G == 0 && TS_NG % TS_PF == 0, "group size must tile the block");
    TS_SKIP_IF(skip);
    extern __shared__ double dblk[];
    __shared__ double xb[2][TS_BS][K];
    __shared__ int stamp[2][TS_BS];
    __shared__ int done;
    const int nblk = gridDim.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = nblk - 1 - (int)blockIdx.x;
    const int64_t r0 = (int64_t)b * TS_BS;
    const int bsz = (int)((n - r0) < TS_BS ? (n - r0) : TS_BS);
    const int64_t i = r0 + lane;
    const bool act = lane < bsz;
#pragma unroll 2
    for (int c = wave; c < bsz; c += 2)
        if (act)
#pragma unroll
            for (int w = 0; w < K; ++w)
                dblk[(w * TS_BS + c) * TS_BS + lane] = LU[w * ldp + (r0 + c) * lda + i];
    stamp[wave][lane] = 0;
    if (threadIdx.x == 0)
        done = 0;
    __syncthreads();
    // the blocks after this one, in solve order e = 0.. (block nblk-1-e;
    // only e = 0 can be short)
    const int ne = nblk - 1 - b;
    unsigned spins = 0;
    if (wave == 1) {
        for (int e = 0; e < ne; ++e) {
            const int64_t k0 = (int64_t)(nblk - 1 - e) * TS_BS;
            const int bc = (int)((n - k0) < TS_BS ? (n - k0) : TS_BS);
            if (e >= 2)
                ts_wait_done(&done, e - 1, spins, abort_flag);
            ts_fetch<K>(xo + k0, n, bc, e + 1, xb[e & 1], stamp[e & 1], spins, abort_flag);
        }
        return;
    }
    double v[K], rk[K];
#pragma unroll
    for (int w = 0; w < K; ++w) {
        v[w] = act ? x[w * n + i] : 0.0;
        rk[w] = act ? rd[w * n + i] : 0.0;
    }
    // group G: sweep positions (G % TS_NG)*TS_G.. of block e = G / TS_NG,
    // position p being column bc-1-p of the block (columns in decreasing
    // order); U entries loaded TS_PF groups ahead from clamped in-bounds
    // addresses, as in the lower solve
    const int64_t ic = r0 + (act ? lane : bsz - 1);
    const int NG = ne * TS_NG;
    double tr[TS_PF][TS_G][K];
    auto fetch = [&](int G, double (&t)[TS_G][K]) {
        const int Gc = G < NG ? G : NG - 1;
        const int64_t k0 = (int64_t)(nblk - 1 - Gc / TS_NG) * TS_BS;
        const int bc = (int)((n - k0) < TS_BS ? (n - k0) : TS_BS);
#pragma unroll
        for (int q = 0; q < TS_G; ++q) {
            const int ps = (Gc % TS_NG) * TS_G + q;
            const int pc = ps < bc ? ps : bc - 1;
#pragma unroll
            for (int w = 0; w < K; ++w)
                t[q][w] = LU[w * ldp + (k0 + bc - 1 - pc) * lda + ic];
        }
    };
    if (NG > 0)
#pragma unroll
        for (int p = 0; p < TS_PF; ++p)
            fetch(p, tr[p]);
    for (int G0 = 0; G0 < NG; G0 += TS_PF) {  // NG is a multiple of TS_PF
#pragma unroll
        for (int p = 0; p < TS_PF; ++p) {
            const int G = G0 + p;
            const int e = G / TS_NG, g0 = (G % TS_NG) * TS_G;
            const int64_t k0 = (int64_t)(nblk - 1 - e) * TS_BS;
            const int bc = (int)((n - k0) < TS_BS ? (n - k0) : TS_BS);
            if (g0 < bc) {
                // the block's lanes bc-1-g0-q for q < TS_G (those >= 0)
                const int hi = bc - 1 - g0, lo = (hi - TS_G + 1) > 0 ? (hi - TS_G + 1) : 0;
                const unsigned long long need = ((1ull << (hi - lo + 1)) - 1) << lo;
                ts_wait(stamp[e & 1], need, e + 1, spins, abort_flag);
#pragma unroll
                for (int q = 0; q < TS_G; ++q) {
                    if (g0 + q < bc) {
                        double xk[K], o[K];
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            xk[w] = xb[e & 1][bc - 1 - (g0 + q)][w];
                        fms<K>(v, tr[p][q], xk, o);
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            v[w] = o[w];
                    }
                }
            }
#pragma unroll
            for (int w = 0; w < K; ++w)  // as in the lower solve
                __asm__ volatile("" ::"v"(v[w]) : "memory");
            if (g0 + TS_G == TS_BS && lane == 0)
                __hip_atomic_store(&done, e + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_sched_barrier(0);  // as in the lower solve
            fetch(G + TS_PF, tr[p]);
        }
    }
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
// the abort flag of the persistent launches).  info (nullable): set to -1
// when a bounded wait of the pair gave up (never cleared here).
template <int K>
int trsv_pair(int64_t n, const double *LU, int64_t lda, int64_t ldp, const double *rd, double *y, int64_t ldy,
              void *ws, hipStream_t s, int64_t *info, const int *skip)
{
    if (n == 0)
        return BNC_OK;
    allow_lds<K>();
    const size_t lds = block_lds<K>();
    const int64_t nblk = ceil_div(n, TS_BS);
    double *x1 = (double *)ws, *x2 = x1 + (size_t)K * n;
    int *abort_flag = (int *)(x2 + (size_t)K * n);
    hipLaunchKernelGGL(k_ts_reset, dim3((unsigned)(ceil_div(2 * K * n, 256) < 64 ? ceil_div(2 * K * n, 256) : 64)),
                       dim3(256), 0, s, (uint64_t *)x1, (int64_t)(2 * K * n), abort_flag, skip);
    BNC_LAUNCH_CHECK();
    if (force_timeout_bits() & 2) {
        hipLaunchKernelGGL(k_ts_raise, dim3(1), dim3(64), 0, s, abort_flag);
        BNC_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_trsv_lower<K>), dim3((unsigned)nblk), dim3(2 * TS_BS), lds, s, LU, lda, ldp, y, ldy, n, x1,
                       abort_flag, skip);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_trsv_upper<K>), dim3((unsigned)nblk), dim3(2 * TS_BS), lds, s, LU, lda, ldp, rd, x1, x2, y, ldy,
                       n, abort_flag, skip);
    BNC_LAUNCH_CHECK();
    if (info) {
        hipLaunchKernelGGL(k_ts_info, dim3(1), dim3(64), 0, s, (const int *)abort_flag, info, skip);
        BNC_LAUNCH_CHECK();
    }
    return BNC_OK;
}

// up to four words per value
static constexpr size_t trsv_ws_bytes_c(int64_t n) { return 2 * 4 * (size_t)(n > 0 ? n : 1) * sizeof(double) + 256; }
size_t trsv_ws_bytes(int64_t n) { return trsv_ws_bytes_c(n); }

static constexpr size_t getrs_ws_bytes_c(int K, int64_t n)
{
    return n <= 0 ? 0
                  : align256((size_t)n * sizeof(int32_t)) + 2 * (size_t)K * n * sizeof(double) + trsv_ws_bytes_c(n) +
                        1024;
}
size_t getrs_workspace_bytes(int K, int64_t n) { return getrs_ws_bytes_c(K, n); }

// ---- fixed scratch of the no-allocation solve (bnc_getrs_noalloc) -----------
// The workspace of a quad-double solve of the largest order it accepts, in
// one file-scope device array: each device holds its own copy until the
// process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_BYTES = getrs_ws_bytes_c(4, GETRS_NOALLOC_NMAX);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_DEVS = 16;
void *g_noalloc_ptr[NOALLOC_DEVS];
hipError_t g_noalloc_err[NOALLOC_DEVS];
std::once_flag g_noalloc_once[NOALLOC_DEVS];
}  // namespace

// Device address of this device's scratch array (looked up on the first
// call with the device current) and its size.
int noalloc_scratch(void **ptr, size_t *bytes)
{
    int dev = 0;
    BNC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_DEVS)
        return fail_arg(BNC_ERR_UNSUPPORTED, "getrs_noalloc: device index out of range");
    std::call_once(g_noalloc_once[dev], [dev] {
        void *p = nullptr;
        g_noalloc_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_noalloc_ptr[dev] = g_noalloc_err[dev] == hipSuccess ? p : nullptr;
    });
    if (g_noalloc_err[dev] != hipSuccess)
        return fail_hip(g_noalloc_err[dev], "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    *ptr = g_noalloc_ptr[dev];
    *bytes = NOALLOC_BYTES;
    return BNC_OK;
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
               const double *b, int64_t ldb, double *y, int64_t ldy, void *ws, hipStream_t s, int64_t *info,
               const int *skip)
{
    if (n == 0)
        return BNC_OK;
    hipLaunchKernelGGL((k_gather<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, perm, b, ldb, y, ldy,
                       skip);
    BNC_LAUNCH_CHECK();
    return trsv_pair<K>(n, LU, lda, ldp, rd, y, ldy, ws, s, info, skip);
}

// scr: getrs_workspace_bytes(K, n) bytes; info (nullable) gets 0, or -1 if
// a bounded wait of the substitutions gave up
template <int K>
int getrs_run(int64_t n, int64_t nrhs, const double *LU, int64_t lda, int64_t ldp, const int64_t *ipiv, double *B,
              int64_t ldb, int64_t ldpb, int64_t *info, void *scr, hipStream_t s)
{
    if (info) {
        hipLaunchKernelGGL(k_ts_zero, dim3(1), dim3(64), 0, s, info);
        BNC_LAUNCH_CHECK();
    }
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
        rc = getrs_perm<K>(n, LU, lda, ldp, perm, rd, bc, ldpb, y, n, ws, s, info, nullptr);
        if (rc)
            return rc;
        hipLaunchKernelGGL((k_copy_vec<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, y, n, bc, ldpb);
        BNC_LAUNCH_CHECK();
    }
    return BNC_OK;
}

#define INST(K)                                                                                                     \
    template int getrs_perm<K>(int64_t, const double *, int64_t, int64_t, const int32_t *, const double *,          \
                               const double *, int64_t, double *, int64_t, void *, hipStream_t, int64_t *,          \
                               const int *);                                                                        \
    template int diag_recip_run<K>(int64_t, const double *, int64_t, int64_t, double *, hipStream_t);               \
    template int getrs_run<K>(int64_t, int64_t, const double *, int64_t, int64_t, const int64_t *, double *,        \
                              int64_t, int64_t, int64_t *, void *, hipStream_t);
INST(1)
INST(2)
INST(3)
INST(4)
#undef INST

}  // namespace bnc

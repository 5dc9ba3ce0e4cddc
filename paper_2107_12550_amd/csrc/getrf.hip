// Blocked right-looking LU with partial pivoting in K-word arithmetic
// (Kouya 2021, Sec. 2: LU decomposition with partial pivoting in DD/TD/QD).
//
// Per panel of nb columns starting at column j0:
//   1. k_panel: one cooperative launch factors rows j0..n-1 of the panel.
//      Each workgroup keeps R <= 64 panel rows in LDS.  Per column: every
//      workgroup publishes its best candidate row, one grid barrier, every
//      workgroup picks the same global pivot, swaps rows in LDS, scales the
//      column by the pivot reciprocal and updates its rows; the next
//      column is updated and published first so that the barrier overlaps
//      the rest of the update.  Workgroup 0 then turns the nb swaps into
//      (dst, src) row pairs.
//   2. k_laswp_trsm: the same row pairs applied to every column outside the
//      panel; right of the panel it also solves U12 = L11^-1 A12 (one wave
//      per column, lanes = panel rows, one broadcast per pivot row).
//   3. k_update: A22 <- A22 - L21 U12, LDS tiles, one K-word multiply-subtract
//      per (i, j, k) in increasing k.
// Every matrix entry sees exactly the operations of the unblocked algorithm
// in the same order (row moves commute with the updates, each entry is
// updated in increasing k), so the factors equal the unblocked ones bit for
// bit.
#include "common.hpp"
#include "mw.hpp"

namespace bnc {

constexpr int PANEL_THREADS = 256;
constexpr int UPD_THREADS = 256;

// ---------------------------------------------------------------------------
// panel
// ---------------------------------------------------------------------------

// candidate (key, row) reduction: keep b when its key is larger, or equal
// with a smaller row; rows < 0 mark "no candidate".
template <int K>
__device__ __forceinline__ bool cand_better(const double (&kb)[K], int64_t rb, const double (&ka)[K], int64_t ra)
{
    if (rb < 0)
        return false;
    if (ra < 0)
        return true;
    if (key_gt<K>(kb, ka))
        return true;
    if (key_gt<K>(ka, kb))
        return false;
    return rb < ra;
}

// Lane-wise argmax across one wave (xor butterfly); every lane ends with
// the same (key, row): the largest key, ties to the smallest row.
template <int K>
__device__ __forceinline__ void wave_argmax(double (&key)[K], int &row)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double ok[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            ok[w] = __shfl_xor(key[w], off, 64);
        const int orow = __shfl_xor(row, off, 64);
        if (cand_better<K>(ok, orow, key, row)) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                key[w] = ok[w];
            row = orow;
        }
    }
}

// Cross-workgroup exchange inside the panel.  Every word another workgroup
// reads (candidate rows, their row indices, the row at the pivot position,
// the arrival counter) is written and read with device-scope relaxed
// atomics, which the hardware keeps coherent across the XCDs' L2 caches on
// their own (write-through stores, loads that miss the non-coherent caches).
// That makes a full device fence, which would write back and invalidate the
// whole L2 while the concurrent trailing update keeps it full of dirty
// lines, unnecessary: a workgroup waits for its own stores to complete
// before it bumps the counter, and readers load the data only after they
// have seen the counter reach its target.
__device__ __forceinline__ void sh_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sh_store(int64_t *p, int64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double sh_load(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t sh_load(const int64_t *p)
{
    return __hip_atomic_load(const_cast<int64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier on a monotonic counter, split into arrive and wait so that
// work can overlap the wait.  The spin is bounded: on timeout the workgroup
// records the failure and every later wait returns at once, so the grid
// always drains.
constexpr unsigned SPIN_LIMIT = 1u << 21;

__device__ __forceinline__ void bar_arrive_wave(unsigned *bar)
{
    // called by one whole wave after its sh_store()s: wait until they have
    // completed, then count this workgroup in
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    if ((threadIdx.x & 63) == 0)
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void bar_wait(unsigned *bar, unsigned target, int *abort_flag)
{
    if (threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The same wait for one wave only (the other waves keep working).
__device__ __forceinline__ void bar_wait_wave(unsigned *bar, unsigned target, int *abort_flag)
{
    if ((threadIdx.x & 63) == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// LDS tile layout: word w, panel column c, local row r at ((w*jb + c)*R + r);
// R <= 64, so one wave holds one row per lane.
//
// Column kk of the panel (global k = j0 + kk), per workgroup:
//   wait for every workgroup's candidate for column kk
//   pick the pivot (largest key, smallest row); rebuild the pivot row and
//   the displaced row k from their published copies, which were taken after
//   column kk was updated but before columns > kk were: finish those columns
//   with the previous pivot row, exactly as their owner does
//   swap, record ipiv, reciprocal of the pivot, scale column kk
//   wave 0: update column kk+1, find the local candidate for column kk+1,
//   copy it (and row k+1 if owned) to LDS; then, while waves 1.. update
//   columns kk+2.., publish the copies and arrive, wait for the others and
//   do the next column's pivot choice and row rebuild: the update of the
//   panel's remaining columns leaves the critical path.
template <int K>
__global__ void __launch_bounds__(PANEL_THREADS)
    k_panel(double *__restrict__ A, int64_t lda, int64_t ldp, int64_t n, int64_t j0, int jb, int R,
            int64_t *__restrict__ ipiv, int64_t *__restrict__ info, double *__restrict__ cand,
            int64_t *__restrict__ cidx, double *__restrict__ rowk, int64_t *__restrict__ pairs,
            unsigned *__restrict__ bar, int *__restrict__ abort_flag)
{
    extern __shared__ double smem[];
    double *tile = smem;                          // K*jb*R
    double *prow = tile + (size_t)K * jb * R;     // [2][K*jb] pivot rows of this and the previous column
    double *orow = prow + 2 * (size_t)K * jb;     // [K*jb]    displaced row k
    __shared__ int s_p;
    __shared__ double s_rcp[K];
    __shared__ int s_piv[PANEL_NB_MAX];

    const int P = gridDim.x;
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t gr0 = j0 + (int64_t)g * R;
    const int nr = (int)((n - gr0) < R ? (n - gr0) : R);

    for (int e = tid; e < jb * R; e += PANEL_THREADS) {
        const int r = e % R, c = e / R;
#pragma unroll
        for (int w = 0; w < K; ++w)
            tile[(w * jb + c) * R + r] = r < nr ? A[w * ldp + (j0 + c) * lda + gr0 + r] : 0.0;
    }
    __syncthreads();

    double *pubc = orow + (size_t)K * jb;  // [K*jb] staged copy of this workgroup's candidate row
    double *pubk = pubc + (size_t)K * jb;  // [K*jb] staged copy of the row at the next pivot position

    // stage (wave 0): this workgroup's candidate for column cc (rows >=
    // j0+cc) and the row at position j0+cc if owned, copied from the tile;
    // returns the candidate row (-1: none), wave-uniform
    auto stage = [&](int cc, bool &own) -> int {
        const int64_t kc = j0 + cc;
        double key[K];
        int row = -1;
        if (lane < nr && gr0 + lane >= kc) {
            row = (int)(gr0 + lane);
#pragma unroll
            for (int w = 0; w < K; ++w)
                key[w] = tile[(w * jb + cc) * R + lane];
        } else {
#pragma unroll
            for (int w = 0; w < K; ++w)
                key[w] = 0.0;
        }
        wave_argmax<K>(key, row);
        if (row >= 0) {
            const int lr = (int)(row - gr0);
            for (int e = lane; e < K * jb; e += 64) {
                const int w = e / jb, c = e % jb;
                pubc[e] = tile[(w * jb + c) * R + lr];
            }
        }
        own = kc >= gr0 && kc < gr0 + nr;
        if (own) {
            const int lr = (int)(kc - gr0);
            for (int e = lane; e < K * jb; e += 64) {
                const int w = e / jb, c = e % jb;
                pubk[e] = tile[(w * jb + c) * R + lr];
            }
        }
        return row;
    };
    // emit (wave 0): publish the staged copies for column cc and arrive
    auto emit = [&](int cc, int row, bool own) {
        const int b = cc & 1;
        double *cb = cand + ((size_t)(b * P + g) * K) * jb;
        if (row >= 0)
            for (int e = lane; e < K * jb; e += 64)
                sh_store(cb + e, pubc[e]);
        if (lane == 0)
            sh_store(cidx + b * P + g, (int64_t)row);
        if (own) {
            double *rb = rowk + (size_t)b * K * jb;
            for (int e = lane; e < K * jb; e += 64)
                sh_store(rb + e, pubk[e]);
        }
        bar_arrive_wave(bar);
    };

    if (wave == 0) {
        bool own0;
        const int row0 = stage(0, own0);
        emit(0, row0, own0);
    }

    bool nz_prev = false;
    for (int kk = 0; kk < jb; ++kk) {
        const int64_t k = j0 + kk;
        const int b = kk & 1;
        double *pcur = prow + (size_t)b * K * jb;
        const double *pprev = prow + (size_t)(b ^ 1) * K * jb;
        if (wave == 0) {
            bar_wait_wave(bar, (unsigned)(kk + 1) * (unsigned)P, abort_flag);
            // ---- global pivot
            double key[K];
            int row = -1;
#pragma unroll
            for (int w = 0; w < K; ++w)
                key[w] = 0.0;
            for (int t = lane; t < P; t += 64) {
                // index and key in one round trip (the key of a workgroup
                // without a candidate is ignored)
                const double *cc = cand + ((size_t)(b * P + t) * K) * jb;
                double kv[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    kv[w] = sh_load(cc + w * jb + kk);
                const int rr = (int)sh_load(cidx + b * P + t);
                if (rr < 0)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        kv[w] = 0.0;
                if (cand_better<K>(kv, rr, key, row)) {
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        key[w] = kv[w];
                    row = rr;
                }
            }
            wave_argmax<K>(key, row);
            const int64_t p = row;
            const int gw = (int)((p - j0) / R);
            // the winner's key is the pivot (column kk of a published
            // candidate is final): its reciprocal, while the row loads
            if (lane == 0 && !is_zero<K>(key)) {
                double rcp[K];
                recip<K>(key, rcp);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    s_rcp[w] = rcp[w];
            }
            // ---- rebuild the pivot row (and the displaced row k for p's
            //      owner) from their published copies; lane = column
            const double *cc = cand + ((size_t)(b * P + gw) * K) * jb;
            const double *rb = rowk + (size_t)b * K * jb;
            const bool need_o = p != k && p >= gr0 && p < gr0 + nr;
            const int c = lane;
            if (c < jb) {
                double v[K], o[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    v[w] = sh_load(cc + w * jb + c);
                if (nz_prev && c > kk) {
                    double l[K], u[K];
#pragma unroll
                    for (int w = 0; w < K; ++w) {
                        l[w] = sh_load(cc + w * jb + kk - 1);
                        u[w] = pprev[w * jb + c];
                    }
                    fms<K>(v, l, u, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        v[w] = o[w];
                }
#pragma unroll
                for (int w = 0; w < K; ++w)
                    pcur[w * jb + c] = v[w];
                if (need_o) {
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        v[w] = sh_load(rb + w * jb + c);
                    if (nz_prev && c > kk) {
                        double l[K], u[K];
#pragma unroll
                        for (int w = 0; w < K; ++w) {
                            l[w] = sh_load(rb + w * jb + kk - 1);
                            u[w] = pprev[w * jb + c];
                        }
                        fms<K>(v, l, u, o);
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            v[w] = o[w];
                    }
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        orow[w * jb + c] = v[w];
                }
            }
            if (lane == 0)
                s_p = (int)p;
        } else if (nz_prev) {
            // ---- waves 1..: the previous column's update of columns
            //      kk+1.. (rows below the previous pivot)
            const int kp = kk - 1;
            const int64_t kprev = j0 + kp;
            const int ncol = jb - kp - 2;
            for (int e = tid - 64; e < nr * ncol; e += PANEL_THREADS - 64) {
                const int r = e % nr, c = kp + 2 + e / nr;
                if (gr0 + r > kprev) {
                    double a[K], l[K], u[K], o[K];
#pragma unroll
                    for (int w = 0; w < K; ++w) {
                        a[w] = tile[(w * jb + c) * R + r];
                        l[w] = tile[(w * jb + kp) * R + r];
                        u[w] = pprev[w * jb + c];
                    }
                    fms<K>(a, l, u, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        tile[(w * jb + c) * R + r] = o[w];
                }
            }
        }
        __syncthreads();
        const int64_t p = s_p;
        // ---- row interchange k <-> p inside the tiles
        if (k >= gr0 && k < gr0 + nr) {
            const int lr = (int)(k - gr0);
            for (int e = tid; e < K * jb; e += PANEL_THREADS) {
                const int w = e / jb, c = e % jb;
                tile[(w * jb + c) * R + lr] = pcur[w * jb + c];
            }
        }
        if (p != k && p >= gr0 && p < gr0 + nr) {
            const int lr = (int)(p - gr0);
            for (int e = tid; e < K * jb; e += PANEL_THREADS) {
                const int w = e / jb, c = e % jb;
                tile[(w * jb + c) * R + lr] = orow[w * jb + c];
            }
        }
        if (tid == 0) {
            s_piv[kk] = (int)p;
            if (g == 0)
                ipiv[k] = p;
        }
        double pv[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            pv[w] = pcur[w * jb + kk];
        const bool nz = !is_zero<K>(pv);
        if (!nz && g == 0 && tid == 0 && *info == 0)
            *info = k + 1;
        __syncthreads();
        // ---- multipliers l_ik = a_ik * (1/a_kk), rows > k (wave 0, lane = row)
        if (nz && wave == 0 && lane < nr && gr0 + lane > k) {
            double rcp[K], a[K], l[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                rcp[w] = s_rcp[w];
#pragma unroll
            for (int w = 0; w < K; ++w)
                a[w] = tile[(w * jb + kk) * R + lane];
            mul<K>(a, rcp, l);
#pragma unroll
            for (int w = 0; w < K; ++w)
                tile[(w * jb + kk) * R + lane] = l[w];
        }
        __syncthreads();
        // ---- wave 0: column kk+1 first, then the next candidate, staged
        int crow = -1;
        bool cown = false;
        if (wave == 0 && kk + 1 < jb) {
            if (nz && lane < nr && gr0 + lane > k) {
                double a[K], l[K], u[K], o[K];
#pragma unroll
                for (int w = 0; w < K; ++w) {
                    a[w] = tile[(w * jb + kk + 1) * R + lane];
                    l[w] = tile[(w * jb + kk) * R + lane];
                    u[w] = pcur[w * jb + kk + 1];
                }
                fms<K>(a, l, u, o);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    tile[(w * jb + kk + 1) * R + lane] = o[w];
            }
            crow = stage(kk + 1, cown);
        }
        // the staged copies are taken before columns kk+2.. change
        __syncthreads();
        if (wave == 0 && kk + 1 < jb)
            emit(kk + 1, crow, cown);
        nz_prev = nz;
    }
    __syncthreads();

    for (int e = tid; e < jb * R; e += PANEL_THREADS) {
        const int r = e % R, c = e / R;
        if (r < nr) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                A[w * ldp + (j0 + c) * lda + gr0 + r] = tile[(w * jb + c) * R + r];
        }
    }
    if (g == 0 && tid == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        *info = -1;

    // ---- net row permutation of the nb swaps, as (dst, src) pairs:
    //      after the swaps, row dst holds the original row src.
    //      Lane l tracks block position j0+l and one outside slot.
    if (g == 0 && wave == 0) {
        int64_t in_c = j0 + lane;
        int64_t out_pos = -1, out_c = -1;
        int nout = 0;
        for (int q = 0; q < jb; ++q) {
            const int64_t pq = s_piv[q];
            if (pq == j0 + q)
                continue;
            const int64_t ck = __shfl(in_c, q, 64);
            if (pq < j0 + jb) {
                const int64_t cp = __shfl(in_c, (int)(pq - j0), 64);
                if (lane == q)
                    in_c = cp;
                if (lane == (int)(pq - j0))
                    in_c = ck;
            } else {
                const unsigned long long m = __ballot(lane < nout && out_pos == pq);
                int slot;
                if (m) {
                    slot = __ffsll(m) - 1;
                } else {
                    slot = nout;
                    if (lane == slot) {
                        out_pos = pq;
                        out_c = pq;
                    }
                    ++nout;
                }
                const int64_t co = __shfl(out_c, slot, 64);
                if (lane == q)
                    in_c = co;
                if (lane == slot)
                    out_c = ck;
            }
        }
        // pairs layout: dst[2*nbmax], src[2*nbmax]; -1 = unused
        int64_t *dst = pairs, *src = pairs + 2 * PANEL_NB_MAX;
        const bool in_ok = lane < jb && in_c != j0 + lane;
        dst[lane] = in_ok ? j0 + lane : -1;
        src[lane] = in_ok ? in_c : -1;
        const bool out_ok = lane < nout && out_c != out_pos;
        dst[PANEL_NB_MAX + lane] = out_ok ? out_pos : -1;
        src[PANEL_NB_MAX + lane] = out_ok ? out_c : -1;
    }
}

// ---------------------------------------------------------------------------
// row interchanges outside the panel (+ U12 solve right of the panel)
// one workgroup of 64 threads per column
// ---------------------------------------------------------------------------
template <int K, bool TRSM>
__global__ void __launch_bounds__(64)
    k_laswp_trsm(double *__restrict__ A, int64_t lda, int64_t ldp, int64_t j0, int jb, int64_t col0,
                 const int64_t *__restrict__ pairs)
{
    __shared__ double stage[2 * PANEL_NB_MAX][K];
    __shared__ double ub[K];
    const int64_t c = col0 + blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t *dst = pairs, *src = pairs + 2 * PANEL_NB_MAX;
    double *colp = A + c * lda;
    for (int t = lane; t < 2 * PANEL_NB_MAX; t += 64) {
        const int64_t s = src[t];
        if (s >= 0) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                stage[t][w] = colp[w * ldp + s];
        }
    }
    __syncthreads();
    for (int t = lane; t < 2 * PANEL_NB_MAX; t += 64) {
        const int64_t d = dst[t];
        if (d >= 0) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                colp[w * ldp + d] = stage[t][w];
        }
    }
    if (!TRSM)
        return;
    __syncthreads();
    __threadfence_block();
    // forward substitution with the unit lower L11 (rows/cols j0..j0+jb-1)
    double u[K];
    if (lane < jb) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            u[w] = colp[w * ldp + j0 + lane];
    }
    for (int kk = 0; kk < jb; ++kk) {
        if (lane == kk) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                ub[w] = u[w];
        }
        __syncthreads();
        if (lane > kk && lane < jb) {
            double l[K], uk[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w) {
                l[w] = A[w * ldp + (j0 + kk) * lda + j0 + lane];
                uk[w] = ub[w];
            }
            fms<K>(u, l, uk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                u[w] = o[w];
        }
        __syncthreads();
    }
    if (lane < jb) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            colp[w * ldp + j0 + lane] = u[w];
    }
}

// ---------------------------------------------------------------------------
// trailing update C <- C - L21 * U12
// C(i,j) = A[r0+i, c0+j], L21(i,k) = A[r0+i, j0+k], U12(k,j) = A[j0+k, c0+j]
// workgroup tile BM x BN, thread tile TM x TN (rows tx + (BM/TM) a,
// columns ty + (BN/TN) b), k staged through LDS in chunks of KB.
// ---------------------------------------------------------------------------
template <int K, int BM, int BN, int TM, int TN, int KB>
__global__ void __launch_bounds__(UPD_THREADS)
    k_update(double *__restrict__ A, int64_t lda, int64_t ldp, int64_t r0, int64_t c0, int64_t m, int64_t nc,
             int64_t j0, int kd)
{
    static_assert((BM / TM) * (BN / TN) == UPD_THREADS, "thread tile");
    __shared__ double Ls[K][KB][BM];
    __shared__ double Us[K][KB][BN];
    constexpr int TX = BM / TM;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int64_t bi = (int64_t)blockIdx.x * BM, bj = (int64_t)blockIdx.y * BN;

    double acc[TM][TN][K];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int64_t i = bi + tx + a * TX, j = bj + ty + b * (BN / TN);
#pragma unroll
            for (int w = 0; w < K; ++w)
                acc[a][b][w] = (i < m && j < nc) ? A[w * ldp + (c0 + j) * lda + r0 + i] : 0.0;
        }

    for (int k0 = 0; k0 < kd; k0 += KB) {
        const int kc = (kd - k0) < KB ? (kd - k0) : KB;
        for (int e = tid; e < KB * BM; e += UPD_THREADS) {
            const int i = e % BM, kk = e / BM;
            const bool ok = kk < kc && bi + i < m;
#pragma unroll
            for (int w = 0; w < K; ++w)
                Ls[w][kk][i] = ok ? A[w * ldp + (j0 + k0 + kk) * lda + r0 + bi + i] : 0.0;
        }
        for (int e = tid; e < KB * BN; e += UPD_THREADS) {
            const int kk = e % KB, j = e / KB;
            const bool ok = kk < kc && bj + j < nc;
#pragma unroll
            for (int w = 0; w < K; ++w)
                Us[w][kk][j] = ok ? A[w * ldp + (c0 + bj + j) * lda + j0 + k0 + kk] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < kc; ++kk) {
            double l[TM][K], u[TN][K];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int w = 0; w < K; ++w)
                    l[a][w] = Ls[w][kk][tx + a * TX];
#pragma unroll
            for (int b = 0; b < TN; ++b)
#pragma unroll
                for (int w = 0; w < K; ++w)
                    u[b][w] = Us[w][kk][ty + b * (BN / TN)];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    double o[K];
                    fms<K>(acc[a][b], l[a], u[b], o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        acc[a][b][w] = o[w];
                }
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int64_t i = bi + tx + a * TX, j = bj + ty + b * (BN / TN);
            if (i < m && j < nc) {
#pragma unroll
                for (int w = 0; w < K; ++w)
                    A[w * ldp + (c0 + j) * lda + r0 + i] = acc[a][b][w];
            }
        }
}

// thin variant for the look-ahead columns (n x 64 blocks): more workgroups
template <int K>
struct UpdCfgThin {
    static constexpr int BM = 64, BN = 16, TM = 4, TN = 1, KB = 16;
};

template <int K>
struct UpdCfg;
template <>
struct UpdCfg<1> {
    static constexpr int BM = 64, BN = 64, TM = 4, TN = 4, KB = 16;
};
template <>
struct UpdCfg<2> {
    static constexpr int BM = 64, BN = 64, TM = 4, TN = 4, KB = 16;
};
template <>
struct UpdCfg<3> {  // 32 x 64: 36.9 TFLOP/s on a 4032^2 x 64 update (64 x 64: 31.3)
    static constexpr int BM = 32, BN = 64, TM = 2, TN = 4, KB = 16;
};
template <>
struct UpdCfg<4> {
    static constexpr int BM = 64, BN = 32, TM = 4, TN = 2, KB = 16;
};

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
size_t getrf_scratch_bytes(int K)
{
    const size_t cand = 2ull * PANEL_WG_MAX * K * PANEL_NB_MAX * sizeof(double);
    const size_t cidx = 2ull * PANEL_WG_MAX * sizeof(int64_t);
    const size_t rowk = 2ull * K * PANEL_NB_MAX * sizeof(double);
    const size_t pairs = 8ull * PANEL_NB_MAX * sizeof(int64_t);  // two panels' pairs
    return cand + cidx + rowk + pairs + 4 * 256 + 256;
}

__global__ void k_zero_i64(int64_t *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *p = 0;
}

static size_t panel_lds_bytes(int K, int jb, int R)
{
    // tile, two pivot rows, the displaced row, two staged copies
    return ((size_t)K * jb * R + 5 * (size_t)K * jb) * sizeof(double);
}

// reset the grid-barrier counter and abort flag of one panel launch
__global__ void k_bar_reset(unsigned *bar, int *abort_flag)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *bar = 0;
        *abort_flag = 0;
    }
}

// Side stream and two events per device for the look-ahead: the next panel
// runs on the side stream while the rest of the trailing update runs on the
// caller's stream.  Default priority, created once.
namespace {
struct LookAhead {
    hipStream_t side = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
};
LookAhead g_la[16];
}  // namespace

static int lookahead_get(LookAhead *&la)
{
    int dev = 0;
    BNC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16)
        return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: device index out of range");
    la = &g_la[dev];
    if (!la->side) {
        BNC_HIP(hipStreamCreateWithFlags(&la->side, hipStreamNonBlocking));
        BNC_HIP(hipEventCreateWithFlags(&la->ready, hipEventDisableTiming));
        BNC_HIP(hipEventCreateWithFlags(&la->done, hipEventDisableTiming));
    }
    return BNC_OK;
}

template <int K>
int oz_split_rows_run(const double *A, int64_t lda, int64_t ldp, int64_t r0, int64_t m, int64_t j0, int kb, int s,
                      double *SL, int64_t ldsl, hipStream_t st);
template <int K>
int oz_split_cols_run(const double *A, int64_t lda, int64_t ldp, int64_t j0, int kb, int64_t c0, int64_t nc, int s,
                      double *SU, int64_t ldsu, hipStream_t st);
template <int K>
int oz_update_run(int s, bool thin, double *A, int64_t lda, int64_t ldp, int64_t r0, int64_t c0, int64_t m,
                  int64_t nc, int kb, const double *SL, int64_t ldsl, const double *SU, int64_t ldsu, hipStream_t st);

// oz = 0: K-word trailing updates (bit-identical to the unblocked LU).
// oz = S in 1..OZ_SMAX: split updates with S slices (ozaki.hip); oz_buf
// holds the slices, >= oz_slices_bytes(n) bytes.
template <int K>
int getrf_run(int64_t n, double *A, int64_t lda, int64_t ldp, int64_t *ipiv, int64_t *info, void *scr,
              hipStream_t s, int oz, double *oz_buf)
{
    if (n == 0)
        return BNC_OK;
    const int nb = PANEL_NB_MAX;
    char *base = (char *)scr;
    double *cand = (double *)base;
    base += 2ull * PANEL_WG_MAX * K * PANEL_NB_MAX * sizeof(double);
    int64_t *cidx = (int64_t *)base;
    base += 2ull * PANEL_WG_MAX * sizeof(int64_t);
    double *rowk = (double *)base;
    base += 2ull * K * PANEL_NB_MAX * sizeof(double);
    int64_t *pairs[2] = {(int64_t *)base, (int64_t *)base + 4 * PANEL_NB_MAX};
    base += 8ull * PANEL_NB_MAX * sizeof(int64_t);
    unsigned *bar = (unsigned *)base;
    int *abort_flag = (int *)(base + 64);

    int dev = 0;
    BNC_HIP(hipGetDevice(&dev));
    int ncu = 0, lds_max = 0;
    BNC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    BNC_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t lds_static = 512;
    LookAhead *la = nullptr;
    int rc = lookahead_get(la);
    if (rc)
        return rc;

    // one panel: rows pj0..n-1, columns pj0..pj0+pjb-1
    auto panel = [&](int64_t pj0, int pjb, int64_t *pr, hipStream_t st) -> int {
        const int64_t m = n - pj0;
        void *kfn = (void *)k_panel<K>;
        int R = 64;
        while (R > 8 && panel_lds_bytes(K, pjb, R) + lds_static > (size_t)lds_max)
            R /= 2;
        const size_t lds = panel_lds_bytes(K, pjb, R);
        if (lds + lds_static > (size_t)lds_max)
            return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: panel does not fit in LDS");
        if (hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            (void)hipGetLastError();
        int per_cu = 0;
        BNC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, PANEL_THREADS, lds));
        int64_t cap = (int64_t)per_cu * ncu;
        if (cap > PANEL_WG_MAX)
            cap = PANEL_WG_MAX;
        const int P = (int)ceil_div(m, R);
        if (P > cap)
            return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: panel needs more workgroups than can be co-resident");
        hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, st, bar, abort_flag);
        BNC_LAUNCH_CHECK();
        // All P workgroups fit on the device at once (checked above); the
        // grid barrier inside the kernel has a bounded spin, so a workgroup
        // that starts late (the other stream's kernels still hold CUs) only
        // delays the panel.
        hipLaunchKernelGGL((k_panel<K>), dim3(P), dim3(PANEL_THREADS), lds, st, A, lda, ldp, n, pj0, pjb, R, ipiv,
                           info, cand, cidx, rowk, pr, bar, abort_flag);
        BNC_LAUNCH_CHECK();
        return BNC_OK;
    };
    auto swaps = [&](int64_t j0, int jb, int64_t c0, int64_t nc, const int64_t *pr, bool trsm) -> int {
        if (nc <= 0)
            return BNC_OK;
        if (trsm)
            hipLaunchKernelGGL((k_laswp_trsm<K, true>), dim3((unsigned)nc), dim3(64), 0, s, A, lda, ldp, j0, jb, c0,
                               pr);
        else
            hipLaunchKernelGGL((k_laswp_trsm<K, false>), dim3((unsigned)nc), dim3(64), 0, s, A, lda, ldp, j0, jb,
                               c0, pr);
        BNC_LAUNCH_CHECK();
        return BNC_OK;
    };
    // A[r0.., c0..c0+nc) -= L21 (columns j0..j0+jb) * U12
    // split form: SL holds the sliced rows cn..n-1 of the current panel,
    // SU the sliced columns cn..n-1 of its U12 (both with leading dimension n)
    double *SL = oz_buf, *SU = oz_buf ? oz_buf + (size_t)OZ_SMAX * PANEL_NB_MAX * n : nullptr;
    auto update = [&](int64_t r0, int64_t c0, int64_t m, int64_t nc, int64_t j0, int jb, bool thin) -> int {
        if (m <= 0 || nc <= 0)
            return BNC_OK;
        if (oz) {
            int rc2 = oz_split_cols_run<K>(A, lda, ldp, j0, jb, c0, nc, oz, SU + (c0 - r0), n, s);
            if (rc2)
                return rc2;
            const int ev = UpdateTimer::begin(s);
            rc2 = oz_update_run<K>(oz, thin, A, lda, ldp, r0, c0, m, nc, jb, SL, n, SU + (c0 - r0), n, s);
            UpdateTimer::end(ev, s, 2.0 * (oz * (oz + 1) / 2) * (double)m * (double)nc * (double)jb);
            return rc2;
        }
        const int ev = UpdateTimer::begin(s);
        if (thin) {
            using C = UpdCfgThin<K>;
            dim3 grid((unsigned)ceil_div(m, C::BM), (unsigned)ceil_div(nc, C::BN));
            hipLaunchKernelGGL((k_update<K, C::BM, C::BN, C::TM, C::TN, C::KB>), grid, dim3(UPD_THREADS), 0, s, A,
                               lda, ldp, r0, c0, m, nc, j0, jb);
        } else {
            using C = UpdCfg<K>;
            dim3 grid((unsigned)ceil_div(m, C::BM), (unsigned)ceil_div(nc, C::BN));
            hipLaunchKernelGGL((k_update<K, C::BM, C::BN, C::TM, C::TN, C::KB>), grid, dim3(UPD_THREADS), 0, s, A,
                               lda, ldp, r0, c0, m, nc, j0, jb);
        }
        BNC_LAUNCH_CHECK();
        UpdateTimer::end(ev, s, (double)m * (double)nc * (double)jb * fms_flops(K));
        return BNC_OK;
    };

    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, info);
    BNC_LAUNCH_CHECK();
    if ((rc = panel(0, (int)(n < nb ? n : nb), pairs[0], s)))
        return rc;
    int J = 0;
    for (int64_t j0 = 0; j0 < n; j0 += nb, ++J) {
        const int jb = (int)((n - j0) < nb ? (n - j0) : nb);
        const int64_t *pr = pairs[J & 1];
        if ((rc = swaps(j0, jb, 0, j0, pr, false)))
            return rc;
        const int64_t cn = j0 + jb;
        if (cn >= n)
            break;
        const int nbn = (int)((n - cn) < nb ? (n - cn) : nb);
        if (oz && (rc = oz_split_rows_run<K>(A, lda, ldp, cn, n - cn, j0, jb, oz, SL, n, s)))
            return rc;
        // look-ahead: the next panel's columns first
        if ((rc = swaps(j0, jb, cn, nbn, pr, true)) || (rc = update(cn, cn, n - cn, nbn, j0, jb, true)))
            return rc;
        BNC_HIP(hipEventRecord(la->ready, s));
        BNC_HIP(hipStreamWaitEvent(la->side, la->ready, 0));
        if ((rc = panel(cn, nbn, pairs[(J + 1) & 1], la->side)))
            return rc;
        BNC_HIP(hipEventRecord(la->done, la->side));
        // the rest of the trailing matrix, concurrently with that panel
        const int64_t cr = cn + nbn;
        if ((rc = swaps(j0, jb, cr, n - cr, pr, true)) || (rc = update(cn, cr, n - cn, n - cr, j0, jb, false)))
            return rc;
        BNC_HIP(hipStreamWaitEvent(s, la->done, 0));
    }
    return BNC_OK;
}

template int getrf_run<1>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);
template int getrf_run<2>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);
template int getrf_run<3>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);
template int getrf_run<4>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);

}  // namespace bnc

// Blocked right-looking LU with partial pivoting in K-word arithmetic
// (Kouya 2021, Sec. 2: LU decomposition with partial pivoting in DD/TD/QD).
//
// Per panel of nb columns starting at column j0:
//   1. k_panel: one cooperative launch factors rows j0..n-1 of the panel.
//      Each workgroup keeps R <= 64 panel rows in LDS.  Per column: every
//      workgroup publishes its best candidate row into an exchange slot and
//      reads everyone else's (polling the words themselves), every
//      workgroup picks the same global pivot, swaps rows in LDS, scales the
//      column by the pivot reciprocal and updates its rows; the next
//      column is updated and published first, so the exchange overlaps the
//      rest of the update.  Workgroup 0 then turns the nb swaps into
//      (dst, src) row pairs.  In the split form the panel also cuts its
//      finished L21 rows into slices.
//   2. k_laswp_trsm: the same row pairs applied to every column outside the
//      panel; right of the panel it also solves U12 = L11^-1 A12 (one wave
//      per column, lanes = panel rows, one broadcast per pivot row) and, for
//      the look-ahead columns of the split form, cuts them into slices.
//   3. k_update: A22 <- A22 - L21 U12, LDS tiles, one K-word multiply-subtract
//      per (i, j, k) in increasing k (or the split form, ozaki.hip).
// The next panel's columns are updated first and that panel runs on a side
// stream while the rest of the trailing update proceeds (look-ahead).
// Every matrix entry sees exactly the operations of the unblocked algorithm
// in the same order (row moves commute with the updates, each entry is
// updated in increasing k), so the factors equal the unblocked ones bit for
// bit.
#include <cstdlib>
#include <mutex>

#include "common.hpp"
#include "mw.hpp"
#include "ozsplit.hpp"

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

// Cross-workgroup exchange inside the panel.  Each panel launch has an
// exchange buffer (two, alternating between consecutive panels) holding,
// per column kk of the panel, the row index of every workgroup's pivot
// candidate (-1: none), a copy of every candidate row and a copy of the row
// at position j0 + kk.  Every word of it starts as XSENT, a signalling NaN
// that no arithmetic produces, and is written at most once per panel, so a
// reader polls the words it needs until none is XSENT: no counters, no
// fences, and a writer never waits for its own stores.  Words are written
// and read with device-scope relaxed atomics, which the hardware keeps
// coherent across the XCDs' L2 caches (write-through stores, loads that
// miss the non-coherent caches).  A matrix that holds the XSENT bit pattern
// itself can stall a poll; every poll is bounded and such a panel ends with
// info = -1.
constexpr int64_t XSENT = (int64_t)0xFFF40000DEADBEEFull;

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
__device__ __forceinline__ bool xsent(double v) { return __double_as_longlong(v) == (long long)XSENT; }

// Bounded polling: after SPIN_LIMIT retries (or once another workgroup has
// given up) the lane marks the panel failed and goes on with what it has,
// so the grid always drains.
constexpr unsigned SPIN_LIMIT = 1u << 21;

struct Poll {
    unsigned spins = 0;
    bool dead = false;
    // one more retry allowed?
    __device__ __forceinline__ bool again(int *abort_flag)
    {
        if (dead)
            return false;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT ||
            ((spins & 1023u) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            dead = true;
            return false;
        }
        return true;
    }
};

// K words at p[w * stride], polled until none is XSENT
template <int K>
__device__ __forceinline__ void xpoll(const double *p, int stride, double (&v)[K], Poll &pl, int *abort_flag)
{
    bool any;
    do {
        // every word is written once: reloading one already seen is harmless
        any = false;
#pragma unroll
        for (int w = 0; w < K; ++w) {
            v[w] = sh_load(p + w * stride);
            any |= xsent(v[w]);
        }
    } while (any && pl.again(abort_flag));
}

// Exchange buffer layout (in doubles), for up to ps workgroups: idx
// [ps][64] (int64), rows [ps][64][K * 64] (word w, column c at w * jb + c),
// own [64][K * 64].
static size_t xbuf_words(int K, int ps)
{
    return (size_t)ps * PANEL_NB_MAX * (1 + K * PANEL_NB_MAX) + (size_t)PANEL_NB_MAX * K * PANEL_NB_MAX;
}

// workgroup slots of a factorisation of order n: panels have at least 8
// rows per workgroup
static int panel_slots(int64_t n)
{
    const int64_t s = (n + 7) / 8;
    return (int)(s < 1 ? 1 : (s > PANEL_WG_MAX ? PANEL_WG_MAX : s));
}

// Broadcast of lane l's double (l wave-uniform) through scalar registers.
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// wave_argmax with a fast path: the key order compares |leading word|
// first, so when exactly one lane holds the largest |leading word| it wins
// outright; ties on it (or no candidate at all) take the full reduction.
// DPP lane move of a double (both halves with the same control)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// fmax over the wave, in every lane: within each row of 16 lanes by DPP
// (quad swaps, then half-row and row mirrors), across the four rows through
// scalar registers
__device__ __forceinline__ double wave_fmax(double m)
{
    m = fmax(m, dpp_d<0xB1>(m));   // quad_perm [1,0,3,2]
    m = fmax(m, dpp_d<0x4E>(m));   // quad_perm [2,3,0,1]
    m = fmax(m, dpp_d<0x141>(m));  // row_half_mirror
    m = fmax(m, dpp_d<0x140>(m));  // row_mirror
    return fmax(fmax(readlane_d(m, 0), readlane_d(m, 16)), fmax(readlane_d(m, 32), readlane_d(m, 48)));
}

template <int K>
__device__ __forceinline__ void wave_argmax_fast(double (&key)[K], int &row)
{
    const double m = row >= 0 ? fabs(key[0]) : -1.0;
    const double mx = wave_fmax(m);
    const unsigned long long at = __ballot(row >= 0 && m == mx);
    if (__popcll(at) == 1) {
        const int src = __builtin_ctzll(at);
#pragma unroll
        for (int w = 0; w < K; ++w)
            key[w] = readlane_d(key[w], src);
        row = __builtin_amdgcn_readlane(row, src);
        return;
    }
    wave_argmax<K>(key, row);
}

// LDS tile layout: word w, panel column c, local row r at
// ((w*jb + c)*(R+1) + r); R <= 64, so one wave holds one row per lane, and
// the odd stride R+1 keeps row-wise access (lane = column) free of bank
// conflicts.
//
// Column kk of the panel (global k = j0 + kk), per workgroup:
//   wait for every workgroup's candidate for column kk
//   pick the pivot (largest key, smallest row); rebuild the pivot row and
//   the displaced row k from their published copies, which were taken after
//   column kk was updated but before columns > kk were: finish those columns
//   with the previous pivot row, exactly as their owner does
//   swap, record ipiv, reciprocal of the pivot, scale column kk
//   wave 0: update column kk+1, find the local candidate for column kk+1
//   and publish it (and row k+1 if owned); then, while waves 1.. update
//   columns kk+2.., wait for the others and do the next column's pivot
//   choice and row rebuild: the update of the panel's remaining columns
//   leaves the critical path.
template <int K>
__global__ void __launch_bounds__(PANEL_THREADS)
    k_panel(double *__restrict__ A, int64_t lda, int64_t ldp, int64_t n, int64_t j0, int jb, int R,
            int64_t *__restrict__ ipiv, int64_t *__restrict__ info, double *__restrict__ xcur,
            double *__restrict__ xnext, int ps, int64_t *__restrict__ pairs, int *__restrict__ abort_flag, int ozs,
            double *__restrict__ SL, int64_t ldsl)
{
    constexpr int KJ = K * PANEL_NB_MAX;
    constexpr int NW = PANEL_THREADS / 64;
    int64_t *xidx = (int64_t *)xcur;
    double *xrow = xcur + (size_t)ps * PANEL_NB_MAX;
    double *xown = xrow + (size_t)ps * PANEL_NB_MAX * KJ;
    const int RS = R + 1;
    extern __shared__ double smem[];
    double *tile = smem;                        // K*jb*RS
    double *prow = tile + (size_t)K * jb * RS;  // [2][K*jb] pivot rows of this and the previous column
    double *orow = prow + 2 * (size_t)K * jb;   // [K*jb]    displaced row k
    __shared__ int s_p;
    __shared__ double s_rcp[K];
    __shared__ int s_piv[PANEL_NB_MAX];
    auto T = [&](int w, int c, int r) -> double & { return tile[(w * jb + c) * RS + r]; };

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
            T(w, c, r) = r < nr ? A[w * ldp + (j0 + c) * lda + gr0 + r] : 0.0;
    }
    __syncthreads();

    // wave 0: this workgroup's candidate for column cc (rows >= j0+cc) and
    // the row at position j0+cc if owned, published straight from the tile
    // (lane = column); returns nothing, the copies are what the others need
    auto publish = [&](int cc) {
        const int64_t kc = j0 + cc;
        double key[K];
        int row = -1;
        const bool cand = lane < nr && gr0 + lane >= kc;
#pragma unroll
        for (int w = 0; w < K; ++w)
            key[w] = 0.0;
        if (cand) {
            row = (int)(gr0 + lane);
#pragma unroll
            for (int w = 0; w < K; ++w)
                key[w] = T(w, cc, lane);
        }
        wave_argmax_fast<K>(key, row);
        if (row >= 0 && lane < jb) {
            const int lr = (int)(row - gr0);
            double *rb = xrow + ((size_t)g * PANEL_NB_MAX + cc) * KJ;
#pragma unroll
            for (int w = 0; w < K; ++w)
                sh_store(rb + w * jb + lane, T(w, lane, lr));
        }
        if (kc >= gr0 && kc < gr0 + nr && lane < jb) {
            const int lr = (int)(kc - gr0);
            double *ob = xown + (size_t)cc * KJ;
#pragma unroll
            for (int w = 0; w < K; ++w)
                sh_store(ob + w * jb + lane, T(w, lane, lr));
        }
        // the index last: a reader that sees it still polls the row words
        if (lane == 0)
            sh_store(xidx + g * PANEL_NB_MAX + cc, (int64_t)row);
    };

    if (wave == 0)
        publish(0);

    bool nz_prev = false;
    Poll pl;  // wave 0's polls; none once an earlier panel has failed
    pl.dead = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    for (int kk = 0; kk < jb; ++kk) {
        const int64_t k = j0 + kk;
        const int b = kk & 1;
        double *pcur = prow + (size_t)b * K * jb;
        const double *pprev = prow + (size_t)(b ^ 1) * K * jb;
        if (wave == 0) {
            // ---- global pivot: every workgroup's candidate index and key
            double key[K];
            int row = -1;
#pragma unroll
            for (int w = 0; w < K; ++w)
                key[w] = 0.0;
            for (int t = lane; t < P; t += 64) {
                const int64_t *ip = xidx + t * PANEL_NB_MAX + kk;
                const double *kp = xrow + ((size_t)t * PANEL_NB_MAX + kk) * KJ + kk;
                int64_t rr;
                double kv[K];
                bool wait;
                do {
                    rr = sh_load(ip);
                    bool ks = false;
#pragma unroll
                    for (int w = 0; w < K; ++w) {
                        kv[w] = sh_load(kp + w * jb);
                        ks |= xsent(kv[w]);
                    }
                    wait = rr == XSENT || (rr >= 0 && ks);
                } while (wait && pl.again(abort_flag));
                const int ri = (rr >= k && rr < n) ? (int)rr : -1;
                if (cand_better<K>(kv, ri, key, row)) {
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        key[w] = kv[w];
                    row = ri;
                }
            }
            wave_argmax_fast<K>(key, row);
            // a failed poll can leave no valid row: keep indexing in range
            const int64_t p = row >= 0 ? row : k;
            const int gw = (int)((p - j0) / R);
            // ---- rebuild the pivot row (and the displaced row k for p's
            //      owner) from their published copies, lane = column: every
            //      load is issued first, the pivot's reciprocal (its key:
            //      column kk of a published candidate is final) is formed
            //      while they are in flight
            const double *cc = xrow + ((size_t)gw * PANEL_NB_MAX + kk) * KJ;
            const double *rb = xown + (size_t)kk * KJ;
            const bool need_o = p != k && p >= gr0 && p < gr0 + nr;
            const int c = lane;
            const bool live = c < jb;
            const bool fin = nz_prev && c > kk && c < jb;
            double v[K], l[K], vo[K], lo[K];
#pragma unroll
            for (int w = 0; w < K; ++w) {
                v[w] = live ? sh_load(cc + w * jb + c) : 0.0;
                l[w] = fin ? sh_load(cc + w * jb + kk - 1) : 0.0;
                vo[w] = (need_o && live) ? sh_load(rb + w * jb + c) : 0.0;
                lo[w] = (need_o && fin) ? sh_load(rb + w * jb + kk - 1) : 0.0;
            }
            if (lane == 0 && !is_zero<K>(key)) {
                double rcp[K];
                recip<K>(key, rcp);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    s_rcp[w] = rcp[w];
            }
            for (;;) {
                bool any = false;
#pragma unroll
                for (int w = 0; w < K; ++w)
                    any |= xsent(v[w]) | xsent(l[w]) | xsent(vo[w]) | xsent(lo[w]);
                if (!any || !pl.again(abort_flag))
                    break;
#pragma unroll
                for (int w = 0; w < K; ++w) {  // written once: reloading is harmless
                    v[w] = live ? sh_load(cc + w * jb + c) : 0.0;
                    l[w] = fin ? sh_load(cc + w * jb + kk - 1) : 0.0;
                    vo[w] = (need_o && live) ? sh_load(rb + w * jb + c) : 0.0;
                    lo[w] = (need_o && fin) ? sh_load(rb + w * jb + kk - 1) : 0.0;
                }
            }
            if (fin) {
                double u[K], o[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    u[w] = pprev[w * jb + c];
                fms<K>(v, l, u, o);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    v[w] = o[w];
                if (need_o) {
                    fms<K>(vo, lo, u, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        vo[w] = o[w];
                }
            }
            if (live) {
#pragma unroll
                for (int w = 0; w < K; ++w) {
                    pcur[w * jb + c] = v[w];
                    if (need_o)
                        orow[w * jb + c] = vo[w];
                }
            }
            if (lane == 0)
                s_p = (int)p;
        } else if (nz_prev) {
            // ---- waves 1..: the previous column's update of columns
            //      kk+1.. (rows below the previous pivot), lane = row
            const int kp = kk - 1;
            const int r = lane;
            if (r < nr && gr0 + r > j0 + kp) {
                double l[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    l[w] = T(w, kp, r);
#pragma unroll 2
                for (int c = kp + 1 + wave; c < jb; c += NW - 1) {
                    double a[K], u[K], o[K];
#pragma unroll
                    for (int w = 0; w < K; ++w) {
                        a[w] = T(w, c, r);
                        u[w] = pprev[w * jb + c];
                    }
                    fms<K>(a, l, u, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        T(w, c, r) = o[w];
                }
            }
        }
        __syncthreads();
        const int64_t p = s_p;
        // ---- row interchange k <-> p inside the tiles (wave w: word w)
        if (wave < K && lane < jb) {
            if (k >= gr0 && k < gr0 + nr)
                T(wave, lane, (int)(k - gr0)) = pcur[wave * jb + lane];
            if (p != k && p >= gr0 && p < gr0 + nr)
                T(wave, lane, (int)(p - gr0)) = orow[wave * jb + lane];
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
        if (wave == 0) {
            // ---- multipliers l_ik = a_ik * (1/a_kk), rows > k (lane = row)
            const bool mine = nz && lane < nr && gr0 + lane > k;
            if (mine) {
                double rcp[K], a[K], l[K];
#pragma unroll
                for (int w = 0; w < K; ++w) {
                    rcp[w] = s_rcp[w];
                    a[w] = T(w, kk, lane);
                }
                mul<K>(a, rcp, l);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    T(w, kk, lane) = l[w];
                // ---- column kk+1 first, then the next candidate is published
                if (kk + 1 < jb) {
                    double a1[K], u[K], o[K];
#pragma unroll
                    for (int w = 0; w < K; ++w) {
                        a1[w] = T(w, kk + 1, lane);
                        u[w] = pcur[w * jb + kk + 1];
                    }
                    fms<K>(a1, l, u, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        T(w, kk + 1, lane) = o[w];
                }
            }
            if (kk + 1 < jb)
                publish(kk + 1);
        }
        // waves 1.. may change columns kk+2.. only after the copies are out
        __syncthreads();
        nz_prev = nz;
    }

    for (int e = tid; e < jb * R; e += PANEL_THREADS) {
        const int r = e % R, c = e / R;
        if (r < nr) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                A[w * ldp + (j0 + c) * lda + gr0 + r] = T(w, c, r);
        }
    }
    // split form: slices of the finished rows below the panel block (L21),
    // SL[(q jb + c) ldsl + i] for row j0 + jb + i; PANEL_THREADS / R threads
    // per row, each a share of the columns, the row's scale from the
    // largest leading word over all shares
    if (ozs > 0) {
        __shared__ double s_mx[PANEL_THREADS];
        const int r = tid % R, qt = tid / R, nq = PANEL_THREADS / R;
        const int per = (jb + nq - 1) / nq;
        const int cb = qt * per, ce = (cb + per) < jb ? (cb + per) : jb;
        const int64_t row = gr0 + r;
        const bool mine = r < nr && row >= j0 + jb;
        double mx = 0.0;
        if (mine)
            for (int c = cb; c < ce; ++c)
                mx = fmax(mx, fabs(T(0, c, r)));
        s_mx[tid] = mx;  // tid = qt R + r
        __syncthreads();
        if (mine) {
            for (int t = 0; t < nq; ++t)
                mx = fmax(mx, s_mx[t * R + r]);
            const int E = oz_scale(mx);
            const int beta = oz_beta(K, ozs);
            if (mx != 0.0 && E < oz_emin(K, ozs))  // below the exact range: info -3 at the end
                __hip_atomic_store(abort_flag + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            double *out = SL + (row - j0 - jb);
            for (int c = cb; c < ce; ++c) {
                double v[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    v[w] = T(w, c, r);
                oz_cut_store<K>(v, E, ozs, beta, out + (int64_t)c * ldsl, (int64_t)jb * ldsl);
            }
        }
    }
    // the next panel's exchange buffer back to XSENT: this workgroup's
    // slots (the next panel has no more workgroups than this one) and every
    // P-th row copy at the pivot position
    {
        int64_t *nidx = (int64_t *)xnext;
        double *nrow = xnext + (size_t)ps * PANEL_NB_MAX;
        double *nown = nrow + (size_t)ps * PANEL_NB_MAX * KJ;
        const double sent = __longlong_as_double((long long)XSENT);
        if (tid < PANEL_NB_MAX)
            sh_store(nidx + g * PANEL_NB_MAX + tid, XSENT);
        double *rb = nrow + (size_t)g * PANEL_NB_MAX * KJ;
        for (int e = tid; e < PANEL_NB_MAX * KJ; e += PANEL_THREADS)
            sh_store(rb + e, sent);
        for (int c = g; c < PANEL_NB_MAX; c += P)
            for (int e = tid; e < KJ; e += PANEL_THREADS)
                sh_store(nown + (size_t)c * KJ + e, sent);
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
// one workgroup of one wave per column
// ---------------------------------------------------------------------------
// Lane l moves pairs l and PANEL_NB_MAX + l.  Every source is read before
// any destination is written: the stores use the loaded words, so they
// issue only after the wave's loads have returned.  Pairs l < PANEL_NB_MAX
// are the block rows (destination j0 + l); with the U12 solve, row j0 + l
// after the interchanges is lane l's own loaded word (or the untouched
// row), so the solve starts from registers and its result is the only
// store to the block rows.
template <int K, bool TRSM>
__global__ void __launch_bounds__(64)
    k_laswp_trsm(double *__restrict__ A, int64_t lda, int64_t ldp, int64_t j0, int jb, int64_t col0,
                 const int64_t *__restrict__ pairs, int ozs, double *__restrict__ SU, int64_t ldsu,
                 int *__restrict__ ozlow)
{
    const int64_t c = col0 + blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t *dst = pairs, *src = pairs + 2 * PANEL_NB_MAX;
    double *colp = A + c * lda;
    const int64_t s0 = src[lane], s1 = src[PANEL_NB_MAX + lane];
    const int64_t d0 = dst[lane], d1 = dst[PANEL_NB_MAX + lane];
    double v0[K], v1[K];
#pragma unroll
    for (int w = 0; w < K; ++w) {
        v0[w] = s0 >= 0 ? colp[w * ldp + s0] : 0.0;
        v1[w] = s1 >= 0 ? colp[w * ldp + s1] : 0.0;
    }
    // L11 columns are read PF steps ahead of their use (they do not
    // depend on the solve), so the chain only waits for the arithmetic
    constexpr int PF = 8;
    // (every prefetch is an unconditional load from an in-bounds address:
    // lanes past jb read row j0 + jb - 1 and steps past the end re-read the
    // last column, so the compiler can count the loads in flight)
    double lp[PF][K], u[K];
    const double *l11 = A + j0 * lda + j0 + (lane < jb ? lane : jb - 1);
    if (TRSM) {
        // the block row as it stands, loaded with the pairs' words (one
        // round trip); lane l's own pair replaces it when there is one
#pragma unroll
        for (int w = 0; w < K; ++w)
            u[w] = lane < jb ? colp[w * ldp + j0 + lane] : 0.0;
#pragma unroll
        for (int q = 0; q < PF; ++q)
#pragma unroll
            for (int w = 0; w < K; ++w)
                lp[q][w] = l11[w * ldp + (int64_t)(q < jb ? q : jb - 1) * lda];
#pragma unroll
        for (int w = 0; w < K; ++w)
            u[w] = s0 >= 0 ? v0[w] : u[w];
    }
    if (d1 >= 0)
#pragma unroll
        for (int w = 0; w < K; ++w)
            colp[w * ldp + d1] = v1[w];
    if (!TRSM) {
        if (d0 >= 0)
#pragma unroll
            for (int w = 0; w < K; ++w)
                colp[w * ldp + d0] = v0[w];
        return;
    }
    // forward substitution with the unit lower L11 (rows/cols j0..j0+jb-1):
    // lane kk's finished value is broadcast through scalar registers.  The
    // steps run in whole groups of PF (at most 64 steps); a step past jb
    // changes no lane.
    for (int k0 = 0; k0 < jb; k0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int kk = k0 + q;
            double uk[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                uk[w] = readlane_d(u[w], kk);
            if (lane > kk && lane < jb) {
                double o[K];
                fms<K>(u, lp[q], uk, o);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    u[w] = o[w];
            }
            const int kn = kk + PF < jb ? kk + PF : jb - 1;
#pragma unroll
            for (int w = 0; w < K; ++w)
                lp[q][w] = l11[w * ldp + (int64_t)kn * lda];
        }
    }
    if (lane < jb) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            colp[w * ldp + j0 + lane] = u[w];
    }
    // split form: the finished column's slices, SU[(q jb + k) ldsu + blockIdx.x]
    if (ozs > 0) {
        double mx = lane < jb ? fabs(u[0]) : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            mx = fmax(mx, __shfl_xor(mx, off, 64));
        if (lane == 0 && mx != 0.0 && oz_scale(mx) < oz_emin(K, ozs))
            __hip_atomic_store(ozlow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane < jb)
            oz_cut_store<K>(u, oz_scale(mx), ozs, oz_beta(K, ozs), SU + (int64_t)lane * ldsu + blockIdx.x,
                            (int64_t)jb * ldsu);
    }
}

// ---------------------------------------------------------------------------
// multiply-subtract C <- C - L U on K-plane views (pointer, column stride,
// plane stride): C m x nc, L m x kd, U kd x nc.  The trailing update of the
// LU passes views of its own matrix: C(i,j) = A[r0+i, c0+j],
// L21(i,k) = A[r0+i, j0+k], U12(k,j) = A[j0+k, c0+j]; the multi-word GEMM
// passes three matrices.  Each entry of C is updated in increasing k, one
// K-word multiply-subtract per k.
// workgroup tile BM x BN, thread tile TM x TN (rows tx + (BM/TM) a,
// columns ty + (BN/TN) b), k staged through LDS in chunks of KB.
// ---------------------------------------------------------------------------
struct MwView {
    const double *p;
    int64_t ld, ldp;
};

template <int K, int BM, int BN, int TM, int TN, int KB>
__global__ void __launch_bounds__(UPD_THREADS)
    k_update(double *__restrict__ Cp, int64_t ldc, int64_t ldpc, MwView Lv, MwView Uv, int64_t m, int64_t nc, int kd)
{
    const double *__restrict__ Lp = Lv.p;
    const double *__restrict__ Up = Uv.p;
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
                acc[a][b][w] = (i < m && j < nc) ? Cp[w * ldpc + j * ldc + i] : 0.0;
        }

    for (int k0 = 0; k0 < kd; k0 += KB) {
        const int kc = (kd - k0) < KB ? (kd - k0) : KB;
        for (int e = tid; e < KB * BM; e += UPD_THREADS) {
            const int i = e % BM, kk = e / BM;
            const bool ok = kk < kc && bi + i < m;
#pragma unroll
            for (int w = 0; w < K; ++w)
                Ls[w][kk][i] = ok ? Lp[w * Lv.ldp + (k0 + kk) * Lv.ld + bi + i] : 0.0;
        }
        for (int e = tid; e < KB * BN; e += UPD_THREADS) {
            const int kk = e % KB, j = e / KB;
            const bool ok = kk < kc && bj + j < nc;
#pragma unroll
            for (int w = 0; w < K; ++w)
                Us[w][kk][j] = ok ? Up[w * Uv.ldp + (bj + j) * Uv.ld + k0 + kk] : 0.0;
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
                    Cp[w * ldpc + j * ldc + i] = acc[a][b][w];
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
size_t getrf_scratch_bytes(int K, int64_t n)
{
    const size_t xb = 2 * xbuf_words(K, panel_slots(n)) * sizeof(double);  // two exchange buffers
    const size_t pairs = 8ull * PANEL_NB_MAX * sizeof(int64_t);           // two panels' pairs
    return xb + pairs + 256;
}

size_t oz_slices_bytes(int64_t n);

// Workspace of a stand-alone factorisation: the exchange buffers, pairs and
// abort flag, then (split form) the slices.
size_t getrf_workspace_bytes(int K, int64_t n, int oz)
{
    if (n <= 0)
        return 0;
    return align256(getrf_scratch_bytes(K, n)) + (oz ? oz_slices_bytes(n) : 0);
}

__global__ void k_zero_i64(int64_t *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *p = 0;
}

static size_t panel_lds_bytes(int K, int jb, int R)
{
    // tile (row stride R + 1), two pivot rows, the displaced row
    return ((size_t)K * jb * (R + 1) + 3 * (size_t)K * jb) * sizeof(double);
}

// start of a factorisation: clear the abort flag and the split form's
// range flag after it, and set words [0, nw) of the first panel's exchange
// buffer to XSENT
__global__ void k_xbuf_init(uint64_t *x, int64_t nw, int *abort_flag)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride)
        x[i] = (uint64_t)XSENT;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        abort_flag[0] = 0;
        abort_flag[1] = 0;
    }
}

// the timeout test hook: every poll of the factorisation gives up at once
__global__ void k_xbuf_raise(int *abort_flag)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *abort_flag = 1;
}

// end of a factorisation: a failed panel exchange makes info -1; else a
// split-form row or column scale below the exact range makes a nonsingular
// factorisation's info -3
__global__ void k_abort_check(const int *abort_flag, int64_t *info)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (abort_flag[0])
            *info = -1;
        else if (abort_flag[1] && *info == 0)
            *info = -3;
    }
}

// Side stream and four events per device for the look-ahead: the panels
// and the look-ahead columns' interchanges and update run in order on the
// side stream (no cross-stream wait between a panel and the next one when
// the trailing update keeps up), the rest of each trailing update on the
// caller's stream.  The big update waits until the look-ahead is through,
// so that the next panel's workgroups are resident before it fills the
// device.  Default priority, created once.
namespace {
struct LookAhead {
    hipStream_t side = nullptr;
    hipEvent_t start = nullptr, panel = nullptr, look = nullptr, rest = nullptr;
};
LookAhead g_la[16];
std::once_flag g_la_exit;

// at process exit, before the HIP runtime's own teardown (registered
// earlier, so it runs later): release every device's stream and events
void lookahead_release()
{
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess)
        return;
    for (int d = 0; d < 16; ++d) {
        LookAhead &la = g_la[d];
        if (!la.side || hipSetDevice(d) != hipSuccess)
            continue;
        (void)hipStreamSynchronize(la.side);
        (void)hipEventDestroy(la.start);
        (void)hipEventDestroy(la.panel);
        (void)hipEventDestroy(la.look);
        (void)hipEventDestroy(la.rest);
        (void)hipStreamDestroy(la.side);
        la = LookAhead{};
    }
    (void)hipSetDevice(cur);
}
}  // namespace

static int lookahead_get(LookAhead *&la)
{
    int dev = 0;
    BNC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16)
        return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: device index out of range");
    std::call_once(g_la_exit, [] { std::atexit(lookahead_release); });
    la = &g_la[dev];
    if (!la->side) {
        BNC_HIP(hipStreamCreateWithFlags(&la->side, hipStreamNonBlocking));
        BNC_HIP(hipEventCreateWithFlags(&la->start, hipEventDisableTiming));
        BNC_HIP(hipEventCreateWithFlags(&la->panel, hipEventDisableTiming));
        BNC_HIP(hipEventCreateWithFlags(&la->look, hipEventDisableTiming));
        BNC_HIP(hipEventCreateWithFlags(&la->rest, hipEventDisableTiming));
    }
    return BNC_OK;
}

template <int K>
int oz_split_cols_run(const double *A, int64_t lda, int64_t ldp, int64_t j0, int kb, int64_t c0, int64_t nc, int s,
                      double *SU, int64_t ldsu, int *ozlow, hipStream_t st);
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
    const int ps = panel_slots(n);
    const size_t xw = xbuf_words(K, ps);
    double *xb[2] = {(double *)base, (double *)base + xw};
    base += 2 * xw * sizeof(double);
    int64_t *pairs[2] = {(int64_t *)base, (int64_t *)base + 4 * PANEL_NB_MAX};
    base += 8ull * PANEL_NB_MAX * sizeof(int64_t);
    int *abort_flag = (int *)base;

    int dev = 0;
    BNC_HIP(hipGetDevice(&dev));
    int ncu = 0, lds_max = 0;
    BNC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    BNC_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t lds_static = 4096;  // bound on the panel kernel's static LDS
    LookAhead *la = nullptr;
    int rc = lookahead_get(la);
    if (rc)
        return rc;

    // one panel: rows pj0..n-1, columns pj0..pj0+pjb-1
    // panel number pn (its exchange buffer is xb[pn & 1]; it resets the other)
    auto panel = [&](int pn, int64_t pj0, int pjb, int64_t *pr, double *psl, hipStream_t st) -> int {
        const int64_t m = n - pj0;
        void *kfn = (void *)k_panel<K>;
        int R = 64;
        while (R > 8 && panel_lds_bytes(K, pjb, R) + lds_static > (size_t)lds_max)
            R /= 2;
        if (panel_lds_bytes(K, pjb, R) + lds_static > (size_t)lds_max)
            return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: panel does not fit in LDS");
        // split form: the panel asks for all of a CU's LDS, so no update
        // workgroup shares its CU (the matrix-core update would slow the
        // latency-bound panel down; the vector update is the bottleneck of
        // the K-word form, which keeps every CU for it)
        const size_t lds = oz ? (size_t)lds_max - lds_static : panel_lds_bytes(K, pjb, R);
        if (hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            (void)hipGetLastError();
        int per_cu = 0;
        BNC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, PANEL_THREADS, lds));
        int64_t cap = (int64_t)per_cu * ncu;
        if (cap > ps)
            cap = ps;
        const int P = (int)ceil_div(m, R);
        if (P > cap)
            return fail_arg(BNC_ERR_UNSUPPORTED, "getrf: panel needs more workgroups than can be co-resident");
        if (pn == 0) {
            // slots of workgroups 0..P-1 and the pivot-row copies
            const int64_t nw = (int64_t)ps * PANEL_NB_MAX + (int64_t)P * PANEL_NB_MAX * K * PANEL_NB_MAX;
            hipLaunchKernelGGL(k_xbuf_init, dim3(256), dim3(256), 0, st, (uint64_t *)xb[0], nw, abort_flag);
            BNC_LAUNCH_CHECK();
            const int64_t own_off = (int64_t)ps * PANEL_NB_MAX * (1 + K * PANEL_NB_MAX);
            hipLaunchKernelGGL(k_xbuf_init, dim3(16), dim3(256), 0, st, (uint64_t *)(xb[0] + own_off),
                               (int64_t)PANEL_NB_MAX * K * PANEL_NB_MAX, abort_flag);
            BNC_LAUNCH_CHECK();
            if (force_timeout_bits() & 1) {
                hipLaunchKernelGGL(k_xbuf_raise, dim3(1), dim3(64), 0, st, abort_flag);
                BNC_LAUNCH_CHECK();
            }
        }
        // All P workgroups fit on the device at once (checked above); the
        // grid barrier inside the kernel has a bounded spin, so a workgroup
        // that starts late (the other stream's kernels still hold CUs) only
        // delays the panel.
        hipLaunchKernelGGL((k_panel<K>), dim3(P), dim3(PANEL_THREADS), lds, st, A, lda, ldp, n, pj0, pjb, R, ipiv,
                           info, xb[pn & 1], xb[(pn + 1) & 1], ps, pr, abort_flag, oz, psl, n);
        BNC_LAUNCH_CHECK();
        return BNC_OK;
    };
    // split form: SLb[J & 1] holds the sliced rows cn..n-1 of panel J
    // (written by the panel itself; the next panel, which runs beside this
    // panel's trailing update, writes the other buffer), SU the sliced
    // columns cn..n-1 of its U12; all with leading dimension n
    double *SLb[2] = {oz_buf, oz_buf ? oz_buf + (size_t)OZ_SMAX * PANEL_NB_MAX * n : nullptr};
    double *SU = oz_buf ? oz_buf + 2 * (size_t)OZ_SMAX * PANEL_NB_MAX * n : nullptr;
    // row interchanges of columns c0..c0+nc-1; with trsm also U12 = L11^-1 A12
    // there, and with osu (split form, look-ahead columns) its slices,
    // column c0 + t at osu[t]
    auto swaps = [&](int64_t j0, int jb, int64_t c0, int64_t nc, const int64_t *pr, bool trsm, double *osu,
                     hipStream_t st) -> int {
        if (nc <= 0)
            return BNC_OK;
        const int ozs = osu ? oz : 0;
        if (trsm)
            hipLaunchKernelGGL((k_laswp_trsm<K, true>), dim3((unsigned)nc), dim3(64), 0, st, A, lda, ldp, j0, jb,
                               c0, pr, ozs, osu, n, abort_flag + 1);
        else
            hipLaunchKernelGGL((k_laswp_trsm<K, false>), dim3((unsigned)nc), dim3(64), 0, st, A, lda, ldp, j0, jb,
                               c0, pr, 0, nullptr, n, abort_flag + 1);
        BNC_LAUNCH_CHECK();
        return BNC_OK;
    };
    // A[r0.., c0..c0+nc) -= L21 (columns j0..j0+jb) * U12; split form:
    // the rows' slices in SL, the columns' slices already in SU (split) or
    // cut here
    auto update = [&](int64_t r0, int64_t c0, int64_t m, int64_t nc, int64_t j0, int jb, bool thin,
                      const double *SL, bool split, hipStream_t st) -> int {
        if (m <= 0 || nc <= 0)
            return BNC_OK;
        if (oz) {
            int rc2 = split ? BNC_OK : oz_split_cols_run<K>(A, lda, ldp, j0, jb, c0, nc, oz, SU + (c0 - r0), n, abort_flag + 1, st);
            if (rc2)
                return rc2;
            // profiling brackets the big-tile launches only: the thin ones sit
            // on the look-ahead chain, where the events would cost more time
            const int ev = thin ? -1 : UpdateTimer::begin(st);
            rc2 = oz_update_run<K>(oz, thin, A, lda, ldp, r0, c0, m, nc, jb, SL, n, SU + (c0 - r0), n, st);
            UpdateTimer::end(ev, st, 2.0 * (oz * (oz + 1) / 2) * (double)m * (double)nc * (double)jb);
            return rc2;
        }
        const int ev = thin ? -1 : UpdateTimer::begin(st);
        double *Cv = A + c0 * lda + r0;
        const MwView Lv{A + j0 * lda + r0, lda, ldp}, Uv{A + c0 * lda + j0, lda, ldp};
        if (thin) {
            using C = UpdCfgThin<K>;
            dim3 grid((unsigned)ceil_div(m, C::BM), (unsigned)ceil_div(nc, C::BN));
            hipLaunchKernelGGL((k_update<K, C::BM, C::BN, C::TM, C::TN, C::KB>), grid, dim3(UPD_THREADS), 0, st, Cv,
                               lda, ldp, Lv, Uv, m, nc, jb);
        } else {
            using C = UpdCfg<K>;
            dim3 grid((unsigned)ceil_div(m, C::BM), (unsigned)ceil_div(nc, C::BN));
            hipLaunchKernelGGL((k_update<K, C::BM, C::BN, C::TM, C::TN, C::KB>), grid, dim3(UPD_THREADS), 0, st, Cv,
                               lda, ldp, Lv, Uv, m, nc, jb);
        }
        BNC_LAUNCH_CHECK();
        UpdateTimer::end(ev, st, (double)m * (double)nc * (double)jb * fms_flops(K));
        return BNC_OK;
    };

    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, info);
    BNC_LAUNCH_CHECK();
    hipStream_t side = la->side;
    BNC_HIP(hipEventRecord(la->start, s));
    BNC_HIP(hipStreamWaitEvent(side, la->start, 0));
    if ((rc = panel(0, 0, (int)(n < nb ? n : nb), pairs[0], SLb[0], side)))
        return rc;
    BNC_HIP(hipEventRecord(la->panel, side));
    int J = 0;
    for (int64_t j0 = 0; j0 < n; j0 += nb, ++J) {
        const int jb = (int)((n - j0) < nb ? (n - j0) : nb);
        const int64_t *pr = pairs[J & 1];
        const int64_t cn = j0 + jb;
        // the caller's stream continues once panel J is done
        BNC_HIP(hipStreamWaitEvent(s, la->panel, 0));
        if (cn >= n) {
            if ((rc = swaps(j0, jb, 0, j0, pr, false, nullptr, s)))
                return rc;
            break;
        }
        const int nbn = (int)((n - cn) < nb ? (n - cn) : nb);
        double *SL = SLb[J & 1];
        // side stream: once the previous trailing update is through, the next
        // panel's columns (interchanges, U12 and, in the split form, its
        // slices in one kernel; then their update), then that panel
        if (J > 0)
            BNC_HIP(hipStreamWaitEvent(side, la->rest, 0));
        if ((rc = swaps(j0, jb, cn, nbn, pr, true, oz ? SU : nullptr, side)) ||
            (rc = update(cn, cn, n - cn, nbn, j0, jb, true, SL, oz != 0, side)))
            return rc;
        BNC_HIP(hipEventRecord(la->look, side));
        if ((rc = panel(J + 1, cn, nbn, pairs[(J + 1) & 1], SLb[(J + 1) & 1], side)))
            return rc;
        BNC_HIP(hipEventRecord(la->panel, side));
        // caller's stream, concurrently: the interchanges left of this panel
        // and the rest of the trailing matrix; in the split form the rest
        // columns are sliced before the wait for the look-ahead columns (the
        // slices of the two column ranges are disjoint)
        const int64_t cr = cn + nbn;
        if ((rc = swaps(j0, jb, 0, j0, pr, false, nullptr, s)) ||
            (rc = swaps(j0, jb, cr, n - cr, pr, true, nullptr, s)))
            return rc;
        if (oz && cr < n && (rc = oz_split_cols_run<K>(A, lda, ldp, j0, jb, cr, n - cr, oz, SU + nbn, n, abort_flag + 1, s)))
            return rc;
        BNC_HIP(hipStreamWaitEvent(s, la->look, 0));
        if ((rc = update(cn, cr, n - cn, n - cr, j0, jb, false, SL, oz != 0, s)))
            return rc;
        BNC_HIP(hipEventRecord(la->rest, s));
    }
    hipLaunchKernelGGL(k_abort_check, dim3(1), dim3(64), 0, s, abort_flag, info);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// C <- C - A B on K-plane matrices (A m x k, B k x n, C m x n), one launch
// of the trailing-update kernel with its big tile; every entry of C sees
// its k multiply-subtracts in increasing k.
template <int K>
int gemm_run(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
             int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, hipStream_t s)
{
    if (m == 0 || n == 0 || k == 0)
        return BNC_OK;
    using Cf = UpdCfg<K>;
    const dim3 grid((unsigned)ceil_div(m, Cf::BM), (unsigned)ceil_div(n, Cf::BN));
    const MwView Lv{A, lda, ldpa}, Uv{B, ldb, ldpb};
    hipLaunchKernelGGL((k_update<K, Cf::BM, Cf::BN, Cf::TM, Cf::TN, Cf::KB>), grid, dim3(UPD_THREADS), 0, s, C, ldc,
                       ldpc, Lv, Uv, m, n, (int)k);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}
#define GEMM_INST(K)                                                                                               \
    template int gemm_run<K>(int64_t, int64_t, int64_t, const double *, int64_t, int64_t, const double *, int64_t, \
                             int64_t, double *, int64_t, int64_t, hipStream_t);
GEMM_INST(1)
GEMM_INST(2)
GEMM_INST(3)
GEMM_INST(4)

template int getrf_run<1>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);
template int getrf_run<2>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);
template int getrf_run<3>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);
template int getrf_run<4>(int64_t, double *, int64_t, int64_t, int64_t *, int64_t *, void *, hipStream_t, int,
                            double *);

}  // namespace bnc

// Batched refined solves: Listing 1 of Kouya 2021 (Sec. 2) applied to many
// independent systems of order n <= 512 in one persistent launch.
//
// Persistent workgroups (64..512 threads, one per row of the largest system
// they take) take systems from an atomic queue in
// the order the caller gives (largest first balances the load) and run the
// whole path for one system at a time, every step in the same operation
// order as the single-system solver, so each result equals it bit for bit:
//   stage A (binary64 or quad-double words per entry, system by system)
//   to K words; blocked right-looking LU with 8-column panels held
//   in LDS (pivot search by wave shuffles, row interchanges as swaps in a
//   row map instead of data movement, reciprocal and scaling, rank-1 panel
//   updates), U12 by forward substitution, trailing
//   update with each thread's L21 row in registers and U12 in LDS; diagonal
//   reciprocals; substitutions with one thread per row and one LDS broadcast
//   per pivot; the exact residual with one thread per row; the stopping
//   tests on workgroup reductions; the update x <- x + 2^e z.
// Each system records its status, corrections, info and start/end wall-clock
// ticks.
//
// Built once per factor word count: with BNC_BATCH_K = k this unit holds the
// kernels of K = k only (the K-independent host functions go with k = 1), so
// the four units compile in parallel; left undefined, it holds every K.
#ifndef BNC_BATCH_K
#define BNC_BATCH_K 0
#endif
#include "common.hpp"
#include "exact.hpp"
#include "mw.hpp"

namespace bnc {

constexpr int BT_MAX = 512;  // most threads per workgroup (= largest order)
constexpr int BT_DEFAULT = 256;  // threads per workgroup unless chosen
constexpr size_t BLDS_MAX = 160 * 1024;  // LDS of one compute unit
constexpr int BNB_DEFAULT = 8;  // LU panel width unless tuned (4, 8 or 16)
// Residual bins: a row of order n <= 512 has at most 32 n + 4 < 2^15 terms
// (eight per word of A and column, four of b), so 38-bit digits still sum
// exactly; 22 of them span 836 bits (34-bit digits would need 24 bins)
constexpr int BRB_W = 38;   // residual bin width (bits)
constexpr int BRB = 22;     // residual bins per row
constexpr int BJ = 4;       // trailing-update columns per thread at once
constexpr int RPF = 4;      // residual: columns of A loaded ahead

// Per persistent workgroup of NT threads, reused across the systems it
// solves: the LU (K planes of NT*NT, lda = n), then 1/u_kk (K planes of NT).
template <int K, int NT>
constexpr size_t slot_doubles()
{
    return (size_t)K * NT * NT + (size_t)K * NT;
}

template <int K, int PW, int NT>
struct BatchLds {
    double tile[K * PW * NT];  // panel [w][c][r]; reused as U12 [w][k][j]
    double l11[K][PW][PW];      // the panel's unit lower triangle [w][k][r]
    double ybuf[NT][K];         // broadcast slots of the substitutions
    double xq[4][NT];           // current solution (quad-double)
    double red[NT];                // reduction scratch
    int redi[NT];
    double wkey[NT / 64][K];       // per-wave argmax
    int wrow[NT / 64];
    int perm[NT];  // row map of the factorisation, then its permutation
    int s_int[4];
};

// ---- workgroup reductions ----------------------------------------------------

template <int NT>
__device__ __forceinline__ double wg_max(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s)
            red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ double wg_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s)
            red[t] = red[t] + red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ int wg_min_i(int v, int *redi)
{
    const int t = threadIdx.x;
    redi[t] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s)
            redi[t] = redi[t + s] < redi[t] ? redi[t + s] : redi[t];
        __syncthreads();
    }
    const int r = redi[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ __forceinline__ int wg_or(int v, int *redi)
{
    const int t = threadIdx.x;
    redi[t] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s)
            redi[t] = redi[t] | redi[t + s];
        __syncthreads();
    }
    const int r = redi[0];
    __syncthreads();
    return r;
}

template <int K>
__device__ __forceinline__ bool cand_better_b(const double (&kb)[K], int rb, const double (&ka)[K], int ra)
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

// 2-norm of v over threads t < n (binary64, power-of-two scaled; the tree
// order is fixed)
template <int NT>
__device__ __forceinline__ double wg_norm2(double v, bool active, double vmax, double *red)
{
    const double sc = pow2(-(norm_exp(vmax) + 1));
    const double t = active ? v * sc : 0.0;
    const double s = wg_sum<NT>(t * t, red);
    return vmax == 0.0 ? 0.0 : sqrt(s) * pow2(norm_exp(vmax) + 1);
}

// ---- substitutions (thread i holds y_i) ---------------------------------------

template <int K, int NT, class LDS>
__device__ __forceinline__ void bsolve(int n, const double *__restrict__ lu, int64_t ldp, const double *__restrict__ rd,
                                       double (&y)[K], LDS &S)
{
    const int t = threadIdx.x;
    const int tc = t < n ? t : n - 1;  // in-bounds row for the prefetches
    const int64_t pt = S.perm[tc];      // its stored row (rows are never moved)
    // forward: y_i <- y_i - l_ik y_k, k increasing; column k + 1's entry is
    // loaded a step ahead (unconditionally, from an in-bounds address)
    double ln[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        ln[w] = lu[w * ldp + pt];
    for (int k = 0; k < n; ++k) {
        double l[K];
        const int kn = k + 1 < n ? k + 1 : k;
#pragma unroll
        for (int w = 0; w < K; ++w) {
            l[w] = ln[w];
            ln[w] = lu[w * ldp + (int64_t)kn * n + pt];
        }
        if (t == k) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                S.ybuf[k][w] = y[w];
        }
        __syncthreads();
        if (t > k && t < n) {
            double yk[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                yk[w] = S.ybuf[k][w];
            fms<K>(y, l, yk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                y[w] = o[w];
        }
    }
    __syncthreads();
    // backward: x_k = y_k * (1/u_kk), then y_i <- y_i - u_ik x_k, k
    // decreasing; column k - 1's entry loaded a step ahead
    double un[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        un[w] = lu[w * ldp + (int64_t)(n - 1) * n + pt];
    for (int k = n - 1; k >= 0; --k) {
        double u[K];
        const int kn = k > 0 ? k - 1 : 0;
#pragma unroll
        for (int w = 0; w < K; ++w) {
            u[w] = un[w];
            un[w] = lu[w * ldp + (int64_t)kn * n + pt];
        }
        if (t == k) {
            double rk[K], xk[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                rk[w] = rd[w * NT + k];
            mul<K>(y, rk, xk);
#pragma unroll
            for (int w = 0; w < K; ++w) {
                y[w] = xk[w];
                S.ybuf[k][w] = xk[w];
            }
        }
        __syncthreads();
        if (t < k) {
            double xk[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                xk[w] = S.ybuf[k][w];
            fms<K>(y, u, xk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                y[w] = o[w];
        }
    }
    __syncthreads();
}

// y_i = rf_perm[i]: gather of the K-word copy held per thread through perm
template <int K, int NT, class LDS>
__device__ __forceinline__ void bgather(int n, double (&v)[K], LDS &S)
{
    const int t = threadIdx.x;
    if (t < n) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            S.ybuf[t][w] = v[w];
    }
    __syncthreads();
    if (t < n) {
        const int s = S.perm[t];
#pragma unroll
        for (int w = 0; w < K; ++w)
            v[w] = S.ybuf[s][w];
    }
    __syncthreads();
}

// ---- exact residual ------------------------------------------------------------

// Deposits of -A(t, :) x into row t's bins: each product of a word of
// A(t, j) and a word of x_j as its two exact halves, column by column (the
// sum is exact, so the order of the deposits does not matter).  A's words
// are loaded PF columns ahead, unconditionally from clamped columns.
template <int AW, int NT>
__device__ __forceinline__ void resid_row_terms(int n, const double *__restrict__ Arow, int64_t nn2,
                                                const double (&xq)[4][NT], double sg0, double (&bins)[BRB], int nb,
                                                int nbu, double lim0, bool &bd)
{
    constexpr int PF = AW == 1 ? RPF : 2;
    double apf[PF][AW];
#pragma unroll
    for (int p = 0; p < PF; ++p)
#pragma unroll
        for (int u = 0; u < AW; ++u)
            apf[p][u] = Arow[u * nn2 + (int64_t)(p < n ? p : n - 1) * n];
    for (int j0 = 0; j0 < n; j0 += PF) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int j = j0 + p;
            double a[AW];
            const int jn = j + PF < n ? j + PF : n - 1;
#pragma unroll
            for (int u = 0; u < AW; ++u) {
                a[u] = apf[p][u];
                apf[p][u] = Arow[u * nn2 + (int64_t)jn * n];
            }
            if (j < n) {
#pragma unroll
                for (int u = 0; u < AW; ++u) {
                    // a word that is zero on every row of the wave adds
                    // nothing (its products are exact zeros): skipped
                    if (AW > 1 && !__any(a[u] != 0.0))
                        continue;
                    double tt[8];
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        double lo;
                        const double hi = two_prod(a[u], xq[w][j], lo);
                        tt[2 * w] = -hi;
                        tt[2 * w + 1] = -lo;
                    }
                    deposit_many<BRB, 8, BRB_W>(tt, sg0, bins, nb, nbu, lim0, bd);
                }
            }
        }
    }
}

// ---- the batched solver ---------------------------------------------------------

// Register budget: two waves per SIMD (512 / NT workgroups of NT threads per
// compute unit, where the LDS allows).  The whole solve in one kernel needs
// about 430 registers; capped at 256 it spills (about 720 bytes per lane),
// and the second wave still wins: orders 129..256 (8-wide panels, 256
// threads) ran 24% faster than at one wave per SIMD without spills.
template <int K, int PW, int NT>
__global__ void __launch_bounds__(NT, 512 / NT)
    k_batch(int64_t count, const int64_t *__restrict__ nn, const int32_t *__restrict__ aws,
            const double *const *__restrict__ As,
            const double *const *__restrict__ bs, double *const *__restrict__ xs, const int32_t *__restrict__ order,
            unsigned *__restrict__ queue, double *__restrict__ work, bnc_refine_opts o,
            bnc_batch_result *__restrict__ res)
{
    extern __shared__ double smem_raw[];
    BatchLds<K, PW, NT> &S = *reinterpret_cast<BatchLds<K, PW, NT> *>(smem_raw);
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int64_t ldp = (int64_t)NT * NT;
    double *lu = work + (size_t)blockIdx.x * slot_doubles<K, NT>();
    double *rd = lu + (size_t)K * NT * NT;

    for (;;) {
        if (t == 0)
            S.s_int[0] = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t qi = S.s_int[0];
        __syncthreads();
        if (qi >= count)
            break;
        const int64_t sys = order ? order[qi] : qi;
        const uint64_t t0 = wall_clock64();
        const int64_t n64 = nn[sys];
        const int aw = aws ? aws[sys] : 1;  // words per entry of A
        bnc_batch_result out{};
        double *x = xs[sys];
        if (n64 < 1 || n64 > NT || (aw != 1 && aw != 4)) {
            if (t == 0) {
                out.status = BNC_BAD_SIZE;
                out.t_start = t0;
                out.t_factored = t0;
                out.t_end = wall_clock64();
                res[sys] = out;
            }
            continue;
        }
        const int n = (int)n64;
        const double *A = As[sys];
        const double *b = bs[sys];

        const int64_t nn2 = (int64_t)n * n;  // plane stride of A's words

        // ---- checks, row maxima (leading words), exponent bounds (every
        // word): the leading words by rows (thread t = row t, one pass),
        // the other words, if any, after
        int bad = 0;
        double rmax_i = 0.0;
        int ea = 2000, eb = 2000;
        if (t < n) {
            for (int j = 0; j < n; ++j) {
                const double v = A[(int64_t)j * n + t];
                bad |= !isfinite(v);
                if (v != 0.0) {
                    const int ex = ilogb_bits(v);
                    ea = ex < ea ? ex : ea;
                }
                rmax_i = fmax(rmax_i, fabs(v));
            }
            for (int w = 0; w < 4; ++w) {
                const double v = b[w * n + t];
                bad |= !isfinite(v);
                if (v != 0.0) {
                    const int ex = ilogb_bits(v);
                    eb = ex < eb ? ex : eb;
                }
            }
        }
        for (int64_t e = nn2 + t; e < (int64_t)aw * nn2; e += NT) {
            const double v = A[e];
            bad |= !isfinite(v);
            if (v != 0.0) {
                const int ex = ilogb_bits(v);
                ea = ex < ea ? ex : ea;
            }
        }
        if (wg_or<NT>(bad, S.redi)) {
            for (int e = t; e < 4 * n; e += NT)
                x[(e / n) * n + e % n] = 0.0;
            if (t == 0) {
                out.status = BNC_NONFINITE;
                out.t_start = t0;
                out.t_factored = t0;
                out.t_end = wall_clock64();
                res[sys] = out;
            }
            continue;
        }
        ea = wg_min_i<NT>(ea, S.redi);
        eb = wg_min_i<NT>(eb, S.redi);

        // ---- K-word copy of A (quad-double words renormalised to K) and,
        // in the same pass, ||A||_F from the leading words (power-of-two
        // scaled by the largest entry)
        double anorm;
        {
            const double am = wg_max<NT>(rmax_i, S.red);  // max |a_ij| (leading words)
            const double sc = pow2(-(norm_exp(am) + 1));
            double acc = 0.0;
            if (aw == 1) {
                for (int64_t e = t; e < nn2; e += NT) {
                    const double a0 = A[e];
                    lu[e] = a0;
#pragma unroll
                    for (int w = 1; w < K; ++w)
                        lu[w * ldp + e] = 0.0;
                    const double v = a0 * sc;
                    acc = acc + v * v;
                }
            } else {
                for (int64_t e = t; e < nn2; e += NT) {
                    double v[4], o[K];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        v[u] = A[u * nn2 + e];
                    renorm<K, 4>(v, o);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        lu[w * ldp + e] = o[w];
                    const double s0 = v[0] * sc;
                    acc = acc + s0 * s0;
                }
            }
            const double ss = wg_sum<NT>(acc, S.red);
            anorm = am == 0.0 ? 0.0 : sqrt(ss) * pow2(norm_exp(am) + 1);
        }
        __syncthreads();

        // ---- blocked LU.  Rows are never moved in the workspace: S.perm[i]
        // is the stored row that holds row i of the factorisation (the
        // original row index, since A is staged unpermuted), and a pivot
        // interchange swaps two entries of it.  Every access to row i goes
        // through S.perm, so the values are those of whole-row swaps.
        for (int i = t; i < n; i += NT)
            S.perm[i] = i;
        __syncthreads();
        int64_t info = 0;
        for (int j0 = 0; j0 < n; j0 += PW) {
            const int jb = (n - j0) < PW ? (n - j0) : PW;
            const int m = n - j0;
            for (int e = t; e < m * jb; e += NT) {
                const int r = e % m, c = e / m;
                const int pr = S.perm[j0 + r];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    S.tile[(w * PW + c) * NT + r] = lu[w * ldp + (int64_t)(j0 + c) * n + pr];
            }
            __syncthreads();
            for (int kk = 0; kk < jb; ++kk) {
                const int k = j0 + kk;
                // pivot: rows kk..m-1 of the tile, thread = row
                double key[K];
                int row = -1;
                if (t < m && t >= kk) {
                    row = t;
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        key[w] = S.tile[(w * PW + kk) * NT + t];
                } else {
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        key[w] = 0.0;
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    double ok[K];
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        ok[w] = __shfl_xor(key[w], off, 64);
                    const int orow = __shfl_xor(row, off, 64);
                    if (cand_better_b<K>(ok, orow, key, row)) {
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            key[w] = ok[w];
                        row = orow;
                    }
                }
                if (lane == 0) {
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        S.wkey[wave][w] = key[w];
                    S.wrow[wave] = row;
                }
                __syncthreads();
                if (t == 0) {
                    double bk[K];
                    int br = -1;
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        bk[w] = 0.0;
                    for (int q = 0; q < NT / 64; ++q) {
                        double kq[K];
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            kq[w] = S.wkey[q][w];
                        if (cand_better_b<K>(kq, S.wrow[q], bk, br)) {
#pragma unroll
                            for (int w = 0; w < K; ++w)
                                bk[w] = kq[w];
                            br = S.wrow[q];
                        }
                    }
                    S.s_int[1] = br;
                }
                __syncthreads();
                const int pr = S.s_int[1];  // tile row of the pivot
                if (pr != kk) {
                    // panel columns in the tile, the rest through the row map
                    for (int e = t; e < jb * K; e += NT) {
                        const int c = e % jb, w = e / jb;
                        double *a = &S.tile[(w * PW + c) * NT];
                        const double tmp = a[kk];
                        a[kk] = a[pr];
                        a[pr] = tmp;
                    }
                    if (t == 0) {
                        const int tmp = S.perm[k];
                        S.perm[k] = S.perm[j0 + pr];
                        S.perm[j0 + pr] = tmp;
                    }
                }
                __syncthreads();
                double pv[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    pv[w] = S.tile[(w * PW + kk) * NT + kk];
                if (is_zero<K>(pv)) {
                    if (info == 0)
                        info = k + 1;
                    continue;
                }
                if (t < m && t > kk) {
                    double rc[K], a[K], l[K];
                    recip<K>(pv, rc);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        a[w] = S.tile[(w * PW + kk) * NT + t];
                    mul<K>(a, rc, l);
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        S.tile[(w * PW + kk) * NT + t] = l[w];
                }
                __syncthreads();
                const int nc = jb - kk - 1;
                for (int e = t; e < m * nc; e += NT) {
                    const int r = e % m, c = kk + 1 + e / m;
                    if (r > kk) {
                        double a[K], l[K], u[K], oo[K];
#pragma unroll
                        for (int w = 0; w < K; ++w) {
                            a[w] = S.tile[(w * PW + c) * NT + r];
                            l[w] = S.tile[(w * PW + kk) * NT + r];
                            u[w] = S.tile[(w * PW + c) * NT + kk];
                        }
                        fms<K>(a, l, u, oo);
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            S.tile[(w * PW + c) * NT + r] = oo[w];
                    }
                }
                __syncthreads();
            }
            // panel back to the workspace (rows through the map, final for
            // this panel: later interchanges only swap entries past it)
            for (int e = t; e < m * jb; e += NT) {
                const int r = e % m, c = e / m;
                const int pr = S.perm[j0 + r];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    lu[w * ldp + (int64_t)(j0 + c) * n + pr] = S.tile[(w * PW + c) * NT + r];
            }
            // every later phase reads the panel back from the workspace,
            // written above by other threads
            __syncthreads();
            const int c0 = j0 + jb;
            const int m2 = n - c0;
            if (m2 <= 0)
                break;
            // trailing-update mapping: thread = (row r, column group q)
            int R2 = 1;
            while (R2 < m2)
                R2 <<= 1;
            const int G = NT / R2;
            const int r = t % R2, q = t / R2;
            double l21[PW][K];
            if (r < m2) {
#pragma unroll
                for (int kk = 0; kk < PW; ++kk)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        l21[kk][w] = kk < jb ? S.tile[(w * PW + kk) * NT + jb + r] : 0.0;
            }
            // L11 to its own block (U12 overwrites the tile below)
            for (int e = t; e < K * PW * PW; e += NT) {
                const int rr = e % PW, kk = (e / PW) % PW, w = e / (PW * PW);
                S.l11[w][kk][rr] = (kk < jb && rr < jb) ? S.tile[(w * PW + kk) * NT + rr] : 0.0;
            }
            __syncthreads();
            // U12 = L11^-1 A12: thread per column of A12
            int prow[PW];  // stored rows of the panel's rows
#pragma unroll
            for (int kk = 0; kk < PW; ++kk)
                prow[kk] = kk < jb ? S.perm[j0 + kk] : 0;
            for (int j = t; j < m2; j += NT) {
                double u[PW][K];
#pragma unroll
                for (int kk = 0; kk < PW; ++kk)
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        u[kk][w] = kk < jb ? lu[w * ldp + (int64_t)(c0 + j) * n + prow[kk]] : 0.0;
#pragma unroll
                for (int kk = 0; kk < PW; ++kk) {
                    if (kk < jb) {
#pragma unroll
                        for (int rr = 0; rr < PW; ++rr) {
                            if (rr > kk && rr < jb) {
                                double l[K], oo[K];
#pragma unroll
                                for (int w = 0; w < K; ++w)
                                    l[w] = S.l11[w][kk][rr];
                                fms<K>(u[rr], l, u[kk], oo);
#pragma unroll
                                for (int w = 0; w < K; ++w)
                                    u[rr][w] = oo[w];
                            }
                        }
                    }
                }
#pragma unroll
                for (int kk = 0; kk < PW; ++kk)
                    if (kk < jb) {
#pragma unroll
                        for (int w = 0; w < K; ++w) {
                            lu[w * ldp + (int64_t)(c0 + j) * n + prow[kk]] = u[kk][w];
                            S.tile[(w * PW + kk) * NT + j] = u[kk][w];
                        }
                    }
            }
            __syncthreads();
            // A22 <- A22 - L21 U12, each entry in increasing k.  A thread
            // takes BJ of its columns at once: their multiply-subtract
            // chains are independent, so they interleave and hide each
            // other's latency (one chain per thread left the FP64 pipes
            // idle at one wave per SIMD)
            if (r < m2) {
                const int64_t prr = S.perm[c0 + r];  // stored row of row c0 + r
                int j = q;
                // the next group's entries are loaded while this group is
                // updated (unconditional loads from clamped columns)
                double c[BJ][K];
                auto load_group = [&](int jg, double (&cc)[BJ][K]) {
#pragma unroll
                    for (int bj = 0; bj < BJ; ++bj) {
                        const int jc = jg + bj * G < m2 ? jg + bj * G : m2 - 1;
                        const double *cp = lu + (int64_t)(c0 + jc) * n + prr;
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            cc[bj][w] = cp[w * ldp];
                    }
                };
                if (j + (BJ - 1) * G < m2)
                    load_group(j, c);
                for (; j + (BJ - 1) * G < m2; j += BJ * G) {
                    double cn[BJ][K];
                    load_group(j + BJ * G, cn);
#pragma unroll
                    for (int kk = 0; kk < PW; ++kk) {
                        if (kk < jb) {
#pragma unroll
                            for (int bj = 0; bj < BJ; ++bj) {
                                double u[K], oo[K];
#pragma unroll
                                for (int w = 0; w < K; ++w)
                                    u[w] = S.tile[(w * PW + kk) * NT + j + bj * G];
                                fms<K>(c[bj], l21[kk], u, oo);
#pragma unroll
                                for (int w = 0; w < K; ++w)
                                    c[bj][w] = oo[w];
                            }
                        }
                    }
#pragma unroll
                    for (int bj = 0; bj < BJ; ++bj) {
                        double *cp = lu + (int64_t)(c0 + j + bj * G) * n + prr;
#pragma unroll
                        for (int w = 0; w < K; ++w) {
                            cp[w * ldp] = c[bj][w];
                            c[bj][w] = cn[bj][w];
                        }
                    }
                }
                for (; j < m2; j += G) {
                    double c[K];
                    double *cp = lu + (int64_t)(c0 + j) * n + prr;
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        c[w] = cp[w * ldp];
#pragma unroll
                    for (int kk = 0; kk < PW; ++kk) {
                        if (kk < jb) {
                            double u[K], oo[K];
#pragma unroll
                            for (int w = 0; w < K; ++w)
                                u[w] = S.tile[(w * PW + kk) * NT + j];
                            fms<K>(c, l21[kk], u, oo);
#pragma unroll
                            for (int w = 0; w < K; ++w)
                                c[w] = oo[w];
                        }
                    }
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        cp[w * ldp] = c[w];
                }
            }
            __syncthreads();
        }
        const uint64_t t_fact = wall_clock64();
        if (info != 0) {
            for (int e = t; e < 4 * n; e += NT)
                x[(e / n) * n + e % n] = 0.0;
            if (t == 0) {
                out.status = BNC_SINGULAR;
                out.info = info;
                out.t_start = t0;
                out.t_factored = t_fact;
                out.t_end = wall_clock64();
                res[sys] = out;
            }
            __syncthreads();
            continue;
        }
        // diagonal reciprocals; S.perm is the row permutation of P A = L U
        if (t < n) {
            double d[K], rc[K];
#pragma unroll
            for (int w = 0; w < K; ++w)
                d[w] = lu[w * ldp + (int64_t)t * n + S.perm[t]];
            recip<K>(d, rc);
#pragma unroll
            for (int w = 0; w < K; ++w)
                rd[w * NT + t] = rc[w];
        }
        __syncthreads();

        // ---- first solution: K-word copy of b, substitution, extend
        double y[K];
        if (t < n) {
            double bw[4];
#pragma unroll
            for (int w = 0; w < 4; ++w)
                bw[w] = b[w * n + t];
            renorm<K, 4>(bw, y);
        }
        bgather<K, NT>(n, y, S);
        bsolve<K, NT>(n, lu, ldp, rd, y, S);
        if (t < n) {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                S.xq[w][t] = w < K ? y[w] : 0.0;
        }
        __syncthreads();

        // ---- refinement loop (same tests and order as the single solver)
        const int h = [&] {
            const int64_t N = 8 * (int64_t)n + 4;
            int hh = 1;
            while (((int64_t)1 << hh) < 2 * N)
                ++hh;
            return hh;
        }();
        const double thresh_c = sqrt((double)n) * o.rtol * anorm;
        bool have_z = false;
        double zmax = 0.0, zprev = 0.0;
        int iters = 0, status = BNC_MAX_ITER, inexact = 0;
        for (int it = 0; it <= o.max_iter; ++it) {
            // x bounds
            double xv0 = t < n ? S.xq[0][t] : 0.0;
            int ex = 2000;
            if (t < n)
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    if (S.xq[w][t] != 0.0) {
                        const int e2 = ilogb_bits(S.xq[w][t]);
                        ex = e2 < ex ? e2 : ex;
                    }
            const double xmax = wg_max<NT>(fabs(xv0), S.red);
            // the forward test needs no residual: when it decides, this
            // pass's residual (whose test could only agree) is not formed
            if (have_z && zmax <= o.ctol * xmax) {
                status = BNC_CONVERGED;
                break;
            }
            ex = wg_min_i<NT>(ex, S.redi);
            // exact residual, thread per row; the wave's lanes deposit into
            // a common number of bins (the largest row's) so that the bin
            // loop is uniform and each column's eight terms interleave
            double rr[4] = {0.0, 0.0, 0.0, 0.0};
            int rbad = 0;
            RowAnchor an{};
            an.any = false;
            if (t < n) {
                ExpBounds ebnd;
                ebnd.a = ea;
                ebnd.x = ex;
                ebnd.b = eb;
                an = row_anchor<BRB, BRB_W>(rmax_i, xmax, b[t], h, lowest_bit(ebnd));
            }
            const int nbu = wave_max_nb(t < n && an.any ? an.nb : 0);
            if (t < n && an.any) {
                double bins[BRB];
#pragma unroll
                for (int qb = 0; qb < BRB; ++qb)
                    bins[qb] = 0.0;
                const double sg0 = 1.5 * pow2(an.e0 + 52);  // bin 0's extraction constant
                const double lim0 = pow2(an.e0 + 51);
                bool bd = false;
                if (aw == 1)
                    resid_row_terms<1>(n, A + t, nn2, S.xq, sg0, bins, an.nb, nbu, lim0, bd);
                else
                    resid_row_terms<4>(n, A + t, nn2, S.xq, sg0, bins, an.nb, nbu, lim0, bd);
                double tb[4];
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    tb[w] = b[w * n + t];
                deposit_many<BRB, 4, BRB_W>(tb, sg0, bins, an.nb, nbu, lim0, bd);
                bd = bins_to_qd<BRB, BRB_W>(bins, an.nb, an.e0, rr) || bd;
                rbad = bd ? 1 : 0;
            }
            inexact |= wg_or<NT>(rbad, S.redi);
            const double rmax = wg_max<NT>(fabs(rr[0]), S.red);
            const double nr = wg_norm2<NT>(rr[0], t < n, rmax, S.red);
            const double nx = wg_norm2<NT>(xv0, t < n, xmax, S.red);
            if (nr < thresh_c * nx + o.atol || (have_z && zmax <= o.ctol * xmax)) {
                status = BNC_CONVERGED;
                break;
            }
            if (o.stagnation_ratio > 0.0 && iters >= 2 && zmax > o.stagnation_ratio * zprev) {
                status = BNC_STAGNATED;
                break;
            }
            if (iters == o.max_iter)
                break;
            // K-word copy of r * 2^-e, correction, x <- x + 2^e z
            const int e = norm_exp(rmax);
            double v[K];
            if (t < n) {
                double sr[4];
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    sr[w] = rr[w] * pow2(-e);
                renorm<K, 4>(sr, v);
            }
            bgather<K, NT>(n, v, S);
            bsolve<K, NT>(n, lu, ldp, rd, v, S);
            double z0 = 0.0;
            if (t < n) {
                double zv[4], xv[4], oo[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    zv[w] = w < K ? v[w] * pow2(e) : 0.0;
                    xv[w] = S.xq[w][t];
                }
                add<4>(xv, zv, oo);
                z0 = zv[0];
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    S.xq[w][t] = oo[w];
            }
            zprev = zmax;
            zmax = wg_max<NT>(fabs(z0), S.red);
            have_z = true;
            ++iters;
        }
        for (int e = t; e < 4 * n; e += NT)
            x[e] = S.xq[e / n][e % n];
        if (t == 0) {
            out.status = status;
            out.iters = iters;
            out.info = 0;
            out.residual_inexact = inexact;
            out.t_start = t0;
            out.t_factored = t_fact;
            out.t_end = wall_clock64();
            res[sys] = out;
        }
        __syncthreads();
    }
}

static __global__ void k_queue_reset(unsigned *q)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *q = 0;
}

#if BNC_BATCH_K == 0 || BNC_BATCH_K == 1
// the queue counter (256 bytes), then one slot per workgroup
size_t batch_workspace_bytes(int K, int slots, int threads)
{
    const size_t nt = threads ? (size_t)threads : (size_t)BT_DEFAULT;
    return (size_t)slots * ((size_t)K * nt * nt + (size_t)K * nt) * sizeof(double) + 256;
}
#endif

// persistent workgroups per compute unit: as many as registers and LDS allow
template <int K, int PW, int NT>
static int occupancy_per_cu()
{
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_batch<K, PW, NT>, NT,
                                                     sizeof(BatchLds<K, PW, NT>)) != hipSuccess ||
        per < 1)
        per = 1;
    return per;
}

// Panel widths a launch of NT threads offers: 16 from 128 threads up, when
// its LDS fits a compute unit; 8 when it fits; 4 always.
template <int K, int PW, int NT>
constexpr bool panel_offered()
{
    return sizeof(BatchLds<K, PW, NT>) <= BLDS_MAX && (PW != 16 || NT >= 128);
}

// The panel width actually launched: the widest offered one not above the
// request (0 = 8).  The width changes no result.
template <int K, int NT>
constexpr int panel_fit(int pw)
{
    if (pw == 0)
        pw = BNB_DEFAULT;
    if (pw >= 16 && panel_offered<K, 16, NT>())
        return 16;
    if (pw >= 8 && panel_offered<K, 8, NT>())
        return 8;
    return 4;
}

template <int K, int NT>
static int occupancy_pw(int pw)
{
    static_assert(sizeof(BatchLds<K, 4, NT>) <= BLDS_MAX, "batched LDS exceeds a compute unit");
    const int f = panel_fit<K, NT>(pw);
    if constexpr (panel_offered<K, 16, NT>()) {
        if (f == 16)
            return occupancy_per_cu<K, 16, NT>();
    }
    if constexpr (panel_offered<K, 8, NT>()) {
        if (f == 8)
            return occupancy_per_cu<K, 8, NT>();
    }
    return occupancy_per_cu<K, 4, NT>();
}

// persistent workgroups per compute unit of the K-word launch of nt threads
// (defined in the unit that holds that K's kernels)
template <int K>
int occupancy_k(int pw, int nt)
{
    switch (nt) {
    case 64:
        return occupancy_pw<K, 64>(pw);
    case 128:
        return occupancy_pw<K, 128>(pw);
    case 256:
        return occupancy_pw<K, 256>(pw);
    default:
        return occupancy_pw<K, 512>(pw);
    }
}

#if BNC_BATCH_K != 0
// the other word counts' kernels live in their own units
#define EXT(K)                                                                                                  \
    extern template int occupancy_k<K>(int, int);                                                              \
    extern template int batch_run<K>(int64_t, const int64_t *, const int32_t *, const double *const *,         \
                                     const double *const *, double *const *, const int32_t *, void *, int,     \
                                     const bnc_refine_opts *, bnc_batch_result *, hipStream_t);
template <int K>
int batch_run(int64_t count, const int64_t *n, const int32_t *aw, const double *const *A, const double *const *b,
              double *const *x, const int32_t *order, void *work, int slots, const bnc_refine_opts *o,
              bnc_batch_result *res, hipStream_t s);
#if BNC_BATCH_K != 1
EXT(1)
#endif
#if BNC_BATCH_K != 2
EXT(2)
#endif
#if BNC_BATCH_K != 3
EXT(3)
#endif
#if BNC_BATCH_K != 4
EXT(4)
#endif
#undef EXT
#endif

#if BNC_BATCH_K == 0 || BNC_BATCH_K == 1
bool batch_panel_ok(int pw) { return pw == 0 || pw == 4 || pw == 8 || pw == 16; }
bool batch_threads_ok(int nt) { return nt == 0 || nt == 64 || nt == 128 || nt == 256 || nt == 512; }

int batch_default_slots(int K, int pw, int nt)
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    if (pw == 0)
        pw = BNB_DEFAULT;
    if (nt == 0)
        nt = BT_DEFAULT;
    const int per = K == 1 ? occupancy_k<1>(pw, nt) : K == 2 ? occupancy_k<2>(pw, nt)
                                                  : K == 3 ? occupancy_k<3>(pw, nt) : occupancy_k<4>(pw, nt);
    return per * ncu;
}
#endif

template <int K, int PW, int NT>
static int batch_launch(int64_t count, const int64_t *n, const int32_t *aw, const double *const *A,
                        const double *const *b, double *const *x, const int32_t *order, unsigned *queue, double *ws,
                        int slots, const bnc_refine_opts *o, bnc_batch_result *res, hipStream_t s)
{
    const size_t lds = sizeof(BatchLds<K, PW, NT>);
    if (hipFuncSetAttribute((const void *)k_batch<K, PW, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        (void)hipGetLastError();
    hipLaunchKernelGGL((k_batch<K, PW, NT>), dim3((unsigned)slots), dim3(NT), lds, s, count, n, aw, A, b, x, order,
                       queue, ws, *o, res);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

template <int K, int NT>
static int batch_launch_pw(int64_t count, const int64_t *n, const int32_t *aw, const double *const *A,
                           const double *const *b, double *const *x, const int32_t *order, unsigned *queue,
                           double *ws, int slots, const bnc_refine_opts *o, bnc_batch_result *res, hipStream_t s)
{
    const int f = panel_fit<K, NT>(o->batch_panel);
    if constexpr (panel_offered<K, 16, NT>()) {
        if (f == 16)
            return batch_launch<K, 16, NT>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
    }
    if constexpr (panel_offered<K, 8, NT>()) {
        if (f == 8)
            return batch_launch<K, 8, NT>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
    }
    return batch_launch<K, 4, NT>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
}

template <int K>
int batch_run(int64_t count, const int64_t *n, const int32_t *aw, const double *const *A, const double *const *b,
              double *const *x, const int32_t *order, void *work, int slots, const bnc_refine_opts *o,
              bnc_batch_result *res, hipStream_t s)
{
    if (count == 0)
        return BNC_OK;
    unsigned *queue = (unsigned *)work;
    double *ws = (double *)((char *)work + 256);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, queue);
    BNC_LAUNCH_CHECK();
    switch (o->batch_threads ? o->batch_threads : BT_DEFAULT) {
    case 64:
        return batch_launch_pw<K, 64>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
    case 128:
        return batch_launch_pw<K, 128>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
    case 256:
        return batch_launch_pw<K, 256>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
    default:
        return batch_launch_pw<K, 512>(count, n, aw, A, b, x, order, queue, ws, slots, o, res, s);
    }
}

#define INST(K)                                                                                                 \
    template int occupancy_k<K>(int, int);                                                                     \
    template int batch_run<K>(int64_t, const int64_t *, const int32_t *, const double *const *,                 \
                              const double *const *, double *const *, const int32_t *, void *, int,            \
                              const bnc_refine_opts *, bnc_batch_result *, hipStream_t);
#if BNC_BATCH_K == 0
INST(1)
INST(2)
INST(3)
INST(4)
#else
INST(BNC_BATCH_K)
#endif
#undef INST

}  // namespace bnc

// Learned choice of the factor precision (not in the paper; the project's
// addition on top of its mixed-precision refinement, Sec. 2 / Listing 1).
//
//   k_features  24 cheap binary64 features of each system (order <= 512,
//               the leading words of A):
//               norms and their ratios, diagonal dominance, symmetry, a
//               binary64 LU with partial pivoting (pivot growth, spread of
//               U's diagonal), three steps of Hager's 1-norm estimate of
//               ||A^-1||_1 (Hager 1984; Higham 1988) from solves with A and
//               A^T, and the binary64 solution of A x = b (its size and
//               backward error).  One workgroup per system, thread t owns
//               row t (256 threads up to order 256, 512 above); every sum
//               runs in index order on one thread and
//               every maximum, minimum and arg-maximum is exact, so the
//               numbers do not depend on the launch shape.
//   k_mlp_*     a multilayer perceptron 24 -> 64 -> 64 -> 5 (ReLU) in
//               binary32: 4 logits for the factor precision (1..4 words)
//               and a regression of log2(1 + corrections); forward pass,
//               loss (cross-entropy + 0.5 Huber), backward pass with
//               per-parameter batch sums in sample order, Adam.
#include "common.hpp"
#include "mw.hpp"

namespace bnc {

constexpr int FNMAX = 512;  // largest order (workspace slots are FNMAX^2)
constexpr int NFEAT = 24;
constexpr int HAGER_STEPS = 3;
constexpr int FB = 8;       // LU panel width
constexpr double LG_CAP = 1100.0;

// FT threads per workgroup = the largest order it takes
template <int FT>
struct FeatLds {
    double y[FT];       // vector being solved
    double a[FT];       // per-row / per-column partials
    double b[FT];
    double c[FT];
    double d[FT];
    double e[FT];
    double rv[FT / 64]; // reduction scratch: one value per wave
    int ri[FT / 64];
    int ipiv[FT];
    double prow[FB], rowk[FB], rowp[FB];  // pivot row and the two swapped rows of a panel
    double ub[FB][FT];                    // the panel's rows of U12
    double bc[4];
    int s_i[4];
};

__device__ __forceinline__ double lg(double x)
{
    if (!(x > 0.0))
        return -LG_CAP;
    const double v = log2(x);
    return v > LG_CAP ? LG_CAP : (v < -LG_CAP ? -LG_CAP : v);
}

// exact maximum of the threads' values (every thread gets it): a
// butterfly inside each wave, then the four wave results in order
template <int FT>
__device__ double wg_max_exact(double v, FeatLds<FT> &S)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    if (lane == 0)
        S.rv[wave] = v;
    __syncthreads();
    double r = S.rv[0];
#pragma unroll
    for (int w = 1; w < FT / 64; ++w)
        r = fmax(r, S.rv[w]);
    __syncthreads();
    return r;
}

template <int FT>
__device__ double wg_min_exact(double v, FeatLds<FT> &S)
{
    return -wg_max_exact(-v, S);
}

// arg-maximum of key (ties: smallest index; keys < 0 never win)
template <int FT>
__device__ int wg_argmax(double key, FeatLds<FT> &S)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int idx = t;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double k2 = __shfl_xor(key, off, 64);
        const int i2 = __shfl_xor(idx, off, 64);
        if (k2 > key || (k2 == key && i2 < idx)) {
            key = k2;
            idx = i2;
        }
    }
    if (lane == 0) {
        S.rv[wave] = key;
        S.ri[wave] = idx;
    }
    __syncthreads();
    double bk = S.rv[0];
    int bi = S.ri[0];
#pragma unroll
    for (int w = 1; w < FT / 64; ++w)
        if (S.rv[w] > bk || (S.rv[w] == bk && S.ri[w] < bi)) {
            bk = S.rv[w];
            bi = S.ri[w];
        }
    __syncthreads();
    return bi;
}

// sum of p[0..n) in index order (thread 0), broadcast
template <int FT>
__device__ double seq_sum(const double *p, int n, FeatLds<FT> &S)
{
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i)
            s += p[i];
        S.bc[0] = s;
    }
    __syncthreads();
    const double r = S.bc[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double fms1(double c, double a, double b)
{
    double cc[1] = {c}, aa[1] = {a}, bb[1] = {b}, o[1];
    fms<1>(cc, aa, bb, o);
    return o[0];
}
__device__ __forceinline__ double mul1(double a, double b)
{
    double aa[1] = {a}, bb[1] = {b}, o[1];
    mul<1>(aa, bb, o);
    return o[0];
}
__device__ __forceinline__ double recip1(double a)
{
    double aa[1] = {a}, o[1];
    recip<1>(aa, o);
    return o[0];
}

// S.y <- A^-1 S.y with the binary64 factors W (column-major n x n) and
// S.ipiv: swaps in order, forward substitution with the unit lower factor
// (increasing k), backward substitution x_k = y_k (1/u_kk) then
// y_i -= u_ik x_k (decreasing k)
constexpr int PF = 8;  // substitution steps whose factor entries are loaded together

template <int FT>
__device__ void lu_solve(const double *W, int n, FeatLds<FT> &S)
{
    const int t = threadIdx.x;
    if (t == 0)
        for (int k = 0; k < n; ++k) {
            const int p = S.ipiv[k];
            if (p != k) {
                const double tmp = S.y[k];
                S.y[k] = S.y[p];
                S.y[p] = tmp;
            }
        }
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += PF) {
        double l[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            l[q] = (k < n && t > k && t < n) ? W[(int64_t)k * n + t] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            if (k < n) {
                const double yk = S.y[k];
                if (t > k && t < n)
                    S.y[t] = fms1(S.y[t], l[q], yk);
                __syncthreads();
            }
        }
    }
    // every thread forms x_k from y_k; the finished x_k go to S.d so that
    // no thread overwrites y_k while another still reads it
    for (int k0 = n - 1; k0 >= 0; k0 -= PF) {
        double u[PF], d[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 - q;
            u[q] = (k >= 0 && t < k) ? W[(int64_t)k * n + t] : 0.0;
            d[q] = k >= 0 ? W[(int64_t)k * n + k] : 1.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 - q;
            if (k >= 0) {
                const double xk = mul1(S.y[k], recip1(d[q]));
                if (t < k)
                    S.y[t] = fms1(S.y[t], u[q], xk);
                else if (t == k)
                    S.d[t] = xk;
                __syncthreads();
            }
        }
    }
    if (t < n)
        S.y[t] = S.d[t];
    __syncthreads();
}

// S.y <- A^-T S.y: U^T w = c (forward: w_k = w_k (1/u_kk), then
// w_i -= u_ki w_k for i > k), L^T v = w (backward: v_i -= l_ki v_k for
// i < k), then the swaps undone in reverse order
template <int FT>
__device__ void lu_solve_t(const double *W, int n, FeatLds<FT> &S)
{
    const int t = threadIdx.x;
    for (int k0 = 0; k0 < n; k0 += PF) {
        double u[PF], d[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            u[q] = (k < n && t > k && t < n) ? W[(int64_t)t * n + k] : 0.0;
            d[q] = k < n ? W[(int64_t)k * n + k] : 1.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            if (k < n) {
                const double wk = mul1(S.y[k], recip1(d[q]));
                if (t > k && t < n)
                    S.y[t] = fms1(S.y[t], u[q], wk);
                else if (t == k)
                    S.d[t] = wk;
                __syncthreads();
            }
        }
    }
    if (t < n)
        S.y[t] = S.d[t];
    __syncthreads();
    for (int k0 = n - 1; k0 >= 0; k0 -= PF) {
        double l[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 - q;
            l[q] = (k >= 0 && t < k) ? W[(int64_t)t * n + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 - q;
            if (k >= 0) {
                const double vk = S.y[k];
                if (t < k)
                    S.y[t] = fms1(S.y[t], l[q], vk);
                __syncthreads();
            }
        }
    }
    if (t == 0)
        for (int k = n - 1; k >= 0; --k) {
            const int p = S.ipiv[k];
            if (p != k) {
                const double tmp = S.y[k];
                S.y[k] = S.y[p];
                S.y[p] = tmp;
            }
        }
    __syncthreads();
}

// Systems of order in (n_lo, FT] get their features here; a launch with
// n_lo = 0 writes zeros for orders outside 1..FT, a launch with n_lo > 0
// leaves every other system alone.
template <int FT>
__global__ void __launch_bounds__(FT)
    k_features(int64_t count, const int64_t *__restrict__ nn, const double *const *__restrict__ As,
               const double *const *__restrict__ bs, const int32_t *__restrict__ order, float *__restrict__ F,
               unsigned *__restrict__ queue, double *__restrict__ work, int64_t n_lo)
{
    __shared__ FeatLds<FT> S;
    const int t = threadIdx.x;
    double *W = work + (size_t)blockIdx.x * FNMAX * FNMAX;
    for (;;) {
        if (t == 0)
            S.s_i[0] = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t qi = S.s_i[0];
        __syncthreads();
        if (qi >= count)
            break;
        const int64_t sys = order ? order[qi] : qi;
        const int64_t n64 = nn[sys];
        float *out = F + sys * NFEAT;
        if (n_lo > 0 && (n64 <= n_lo || n64 > FT))
            continue;
        if (n64 < 1 || n64 > FT) {
            if (t < NFEAT)
                out[t] = 0.0f;
            continue;
        }
        const int n = (int)n64;
        const double *A = As[sys];
        const double *b = bs[sys];
        double f[NFEAT];
#pragma unroll
        for (int q = 0; q < NFEAT; ++q)
            f[q] = 0.0;

        // ---- statistics of A: thread t as row t and as column t
        double rowabs = 0.0, rowsq = 0.0, off = 0.0, colabs = 0.0, colsq = 0.0, symsq = 0.0, amax_t = 0.0;
        if (t < n) {
#pragma unroll 4
            for (int j = 0; j < n; ++j) {
                const double v = A[(int64_t)j * n + t];
                rowabs += fabs(v);
                rowsq += v * v;
                if (j != t)
                    off += fabs(v);
                amax_t = fmax(amax_t, fabs(v));
            }
#pragma unroll 4
            for (int i = 0; i < n; ++i) {
                const double v = A[(int64_t)t * n + i];
                const double d = v - A[(int64_t)i * n + t];
                colabs += fabs(v);
                colsq += v * v;
                symsq += d * d;
            }
        }
        const double diag = t < n ? fabs(A[(int64_t)t * n + t]) : 0.0;
        const double ratio = t < n ? (off > 0.0 ? diag / off : 0x1p100) : 0.0;
        S.a[t] = colsq;
        S.b[t] = symsq;
        S.c[t] = diag * diag;
        S.d[t] = ratio;
        S.e[t] = (t < n && ratio > 1.0) ? 1.0 : 0.0;
        __syncthreads();
        const double fro2 = seq_sum(S.a, n, S);
        const double sym2 = seq_sum(S.b, n, S);
        const double dg2 = seq_sum(S.c, n, S);
        const double rsum = seq_sum(S.d, n, S);
        const double ndom = seq_sum(S.e, n, S);
        const double norm1 = wg_max_exact(colabs, S);
        const double norminf = wg_max_exact(rowabs, S);
        const double amax = wg_max_exact(amax_t, S);
        const double rmin = wg_min_exact(t < n ? ratio : INFINITY, S);
        const double cmax = wg_max_exact(t < n ? colsq : 0.0, S), cmin = wg_min_exact(t < n ? colsq : INFINITY, S);
        const double wmax = wg_max_exact(t < n ? rowsq : 0.0, S), wmin = wg_min_exact(t < n ? rowsq : INFINITY, S);
        const double fro = sqrt(fro2);
        const double lfro = lg(fro);
        f[0] = lg((double)n);
        f[1] = lfro;
        f[2] = lg(norm1) - lfro;
        f[3] = lg(norminf) - lfro;
        f[4] = lg(amax) - lfro;
        f[5] = lg(rmin);
        f[6] = lg(rsum / n);
        f[7] = ndom / n;
        f[8] = 0.5 * lg(dg2) - lfro;
        f[9] = 0.5 * (lg(cmin) - lg(cmax));
        f[10] = 0.5 * (lg(wmin) - lg(wmax));
        f[11] = lg(sqrt(sym2) / fro);

        // ---- binary64 LU with partial pivoting in W, in panels of FB
        //      columns: every entry still sees its updates one by one in
        //      increasing k, as in the unblocked algorithm (row swaps
        //      commute with the updates)
        for (int e = t; e < n * n; e += FT)
            W[e] = A[e];
        __syncthreads();
        int info = 0;
        for (int j0 = 0; j0 < n; j0 += FB) {
            const int jb = n - j0 < FB ? n - j0 : FB;
            double pr[FB];  // row t of the panel
#pragma unroll
            for (int c = 0; c < FB; ++c)
                pr[c] = (t < n && c < jb) ? W[(int64_t)(j0 + c) * n + t] : 0.0;
            unsigned zmask = 0;
#pragma unroll
            for (int c = 0; c < FB; ++c) {
                if (c < jb) {
                    const int k = j0 + c;
                    const int p = wg_argmax((t >= k && t < n) ? fabs(pr[c]) : -1.0, S);
                    if (t == 0)
                        S.ipiv[k] = p;
                    if (p != k) {
                        if (t == p)
#pragma unroll
                            for (int q = 0; q < FB; ++q)
                                S.rowp[q] = pr[q];
                        if (t == k)
#pragma unroll
                            for (int q = 0; q < FB; ++q)
                                S.rowk[q] = pr[q];
                        __syncthreads();
                        if (t == p)
#pragma unroll
                            for (int q = 0; q < FB; ++q)
                                pr[q] = S.rowk[q];
                        if (t == k)
#pragma unroll
                            for (int q = 0; q < FB; ++q)
                                pr[q] = S.rowp[q];
                    }
                    if (t == k)
#pragma unroll
                        for (int q = 0; q < FB; ++q)
                            S.prow[q] = pr[q];
                    __syncthreads();
                    const double piv = S.prow[c];
                    if (piv == 0.0) {
                        zmask |= 1u << c;
                        if (info == 0)
                            info = k + 1;
                    } else if (t > k && t < n) {
                        pr[c] = mul1(pr[c], recip1(piv));
#pragma unroll
                        for (int q = c + 1; q < FB; ++q)
                            if (q < jb)
                                pr[q] = fms1(pr[q], pr[c], S.prow[q]);
                    }
                    __syncthreads();
                }
            }
#pragma unroll
            for (int c = 0; c < FB; ++c)
                if (t < n && c < jb)
                    W[(int64_t)(j0 + c) * n + t] = pr[c];
            // the panel's swaps on the other columns, in order
            for (int j = t; j < n; j += FT)
                if (j < j0 || j >= j0 + jb)
                    for (int c = 0; c < jb; ++c) {
                        const int k = j0 + c, p = S.ipiv[k];
                        if (p != k) {
                            const double tmp = W[(int64_t)j * n + k];
                            W[(int64_t)j * n + k] = W[(int64_t)j * n + p];
                            W[(int64_t)j * n + p] = tmp;
                        }
                    }
            __syncthreads();
            // U12: forward substitution with the panel's unit lower block;
            // the finished rows also go to LDS for the trailing update
            for (int j = j0 + jb + t; j < n; j += FT) {
                double u[FB];
#pragma unroll
                for (int c = 0; c < FB; ++c)
                    u[c] = c < jb ? W[(int64_t)j * n + j0 + c] : 0.0;
#pragma unroll
                for (int c = 0; c < FB; ++c)
                    if (c < jb && !((zmask >> c) & 1u))
#pragma unroll
                        for (int q = c + 1; q < FB; ++q)
                            if (q < jb)
                                u[q] = fms1(u[q], W[(int64_t)(j0 + c) * n + j0 + q], u[c]);
#pragma unroll
                for (int c = 0; c < FB; ++c)
                    if (c < jb) {
                        W[(int64_t)j * n + j0 + c] = u[c];
                        S.ub[c][j] = u[c];
                    }
            }
            __syncthreads();
            // trailing rows: a_tj -= l_tk u_kj for k = j0.. in order
            if (t >= j0 + jb && t < n) {
#pragma unroll 4
                for (int j = j0 + jb; j < n; ++j) {
                    double w = W[(int64_t)j * n + t];
#pragma unroll
                    for (int c = 0; c < FB; ++c)
                        if (c < jb && !((zmask >> c) & 1u))
                            w = fms1(w, pr[c], S.ub[c][j]);
                    W[(int64_t)j * n + t] = w;
                }
            }
            __syncthreads();
        }
        // U statistics: largest entry, spread of the diagonal
        double umax_t = 0.0;
        if (t < n)
            for (int i = 0; i <= t; ++i)
                umax_t = fmax(umax_t, fabs(W[(int64_t)t * n + i]));
        const double umax = wg_max_exact(umax_t, S);
        const double ud = t < n ? fabs(W[(int64_t)t * n + t]) : 0.0;
        const double udmax = wg_max_exact(ud, S);
        const double udmin = wg_min_exact(t < n ? ud : INFINITY, S);
        S.a[t] = t < n ? lg(ud) : 0.0;
        S.b[t] = (t < n && ud < 0x1p-26 * udmax) ? 1.0 : 0.0;
        __syncthreads();
        const double lgsum = seq_sum(S.a, n, S);
        const double ntiny = seq_sum(S.b, n, S);
        f[12] = lg(umax) - lg(amax);
        f[13] = lg(udmin) - lg(udmax);
        f[14] = lg(udmax) - lfro;
        f[15] = lgsum / n - lg(udmax);
        f[16] = ntiny / n;

        // ---- Hager's estimate of ||A^-1||_1 and the binary64 solve
        double est0 = 0x1p1000, est1 = 0x1p1000, est2 = 0x1p1000;
        int steps = 0;
        if (info) {
            f[20] = LG_CAP;
            f[21] = 0.0;
        } else {
            S.y[t] = t < n ? 1.0 / (double)n : 0.0;
            S.e[t] = S.y[t];  // x
            __syncthreads();
            int jprev = -1;
            for (int it = 0; it < HAGER_STEPS; ++it) {
                lu_solve(W, n, S);
                S.a[t] = t < n ? fabs(S.y[t]) : 0.0;
                __syncthreads();
                const double g = seq_sum(S.a, n, S);
                steps = it + 1;
                est0 = it == 0 ? g : est0;
                est1 = it <= 1 ? g : est1;
                est2 = g;
                const double xi = (t < n && S.y[t] < 0.0) ? -1.0 : 1.0;
                __syncthreads();
                S.y[t] = t < n ? xi : 0.0;
                __syncthreads();
                lu_solve_t(W, n, S);
                const int j = wg_argmax(t < n ? fabs(S.y[t]) : -1.0, S);
                double zx;
                if (jprev < 0) {
                    S.a[t] = t < n ? S.y[t] * S.e[t] : 0.0;
                    __syncthreads();
                    zx = seq_sum(S.a, n, S);
                } else {
                    zx = S.y[jprev];
                }
                const double zj = fabs(S.y[j]);
                __syncthreads();
                if (zj <= zx)
                    break;
                jprev = j;
                S.y[t] = (t == j) ? 1.0 : 0.0;
                S.e[t] = S.y[t];
                __syncthreads();
            }
            // (estimates after an early stop repeat the last one)
            // binary64 solution of A x = b (leading words) and its residual
            const double b0 = t < n ? b[t] : 0.0;
            S.y[t] = b0;
            __syncthreads();
            lu_solve(W, n, S);
            double r = b0;
            if (t < n)
                for (int j = 0; j < n; ++j)
                    r = r - A[(int64_t)j * n + t] * S.y[j];
            const double xmax = wg_max_exact(t < n ? fabs(S.y[t]) : 0.0, S);
            const double bmax = wg_max_exact(fabs(b0), S);
            const double rmax = wg_max_exact(t < n ? fabs(r) : 0.0, S);
            f[20] = lg(xmax) - lg(bmax) + lg(norminf);
            f[21] = lg(rmax) - lg(norminf) - lg(xmax);
        }
        f[17] = lg(norm1) + lg(est0);
        f[18] = lg(norm1) + lg(est1);
        f[19] = lg(norm1) + lg(est2);
        f[22] = (double)steps;
        f[23] = lg(wg_max_exact(diag, S)) - lg(amax);
        if (t == 0)
#pragma unroll
            for (int q = 0; q < NFEAT; ++q) {
                double v = f[q];
                v = v > LG_CAP ? LG_CAP : (v < -LG_CAP ? -LG_CAP : v);
                out[q] = (float)v;
            }
        __syncthreads();
    }
}

// workspace: the queue counter (256 bytes), then one n x n matrix per slot
size_t features_workspace_bytes(int slots) { return 256 + (size_t)slots * FNMAX * FNMAX * sizeof(double); }

__global__ void k_feat_queue_reset(unsigned *q)
{
    if (threadIdx.x == 0)
        *q = 0u;
}

int features_default_slots()
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_features<256>, 256, 0) != hipSuccess ||
        per < 1)
        per = 1;
    return per * ncu;
}

int features_run(int64_t count, const int64_t *n, const double *const *A, const double *const *b,
                 const int32_t *order, float *F, void *work, int slots, hipStream_t s)
{
    if (count == 0)
        return BNC_OK;
    unsigned *queue = (unsigned *)work;
    double *ws = (double *)((char *)work + 256);
    const int64_t g = count < slots ? count : slots;
    // orders up to 256 (and zeros for the invalid ones), then 257..512
    hipLaunchKernelGGL(k_feat_queue_reset, dim3(1), dim3(64), 0, s, queue);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_features<256>, dim3((unsigned)g), dim3(256), 0, s, count, n, A, b, order, F, queue, ws,
                       (int64_t)0);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_feat_queue_reset, dim3(1), dim3(64), 0, s, queue);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_features<512>, dim3((unsigned)g), dim3(512), 0, s, count, n, A, b, order, F, queue, ws,
                       (int64_t)256);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

// ---------------------------------------------------------------------------
// MLP 24 -> 64 -> 64 -> 5 in binary32
// parameters, packed: W1[24][64] b1[64] W2[64][64] b2[64] W3[64][5] b3[5]
// (W[i][j]: input i -> output j); norm[48]: per-feature mean and 1/scale
// applied to the inputs first (not trained)
// ---------------------------------------------------------------------------
constexpr int MI = 24, MH = 64, MO = 5, MC = 4;
constexpr int OW1 = 0, OB1 = OW1 + MI * MH, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH, OB3 = OW3 + MH * MO,
              MLP_NPARAM = OB3 + MO;
constexpr float HUBER_W = 0.5f;

int mlp_param_count() { return MLP_NPARAM; }

// one thread per sample: hidden activations and outputs
__global__ void __launch_bounds__(64) k_mlp_fwd(int64_t B, const float *__restrict__ X, const float *__restrict__ norm,
                          const float *__restrict__ P, float *__restrict__ H1, float *__restrict__ H2,
                          float *__restrict__ O)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B)
        return;
    float x[MI], h1[MH], h2[MH];
#pragma unroll
    for (int i = 0; i < MI; ++i)
        x[i] = (X[s * MI + i] - norm[i]) * norm[MI + i];
#pragma unroll
    for (int j = 0; j < MH; ++j) {
        float a = P[OB1 + j];
#pragma unroll
        for (int i = 0; i < MI; ++i)
            a = fmaf(x[i], P[OW1 + i * MH + j], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < MH; ++j) {
        float a = P[OB2 + j];
#pragma unroll
        for (int i = 0; i < MH; ++i)
            a = fmaf(h1[i], P[OW2 + i * MH + j], a);
        h2[j] = a > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < MO; ++j) {
        float a = P[OB3 + j];
#pragma unroll
        for (int i = 0; i < MH; ++i)
            a = fmaf(h2[i], P[OW3 + i * MO + j], a);
        O[s * MO + j] = a;
    }
    if (H1)
#pragma unroll
        for (int j = 0; j < MH; ++j) {
            H1[s * MH + j] = h1[j];
            H2[s * MH + j] = h2[j];
        }
}

// one thread per sample: loss, output gradient and the back-propagated
// deltas of both hidden layers (already masked by the ReLU)
__global__ void __launch_bounds__(64) k_mlp_delta(int64_t B, const float *__restrict__ P, const float *__restrict__ H1,
                            const float *__restrict__ H2, const float *__restrict__ O, const int32_t *__restrict__ cls,
                            const float *__restrict__ tgt, float *__restrict__ DO, float *__restrict__ D2,
                            float *__restrict__ D1, float *__restrict__ L)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B)
        return;
    const float inv = 1.0f / (float)B;
    float o[MO], dout[MO];
#pragma unroll
    for (int j = 0; j < MO; ++j)
        o[j] = O[s * MO + j];
    float m = o[0];
#pragma unroll
    for (int j = 1; j < MC; ++j)
        m = fmaxf(m, o[j]);
    float z = 0.0f, e[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) {
        e[j] = expf(o[j] - m);
        z += e[j];
    }
    const int c = cls[s];
    float loss = logf(z) + m - o[c];
#pragma unroll
    for (int j = 0; j < MC; ++j)
        dout[j] = (e[j] / z - (j == c ? 1.0f : 0.0f)) * inv;
    const float d = o[MC] - tgt[s];
    const float ad = fabsf(d);
    loss += HUBER_W * (ad <= 1.0f ? 0.5f * d * d : ad - 0.5f);
    dout[MC] = HUBER_W * (ad <= 1.0f ? d : (d > 0.0f ? 1.0f : -1.0f)) * inv;
    L[s] = loss;
#pragma unroll
    for (int j = 0; j < MO; ++j)
        DO[s * MO + j] = dout[j];
    float d2[MH];
#pragma unroll
    for (int i = 0; i < MH; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < MO; ++j)
            a = fmaf(P[OW3 + i * MO + j], dout[j], a);
        d2[i] = H2[s * MH + i] > 0.0f ? a : 0.0f;
        D2[s * MH + i] = d2[i];
    }
#pragma unroll
    for (int i = 0; i < MH; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < MH; ++j)
            a = fmaf(P[OW2 + i * MH + j], d2[j], a);
        D1[s * MH + i] = H1[s * MH + i] > 0.0f ? a : 0.0f;
    }
}

// one thread per parameter: batch sums in sample order
__global__ void k_mlp_grad(int64_t B, const float *__restrict__ X, const float *__restrict__ norm,
                           const float *__restrict__ H1, const float *__restrict__ H2, const float *__restrict__ DO,
                           const float *__restrict__ D2, const float *__restrict__ D1, float *__restrict__ G)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM)
        return;
    float g = 0.0f;
    if (p < OB1) {
        const int i = (p - OW1) / MH, j = (p - OW1) % MH;
        for (int64_t s = 0; s < B; ++s)
            g = fmaf((X[s * MI + i] - norm[i]) * norm[MI + i], D1[s * MH + j], g);
    } else if (p < OW2) {
        const int j = p - OB1;
        for (int64_t s = 0; s < B; ++s)
            g += D1[s * MH + j];
    } else if (p < OB2) {
        const int i = (p - OW2) / MH, j = (p - OW2) % MH;
        for (int64_t s = 0; s < B; ++s)
            g = fmaf(H1[s * MH + i], D2[s * MH + j], g);
    } else if (p < OW3) {
        const int j = p - OB2;
        for (int64_t s = 0; s < B; ++s)
            g += D2[s * MH + j];
    } else if (p < OB3) {
        const int i = (p - OW3) / MO, j = (p - OW3) % MO;
        for (int64_t s = 0; s < B; ++s)
            g = fmaf(H2[s * MH + i], DO[s * MO + j], g);
    } else {
        const int j = p - OB3;
        for (int64_t s = 0; s < B; ++s)
            g += DO[s * MO + j];
    }
    G[p] = g;
}

__global__ void k_sum_f32(int64_t B, const float *__restrict__ v, float *__restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int64_t i = 0; i < B; ++i)
            s += v[i];
        *out = s / (float)B;
    }
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ M, float *__restrict__ V,
                       float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM)
        return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

size_t mlp_workspace_bytes(int64_t B)
{
    // H1, H2, D2, D1 (B x 64), O, DO (B x 5), per-sample loss
    return (size_t)B * (4 * MH + 2 * MO + 1) * sizeof(float);
}

int mlp_forward_run(int64_t B, const float *X, const float *norm, const float *P, float *O, hipStream_t s)
{
    if (B == 0)
        return BNC_OK;
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, s, B, X, norm, P, (float *)nullptr,
                       (float *)nullptr, O);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

int mlp_grad_run(int64_t B, const float *X, const float *norm, const int32_t *cls, const float *tgt, const float *P,
                 float *G, float *loss, void *work, hipStream_t s)
{
    float *H1 = (float *)work, *H2 = H1 + B * MH, *D2 = H2 + B * MH, *D1 = D2 + B * MH, *O = D1 + B * MH,
          *DO = O + B * MO, *L = DO + B * MO;
    const unsigned gs = (unsigned)ceil_div(B, 64);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(gs), dim3(64), 0, s, B, X, norm, P, H1, H2, O);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mlp_delta, dim3(gs), dim3(64), 0, s, B, P, H1, H2, (const float *)O, cls, tgt, DO, D2, D1,
                       L);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)ceil_div(MLP_NPARAM, 64)), dim3(64), 0, s, B, X, norm,
                       (const float *)H1, (const float *)H2, (const float *)DO, (const float *)D2, (const float *)D1,
                       G);
    BNC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(64), 0, s, B, (const float *)L, loss);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

int mlp_adam_run(float *P, const float *G, float *M, float *V, float lr, float b1, float b2, float eps, int64_t step,
                 hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)ceil_div(MLP_NPARAM, 64)), dim3(64), 0, s, P, G, M, V, lr, b1, b2, eps,
                       c1, c2);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

}  // namespace bnc

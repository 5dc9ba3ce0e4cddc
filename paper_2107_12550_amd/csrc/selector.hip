// Learned choice of the factor precision (not in the paper; the project's
// addition on top of its mixed-precision refinement, Sec. 2 / Listing 1).
//
//   k_features  24 cheap binary64 features of each system (order <= 256):
//               norms and their ratios, diagonal dominance, symmetry, a
//               binary64 LU with partial pivoting (pivot growth, spread of
//               U's diagonal), three steps of Hager's 1-norm estimate of
//               ||A^-1||_1 (Hager 1984; Higham 1988) from solves with A and
//               A^T, and the binary64 solution of A x = b (its size and
//               backward error).  One workgroup per system, thread t owns
//               row t; every sum runs in index order on one thread and
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

constexpr int FT = 256;     // threads per workgroup
constexpr int FNMAX = 256;  // largest order
constexpr int NFEAT = 24;
constexpr int HAGER_STEPS = 3;
constexpr double LG_CAP = 1100.0;

struct FeatLds {
    double y[FNMAX];    // vector being solved
    double a[FNMAX];    // per-row / per-column partials
    double b[FNMAX];
    double c[FNMAX];
    double d[FNMAX];
    double e[FNMAX];
    double rv[FT];      // reduction scratch (values)
    int ri[FT];         // reduction scratch (indices)
    int ipiv[FNMAX];
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

// exact maximum over v[0..n) of the threads' values (n <= FT); every thread
// gets it
__device__ double wg_max_exact(double v, FeatLds &S)
{
    const int t = threadIdx.x;
    S.rv[t] = v;
    __syncthreads();
    for (int off = FT / 2; off > 0; off >>= 1) {
        if (t < off)
            S.rv[t] = fmax(S.rv[t], S.rv[t + off]);
        __syncthreads();
    }
    const double r = S.rv[0];
    __syncthreads();
    return r;
}

__device__ double wg_min_exact(double v, FeatLds &S)
{
    return -wg_max_exact(-v, S);
}

// arg-maximum of key (ties: smallest index; keys < 0 never win)
__device__ int wg_argmax(double key, FeatLds &S)
{
    const int t = threadIdx.x;
    S.rv[t] = key;
    S.ri[t] = t;
    __syncthreads();
    for (int off = FT / 2; off > 0; off >>= 1) {
        if (t < off) {
            const double k2 = S.rv[t + off];
            const int i2 = S.ri[t + off];
            if (k2 > S.rv[t] || (k2 == S.rv[t] && i2 < S.ri[t])) {
                S.rv[t] = k2;
                S.ri[t] = i2;
            }
        }
        __syncthreads();
    }
    const int r = S.ri[0];
    __syncthreads();
    return r;
}

// sum of p[0..n) in index order (thread 0), broadcast
__device__ double seq_sum(const double *p, int n, FeatLds &S)
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
__device__ void lu_solve(const double *W, int n, FeatLds &S)
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
    for (int k = 0; k < n; ++k) {
        const double yk = S.y[k];
        if (t > k && t < n)
            S.y[t] = fms1(S.y[t], W[(int64_t)k * n + t], yk);
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        if (t == 0)
            S.y[k] = mul1(S.y[k], recip1(W[(int64_t)k * n + k]));
        __syncthreads();
        const double xk = S.y[k];
        if (t < k)
            S.y[t] = fms1(S.y[t], W[(int64_t)k * n + t], xk);
        __syncthreads();
    }
}

// S.y <- A^-T S.y: U^T w = c (forward: w_k = w_k (1/u_kk), then
// w_i -= u_ki w_k for i > k), L^T v = w (backward: v_i -= l_ki v_k for
// i < k), then the swaps undone in reverse order
__device__ void lu_solve_t(const double *W, int n, FeatLds &S)
{
    const int t = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        if (t == 0)
            S.y[k] = mul1(S.y[k], recip1(W[(int64_t)k * n + k]));
        __syncthreads();
        const double wk = S.y[k];
        if (t > k && t < n)
            S.y[t] = fms1(S.y[t], W[(int64_t)t * n + k], wk);
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const double vk = S.y[k];
        if (t < k)
            S.y[t] = fms1(S.y[t], W[(int64_t)t * n + k], vk);
        __syncthreads();
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

__global__ void __launch_bounds__(FT)
    k_features(int64_t count, const int64_t *__restrict__ nn, const double *const *__restrict__ As,
               const double *const *__restrict__ bs, float *__restrict__ F, double *__restrict__ work)
{
    __shared__ FeatLds S;
    const int t = threadIdx.x;
    double *W = work + (size_t)blockIdx.x * FNMAX * FNMAX;
    for (int64_t sys = blockIdx.x; sys < count; sys += gridDim.x) {
        const int64_t n64 = nn[sys];
        float *out = F + sys * NFEAT;
        if (n64 < 1 || n64 > FNMAX) {
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
            for (int j = 0; j < n; ++j) {
                const double v = A[(int64_t)j * n + t];
                rowabs += fabs(v);
                rowsq += v * v;
                if (j != t)
                    off += fabs(v);
                amax_t = fmax(amax_t, fabs(v));
            }
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

        // ---- binary64 LU with partial pivoting in W
        for (int e = t; e < n * n; e += FT)
            W[e] = A[e];
        __syncthreads();
        int info = 0;
        for (int k = 0; k < n; ++k) {
            const int p = wg_argmax((t >= k && t < n) ? fabs(W[(int64_t)k * n + t]) : -1.0, S);
            if (t == 0)
                S.ipiv[k] = p;
            if (p != k)
                for (int j = t; j < n; j += FT) {
                    const double tmp = W[(int64_t)j * n + k];
                    W[(int64_t)j * n + k] = W[(int64_t)j * n + p];
                    W[(int64_t)j * n + p] = tmp;
                }
            __syncthreads();
            const double piv = W[(int64_t)k * n + k];
            if (piv == 0.0) {
                if (info == 0)
                    info = k + 1;
                continue;
            }
            const double r = recip1(piv);
            if (t > k && t < n) {
                const double l = mul1(W[(int64_t)k * n + t], r);
                W[(int64_t)k * n + t] = l;
                for (int j = k + 1; j < n; ++j)
                    W[(int64_t)j * n + t] = fms1(W[(int64_t)j * n + t], l, W[(int64_t)j * n + k]);
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

size_t features_workspace_bytes(int slots) { return (size_t)slots * FNMAX * FNMAX * sizeof(double); }

int features_default_slots()
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return 2 * ncu;
}

int features_run(int64_t count, const int64_t *n, const double *const *A, const double *const *b, float *F,
                 void *work, int slots, hipStream_t s)
{
    if (count == 0)
        return BNC_OK;
    const int64_t g = count < slots ? count : slots;
    hipLaunchKernelGGL(k_features, dim3((unsigned)g), dim3(FT), 0, s, count, n, A, b, F, (double *)work);
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

// Forward/backward substitution with K-word LU factors (Kouya 2021, Sec. 2:
// the substitution step used for the first solution and every correction of
// Listing 1).
//
// The right-hand side is first gathered through the row permutation that
// the pivot sequence composes to (y = P b).  Each triangle is then solved
// in blocks of 64 rows: one launch per block updates every row beyond the
// block with the block's finished values (one thread per row, the block's
// columns in solve order), and the workgroup that owns the next block also
// finishes that block's triangle (lanes = rows, one broadcast per pivot).
// Per row the updates therefore arrive in increasing k for L and in
// decreasing k for U, exactly as in the unblocked column-oriented solve.
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
template <int K>
__device__ __forceinline__ void stage_block(const double *__restrict__ LU, int64_t lda, int64_t ldp, int64_t b0,
                                            int bsz, double *blk)
{
    const int lane = threadIdx.x;
    for (int c = 0; c < bsz; ++c) {
        if (lane < bsz) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                blk[(w * TS_BS + c) * TS_BS + lane] = LU[w * ldp + (b0 + c) * lda + b0 + lane];
        }
    }
}

// y_i <- y_i - sum over the columns k0..k0+bsz-1 (in the given direction)
// of t_ik y_k, operands fetched eight columns ahead of use
template <int K, bool DESC>
__device__ __forceinline__ void chain_update(const double *__restrict__ LU, int64_t lda, int64_t ldp, int64_t i,
                                             int64_t k0, int bsz, const double (*yb)[K], double (&v)[K])
{
    constexpr int G = 8;
    for (int g0 = 0; g0 < bsz; g0 += G) {
        double t[G][K];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int kk = DESC ? bsz - 1 - (g0 + q) : g0 + q;
            if (g0 + q < bsz) {
#pragma unroll
                for (int w = 0; w < K; ++w)
                    t[q][w] = LU[w * ldp + (k0 + kk) * lda + i];
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int kk = DESC ? bsz - 1 - (g0 + q) : g0 + q;
            if (g0 + q < bsz) {
                double yk[K], o[K];
#pragma unroll
                for (int w = 0; w < K; ++w)
                    yk[w] = yb[kk][w];
                fms<K>(v, t[q], yk, o);
#pragma unroll
                for (int w = 0; w < K; ++w)
                    v[w] = o[w];
            }
        }
    }
}

// ---- lower (unit) triangle -------------------------------------------------

// finish block [b0, b0+bsz) with the block staged in LDS:
// y_r <- y_r - l_rk y_k for k < r inside the block
template <int K>
__device__ __forceinline__ void lower_block(const double *blk, int bsz, double (&v)[K], double (*ub)[K])
{
    const int lane = threadIdx.x;
    for (int kk = 0; kk < bsz; ++kk) {
        if (lane == kk) {
#pragma unroll
            for (int w = 0; w < K; ++w)
                ub[0][w] = v[w];
        }
        __syncthreads();
        if (lane > kk && lane < bsz) {
            double l[K], yk[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w) {
                l[w] = blk[(w * TS_BS + kk) * TS_BS + lane];
                yk[w] = ub[0][w];
            }
            fms<K>(v, l, yk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = o[w];
        }
        __syncthreads();
    }
}

template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_lower_first(const double *__restrict__ LU, int64_t lda, int64_t ldp, double *__restrict__ y, int64_t ldy,
                  int64_t n)
{
    extern __shared__ double blk[];
    __shared__ double ub[1][K];
    const int lane = threadIdx.x;
    const int bsz = (int)(n < TS_BS ? n : TS_BS);
    stage_block<K>(LU, lda, ldp, 0, bsz, blk);
    double v[K];
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            v[w] = y[w * ldy + lane];
    }
    __syncthreads();
    lower_block<K>(blk, bsz, v, ub);
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            y[w * ldy + lane] = v[w];
    }
}

// rows beyond block [b0, b0+bsz) take that block's contribution; workgroup 0
// (rows [b0+bsz, b0+bsz+64)) then finishes its own block.
template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_lower_step(const double *__restrict__ LU, int64_t lda, int64_t ldp, double *__restrict__ y, int64_t ldy,
                 int64_t n, int64_t b0, int bsz)
{
    extern __shared__ double blk[];
    __shared__ double yb[TS_BS][K];
    __shared__ double ub[1][K];
    const int lane = threadIdx.x;
    const int64_t rb = b0 + bsz + (int64_t)blockIdx.x * TS_BS;  // first row of this workgroup
    const int nsz = (int)((n - rb) < TS_BS ? (n - rb) : TS_BS);
    if (blockIdx.x == 0)
        stage_block<K>(LU, lda, ldp, rb, nsz, blk);
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            yb[lane][w] = y[w * ldy + b0 + lane];
    }
    __syncthreads();
    const int64_t i = rb + lane;
    double v[K];
    if (i < n) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            v[w] = y[w * ldy + i];
        chain_update<K, false>(LU, lda, ldp, i, b0, bsz, yb, v);
    }
    if (blockIdx.x == 0)
        lower_block<K>(blk, nsz, v, ub);
    if (i < n) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            y[w * ldy + i] = v[w];
    }
}

// ---- upper triangle --------------------------------------------------------

// finish block [b0, b0+bsz) staged in LDS: for k = bsz-1..0:
// x_k = y_k * r_k (r = 1/u_kk), then y_r <- y_r - u_rk x_k for r < k
template <int K>
__device__ __forceinline__ void upper_block(const double *blk, const double *__restrict__ rd, int64_t n, int64_t b0,
                                            int bsz, double (&v)[K], double (*ub)[K])
{
    const int lane = threadIdx.x;
    double rk[K];
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            rk[w] = rd[w * n + b0 + lane];
    }
    for (int kk = bsz - 1; kk >= 0; --kk) {
        if (lane == kk) {
            double xk[K];
            mul<K>(v, rk, xk);
#pragma unroll
            for (int w = 0; w < K; ++w) {
                v[w] = xk[w];
                ub[0][w] = xk[w];
            }
        }
        __syncthreads();
        if (lane < kk) {
            double u[K], xk[K], o[K];
#pragma unroll
            for (int w = 0; w < K; ++w) {
                u[w] = blk[(w * TS_BS + kk) * TS_BS + lane];
                xk[w] = ub[0][w];
            }
            fms<K>(v, u, xk, o);
#pragma unroll
            for (int w = 0; w < K; ++w)
                v[w] = o[w];
        }
        __syncthreads();
    }
}

template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_upper_first(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ rd, int64_t n,
                  double *__restrict__ y, int64_t ldy, int64_t b0, int bsz)
{
    extern __shared__ double blk[];
    __shared__ double ub[1][K];
    const int lane = threadIdx.x;
    stage_block<K>(LU, lda, ldp, b0, bsz, blk);
    double v[K];
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            v[w] = y[w * ldy + b0 + lane];
    }
    __syncthreads();
    upper_block<K>(blk, rd, n, b0, bsz, v, ub);
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            y[w * ldy + b0 + lane] = v[w];
    }
}

// rows above block [b0, b0+bsz) take its contribution (k decreasing);
// workgroup 0 (rows [b0-64, b0)) then finishes its own block.
template <int K>
__global__ void __launch_bounds__(TS_BS)
    k_upper_step(const double *__restrict__ LU, int64_t lda, int64_t ldp, const double *__restrict__ rd, int64_t n,
                 double *__restrict__ y, int64_t ldy, int64_t b0, int bsz)
{
    extern __shared__ double blk[];
    __shared__ double xb[TS_BS][K];
    __shared__ double ub[1][K];
    const int lane = threadIdx.x;
    const int64_t rb = b0 - (int64_t)(blockIdx.x + 1) * TS_BS;  // first row of this workgroup (b0 % 64 == 0)
    if (blockIdx.x == 0)
        stage_block<K>(LU, lda, ldp, rb, TS_BS, blk);
    if (lane < bsz) {
#pragma unroll
        for (int w = 0; w < K; ++w)
            xb[lane][w] = y[w * ldy + b0 + lane];
    }
    __syncthreads();
    const int64_t i = rb + lane;
    double v[K];
#pragma unroll
    for (int w = 0; w < K; ++w)
        v[w] = y[w * ldy + i];
    chain_update<K, true>(LU, lda, ldp, i, b0, bsz, xb, v);
    if (blockIdx.x == 0)
        upper_block<K>(blk, rd, n, rb, TS_BS, v, ub);
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
    if (hipFuncSetAttribute((const void *)k_lower_first<K>, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_lower_step<K>, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_upper_first<K>, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_upper_step<K>, hipFuncAttributeMaxDynamicSharedMemorySize, b) != hipSuccess)
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
template <int K>
int trsv_pair(int64_t n, const double *LU, int64_t lda, int64_t ldp, const double *rd, double *y, int64_t ldy,
              hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    allow_lds<K>();
    const size_t lds = block_lds<K>();
    const int64_t nblk = ceil_div(n, TS_BS);
    hipLaunchKernelGGL((k_lower_first<K>), dim3(1), dim3(TS_BS), lds, s, LU, lda, ldp, y, ldy, n);
    BNC_LAUNCH_CHECK();
    for (int64_t B = 0; B + 1 < nblk; ++B) {
        const int64_t b0 = B * TS_BS;
        const unsigned g = (unsigned)ceil_div(n - b0 - TS_BS, TS_BS);
        hipLaunchKernelGGL((k_lower_step<K>), dim3(g), dim3(TS_BS), lds, s, LU, lda, ldp, y, ldy, n, b0, TS_BS);
        BNC_LAUNCH_CHECK();
    }
    const int64_t last = (nblk - 1) * TS_BS;
    hipLaunchKernelGGL((k_upper_first<K>), dim3(1), dim3(TS_BS), lds, s, LU, lda, ldp, rd, n, y, ldy, last,
                       (int)(n - last));
    BNC_LAUNCH_CHECK();
    for (int64_t B = nblk - 1; B >= 1; --B) {
        const int64_t b0 = B * TS_BS;
        const int bsz = (int)((n - b0) < TS_BS ? (n - b0) : TS_BS);
        hipLaunchKernelGGL((k_upper_step<K>), dim3((unsigned)B), dim3(TS_BS), lds, s, LU, lda, ldp, rd, n, y, ldy,
                           b0, bsz);
        BNC_LAUNCH_CHECK();
    }
    return BNC_OK;
}

size_t getrs_scratch_bytes(int K, int64_t n)
{
    return (size_t)n * sizeof(int32_t) + 2 * (size_t)K * n * sizeof(double) + 512;
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
               const double *b, int64_t ldb, double *y, int64_t ldy, hipStream_t s)
{
    if (n == 0)
        return BNC_OK;
    hipLaunchKernelGGL((k_gather<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, perm, b, ldb, y, ldy);
    BNC_LAUNCH_CHECK();
    return trsv_pair<K>(n, LU, lda, ldp, rd, y, ldy, s);
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
    int rc = ipiv_to_perm(n, ipiv, perm, s);
    if (rc)
        return rc;
    if ((rc = diag_recip_run<K>(n, LU, lda, ldp, rd, s)))
        return rc;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *bc = B + c * ldb;
        rc = getrs_perm<K>(n, LU, lda, ldp, perm, rd, bc, ldpb, y, n, s);
        if (rc)
            return rc;
        hipLaunchKernelGGL((k_copy_vec<K>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, y, n, bc, ldpb);
        BNC_LAUNCH_CHECK();
    }
    return BNC_OK;
}

#define INST(K)                                                                                                     \
    template int getrs_perm<K>(int64_t, const double *, int64_t, int64_t, const int32_t *, const double *,          \
                               const double *, int64_t, double *, int64_t, hipStream_t);                            \
    template int diag_recip_run<K>(int64_t, const double *, int64_t, int64_t, double *, hipStream_t);               \
    template int getrs_run<K>(int64_t, int64_t, const double *, int64_t, int64_t, const int64_t *, double *,        \
                              int64_t, int64_t, void *, hipStream_t);
INST(1)
INST(2)
INST(3)
INST(4)
#undef INST

}  // namespace bnc

// Split (Ozaki) form of the blocked LU's trailing update on the FP64 matrix
// cores.  Not part of the paper's method: an alternative to the K-word
// multiply-subtract update of its LU (Sec. 2), after Ozaki, Ogita, Oishi and
// Rump, "Error-free transformations of matrix multiplication by using fast
// routines of matrix multiplication and its applications", Numer.
// Algorithms 59 (2012).
//
// For A22 <- A22 - L21 U12 with panel width kb <= 64:
//   * every row i of L21 gets the scale E_i (|l_ik| < 2^E_i for all k, from
//     the leading words) and is cut into S slices; slice q is the sum over
//     the words of what is left of l_ik, each word rounded to the nearest
//     multiple of 2^(E_i - (q+1) beta) (ties to even), beta = oz_beta(K, S)
//     bits (22 for a double-double factor with 5 slices, 21 for
//     triple-double with 5); columns of U12 likewise with scales F_j;
//   * the group sums acc_d = sum_{p+q=d} sum_k L_p(i,k) U_q(k,j), d < S, are
//     formed with v_mfma_f64_16x16x4.  Every product and every partial sum is
//     a multiple of 2^(E_i + F_j - (d+2) beta) below 2^53 of those units
//     (oz_beta is the widest width for which the kb (d+1) <= 64 S products
//     of group d, each bounded by the slices' sizes, stay below 2^53), so
//     each acc_d is exact whatever the order the matrix core adds in;
//   * a_ij <- (((a_ij - acc_0) - acc_1) ...) - acc_{S-1} in K-word addition,
//     in that order.
// Slices with p + q >= S are dropped: the factor is slightly less accurate
// than the K-word one and the refinement recovers the accuracy.  Because
// the group sums are exact, the result does not depend on the tiling, and
// it is bit for bit the same as a plain loop that forms them one by one.
// Exactness needs the grids in the normal binary64 range (rows and columns
// whose scale is above about 2^-700).
#include "common.hpp"
#include "mw.hpp"
#include "ozsplit.hpp"

namespace bnc {

constexpr int OZ_KB = 8;  // k values staged through LDS per step

typedef double d4 __attribute__((ext_vector_type(4)));

// Splitting of U12 columns (the rows of L21 are cut by the panel as it
// writes them back, the look-ahead columns by their triangular solve): a
// workgroup of 256 threads takes 64 columns, four threads per column each
// cutting a quarter of its kb <= 64 entries; the column's scale comes from
// the maximum over the four quarters.
constexpr int OZ_SPLIT_V = 64;  // columns per workgroup
constexpr int OZ_SPLIT_Q = 4;   // threads per column

// Columns c0..c0+nc-1 of the rows j0..j0+kb-1 -> SU[(q kb + k) ldsu + c].
template <int K>
__global__ void __launch_bounds__(OZ_SPLIT_V *OZ_SPLIT_Q)
    k_oz_split_cols(const double *__restrict__ A, int64_t lda, int64_t ldp, int64_t j0, int kb, int64_t c0,
                    int64_t nc, int s, double *__restrict__ SU, int64_t ldsu, int *__restrict__ ozlow)
{
    __shared__ double smax[OZ_SPLIT_Q][OZ_SPLIT_V];
    const int v = threadIdx.x % OZ_SPLIT_V, qt = threadIdx.x / OZ_SPLIT_V;
    const int64_t c = (int64_t)blockIdx.x * OZ_SPLIT_V + v;
    const int per = (kb + OZ_SPLIT_Q - 1) / OZ_SPLIT_Q;
    const int k0 = qt * per, k1 = (k0 + per) < kb ? (k0 + per) : kb;
    const double *a = A + (c0 + c) * lda + j0;
    double mx = 0.0;
    if (c < nc)
        for (int k = k0; k < k1; ++k)
            mx = fmax(mx, fabs(a[k]));
    smax[qt][v] = mx;
    __syncthreads();
    if (c >= nc)
        return;
#pragma unroll
    for (int t = 0; t < OZ_SPLIT_Q; ++t)
        mx = fmax(mx, smax[t][v]);
    const int F = oz_scale(mx);
    const int beta = oz_beta(K, s);
    if (qt == 0 && mx != 0.0 && F < oz_emin(K, s))  // below the exact range: info -3 at the end
        __hip_atomic_store(ozlow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int k = k0; k < k1; ++k) {
        double w4[K];
#pragma unroll
        for (int w = 0; w < K; ++w)
            w4[w] = a[w * ldp + k];
        oz_cut_store<K>(w4, F, s, beta, SU + (int64_t)k * ldsu + c, (int64_t)kb * ldsu);
    }
}

// C(i, j) = A[r0 + i, c0 + j] (i < m, j < nc) minus the group sums of
// SL (rows, i-indexed from r0) and SU (columns, j-indexed from c0).
// Workgroup: WM x WN waves, each FI x FJ blocks of 16 x 16 outputs; the
// matrix core computes the transposed block D(j, i) = sum_k U(k, j) L(i, k)
// so that each output register holds 16 consecutive rows of one column.
template <int K, int S, int WM, int WN, int FI, int FJ>
__global__ void __launch_bounds__(64 * WM * WN)
    k_oz_update(double *__restrict__ A, int64_t lda, int64_t ldp, int64_t r0, int64_t c0, int64_t m, int64_t nc,
                int kb, const double *__restrict__ SL, int64_t ldsl, const double *__restrict__ SU, int64_t ldsu)
{
    constexpr int NT = 64 * WM * WN;
    constexpr int BM = WM * FI * 16, BN = WN * FJ * 16;
    extern __shared__ double oz_lds[];
    double *Ls = oz_lds;                  // [S][OZ_KB][BM]
    double *Us = oz_lds + S * OZ_KB * BM;  // [S][OZ_KB][BN]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi0 = (wave % WM) * FI * 16, wj0 = (wave / WM) * FJ * 16;
    const int64_t bi0 = (int64_t)blockIdx.x * BM, bj0 = (int64_t)blockIdx.y * BN;

    d4 acc[S][FI][FJ];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int a = 0; a < FI; ++a)
#pragma unroll
            for (int b = 0; b < FJ; ++b)
                acc[d][a][b] = d4{0.0, 0.0, 0.0, 0.0};

    // the next chunk's slices are fetched into registers while the current
    // one is multiplied out of LDS
    constexpr int NL = (S * OZ_KB * BM + NT - 1) / NT, NU = (S * OZ_KB * BN + NT - 1) / NT;
    double lr[NL], ur[NU];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int v = 0; v < NL; ++v) {
            const int t = tid + v * NT;
            const int i = t % BM, k = (t / BM) % OZ_KB, q = t / (BM * OZ_KB);
            const int64_t row = bi0 + i;
            const int kk = kc + k;
            lr[v] = (t < S * OZ_KB * BM && row < m && kk < kb) ? SL[((int64_t)q * kb + kk) * ldsl + row] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < NU; ++v) {
            const int t = tid + v * NT;
            const int j = t % BN, k = (t / BN) % OZ_KB, q = t / (BN * OZ_KB);
            const int64_t col = bj0 + j;
            const int kk = kc + k;
            ur[v] = (t < S * OZ_KB * BN && col < nc && kk < kb) ? SU[((int64_t)q * kb + kk) * ldsu + col] : 0.0;
        }
    };
    fetch(0);
    for (int kc = 0; kc < kb; kc += OZ_KB) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NL; ++v)
            if (tid + v * NT < S * OZ_KB * BM)
                Ls[tid + v * NT] = lr[v];
#pragma unroll
        for (int v = 0; v < NU; ++v)
            if (tid + v * NT < S * OZ_KB * BN)
                Us[tid + v * NT] = ur[v];
        __syncthreads();
        if (kc + OZ_KB < kb)
            fetch(kc + OZ_KB);
#pragma unroll 1
        for (int ks = 0; ks < OZ_KB; ks += 4) {
            const int kr = ks + (lane >> 4);
            double lf[S][FI], uf[S][FJ];
#pragma unroll
            for (int q = 0; q < S; ++q) {
#pragma unroll
                for (int a = 0; a < FI; ++a)
                    lf[q][a] = Ls[(q * OZ_KB + kr) * BM + wi0 + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < FJ; ++b)
                    uf[q][b] = Us[(q * OZ_KB + kr) * BN + wj0 + b * 16 + (lane & 15)];
            }
#pragma unroll
            for (int d = 0; d < S; ++d)
#pragma unroll
                for (int p = 0; p <= d; ++p)
#pragma unroll
                    for (int a = 0; a < FI; ++a)
#pragma unroll
                        for (int b = 0; b < FJ; ++b)
                            acc[d][a][b] =
                                __builtin_amdgcn_mfma_f64_16x16x4f64(uf[d - p][b], lf[p][a], acc[d][a][b], 0, 0, 0);
        }
    }

    // epilogue: lane holds rows (lane & 15), columns 4 v + (lane >> 4)
#pragma unroll
    for (int a = 0; a < FI; ++a)
#pragma unroll
        for (int b = 0; b < FJ; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = bi0 + wi0 + a * 16 + (lane & 15);
                const int64_t col = bj0 + wj0 + b * 16 + 4 * v + (lane >> 4);
                if (row < m && col < nc) {
                    double *p = A + (c0 + col) * lda + r0 + row;
                    double c[K];
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        c[w] = p[w * ldp];
#pragma unroll
                    for (int d = 0; d < S; ++d) {
                        double g[K], o[K];
                        g[0] = -acc[d][a][b][v];
#pragma unroll
                        for (int w = 1; w < K; ++w)
                            g[w] = 0.0;
                        add<K>(c, g, o);
#pragma unroll
                        for (int w = 0; w < K; ++w)
                            c[w] = o[w];
                    }
#pragma unroll
                    for (int w = 0; w < K; ++w)
                        p[w * ldp] = c[w];
                }
            }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

size_t oz_slices_bytes(int64_t n)
{
    // two SL (the current panel's and the next one's) and SU, OZ_SMAX
    // slices of a 64-wide panel, n rows/columns each
    return 3ull * OZ_SMAX * PANEL_NB_MAX * (size_t)(n > 0 ? n : 1) * sizeof(double);
}

template <int K>
int oz_split_cols_run(const double *A, int64_t lda, int64_t ldp, int64_t j0, int kb, int64_t c0, int64_t nc, int s,
                      double *SU, int64_t ldsu, int *ozlow, hipStream_t st)
{
    if (nc <= 0)
        return BNC_OK;
    hipLaunchKernelGGL(k_oz_split_cols<K>, dim3((unsigned)ceil_div(nc, OZ_SPLIT_V)), dim3(OZ_SPLIT_V * OZ_SPLIT_Q), 0,
                       st, A, lda, ldp, j0, kb, c0, nc, s, SU, ldsu, ozlow);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

template <int K, int S, int WM, int WN, int FI, int FJ>
static int oz_update_launch(double *A, int64_t lda, int64_t ldp, int64_t r0, int64_t c0, int64_t m, int64_t nc,
                            int kb, const double *SL, int64_t ldsl, const double *SU, int64_t ldsu, hipStream_t st)
{
    constexpr int BM = WM * FI * 16, BN = WN * FJ * 16;
    const size_t lds = (size_t)S * OZ_KB * (BM + BN) * sizeof(double);
    void *fn = (void *)k_oz_update<K, S, WM, WN, FI, FJ>;
    if (lds > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail_arg(BNC_ERR_UNSUPPORTED, "ozaki update: LDS tile too large");
    dim3 grid((unsigned)ceil_div(m, BM), (unsigned)ceil_div(nc, BN));
    hipLaunchKernelGGL((k_oz_update<K, S, WM, WN, FI, FJ>), grid, dim3(64 * WM * WN), lds, st, A, lda, ldp, r0, c0, m,
                       nc, kb, SL, ldsl, SU, ldsu);
    BNC_LAUNCH_CHECK();
    return BNC_OK;
}

template <int K, int S>
static int oz_update_s(bool thin, double *A, int64_t lda, int64_t ldp, int64_t r0, int64_t c0, int64_t m, int64_t nc,
                       int kb, const double *SL, int64_t ldsl, const double *SU, int64_t ldsu, hipStream_t st)
{
    // 8 waves of one 16 x 16 block each (32 x 64 outputs per workgroup):
    // 46.7 TFLOP/s of slice products on a 4032^2 x 64 triple-double update
    // with 8 slices, against 24.3 for 4 waves of 32 x 16; the look-ahead
    // columns (64 of them) take 32 x 32 tiles for twice the workgroups
    if (thin)
        return oz_update_launch<K, S, 2, 2, 1, 1>(A, lda, ldp, r0, c0, m, nc, kb, SL, ldsl, SU, ldsu, st);
    return oz_update_launch<K, S, 2, 4, 1, 1>(A, lda, ldp, r0, c0, m, nc, kb, SL, ldsl, SU, ldsu, st);
}

// A[r0.., c0..] -= the split product of the sliced panel rows and columns.
template <int K>
int oz_update_run(int s, bool thin, double *A, int64_t lda, int64_t ldp, int64_t r0, int64_t c0, int64_t m,
                  int64_t nc, int kb, const double *SL, int64_t ldsl, const double *SU, int64_t ldsu, hipStream_t st)
{
    if (m <= 0 || nc <= 0)
        return BNC_OK;
    if (kb > PANEL_NB_MAX)
        return fail_arg(BNC_ERR_UNSUPPORTED, "ozaki update: panel wider than 64");
    switch (s) {
#define OZ_CASE(SS) \
    case SS:        \
        return oz_update_s<K, SS>(thin, A, lda, ldp, r0, c0, m, nc, kb, SL, ldsl, SU, ldsu, st);
        OZ_CASE(1)
        OZ_CASE(2)
        OZ_CASE(3)
        OZ_CASE(4)
        OZ_CASE(5)
        OZ_CASE(6)
        OZ_CASE(7)
        OZ_CASE(8)
        OZ_CASE(9)
        OZ_CASE(10)
        OZ_CASE(11)
        OZ_CASE(12)
#undef OZ_CASE
    default:
        return fail_arg(BNC_ERR_UNSUPPORTED, "ozaki update: slices outside 1..12");
    }
}

#define OZ_INST(K)                                                                                                   \
    template int oz_split_cols_run<K>(const double *, int64_t, int64_t, int64_t, int, int64_t, int64_t, int,        \
                                      double *, int64_t, int *, hipStream_t);                                       \
    template int oz_update_run<K>(int, bool, double *, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, int,   \
                                  const double *, int64_t, const double *, int64_t, hipStream_t);
OZ_INST(1)
OZ_INST(2)
OZ_INST(3)
OZ_INST(4)
#undef OZ_INST

}  // namespace bnc

// Shared host-side plumbing for the solver library: error reporting,
// workspace sizes, timing of the trailing-update launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/bnc.h"

namespace bnc {

// Record a HIP failure (readable through bnc_last_error) and return the code.
int fail_hip(hipError_t e, const char *what, const char *file, int line);
int fail_arg(int code, const char *msg);

#define BNC_HIP(x)                                                   \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess)                                        \
            return ::bnc::fail_hip(e_, #x, __FILE__, __LINE__);      \
    } while (0)

#define BNC_LAUNCH_CHECK() BNC_HIP(hipGetLastError())

// Every entry point works in memory the caller passes in: no call
// allocates.  Sub-buffers of a workspace start on 256-byte boundaries.
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Largest order bnc_getrs_noalloc accepts (its fixed device scratch holds
// the workspace of a quad-double solve of this order, about 2.1 MB).
constexpr int64_t GETRS_NOALLOC_NMAX = 16384;
int noalloc_scratch(void **ptr, size_t *bytes);

// Test hook: raise the abort flag of the bounded waits right after each
// factorisation (bit 0) or substitution (bit 1) has cleared it, so that every
// wait gives up at once and the timeout paths run (bnc_test_force_timeout).
int force_timeout_bits();

// Timing of trailing-update launches (hipEvents on the launch stream).
struct UpdateTimer {
    static bool enabled();
    // returns an event pair index or -1
    static int begin(hipStream_t s);
    static void end(int idx, hipStream_t s, double flops);
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// FP64 operations per K-word fused multiply-subtract c - a*b of the
// level-accumulation algorithm (a fused multiply-add counts 2): TwoProd 3,
// plain product 1, TwoSum 6, plain add 1, summed over the fixed term lists.
constexpr double fms_flops(int K)
{
    return K == 1 ? 2.0 : (K == 2 ? 27.0 : (K == 3 ? 75.0 : 158.0));
}

// Sizes of the getrf scratch (candidate rows, old pivot-position rows,
// per-panel row-permutation pairs).
constexpr int PANEL_NB_MAX = 64;
constexpr int PANEL_WG_MAX = 256;

// Split (Ozaki) trailing update: at most this many slices per operand.
constexpr int OZ_SMAX = 12;
size_t getrf_scratch_bytes(int K, int64_t n);
template <int K>
int gemm_run(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, int64_t ldpa, const double *B,
             int64_t ldb, int64_t ldpb, double *C, int64_t ldc, int64_t ldpc, hipStream_t s);

}  // namespace bnc

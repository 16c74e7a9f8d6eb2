// Cholesky factorization on the family: the recursive blocked factorization
// the paper names as future work (Sec. 6).  A = U^T U with U upper
// triangular, in the upper triangle of the row-major A (the layout of
// LAPACK's column-major lower factor); the strictly lower triangle is never
// read or written.  Recursive halving:
//
//   [A11 A12; . A22]:  U11 = chol(A11)
//                      U12 = U11^-T A12      (momms_trsm, op(T) = U11^T)
//                      A22 -= U12^T U12      (momms_syrk, upper, transposed)
//                      U22 = chol(A22)
//
// so the flops run as triangular solves and symmetric updates, which are
// themselves family products.  Diagonal blocks of at most 64 rows are
// factored by one workgroup in LDS (right-looking: pivot, scale the row,
// update the trailing triangle).  info: 0, or the 1-based row of the first
// pivot that is not positive (the factorization goes on with NaNs past it).
#include <hip/hip_runtime.h>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {
namespace chol {

constexpr int kBase = 64;

__global__ void k_set_zero(int* p) { *p = 0; }

// Thread (ty, tx) of a 16 x 16 grid owns the entries (ty + 16 p, tx + 16 q)
// of the 64 x 64 block, so no index arithmetic divides.
__global__ __launch_bounds__(256) void k_potrf_base(int s, double* A, int64_t lda, int64_t row0, int* info) {
    __shared__ double a[kBase][kBase + 1];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = ty + 16 * p, j = tx + 16 * q;
            a[i][j] = (i <= j && j < s) ? A[(int64_t)i * lda + j] : 0.0;
        }
    __syncthreads();
    // Step k updates the trailing triangle with the unscaled pivot row,
    // a_ij -= a_ki a_kj / a_kk, and scales row k - 1 (read by nobody in step
    // k): one barrier per step.  Thread 0 alone tracks the first bad pivot.
    int bad = 0;
    double dprev = 1.0;
    for (int k = 0; k <= s; ++k) {
        if (k > 0) {   // row k - 1 becomes u: u_kk = sqrt(d), u_kj = a_kj / sqrt(d)
            const double r = sqrt(dprev);
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = ty + 16 * p, j = tx + 16 * q;
                    if (i == k - 1 && j >= i) a[i][j] = j == i ? r : a[i][j] / r;
                }
        }
        if (k == s) break;
        const double d = a[k][k];
        if (tid == 0 && !(d > 0.0) && bad == 0) bad = k + 1;
        const double inv = 1.0 / d;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = ty + 16 * p, j = tx + 16 * q;
                if (i > k && i <= j) a[i][j] = fma(-a[k][i] * inv, a[k][j], a[i][j]);
            }
        dprev = d;
        __syncthreads();
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = ty + 16 * p, j = tx + 16 * q;
            if (i <= j && j < s) A[(int64_t)i * lda + j] = a[i][j];
        }
    if (tid == 0 && bad != 0 && info != nullptr) atomicCAS(info, 0, (int)(row0 + bad));
}

static inline int64_t split_point(int64_t s) {
    const int64_t h = ((s / 2 + kBase - 1) / kBase) * kBase;
    return h < s ? h : s - kBase;
}

static int rec(int64_t r0, int64_t s, double* A, int64_t lda, int* info, hipStream_t st) {
    if (s <= kBase) {
        hipLaunchKernelGGL(k_potrf_base, dim3(1), dim3(256), 0, st, (int)s, A + r0 * lda + r0, lda, r0, info);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    const int64_t h = split_point(s);
    int rc;
    if ((rc = rec(r0, h, A, lda, info, st)) != 0) return rc;
    double* A11 = A + r0 * lda + r0;
    double* A12 = A11 + h;
    double* A22 = A11 + h * lda + h;
    if ((rc = momms_trsm('U', 1, 'N', h, s - h, 1.0, A11, lda, A12, lda, st)) != 0) return rc;
    if ((rc = momms_syrk('U', 1, s - h, h, -1.0, A12, lda, 1.0, A22, lda, MOMMS_AUTO, st)) != 0) return rc;
    return rec(r0 + h, s - h, A, lda, info, st);
}

}  // namespace chol
}  // namespace momms

extern "C" {

int momms_potrf(int uplo, int64_t n, double* A, int64_t lda, int* info, momms_stream_t stream) {
    using namespace momms::chol;
    if (uplo != 'U') return -1;
    if (n < 0) return -2;
    if (n > 0 && A == nullptr) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > INT32_MAX - 1) return MOMMS_ERR_INFEASIBLE;   // info is a 32-bit row number
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (info != nullptr) {
        hipLaunchKernelGGL(k_set_zero, dim3(1), dim3(1), 0, st, info);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    if (n == 0) return 0;
    return rec(0, n, A, lda, info, st);
}

}  // extern "C"

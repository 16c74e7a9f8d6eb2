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
// factored by one wave with the block in registers (right-looking: publish
// the pivot row, scale it, update the trailing triangle).  info: 0, or the 1-based row of the first
// pivot that is not positive (the factorization goes on with NaNs past it).
#include <hip/hip_runtime.h>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {
namespace chol {

constexpr int kBase = 64;

__global__ void k_set_zero(int* p) { *p = 0; }

// One wave: lane j owns column j of the 64 x 64 block in registers (c[i] =
// a_ij; rows below the diagonal hold values that are never written back).
// Step k: every lane publishes its row-k entry to LDS, then with the pivot
// d = a_kk, r = sqrt(d), lane j forms u_kj = a_kj / r and subtracts
// u_ki u_kj (u_ki = a_ki / r from LDS) from its entries i > k.  An entry
// below the diagonal only ever meets values below the diagonal, so no
// masking is needed.  The padded block is the identity.
__global__ __launch_bounds__(64) void k_potrf_base(int s, double* A, int64_t lda, int64_t row0, int* info) {
    __shared__ double rowbuf[kBase];
    const int j = threadIdx.x;
    double c[kBase];
#pragma unroll
    for (int i = 0; i < kBase; ++i) c[i] = (i <= j && j < s) ? A[(int64_t)i * lda + j] : (i == j ? 1.0 : 0.0);
    int bad = 0;
#pragma clang loop unroll(full)
    for (int k = 0; k < kBase; ++k) {   // fully unrolled: c stays in registers
        rowbuf[j] = c[k];
        __syncthreads();
        const double d = rowbuf[k];
        if (j == 0 && k < s && !(d > 0.0) && bad == 0) bad = k + 1;
        const double r = sqrt(d), rinv = 1.0 / r;
        const double ukj = j == k ? r : c[k] * rinv;
#pragma clang loop unroll(full)
        for (int i0 = k + 1; i0 < kBase; i0 += 8) {   // eight rows at a time keep the loads bounded
            double ui[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < kBase) ui[u] = rowbuf[i0 + u];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < kBase) c[i0 + u] = fma(-(ui[u] * rinv), ukj, c[i0 + u]);
            __builtin_amdgcn_sched_barrier(0);
        }
        c[k] = ukj;
        __syncthreads();   // the next step rewrites rowbuf
    }
#pragma unroll
    for (int i = 0; i < kBase; ++i)
        if (i <= j && j < s) A[(int64_t)i * lda + j] = c[i];
    if (j == 0 && bad != 0 && info != nullptr) atomicCAS(info, 0, (int)(row0 + bad));
}

static inline int64_t split_point(int64_t s) {
    const int64_t h = ((s / 2 + kBase - 1) / kBase) * kBase;
    return h < s ? h : s - kBase;
}

static int rec(int64_t r0, int64_t s, double* A, int64_t lda, int* info, hipStream_t st) {
    if (s <= kBase) {
        hipLaunchKernelGGL(k_potrf_base, dim3(1), dim3(64), 0, st, (int)s, A + r0 * lda + r0, lda, r0, info);
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

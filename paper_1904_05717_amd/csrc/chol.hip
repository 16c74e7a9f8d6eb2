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
// themselves family products.  Diagonal blocks of at most 128 rows are
// factored by one workgroup with the block in registers (right-looking:
// publish the pivot row, scale it, update the trailing triangle).  info: 0, or the 1-based row of the first
// pivot that is not positive (the factorization goes on with NaNs past it).
#include <hip/hip_runtime.h>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {
namespace chol {

constexpr int kBase = 128;   // diagonal blocks factored by one kernel
constexpr int kLeaf = 64;    // the recursion still splits at multiples of 64

__global__ void k_set_zero(int* p) { *p = 0; }

// 1 / sqrt(d) from the hardware estimate and two Newton steps (each squares
// the relative error), and sqrt(d) = d / sqrt(d).
__device__ __forceinline__ void rsqrt_sqrt(double d, double& rinv, double& r) {
    double y = __builtin_amdgcn_rsq(d);
    double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    rinv = y;
    r = d * y;
}

// The update of one wave at pivot K: rows LO .. LO+R-1 of column J are in
// c[0 .. R-1].  u_kJ = a_kJ / sqrt(a_kk) (sqrt(a_kk) on the diagonal), and
// a_iJ -= a_ki u_kJ / sqrt(a_kk) for the rows i > K.  K is a constant once
// the caller's loop is unrolled, which keeps c in registers.
template <int LO, int R>
__device__ __forceinline__ void pivot_update(double (&c)[64], const double* row, int J, int K, int s, int& bad) {
    // every LDS read of the step first: the pivot, this lane's entry of row K
    // and the entries a_ki of the rows i > K this wave holds
    const double d = row[K], akj = row[J];
    double a[R];
#pragma unroll
    for (int i = 0; i < R; ++i)
        if (LO + i > K) a[i] = row[LO + i];
    if (K < s && !(d > 0.0) && bad == 0) bad = K + 1;
    double rinv, r;
    rsqrt_sqrt(d, rinv, r);
    const double ukj = J == K ? r : akj * rinv;
    if (K >= LO && K < LO + R) c[K - LO] = ukj;
    const double sc = ukj * rinv;
#pragma unroll
    for (int i = 0; i < R; ++i)
        if (LO + i > K) c[i] = fma(-a[i], sc, c[i]);
}

// A diagonal block of order s <= 128 factored by one workgroup of four waves,
// the block in registers: wave 0 holds rows 0..63 of columns 0..63, wave 1
// rows 0..63 of columns 64..127, waves 2 and 3 rows 64..95 and 96..127 of
// columns 64..127 (lane j owns one column).  Entries below the diagonal are
// carried along and never written back; the padded block is the identity.
// Row k is published by the wave that holds it, into one of two alternating
// row buffers, so one barrier per pivot suffices.
__global__ __launch_bounds__(256) void k_potrf_base(int s, double* A, int64_t lda, int64_t row0, int* info) {
    __shared__ double rowbuf[2][kBase];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int J = wave == 0 ? lane : 64 + lane;
    const int lo = wave < 2 ? 0 : (wave == 2 ? 64 : 96);
    const int nr = wave < 2 ? 64 : 32;
    double c[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int row = lo + i;
        const bool in = i < nr && row <= J && J < s;
        const double v = A[in ? (int64_t)row * lda + J : 0];
        c[i] = in ? v : (row == J ? 1.0 : 0.0);
    }
    int bad = 0;
#pragma clang loop unroll(full)
    for (int K = 0; K < kBase; ++K) {
        double* row = rowbuf[K & 1];
        if (K < 64) {
            if (wave < 2) row[J] = c[K];
        } else if (K < 96) {
            if (wave == 2) row[J] = c[K - 64];
        } else {
            if (wave == 3) row[J] = c[K - 96];
        }
        __syncthreads();
        if (wave < 2)
            pivot_update<0, 64>(c, row, J, K, s, bad);
        else if (wave == 2)
            pivot_update<64, 32>(c, row, J, K, s, bad);
        else
            pivot_update<96, 32>(c, row, J, K, s, bad);
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int row = lo + i;
        if (i < nr && row <= J && J < s) A[(int64_t)row * lda + J] = c[i];
    }
    if (threadIdx.x == 0 && bad != 0 && info != nullptr) atomicCAS(info, 0, (int)(row0 + bad));
}

static inline int64_t split_point(int64_t s) {   // s > kBase: a multiple of kLeaf in (0, s)
    const int64_t h = ((s / 2 + kLeaf - 1) / kLeaf) * kLeaf;
    return h < s ? h : s - kLeaf;
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

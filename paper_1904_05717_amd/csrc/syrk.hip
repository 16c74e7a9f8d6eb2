// Symmetric rank-k update on the register-resident members of the family:
// C := alpha op(A) op(A)^T + beta C on one triangle of the n x n matrix C,
// op(A) = A (n x k) or A^T (A stored k x n).  The paper names the other
// level-3 BLAS as the family's next target (Sec. 6); SYRK keeps the loop
// nests unchanged and only restricts the C tiles to one triangle:
//
//   * the T(T+1)/2 tiles of the triangle (T tile rows) are folded into a
//     ceil(T/2) x (T+1) rectangle: rectangle row r holds the lower tiles of
//     tile row r followed by those of tile row T-1-r, which together have
//     T+1 tiles.  The rectangle goes through the member's order (C0:
//     row-major; C3C0: grouped rows, each XCD taking a contiguous run), so
//     every XCD gets an equal share (an unfolded band of rows would give the
//     last XCD most of the triangle);
//   * both operands are A: op(A)^T is A read with the opposite transposition;
//   * a diagonal tile stores only its own triangle, so the other triangle of
//     C is never read or written (BLAS semantics).
#include <hip/hip_runtime.h>

#include <climits>

#include "../../include/momms.h"
#include "kernels_f64.hip"
#include "plan_internal.h"

namespace momms {
namespace syrk {

typedef TileCfg<128, 128, 16, 2, 2> Cfg128;
typedef TileCfg<64, 64, 16, 2, 2> Cfg64;

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// TRI = 1: lower triangle (row >= col), 2: upper.
template <class CF, bool TA, int TRI>
__global__ __launch_bounds__(CF::THREADS) __attribute__((amdgpu_waves_per_eu(CF::MT >= 128 ? 2 : 1)))
void k_syrk(int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda, double beta,
            double* __restrict__ C, int64_t ldc, int T, Sched s) {
    static_assert(CF::MT == CF::NT, "square tiles");
    __shared__ double As[2][CF::MT * CF::A_LD];
    __shared__ double Bs[2][CF::KS * CF::B_LD];
    int r, c;
    decode_tile(s, blockIdx.x, r, c);
    // unfold: rectangle (r, c) -> lower tile (tm, tn) of the T x T tile grid
    int tm, tn;
    if (c <= r) {
        tm = r;
        tn = c;
    } else {
        tm = T - 1 - r;
        tn = c - r - 1;
        if (tm <= r) return;   // the middle row of an odd T: the whole workgroup, no barrier pending
    }
    if (TRI == 2) {   // upper triangle: the transposed tile
        const int x = tm;
        tm = tn;
        tn = x;
    }
    const int64_t m0 = (int64_t)tm * CF::MT, n0 = (int64_t)tn * CF::NT;
    if (tm == tn)
        regc_tile<CF, TA, !TA, true, TRI>(N, N, 0, K, alpha, A, lda, A, lda, beta, C, ldc, m0, n0, tm, tn, As, Bs);
    else
        regc_tile<CF, TA, !TA, true, 0>(N, N, 0, K, alpha, A, lda, A, lda, beta, C, ldc, m0, n0, tm, tn, As, Bs);
}

template <class CF, bool TA>
static void launch_t(bool lower, int64_t n, int64_t k, double alpha, const double* A, int64_t lda, double beta,
                     double* C, int64_t ldc, int T, const Sched& s, hipStream_t st) {
    const dim3 grid((unsigned)(s.tiles_m * s.tiles_n));
    if (lower)
        hipLaunchKernelGGL((k_syrk<CF, TA, 1>), grid, dim3(CF::THREADS), 0, st, n, k, alpha, A, lda, beta, C, ldc, T,
                           s);
    else
        hipLaunchKernelGGL((k_syrk<CF, TA, 2>), grid, dim3(CF::THREADS), 0, st, n, k, alpha, A, lda, beta, C, ldc, T,
                           s);
}

}  // namespace syrk
}  // namespace momms

extern "C" {

int momms_syrk(int uplo, int trans, int64_t n, int64_t k, double alpha, const double* A, int64_t lda, double beta,
               double* C, int64_t ldc, int family_member, momms_stream_t stream) {
    using namespace momms;
    using namespace momms::syrk;
    if (uplo != 'L' && uplo != 'U') return -1;
    if (trans != 0 && trans != 1) return -2;
    if (n < 0) return -3;
    if (k < 0) return -4;
    const bool reads_a = alpha != 0.0 && k > 0 && n > 0;
    if (reads_a && A == nullptr) return -6;
    const int64_t contiguous = trans ? n : k;
    if (lda < (contiguous > 1 ? contiguous : 1)) return -7;
    if (n > 0 && C == nullptr) return -9;
    if (ldc < (n > 1 ? n : 1)) return -10;
    int member = family_member == MOMMS_AUTO ? MOMMS_C3C0 : family_member;
    if (member != MOMMS_C0 && member != MOMMS_C3C0) return -11;
    if (cdiv(n, 64) * cdiv(n, 64) >= (int64_t)INT_MAX / 2) return MOMMS_ERR_INFEASIBLE;
    if (n == 0) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;
    momms_plan p;
    if (plan_member(member, n, n, k, &p) != 0) return MOMMS_ERR_INTERNAL;
    const int t = p.mt;
    const int T = (int)cdiv(n, t);
    Sched s;
    s.m_off = 0;
    s.n_off = 0;
    s.m_lim = n;
    s.n_lim = n;
    s.tiles_m = (T + 1) / 2;   // the folded triangle
    s.tiles_n = T + 1;
    s.group_m = member == MOMMS_C3C0 ? (p.group_m < s.tiles_m ? p.group_m : s.tiles_m) : 1;
    if (s.group_m < 1) s.group_m = 1;
    s.xcd = member == MOMMS_C3C0 ? kXcds : 1;
    // alpha = 0 or k = 0: the kernel runs no k slices and only scales the
    // triangle by beta (beta = 0 writes zeros without reading C).
    const int64_t kk = alpha == 0.0 ? 0 : k;
    const bool lower = uplo == 'L';
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (t == 128) {
        if (trans) launch_t<Cfg128, true>(lower, n, kk, alpha, A, lda, beta, C, ldc, T, s, st);
        else       launch_t<Cfg128, false>(lower, n, kk, alpha, A, lda, beta, C, ldc, T, s, st);
    } else {
        if (trans) launch_t<Cfg64, true>(lower, n, kk, alpha, A, lda, beta, C, ldc, T, s, st);
        else       launch_t<Cfg64, false>(lower, n, kk, alpha, A, lda, beta, C, ldc, T, s, st);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"

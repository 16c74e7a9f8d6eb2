// Triangular multiply and solve on the family (the other level-3 BLAS are
// the paper's next target, Sec. 6):
//
//   momms_trmm: C := alpha op(T) B        (out of place)
//   momms_trsm: B := X with op(T) X = alpha B   (in place)
//
// T is the lower or upper triangle of the m x m matrix A (unit diagonal when
// asked, the diagonal of A then not read), op(T) = T or T^T, B and C are
// m x n, all row-major.  Both halve the triangle recursively, so nearly all
// flops run as large family products:
//
//   op(T) lower:  [T11 0; T21 T22]:  solve X1 with T11, B2 -= T21 X1 (product),
//                 solve X2 with T22;   multiply C1 = T11 B1, C2 = T22 B2,
//                 C2 += T21 B1 (product);
//   op(T) upper:  the mirror image (second block first for the solve).
//
// Diagonal blocks of at most 64 rows go to one kernel: a lane owns one column
// of B, held in LDS next to the block of op(T) (read by all lanes at one
// address); four waves share the rows of the triangular product, or run a
// blocked forward or backward substitution.
#include <hip/hip_runtime.h>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {
namespace tri {

constexpr int kBase = 64;   // rows of a diagonal block handled by the base kernel

// The 64 x 64 block of op(T) at op rows R0.., columns C0.. of the s x s
// triangle (A points at its first entry).  Stored entries are read with
// consecutive threads on consecutive stored columns b of a stored row a; the
// op entry is (i, j) = (a, b), or (b, a) when transposed.  Loads and LDS
// stores are split so a kernel can issue every load before it uses any: an
// entry outside the triangle or past s reads A[0] and is replaced by 0 (1 on
// the diagonal past s, and on the diagonal when UNIT).
struct OpBlock {
    int sa0, sb0;   // the stored block's first row and column
};

__device__ __forceinline__ OpBlock op_block_at(bool trans, int R0, int C0) {
    return trans ? OpBlock{C0, R0} : OpBlock{R0, C0};
}

template <bool UNIT>
__device__ __forceinline__ bool op_read(int ga, int gb, int s, bool upper_stored) {
    return ga < s && gb < s && (upper_stored ? ga <= gb : ga >= gb) && !(UNIT && ga == gb);
}

template <bool UNIT>
__device__ __forceinline__ void op_load(double (&tv)[16], const double* A, int64_t lda, int s, bool upper_stored,
                                        OpBlock blk, int tid) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q, ga = blk.sa0 + e / kBase, gb = blk.sb0 + e % kBase;
        tv[q] = A[op_read<UNIT>(ga, gb, s, upper_stored) ? (int64_t)ga * lda + gb : 0];
    }
}

template <bool UNIT>
__device__ __forceinline__ void op_store(double (*Ts)[kBase + 1], double* rdiag, const double (&tv)[16], int s,
                                         bool trans, bool upper_stored, OpBlock blk, int tid) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q, a = e / kBase, b = e % kBase, ga = blk.sa0 + a, gb = blk.sb0 + b;
        const int i = trans ? b : a, j = trans ? a : b;
        const double v = op_read<UNIT>(ga, gb, s, upper_stored) ? tv[q] : (ga == gb ? 1.0 : 0.0);
        Ts[i][j] = v;
        if (rdiag != nullptr && ga == gb) rdiag[i] = 1.0 / v;
    }
}

// Solve the 64-row block of op(T) in Ts (1 / diagonal in rdiag) against the
// 64 columns in xs, in place: four 16-row blocks in solve order.  Wave 0 works
// each 16-row block right-looking in registers (x_u = b_u / t_uu, then x_u is
// subtracted from the block's later rows, the next pivot's column of op(T)
// read from LDS one step ahead); then all four waves subtract the block from
// the rows still to solve.  Callers synchronize before; it ends synchronized.
template <bool LOWER, bool UNIT>
__device__ __forceinline__ void solve_block(const double (*Ts)[kBase + 1], const double* rdiag, double (*xs)[64],
                                            int lane, int wave) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int kb = LOWER ? q : 3 - q;   // block in solve order
        const int b0 = 16 * kb;
        if (wave == 0) {
            double xr[16], rd[16], tc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                xr[u] = xs[b0 + u][lane];
                rd[u] = rdiag[b0 + u];
            }
            {
                const int u = LOWER ? 0 : 15;
#pragma unroll
                for (int i = 0; i < 16; ++i) tc[i] = Ts[b0 + i][b0 + u];
            }
#pragma unroll
            for (int uu = 0; uu < 16; ++uu) {
                const int u = LOWER ? uu : 15 - uu;
                double tn[16];
                if (uu < 15) {
                    const int un = LOWER ? u + 1 : u - 1;
#pragma unroll
                    for (int i = 0; i < 16; ++i) tn[i] = Ts[b0 + i][b0 + un];
                }
                const double x = UNIT ? xr[u] : xr[u] * rd[u];
                xr[u] = x;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (LOWER ? i > u : i < u) xr[i] = fma(-tc[i], x, xr[i]);
                __builtin_amdgcn_sched_barrier(0);   // one pivot at a time: the loads stay one step ahead
                if (uu < 15)
#pragma unroll
                    for (int i = 0; i < 16; ++i) tc[i] = tn[i];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) xs[b0 + u][lane] = xr[u];
        }
        __syncthreads();
        // rows still to solve: after the block (lower) or before it (upper)
        double xb[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) xb[j] = xs[b0 + j][lane];
        const int r0 = LOWER ? b0 + 16 : 0, r1 = LOWER ? kBase : b0;
        for (int i = r0 + wave; i < r1; i += 4) {
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int j = 0; j < 16; j += 2) {
                d0 = fma(Ts[i][b0 + j], xb[j], d0);
                d1 = fma(Ts[i][b0 + j + 1], xb[j + 1], d1);
            }
            xs[i][lane] -= d0 + d1;
        }
        __syncthreads();
    }
}

// MODE 0: solve (x := op(T)^-1 x), 1: multiply (y := alpha op(T) x, written to Y).
// LOWER: op(T) is lower triangular.  A workgroup takes 64 columns with four
// waves; lane c owns column c, held at xs[i][c] (lanes read consecutive
// words).  Multiply: wave w forms rows 16w .. 16w+15, sixteen independent
// sums.  Solve: solve_block.  All 32 loads per thread (16 of op(T), 16 of
// x) are in flight before the first is used.
// The grid's y index picks the diagonal block: block q covers rows 64q ..
// of the `rows`-row triangle (a solve launches one block, the multiply all of
// them at once, since the diagonal products of a multiply are independent).
template <int MODE, bool LOWER, bool UNIT>
__global__ __launch_bounds__(256) void k_tri_base(int64_t rows, int64_t n, const double* __restrict__ A, int64_t lda,
                                                  bool trans, bool upper_stored, double alpha, double* X,
                                                  int64_t ldx, double* Y, int64_t ldy) {
    __shared__ double Ts[kBase][kBase + 1];
    __shared__ double xs[kBase][64];
    __shared__ double rdiag[kBase];   // 1 / t_ii: the substitution multiplies
    const int64_t r0 = (int64_t)blockIdx.y * kBase;
    A += r0 * lda + r0;
    X += r0 * ldx;
    if (MODE == 1) Y += r0 * ldy;
    const int s = (int)(rows - r0 < kBase ? rows - r0 : kBase);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const OpBlock blk = op_block_at(trans, 0, 0);
    double tv[16], xv[16];
    op_load<UNIT>(tv, A, lda, s, upper_stored, blk, tid);
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    const bool live = col < n;   // dead lanes work on zeros and store nothing
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = wave + 4 * q;
        xv[q] = X[(live && i < s) ? (int64_t)i * ldx + col : 0];
    }
    op_store<UNIT>(Ts, rdiag, tv, s, trans, upper_stored, blk, tid);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = wave + 4 * q;
        xs[i][lane] = (live && i < s) ? xv[q] : 0.0;
    }
    __syncthreads();
    if (MODE == 1) {
        double acc[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0;
        const int i0 = 16 * wave;
        // op(T) lower: row i uses j <= i; upper: j >= i.  Columns outside a
        // row's range hold zeros in Ts, so the loop bounds only trim work.
        const int j0 = LOWER ? 0 : i0, j1 = LOWER ? i0 + 16 : kBase;
        for (int j = j0; j < j1; ++j) {
            const double xj = xs[j][lane];
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = fma(Ts[i0 + r][j], xj, acc[r]);
        }
        if (live)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (i0 + r < s) Y[(int64_t)(i0 + r) * ldy + col] = alpha * acc[r];
        return;
    }
    solve_block<LOWER, UNIT>(Ts, rdiag, xs, lane, wave);
    if (live)
        for (int i = wave; i < s; i += 4) X[(int64_t)i * ldx + col] = xs[i][lane];
}

struct Tri {
    bool trans, upper_stored, unit, lower_op;
    const double* A;
    int64_t lda, n;
    hipStream_t st;
};

// Block (R0.., C0..) of op(A) as a product operand: pointer and trans flag.
static inline const double* op_block(const Tri& t, int64_t R0, int64_t C0, int* transA) {
    *transA = t.trans ? 1 : 0;
    return t.trans ? t.A + C0 * t.lda + R0 : t.A + R0 * t.lda + C0;
}

// Diagonal blocks of rows [r0, r0 + s): one block per launch row when s <= 64,
// or every 64-row block of the range at once (blocks > 1, multiply only).
template <int MODE>
static int launch_base(const Tri& t, int64_t r0, int64_t s, double alpha, double* X, int64_t ldx, double* Y,
                       int64_t ldy, unsigned blocks = 1) {
    const dim3 grid((unsigned)((t.n + 63) / 64), blocks);   // 64 columns per workgroup of 256 threads
    const double* Ab = t.A + r0 * t.lda + r0;
    if (t.lower_op) {
        if (t.unit)
            hipLaunchKernelGGL((k_tri_base<MODE, true, true>), grid, dim3(256), 0, t.st, s, t.n, Ab, t.lda,
                               t.trans, t.upper_stored, alpha, X, ldx, Y, ldy);
        else
            hipLaunchKernelGGL((k_tri_base<MODE, true, false>), grid, dim3(256), 0, t.st, s, t.n, Ab, t.lda,
                               t.trans, t.upper_stored, alpha, X, ldx, Y, ldy);
    } else {
        if (t.unit)
            hipLaunchKernelGGL((k_tri_base<MODE, false, true>), grid, dim3(256), 0, t.st, s, t.n, Ab, t.lda,
                               t.trans, t.upper_stored, alpha, X, ldx, Y, ldy);
        else
            hipLaunchKernelGGL((k_tri_base<MODE, false, false>), grid, dim3(256), 0, t.st, s, t.n, Ab, t.lda,
                               t.trans, t.upper_stored, alpha, X, ldx, Y, ldy);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

static inline int64_t split_point(int64_t s) {   // a multiple of kBase in (0, s)
    const int64_t h = ((s / 2 + kBase - 1) / kBase) * kBase;
    return h < s ? h : s - kBase;
}

// Solve op(T)[r0:r0+s, r0:r0+s] X = B[r0:r0+s] in place.
static int solve(const Tri& t, int64_t r0, int64_t s, double* B, int64_t ldb) {
    if (s <= kBase) return launch_base<0>(t, r0, s, 1.0, B + r0 * ldb, ldb, nullptr, 0);
    const int64_t h = split_point(s);
    int ta, rc;
    if (t.lower_op) {
        if ((rc = solve(t, r0, h, B, ldb)) != 0) return rc;
        const double* Ab = op_block(t, r0 + h, r0, &ta);
        if ((rc = momms_gemm_ex(ta, 0, s - h, t.n, h, -1.0, Ab, t.lda, B + r0 * ldb, ldb, 1.0, B + (r0 + h) * ldb,
                                ldb, MOMMS_AUTO, nullptr, 0, t.st)) != 0)
            return rc;
        return solve(t, r0 + h, s - h, B, ldb);
    }
    if ((rc = solve(t, r0 + h, s - h, B, ldb)) != 0) return rc;
    const double* Ab = op_block(t, r0, r0 + h, &ta);
    if ((rc = momms_gemm_ex(ta, 0, h, t.n, s - h, -1.0, Ab, t.lda, B + (r0 + h) * ldb, ldb, 1.0, B + r0 * ldb, ldb,
                            MOMMS_AUTO, nullptr, 0, t.st)) != 0)
        return rc;
    return solve(t, r0, h, B, ldb);
}

// C[r0:r0+s] = alpha op(T)[r0:r0+s, r0:r0+s] B[r0:r0+s].
// The off-diagonal products of the recursion, after every diagonal block has
// been written (leaves == false: the diagonal blocks were launched together).
static int multiply(const Tri& t, int64_t r0, int64_t s, double alpha, const double* B, int64_t ldb, double* C,
                    int64_t ldc, bool leaves) {
    if (s <= kBase)
        return leaves ? launch_base<1>(t, r0, s, alpha, const_cast<double*>(B) + r0 * ldb, ldb, C + r0 * ldc, ldc)
                      : 0;
    const int64_t h = split_point(s);
    int ta, rc;
    if ((rc = multiply(t, r0, h, alpha, B, ldb, C, ldc, leaves)) != 0) return rc;
    if ((rc = multiply(t, r0 + h, s - h, alpha, B, ldb, C, ldc, leaves)) != 0) return rc;
    if (t.lower_op) {   // C2 += alpha T21 B1
        const double* Ab = op_block(t, r0 + h, r0, &ta);
        return momms_gemm_ex(ta, 0, s - h, t.n, h, alpha, Ab, t.lda, B + r0 * ldb, ldb, 1.0, C + (r0 + h) * ldc,
                             ldc, MOMMS_AUTO, nullptr, 0, t.st);
    }
    const double* Ab = op_block(t, r0, r0 + h, &ta);   // C1 += alpha T12 B2
    return momms_gemm_ex(ta, 0, h, t.n, s - h, alpha, Ab, t.lda, B + (r0 + h) * ldb, ldb, 1.0, C + r0 * ldc, ldc,
                         MOMMS_AUTO, nullptr, 0, t.st);
}

static int check_common(int uplo, int trans, int diag, int64_t m, int64_t n, int64_t lda, int64_t ldb) {
    if (uplo != 'L' && uplo != 'U') return -1;
    if (trans != 0 && trans != 1) return -2;
    if (diag != 'N' && diag != 'U') return -3;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (lda < (m > 1 ? m : 1)) return -8;
    if (ldb < (n > 1 ? n : 1)) return -10;
    return 0;
}

}  // namespace tri
}  // namespace momms

extern "C" {

int momms_trmm(int uplo, int trans, int diag, int64_t m, int64_t n, double alpha, const double* A, int64_t lda,
               const double* B, int64_t ldb, double* C, int64_t ldc, momms_stream_t stream) {
    using namespace momms::tri;
    int rc = check_common(uplo, trans, diag, m, n, lda, ldb);
    if (rc != 0) return rc;
    const bool reads = alpha != 0.0 && m > 0 && n > 0;
    if (reads && A == nullptr) return -7;
    if (reads && B == nullptr) return -9;
    if (m > 0 && n > 0 && C == nullptr) return -11;
    if (ldc < (n > 1 ? n : 1)) return -12;
    if (m == 0 || n == 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (alpha == 0.0)   // C = 0, A and B not read
        return momms_gemm_ex(0, 0, m, n, 0, 0.0, nullptr, 1, nullptr, n, 0.0, C, ldc, MOMMS_AUTO, nullptr, 0, st);
    Tri t{trans != 0, uplo == 'U', diag == 'U', (uplo == 'L') != (trans != 0), A, lda, n, st};
    // The diagonal products are independent: all of them in one launch, then
    // the recursion's off-diagonal products add into C.
    const int64_t blocks = (m + kBase - 1) / kBase;
    if (blocks > 65535) return multiply(t, 0, m, alpha, B, ldb, C, ldc, true);
    rc = launch_base<1>(t, 0, m, alpha, const_cast<double*>(B), ldb, C, ldc, (unsigned)blocks);
    if (rc != 0) return rc;
    return multiply(t, 0, m, alpha, B, ldb, C, ldc, false);
}

int momms_trsm(int uplo, int trans, int diag, int64_t m, int64_t n, double alpha, const double* A, int64_t lda,
               double* B, int64_t ldb, momms_stream_t stream) {
    using namespace momms::tri;
    int rc = check_common(uplo, trans, diag, m, n, lda, ldb);
    if (rc != 0) return rc;
    if (alpha != 0.0 && m > 0 && n > 0 && A == nullptr) return -7;
    if (m > 0 && n > 0 && B == nullptr) return -9;
    if (m == 0 || n == 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (alpha != 1.0) {   // B = alpha B (alpha = 0: B = 0 and A is not read)
        rc = momms_gemm_ex(0, 0, m, n, 0, 0.0, nullptr, 1, nullptr, n, alpha, B, ldb, MOMMS_AUTO, nullptr, 0, st);
        if (rc != 0 || alpha == 0.0) return rc;
    }
    Tri t{trans != 0, uplo == 'U', diag == 'U', (uplo == 'L') != (trans != 0), A, lda, n, st};
    return solve(t, 0, m, B, ldb);
}

}  // extern "C"

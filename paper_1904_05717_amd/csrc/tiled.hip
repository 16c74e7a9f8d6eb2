// Tile-major ("prepacked") storage mode of the FP64 family.
//
// The paper's experiments store the matrices so that every block the
// algorithm partitions them into is contiguous, which removes packing and
// separates temporal from spatial locality (Sec. 5.2, varying bandwidth).
// Here op(A) (m x k) and op(B) (k x n) are stored panel-major at the
// granularity of the register-resident kernel:
//
//   A: [m-tile of 128 rows][k-slab of 16][128][16]  row panels of 128-row
//      tiles, each split into contiguous 128 x 16 k-slabs (row-major inside);
//   B: [n-tile of 128 columns][k][128]              column panels, k-major, so
//      every 16 x 128 k-slab is contiguous (Goto's packed B panel, for the
//      whole matrix).
//
// Rows and columns beyond the matrix, and k beyond k, are zero.  The
// register-resident members keep the C tile in registers over all of k
// exactly as in the row-major kernel, with the same k stagger; Goto, B3A2C0,
// C3A2C0 and C4A2C0 run the LDS-resident A-block kernel and A3B2C0 the
// LDS-resident B-block kernel with their row-major loop nests, B read in
// place from the column panels.  So for a given member
// the result is bitwise the one the row-major path computes; only the loads
// differ (one pointer per thread stepping through contiguous slabs, no edge
// predicates).
#include <hip/hip_runtime.h>

#include <climits>

#include "../../include/momms.h"
#include "kernels_f64.hip"
#include "plan_internal.h"

namespace momms {
namespace tiled {

constexpr int kT = 128;      // tile rows of A / columns of B
constexpr int kSlab = 16;    // k depth of a slab
constexpr int kSlabElems = kT * kSlab;

typedef TileCfg<128, 128, 16, 2, 2> Cfg128;
typedef TileCfg<64, 64, 16, 2, 2> Cfg64;
typedef TileCfg<kMCa, kNTa, kKSlds, kMCa / 32, kNTa / 32> CfgA;   // the LDS-resident A-block kernel
typedef TileCfg<kMCa1, kNTa, kKSlds, kMCa1 / 32, kNTa / 32> CfgA1;   // the same, one per CU (C3A2C0)
typedef TileCfg<kMTb, kNCb, kKSlds, kMTb / 32, kNCb / 32> CfgB;   // the LDS-resident B-block kernel

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Padded extents of a tiled operand: A is rows x cols = m x k, B is k x n.
struct Extent {
    int64_t rp, cp;
};
static Extent extent(int operand, int64_t rows, int64_t cols) {
    Extent e;
    if (operand == 'A') {
        e.rp = rup(rows > 0 ? rows : 1, kT);
        e.cp = rup(cols > 0 ? cols : 1, kSlab);
    } else {
        e.rp = rup(rows > 0 ? rows : 1, kSlab);
        e.cp = rup(cols > 0 ? cols : 1, kT);
    }
    return e;
}

// Position of element (r, c) of the padded operand in the tiled buffer.
__device__ __forceinline__ int64_t a_index(int64_t r, int64_t c, int64_t kp) {
    return ((r / kT) * (kp / kSlab) + c / kSlab) * kSlabElems + (r % kT) * kSlab + c % kSlab;
}
__device__ __forceinline__ int64_t b_index(int64_t r, int64_t c, int64_t kp) {
    return ((c / kT) * kp + r) * kT + c % kT;
}

// One thread per element of the padded operand, in tiled order (writes are
// contiguous; a one-time conversion, not the product).  X(r, c) = X[r*ldx+c],
// or X[c*ldx+r] when TRANS.
template <bool B_SIDE, bool TRANS>
__global__ __launch_bounds__(256) void k_to_tiled(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                                   int64_t cols, int64_t rp, int64_t cp, double* __restrict__ T) {
    const int64_t total = rp * cp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r, c;
        if (!B_SIDE) {   // e walks [m-tile][k-slab][row][16]
            const int64_t tile = e / kSlabElems, in = e % kSlabElems;
            const int64_t ks = cp / kSlab;
            r = (tile / ks) * kT + in / kSlab;
            c = (tile % ks) * kSlab + in % kSlab;
        } else {         // e walks [n-tile][k][128]
            const int64_t panel = e / (rp * kT), in = e % (rp * kT);
            r = in / kT;
            c = panel * kT + in % kT;
        }
        double v = 0.0;
        if (r < rows && c < cols) v = TRANS ? X[c * ldx + r] : X[r * ldx + c];
        T[e] = v;
    }
}

template <bool B_SIDE>
__global__ __launch_bounds__(256) void k_from_tiled(const double* __restrict__ T, int64_t rows, int64_t cols,
                                                     int64_t kp, double* __restrict__ X, int64_t ldx) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e % cols;
        X[r * ldx + c] = B_SIDE ? T[b_index(r, c, kp)] : T[a_index(r, c, kp)];
    }
}

// The register-resident tile over k-slabs [s_begin, s_end), reading the
// tiled operands; same stagger, micro-kernel and epilogue as regc_tile.
template <class CF>
__device__ __forceinline__ void regc_tile_tiled(int64_t M, int64_t N, int64_t s_begin, int64_t s_end,
                                                int64_t kp, double alpha, const double* __restrict__ At,
                                                const double* __restrict__ Bt, double beta,
                                                double* __restrict__ C, int64_t ldc, int64_t m0, int64_t n0,
                                                int tm, int tn, double (*As)[CF::MT * CF::A_LD],
                                                double (*Bs)[CF::KS * CF::B_LD]) {
    static_assert(CF::KS == kSlab && kT % CF::MT == 0 && kT % CF::NT == 0, "tile must sit inside a slab");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / CF::WN, wn = wave % CF::WN;
    d4 acc[CF::BM][CF::BN];
    zero_acc<CF>(acc);
    const int64_t nsl = s_end - s_begin;
    if (nsl > 0) {
        const int64_t s0 = (int64_t)((tm + tn) & 7) % nsl;
        const int64_t slabs = kp / kSlab;
        // A slab (i, s) at ((i * slabs) + s) * kSlabElems, rows of 16; B slab
        // (s, j) at (j * kp + 16 s) * 128, rows of 128.  Both advance by one
        // slab (kSlabElems) per step.
        const double* a0 = At + ((m0 / kT) * slabs + s_begin + s0) * kSlabElems + (m0 % kT) * kSlab;
        const double* b0 = Bt + ((n0 / kT) * kp + (s_begin + s0) * kSlab) * kT + n0 % kT;
        FastStage<CF::MT, CF::KS, CF::THREADS, false> fa;
        FastStage<CF::KS, CF::NT, CF::THREADS, false> fb;
        fa.init(a0, kSlab, 0, 0, tid);
        fb.init(b0, kT, 0, 0, tid);
        const int64_t d = kSlabElems;
        fa.load();
        fb.load();
        fa.store(As[0], CF::A_LD, tid);
        fb.store(Bs[0], CF::B_LD, tid);
        __syncthreads();
        for (int64_t sl = 0; sl < nsl; ++sl) {
            const int cur = (int)(sl & 1);
            const bool more = sl + 1 < nsl;
            if (more) {
                const bool wrap = (s0 + sl + 1) == nsl;   // next slab wraps to s_begin
                fa.advance(wrap ? d * (1 - nsl) : d);
                fb.advance(wrap ? d * (1 - nsl) : d);
                fa.load();
                fb.load();
            }
            mma_lds<CF, CF::KS / 4>(As[cur], CF::A_LD, 0, Bs[cur], CF::B_LD, 0, acc, wm, wn, lane);
            if (more) {
                fa.store(As[cur ^ 1], CF::A_LD, tid);
                fb.store(Bs[cur ^ 1], CF::B_LD, tid);
            }
            __syncthreads();
        }
    }
    store_c<CF>(acc, alpha, beta, C, ldc, m0, n0, M, N, wm, wn, lane);
}

template <class CF>
__global__ __launch_bounds__(CF::THREADS) __attribute__((amdgpu_waves_per_eu(CF::MT >= 128 ? 2 : 1)))
void k_regc_tiled(int64_t M, int64_t N, int64_t s_begin, int64_t s_end, int64_t kp, double alpha,
                  const double* __restrict__ At, const double* __restrict__ Bt, double beta, double* __restrict__ C,
                  int64_t ldc, Sched s) {
    __shared__ double As[2][CF::MT * CF::A_LD];
    __shared__ double Bs[2][CF::KS * CF::B_LD];
    int tm, tn;
    decode_tile(s, blockIdx.x, tm, tn);
    const int64_t m0 = s.m_off + (int64_t)tm * CF::MT;
    const int64_t n0 = s.n_off + (int64_t)tn * CF::NT;
    regc_tile_tiled<CF>(M, N, s_begin, s_end, kp, alpha, At, Bt, beta, C, ldc, m0, n0, tm, tn, As, Bs);
}

static Sched sched_of(int64_t m_off, int64_t n_off, int64_t m_lim, int64_t n_lim, int64_t tile, int64_t group_m,
                      bool xcd) {
    Sched s;
    s.m_off = m_off;
    s.n_off = n_off;
    s.m_lim = m_lim;
    s.n_lim = n_lim;
    s.tiles_m = (int)cdiv(m_lim - m_off, tile);
    s.tiles_n = (int)cdiv(n_lim - n_off, tile);
    if (group_m < 1) group_m = 1;
    if (group_m > s.tiles_m) group_m = s.tiles_m;
    s.group_m = (int)group_m;
    s.xcd = xcd ? kXcds : 1;
    return s;
}

struct TArgs {
    int64_t M, N, kp;
    double alpha, beta;
    const double* At;
    const double* Bt;
    double* C;
    int64_t ldc;
    hipStream_t st;
};

static void launch(const TArgs& a, int tile, int64_t s0, int64_t s1, double beta, const Sched& s) {
    const int grid = s.tiles_m * s.tiles_n;
    if (grid <= 0) return;
    if (tile == 128)
        hipLaunchKernelGGL((k_regc_tiled<Cfg128>), dim3(grid), dim3(Cfg128::THREADS), 0, a.st, a.M, a.N, s0, s1,
                           a.kp, a.alpha, a.At, a.Bt, beta, a.C, a.ldc, s);
    else
        hipLaunchKernelGGL((k_regc_tiled<Cfg64>), dim3(grid), dim3(Cfg64::THREADS), 0, a.st, a.M, a.N, s0, s1,
                           a.kp, a.alpha, a.At, a.Bt, beta, a.C, a.ldc, s);
}

// The LDS-resident A-block kernel on tile-major operands: A from its 128 x 16
// slabs, B k-slices straight from the tile-major column panels (the panel
// height is the padded k).  s covers granules of Cfg::MT rows x nj column
// tiles.
template <class Cfg = CfgA>
static void launch_a2(const TArgs& a, int64_t k0, int64_t k1, const Sched& s, int nj, int kc, int64_t slabs) {
    const int grid = s.tiles_m * s.tiles_n;
    if (grid <= 0) return;
    hipLaunchKernelGGL((k_a2<Cfg, kKCa, false, false, true, true>), dim3(grid), dim3(Cfg::THREADS), 0, a.st, a.M,
                       a.N, k0, k1, a.alpha, a.At, slabs, a.Bt, a.kp, a.beta, a.C, a.ldc, s, nj, (int64_t)0,
                       (int64_t)0, kc);
}

// Granules of rows x nj column tiles (kNTa wide) over [m_off, m_lim) x
// [n_off, n_lim).
static Sched granules(int64_t m_off, int64_t n_off, int64_t m_lim, int64_t n_lim, int nj, int64_t group_m,
                      bool xcd, int64_t rows = kMCa) {
    Sched s = sched_of(m_off, n_off, m_lim, n_lim, rows, group_m, xcd);
    s.tiles_n = (int)cdiv(n_lim - n_off, (int64_t)nj * kNTa);
    return s;
}

// The loop nests of the members, as in the row-major path.
static int run(const momms_plan& p, const TArgs& a, int64_t K) {
    if (p.kernel == 1 && (!a2_chunk_ok(p.kc) || !(p.mt == CfgA::MT || (p.member == MOMMS_C3A2C0 && p.mt == CfgA1::MT))))
        return MOMMS_ERR_INTERNAL;
    const int64_t M = a.M, N = a.N, slabs = cdiv(K, kSlab);
    const int t = p.mt;
    switch (p.member) {
        case MOMMS_C0:
            launch(a, t, 0, slabs, a.beta, sched_of(0, 0, M, N, t, 1, false));
            break;
        case MOMMS_C3C0:
            for (int64_t ib = 0; ib < M; ib += p.mc4) {
                const int64_t ie = ib + p.mc4 < M ? ib + p.mc4 : M;
                for (int64_t jb = 0; jb < N; jb += p.nc4) {
                    const int64_t je = jb + p.nc4 < N ? jb + p.nc4 : N;
                    launch(a, t, 0, slabs, a.beta, sched_of(ib, jb, ie, je, t, p.group_m, true));
                }
            }
            break;
        case MOMMS_B3C0:
        case MOMMS_A3C0: {
            const Sched s = sched_of(0, 0, M, N, t, p.group_m, true);
            const int64_t step = p.kc3 / kSlab;
            for (int64_t sb = 0; sb < slabs; sb += step) {
                const int64_t se = sb + step < slabs ? sb + step : slabs;
                launch(a, t, sb, se, sb == 0 ? a.beta : 1.0, s);
            }
            break;
        }
        case MOMMS_A2C0:
            // Goto without packing: n by nc -> k by kc -> the kernel with the
            // A block (128 x kc slabs) in LDS and B k-slices read straight
            // from the tile-major column panels.
            for (int64_t jc = 0; jc < N; jc += p.nc) {
                const int64_t je = jc + p.nc < N ? jc + p.nc : N;
                const Sched s = granules(0, jc, M, je, p.nj, 1, false);
                for (int64_t pc = 0; pc < K; pc += p.kc) {
                    const int64_t pe = pc + p.kc < K ? pc + p.kc : K;
                    launch_a2(a, pc, pe, s, p.nj, (int)p.kc, slabs);
                }
            }
            break;
        case MOMMS_B3A2C0: {
            // k by kc3 -> granules of kMCa rows x nc3 columns in column-major
            // order (one XCD's run shares a kc3 x nc3 B block) -> the kernel
            const Sched s = granules(0, 0, M, N, p.nj, p.group_m, true);
            for (int64_t kb = 0; kb < K; kb += p.kc3) {
                const int64_t ke = kb + p.kc3 < K ? kb + p.kc3 : K;
                launch_a2(a, kb, ke, s, p.nj, (int)p.kc, slabs);
            }
            break;
        }
        case MOMMS_A3B2C0: {
            // k by kc3 -> granules of mc3 rows x kNCb columns, XCD-aware ->
            // the kernel with the B block (kc x kNCb) in LDS, A slices streamed
            Sched s = sched_of(0, 0, M, N, kNCb, 1, true);
            s.tiles_m = (int)cdiv(M, p.mc3);
            for (int64_t kb = 0; kb < K; kb += p.kc3) {
                const int64_t ke = kb + p.kc3 < K ? kb + p.kc3 : K;
                const int grid = s.tiles_m * s.tiles_n;
                if (grid > 0)
                    hipLaunchKernelGGL((k_b2<CfgB, kKC, false, false, true>), dim3(grid), dim3(CfgB::THREADS), 0,
                                       a.st, M, N, kb, ke, a.alpha, a.At, slabs, a.Bt, a.kp, a.beta, a.C, a.ldc, s,
                                       p.mi);
            }
            break;
        }
        case MOMMS_C3A2C0:
            // XCD-grouped C tiles, each walking all of k with its A block in LDS
            if (p.mt == CfgA1::MT)
                launch_a2<CfgA1>(a, 0, K, granules(0, 0, M, N, 1, p.group_m, true, kMCa1), 1, (int)p.kc, slabs);
            else
                launch_a2<CfgA>(a, 0, K, granules(0, 0, M, N, 1, p.group_m, true), 1, (int)p.kc, slabs);
            break;
        case MOMMS_C4A2C0:
            // m, n by the MALL-resident C block -> k by kc3 -> the kernel
            for (int64_t ib = 0; ib < M; ib += p.mc4) {
                const int64_t ie = ib + p.mc4 < M ? ib + p.mc4 : M;
                for (int64_t jb = 0; jb < N; jb += p.nc4) {
                    const int64_t je = jb + p.nc4 < N ? jb + p.nc4 : N;
                    const Sched s = granules(ib, jb, ie, je, p.nj, 1, false);
                    for (int64_t pc = 0; pc < K; pc += p.kc3) {
                        const int64_t pe = pc + p.kc3 < K ? pc + p.kc3 : K;
                        launch_a2(a, pc, pe, s, p.nj, (int)p.kc, slabs);
                    }
                }
            }
            break;
        default:
            return MOMMS_ERR_INTERNAL;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace tiled
}  // namespace momms

extern "C" {

size_t momms_tiled_size(int operand, int64_t rows, int64_t cols) {
    using namespace momms::tiled;
    if ((operand != 'A' && operand != 'B') || rows < 0 || cols < 0) return 0;
    const Extent e = extent(operand, rows, cols);
    return sizeof(double) * (size_t)e.rp * (size_t)e.cp;
}

int momms_to_tiled(int operand, int trans, int64_t rows, int64_t cols, const double* X, int64_t ldx, double* T,
                   momms_stream_t stream) {
    using namespace momms::tiled;
    if (operand != 'A' && operand != 'B') return -1;
    if (trans != 0 && trans != 1) return -2;
    if (rows < 0) return -3;
    if (cols < 0) return -4;
    const int64_t contiguous = trans ? rows : cols;
    if (rows > 0 && cols > 0 && X == nullptr) return -5;
    if (ldx < (contiguous > 1 ? contiguous : 1)) return -6;
    if (T == nullptr) return -7;
    const Extent e = extent(operand, rows, cols);
    if (e.rp * e.cp >= (int64_t)1 << 40) return MOMMS_ERR_INFEASIBLE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t grid = cdiv(e.rp * e.cp, 256);
    if (grid > 65536) grid = 65536;
    const bool b = operand == 'B';
    if (!b && !trans) hipLaunchKernelGGL((k_to_tiled<false, false>), dim3((unsigned)grid), dim3(256), 0, st, X, ldx, rows, cols, e.rp, e.cp, T);
    if (!b && trans)  hipLaunchKernelGGL((k_to_tiled<false, true>), dim3((unsigned)grid), dim3(256), 0, st, X, ldx, rows, cols, e.rp, e.cp, T);
    if (b && !trans)  hipLaunchKernelGGL((k_to_tiled<true, false>), dim3((unsigned)grid), dim3(256), 0, st, X, ldx, rows, cols, e.rp, e.cp, T);
    if (b && trans)   hipLaunchKernelGGL((k_to_tiled<true, true>), dim3((unsigned)grid), dim3(256), 0, st, X, ldx, rows, cols, e.rp, e.cp, T);
    const hipError_t err = hipGetLastError();
    return err == hipSuccess ? 0 : (int)err;
}

int momms_from_tiled(int operand, int64_t rows, int64_t cols, const double* T, double* X, int64_t ldx,
                     momms_stream_t stream) {
    using namespace momms::tiled;
    if (operand != 'A' && operand != 'B') return -1;
    if (rows < 0) return -2;
    if (cols < 0) return -3;
    if (rows == 0 || cols == 0) return 0;
    if (T == nullptr) return -4;
    if (X == nullptr) return -5;
    if (ldx < (cols > 1 ? cols : 1)) return -6;
    const Extent e = extent(operand, rows, cols);
    const int64_t kp = operand == 'A' ? e.cp : e.rp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t grid = cdiv(rows * cols, 256);
    if (grid > 65536) grid = 65536;
    if (operand == 'A')
        hipLaunchKernelGGL((k_from_tiled<false>), dim3((unsigned)grid), dim3(256), 0, st, T, rows, cols, kp, X, ldx);
    else
        hipLaunchKernelGGL((k_from_tiled<true>), dim3((unsigned)grid), dim3(256), 0, st, T, rows, cols, kp, X, ldx);
    const hipError_t err = hipGetLastError();
    return err == hipSuccess ? 0 : (int)err;
}

int momms_gemm_tiled(int64_t m, int64_t n, int64_t k, double alpha, const double* At, const double* Bt, double beta,
                     double* C, int64_t ldc, int family_member, momms_stream_t stream) {
    using namespace momms;
    using namespace momms::tiled;
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (k < 0) return -3;
    const bool reads_ab = alpha != 0.0 && k > 0 && m > 0 && n > 0;
    if (reads_ab && At == nullptr) return -5;
    if (reads_ab && Bt == nullptr) return -6;
    if (m > 0 && n > 0 && C == nullptr) return -8;
    if (ldc < (n > 1 ? n : 1)) return -9;
    int member = family_member;
    if (member == MOMMS_AUTO) {
        member = select_member(m, n, k);
        if (member != MOMMS_C0 && member != MOMMS_B3C0 && member != MOMMS_A3C0) member = MOMMS_C3C0;
    }
    if (member <= MOMMS_AUTO || member >= momms_num_members()) return -10;
    if (cdiv(m, 64) * cdiv(n, 64) >= (int64_t)INT_MAX / 2) return MOMMS_ERR_INFEASIBLE;
    if (m == 0 || n == 0) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;
    momms_plan p;
    if (plan_member(member, m, n, k, &p) != 0) return MOMMS_ERR_INTERNAL;
    TArgs a;
    a.M = m;
    a.N = n;
    a.kp = rup(k > 0 ? k : 1, kSlab);
    a.alpha = alpha;
    a.beta = beta;
    a.At = At;
    a.Bt = Bt;
    a.C = C;
    a.ldc = ldc;
    a.st = static_cast<hipStream_t>(stream);
    if (alpha == 0.0 || k == 0) {
        // C := beta C through a launch over zero slabs (the kernel only scales).
        launch(a, p.mt, 0, 0, beta, sched_of(0, 0, m, n, p.mt, 1, false));
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    return run(p, a, k);
}

}  // extern "C"

// Launch sequences of the MOMMS family members and the plain-FP64 C ABI.
//
// Each member is a loop nest (Sec. 3.2: two loops per level).  The loops
// above a workgroup are realised here: either as host loops over kernel
// launches on one stream (which orders the k passes that update the same C
// tiles), or inside a launch as the workgroup -> tile order that decides
// which blocks the workgroups of one XCD share in its L2.  The loops inside a
// workgroup are the kernels of kernels_f64.hip.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <mutex>

#include "../../include/momms.h"
#include "kernels_f64.hip"
#include "plan_internal.h"

namespace momms {

// C = beta * C over an m x n matrix (beta == 0 writes zeros without reading).
__global__ __launch_bounds__(256) void k_scale_c(int64_t M, int64_t N, double beta, double* __restrict__ C,
                                                 int64_t ldc) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / N, j = e - (e / N) * N;
        double* p = C + i * ldc + j;
        *p = (beta == 0.0) ? 0.0 : beta * (*p);
    }
}

using CfgL = TileCfg<128, 128, 16, 2, 2>;  // register-resident C, large problems
using CfgS = TileCfg<64, 64, 16, 2, 2>;    // register-resident C, small problems
// LDS-resident blocks: waves of 32 x 32, two per SIMD, 32-deep streamed
// slices.  A block kMCa x kKCa (C tiles kMCa x kNTa), four waves, two
// workgroups per CU; for C3A2C0 kMCa1 x kKCa, eight waves, one per CU; B
// block kKC x kNCb (C tiles kMTb x kNCb), eight waves.
using CfgA = TileCfg<kMCa, kNTa, kKSlds, kMCa / 32, kNTa / 32>;
using CfgA1 = TileCfg<kMCa1, kNTa, kKSlds, kMCa1 / 32, kNTa / 32>;
using CfgB = TileCfg<kMTb, kNCb, kKSlds, kMTb / 32, kNCb / 32>;
static_assert(CfgA::THREADS * kWGsPerCuA == 512 && CfgA1::THREADS == 512 && CfgB::THREADS == 512,
              "eight waves per CU");

static hipStream_t g_stream = nullptr;

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static Sched make_sched(int64_t m_off, int64_t n_off, int64_t m_lim, int64_t n_lim, int64_t grain_m,
                        int64_t grain_n, int64_t group_m, bool xcd) {
    Sched s;
    s.m_off = m_off;
    s.n_off = n_off;
    s.m_lim = m_lim;
    s.n_lim = n_lim;
    s.tiles_m = (int)cdiv(m_lim - m_off, grain_m);
    s.tiles_n = (int)cdiv(n_lim - n_off, grain_n);
    if (group_m < 1) group_m = 1;
    if (group_m > s.tiles_m) group_m = s.tiles_m;
    s.group_m = (int)group_m;
    s.xcd = xcd ? kXcds : 1;
    return s;
}

static inline int grid_of(const Sched& s) { return s.tiles_m * s.tiles_n; }

struct Args {
    bool ta, tb;
    int64_t M, N, K;
    double alpha;
    const double* A;
    int64_t lda;
    const double* B;
    int64_t ldb;
    double beta;
    double* C;
    int64_t ldc;
    hipStream_t st;
};

template <class CF, bool TA, bool TB>
static void launch_regc_t(const Args& a, int64_t k0, int64_t k1, double beta, const Sched& s) {
    hipLaunchKernelGGL((k_regc<CF, TA, TB>), dim3(grid_of(s)), dim3(CF::THREADS), 0, a.st, a.M, a.N, k0, k1, a.alpha,
                       a.A, a.lda, a.B, a.ldb, beta, a.C, a.ldc, s);
}

template <class CF>
static void launch_regc(const Args& a, int64_t k0, int64_t k1, double beta, const Sched& s) {
    if (grid_of(s) <= 0) return;
    if (!a.ta && !a.tb) launch_regc_t<CF, false, false>(a, k0, k1, beta, s);
    else if (!a.ta && a.tb) launch_regc_t<CF, false, true>(a, k0, k1, beta, s);
    else if (a.ta && !a.tb) launch_regc_t<CF, true, false>(a, k0, k1, beta, s);
    else launch_regc_t<CF, true, true>(a, k0, k1, beta, s);
}

template <class Cfg, bool TA, bool TB, bool PK>
static void launch_a2_t(const Args& a, int64_t k0, int64_t k1, const Sched& s, int nj, const double* Bsrc,
                        int64_t ldb, int64_t pk0, int64_t pn0, int kc) {
    hipLaunchKernelGGL((k_a2<Cfg, kKCa, TA, TB, PK>), dim3(grid_of(s)), dim3(Cfg::THREADS), 0, a.st, a.M, a.N, k0,
                       k1, a.alpha, a.A, a.lda, Bsrc, ldb, a.beta, a.C, a.ldc, s, nj, pk0, pn0, kc);
}

// beta is applied by the kernel to the pass whose k chunk starts at 0; the
// kernel walks [k0, k1) in chunks of kc (the plan's, checked by run()).  Cfg
// is CfgA1 for C3A2C0 on problems that fill the chip (never packed), CfgA
// otherwise.
template <class Cfg = CfgA>
static void launch_a2(const Args& a, int64_t k0, int64_t k1, const Sched& s, int nj, int kc, const double* packed,
                      int64_t pk0, int64_t pn0) {
    if (grid_of(s) <= 0) return;
    if (packed) {
        if (!a.ta) launch_a2_t<CfgA, false, false, true>(a, k0, k1, s, nj, packed, kKCa, pk0, pn0, kc);
        else launch_a2_t<CfgA, true, false, true>(a, k0, k1, s, nj, packed, kKCa, pk0, pn0, kc);
        return;
    }
    if (!a.ta && !a.tb) launch_a2_t<Cfg, false, false, false>(a, k0, k1, s, nj, a.B, a.ldb, 0, 0, kc);
    else if (!a.ta && a.tb) launch_a2_t<Cfg, false, true, false>(a, k0, k1, s, nj, a.B, a.ldb, 0, 0, kc);
    else if (a.ta && !a.tb) launch_a2_t<Cfg, true, false, false>(a, k0, k1, s, nj, a.B, a.ldb, 0, 0, kc);
    else launch_a2_t<Cfg, true, true, false>(a, k0, k1, s, nj, a.B, a.ldb, 0, 0, kc);
}

template <bool TA, bool TB>
static void launch_b2_t(const Args& a, int64_t k0, int64_t k1, const Sched& s, int mi) {
    hipLaunchKernelGGL((k_b2<CfgB, kKC, TA, TB>), dim3(grid_of(s)), dim3(CfgB::THREADS), 0, a.st, a.M, a.N, k0, k1,
                       a.alpha, a.A, a.lda, a.B, a.ldb, a.beta, a.C, a.ldc, s, mi);
}

static void launch_b2(const Args& a, int64_t k0, int64_t k1, const Sched& s, int mi) {
    if (grid_of(s) <= 0) return;
    if (!a.ta && !a.tb) launch_b2_t<false, false>(a, k0, k1, s, mi);
    else if (!a.ta && a.tb) launch_b2_t<false, true>(a, k0, k1, s, mi);
    else if (a.ta && !a.tb) launch_b2_t<true, false>(a, k0, k1, s, mi);
    else launch_b2_t<true, true>(a, k0, k1, s, mi);
}

static void launch_pack_b(const Args& a, int64_t pk0, int64_t pn0, int64_t ncw, double* P) {
    const int ntiles = (int)cdiv(ncw, CfgA::NT);
    const int64_t total = (int64_t)ntiles * kKCa * CfgA::NT;
    int grid = (int)cdiv(total, 256);
    if (grid > 4 * kCUs * 8) grid = 4 * kCUs * 8;
    if (a.tb)
        hipLaunchKernelGGL((k_pack_b<CfgA::NT, true>), dim3(grid), dim3(256), 0, a.st, a.B, a.ldb, a.K, a.N, pk0, pn0,
                           (int)kKCa, ntiles, P);
    else
        hipLaunchKernelGGL((k_pack_b<CfgA::NT, false>), dim3(grid), dim3(256), 0, a.st, a.B, a.ldb, a.K, a.N, pk0,
                           pn0, (int)kKCa, ntiles, P);
}

// Runs the loop nest of plan p.  Returns 0 or a hipError_t.
static int run_member(const momms_plan& p, const Args& a, void* ws) {
    const int64_t M = a.M, N = a.N, K = a.K;
    if (p.kernel == 1 && (!a2_chunk_ok(p.kc) || !(p.mt == CfgA::MT || (p.member == MOMMS_C3A2C0 && p.mt == CfgA1::MT))))
        return MOMMS_ERR_INTERNAL;
    switch (p.member) {
        case MOMMS_C0: {
            const Sched s = make_sched(0, 0, M, N, p.mt, p.nt, 1, false);
            if (p.mt == 128) launch_regc<CfgL>(a, 0, K, a.beta, s);
            else launch_regc<CfgS>(a, 0, K, a.beta, s);
            break;
        }
        case MOMMS_C3C0: {
            // m, n by the level-4 region (host) -> XCD-aware grouped tiles.
            for (int64_t ib = 0; ib < M; ib += p.mc4) {
                const int64_t ie = ib + p.mc4 < M ? ib + p.mc4 : M;
                for (int64_t jb = 0; jb < N; jb += p.nc4) {
                    const int64_t je = jb + p.nc4 < N ? jb + p.nc4 : N;
                    const Sched s = make_sched(ib, jb, ie, je, p.mt, p.nt, p.group_m, true);
                    if (p.mt == 128) launch_regc<CfgL>(a, 0, K, a.beta, s);
                    else launch_regc<CfgS>(a, 0, K, a.beta, s);
                }
            }
            break;
        }
        case MOMMS_B3C0:
        case MOMMS_A3C0: {
            // k by kc3 (host loop) -> tiles in column-major (B3) or row-major
            // (A3) order, each XCD taking a contiguous run.
            const Sched s = make_sched(0, 0, M, N, p.mt, p.nt, p.group_m, true);
            for (int64_t kb = 0; kb < K; kb += p.kc3) {
                const int64_t ke = kb + p.kc3 < K ? kb + p.kc3 : K;
                const double be = kb == 0 ? a.beta : 1.0;
                if (p.mt == 128) launch_regc<CfgL>(a, kb, ke, be, s);
                else launch_regc<CfgS>(a, kb, ke, be, s);
            }
            break;
        }
        case MOMMS_A2C0: {
            // n by nc -> k by kc (pack the B panel) -> kernel: m by 128 (A
            // block in LDS), n by 128 inside and across workgroups.
            for (int64_t jc = 0; jc < N; jc += p.nc) {
                const int64_t je = jc + p.nc < N ? jc + p.nc : N;
                const Sched s = make_sched(0, jc, M, je, p.mt, (int64_t)p.nj * p.nt, 1, false);
                for (int64_t pc = 0; pc < K; pc += p.kc) {
                    const int64_t pe = pc + p.kc < K ? pc + p.kc : K;
                    if (ws) {
                        double* P = static_cast<double*>(ws);
                        launch_pack_b(a, pc, jc, je - jc, P);
                        launch_a2(a, pc, pe, s, p.nj, (int)p.kc, P, pc, jc);
                    } else {
                        launch_a2(a, pc, pe, s, p.nj, (int)p.kc, nullptr, 0, 0);
                    }
                }
            }
            break;
        }
        case MOMMS_B3A2C0: {
            // k by kc3 (host) -> granules of 128 rows x nc3 columns in
            // column-major order (one XCD's run shares a kc3 x nc3 B block)
            // -> kernel: k by kc inside, A block in LDS, n by 128.
            const Sched s = make_sched(0, 0, M, N, p.mt, p.nc3, p.group_m, true);
            for (int64_t kb = 0; kb < K; kb += p.kc3) {
                const int64_t ke = kb + p.kc3 < K ? kb + p.kc3 : K;
                launch_a2(a, kb, ke, s, p.nj, (int)p.kc, nullptr, 0, 0);
            }
            break;
        }
        case MOMMS_A3B2C0: {
            const Sched s = make_sched(0, 0, M, N, p.mc3, p.nt, 1, true);
            for (int64_t kb = 0; kb < K; kb += p.kc3) {
                const int64_t ke = kb + p.kc3 < K ? kb + p.kc3 : K;
                launch_b2(a, kb, ke, s, p.mi);
            }
            break;
        }
        case MOMMS_C3A2C0: {
            const Sched s = make_sched(0, 0, M, N, p.mt, p.nt, p.group_m, true);
            if (p.mt == CfgA1::MT) launch_a2<CfgA1>(a, 0, K, s, 1, (int)p.kc, nullptr, 0, 0);
            else launch_a2<CfgA>(a, 0, K, s, 1, (int)p.kc, nullptr, 0, 0);
            break;
        }
        case MOMMS_C4A2C0: {
            // m, n by the MALL-resident C block -> k by kc3 (host) -> kernel
            // (k by kc inside).
            for (int64_t ib = 0; ib < M; ib += p.mc4) {
                const int64_t ie = ib + p.mc4 < M ? ib + p.mc4 : M;
                for (int64_t jb = 0; jb < N; jb += p.nc4) {
                    const int64_t je = jb + p.nc4 < N ? jb + p.nc4 : N;
                    const Sched s = make_sched(ib, jb, ie, je, p.mt, (int64_t)p.nj * p.nt, 1, false);
                    for (int64_t pc = 0; pc < K; pc += p.kc3) {
                        const int64_t pe = pc + p.kc3 < K ? pc + p.kc3 : K;
                        launch_a2(a, pc, pe, s, p.nj, (int)p.kc, nullptr, 0, 0);
                    }
                }
            }
            break;
        }
        default:
            return MOMMS_ERR_INTERNAL;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

// Largest grid any member launches for this plan must fit the int tile
// arithmetic of decode_tile.
static bool grid_fits(int64_t M, int64_t N) {
    const int64_t t = cdiv(M, 64) * cdiv(N, 64);
    return t < (int64_t)INT_MAX / 2;
}

// Host-side argument checks shared by the FP64 entry points (argument
// numbers of momms_gemm_ex).  No HIP call.
static int check_args(int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                      int64_t lda, const double* B, int64_t ldb, const double* C, int64_t ldc, int member) {
    const bool ta = transA != 0, tb = transB != 0;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const bool reads_ab = (alpha != 0.0) && k > 0 && m > 0 && n > 0;
    if (reads_ab && A == nullptr) return -7;
    if (lda < (ta ? (m > 1 ? m : 1) : (k > 1 ? k : 1))) return -8;
    if (reads_ab && B == nullptr) return -9;
    if (ldb < (tb ? (k > 1 ? k : 1) : (n > 1 ? n : 1))) return -10;
    if (m > 0 && n > 0 && C == nullptr) return -12;
    if (ldc < (n > 1 ? n : 1)) return -13;
    if (member < 0 || member >= MOMMS_NUM_MEMBERS) return -14;
    if (!grid_fits(m, n)) return MOMMS_ERR_INFEASIBLE;
    return 0;
}

// Scratch of the allocation-free entry point: Goto's packed B panel (k_c rows
// of at most n_c columns, the largest workspace any member asks for)
// in a static device array.  Each GPU holds its own copy for the life of the
// process.  In host code `scratch` names a host-side stand-in, never the
// device memory: its device address is taken once per device with that device
// current, and only that address is passed to kernels.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;   // 4 MiB
static_assert((size_t)kKCa * kGotoNc * sizeof(double) <= kStaticScratchBytes, "Goto's panel fits the scratch");
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

static int static_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return MOMMS_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) return MOMMS_ERR_INTERNAL;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return 0;
}

static_assert(kStaticScratchBytes % 256 == 0, "scratch must keep the workspace alignment");
static_assert(kStaticScratchBytes == MOMMS_STATIC_SCRATCH_BYTES, "header and library disagree on the scratch size");

}  // namespace momms

extern "C" {

int momms_set_stream(momms_stream_t stream) {
    momms::g_stream = static_cast<hipStream_t>(stream);
    return 0;
}

int momms_gemm_ex(int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                  int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int family_member,
                  void* workspace, size_t ws_bytes, momms_stream_t stream) {
    using namespace momms;
    const int bad = check_args(transA, transB, m, n, k, alpha, A, lda, B, ldb, C, ldc, family_member);
    if (bad != 0) return bad;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return -15;

    int member = family_member == MOMMS_AUTO ? select_member(m, n, k) : family_member;
    const size_t need = workspace_bytes(member, m, n, k);
    if (workspace && need > 0 && ws_bytes < need) return -16;

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (m == 0 || n == 0) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;
    if (alpha == 0.0 || k == 0) {
        int64_t total = m * n;
        int grid = (int)cdiv(total, 256);
        if (grid > 8 * kCUs * 8) grid = 8 * kCUs * 8;
        hipLaunchKernelGGL(k_scale_c, dim3(grid), dim3(256), 0, st, m, n, beta, C, ldc);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    momms_plan p;
    if (plan_member(member, m, n, k, &p) != 0) return MOMMS_ERR_INTERNAL;
    Args a{transA != 0, transB != 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, st};
    return run_member(p, a, need > 0 ? workspace : nullptr);
}

int momms_gemm_static(int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                      int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                      int family_member, momms_stream_t stream) {
    using namespace momms;
    const int bad = check_args(transA, transB, m, n, k, alpha, A, lda, B, ldb, C, ldc, family_member);
    if (bad != 0) return bad;
    const int member = family_member == MOMMS_AUTO ? select_member(m, n, k) : family_member;
    const size_t need = workspace_bytes(member, m, n, k);
    if (need > kStaticScratchBytes) return MOMMS_ERR_SCRATCH;
    // Nothing to pack (or nothing to multiply): the workspace-free path.
    const bool multiplies = m > 0 && n > 0 && k > 0 && alpha != 0.0;
    if (need == 0 || !multiplies)
        return momms_gemm_ex(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, member, nullptr, 0,
                             stream);
    void* ws = nullptr;
    const int r = static_scratch(&ws);
    if (r != 0) return r;
    return momms_gemm_ex(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, member, ws,
                         kStaticScratchBytes, stream);
}

int momms_gemm(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda, const double* B,
               int64_t ldb, double beta, double* C, int64_t ldc, int family_member) {
    const int r = momms_gemm_ex(0, 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, family_member, nullptr, 0,
                                momms::g_stream);
    // momms_gemm_ex numbers m as argument 3; momms_gemm numbers it 1.
    return r < 0 ? r + 2 : r;
}

}  // extern "C"

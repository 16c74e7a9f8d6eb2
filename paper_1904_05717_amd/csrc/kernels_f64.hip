// FP64 MFMA kernels of the MOMMS family on gfx950 (CDNA4).
//
// Every member is assembled from three workgroup-level kernels that share one
// register micro-kernel (the paper's "inner kernel", Sec. 5.2: all members
// call the same micro-kernel):
//
//   k_regc : C tile resident in registers (level 0) while the workgroup runs
//            over a k range; A and B k-slices are streamed through a
//            double-buffered LDS stage (LDS holds no resident block).
//   k_a2   : an A block (MT x kc, kc <= KC) resident in LDS (level 2), reused
//            across NJ n-tiles; B slices streamed; C updated once per kc.
//   k_b2   : a B block (KC x NT) resident in LDS, reused across MI m-tiles;
//            A slices streamed; C updated once per KC.
//
// The loops above the workgroup (levels 3 and 4: the per-XCD L2 and the
// MALL) are realised by the host loops in gemm_f64.hip and by the
// workgroup -> tile map `decode_tile` below.
//
// MFMA lane layout of v_mfma_f64_16x16x4_f64 on gfx950 (measured on the
// device): lane l supplies A[l % 16][l / 16] of the 16x4 A block and
// B[l / 16][l % 16] of the 4x16 B block, and holds D[l / 16 + 4 r][l % 16]
// in accumulator element r of the 16x16 result.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sched.h"

namespace momms {

typedef double d4 __attribute__((ext_vector_type(4)));

// A zero in device memory for staged entries outside an operand (see
// Stage::load).  Not const, so that the compiler does not fold its loads.
static __device__ double kZeroEntry = 0.0;

// *(base + off bytes) for a wave-uniform base and a 32-bit lane offset, as a
// global load with a scalar base address and a vector offset: no per-lane
// 64-bit address arithmetic.  The base is opaque to the compiler, which
// otherwise folds the offset in once and steps a 64-bit vector address per
// load.  The offset is opaque at each use too, or its zero extension is
// hoisted into a 64-bit register and the scalar-base form is lost.
typedef __attribute__((address_space(1))) const char gchar;
__device__ __forceinline__ double load_sbase(const double* base, uint32_t off) {
    gchar* b = (gchar*)reinterpret_cast<const char*>(base);
    asm volatile("" : "+s"(b), "+v"(off));
    return *reinterpret_cast<__attribute__((address_space(1))) const double*>(b + off);
}
// The store of the same form.
typedef __attribute__((address_space(1))) char gchar_w;
__device__ __forceinline__ void store_sbase(double* base, uint32_t off, double v) {
    gchar_w* b = (gchar_w*)reinterpret_cast<char*>(base);
    asm volatile("" : "+s"(b), "+v"(off));
    *reinterpret_cast<__attribute__((address_space(1))) double*>(b + off) = v;
}
// A lane offset of that form fits 32 bits for a leading dimension below 2^24.
__device__ __forceinline__ bool sbase_ld(int64_t ld) { return ld < ((int64_t)1 << 24); }

// Register staging of an R x S tile of a logical operand X, where
// X(r, s) = P[(r0 + r) * ld + s0 + s] if !TRANS, P[(s0 + s) * ld + r0 + r] if TRANS.
// Consecutive threads walk the contiguous index, so global loads coalesce.
// Entries outside [0, rlim) x [0, slim) are zero.
template <int R, int S, int THREADS, bool TRANS>
struct Stage {
    static_assert((R * S) % THREADS == 0, "stage must divide evenly over the threads");
    static constexpr int N = (R * S) / THREADS;
    double v[N];

    __device__ __forceinline__ static void coord(int e, int& r, int& s) {
        if (TRANS) { s = e / R; r = e - s * R; }
        else       { r = e / S; s = e - r * S; }
    }
    // Element i of the stage (a stage's loads and stores can then be spread
    // over a step).  Every lane loads, an entry outside from kZeroEntry: a
    // load inside a branch may not have been issued, and the compiler then
    // waits for every load in flight before it uses any older one; a value
    // masked after its load would be waited for where the mask is applied.
    __device__ __forceinline__ void load_elem(int i, const double* __restrict__ P, int64_t ld, int64_t r0,
                                              int64_t s0, int64_t rlim, int64_t slim, int tid) {
        int r, s;
        coord(tid + i * THREADS, r, s);
        const int64_t gr = r0 + r, gs = s0 + s;
        const bool ok = gr < rlim && gs < slim;
        v[i] = *(ok ? P + (TRANS ? gs * ld + gr : gr * ld + gs) : &kZeroEntry);
    }
    __device__ __forceinline__ void load(const double* __restrict__ P, int64_t ld, int64_t r0, int64_t s0,
                                         int64_t rlim, int64_t slim, int tid) {
#pragma unroll
        for (int i = 0; i < N; ++i) load_elem(i, P, ld, r0, s0, rlim, slim, tid);
    }
    // Interior staging: when every entry of the stage lies inside the
    // operand, lane tid's entry i is at a wave-uniform address plus one
    // per-lane 32-bit byte offset (lane_offset), so each load is a scalar
    // base plus that offset with no per-entry address arithmetic.  origin
    // points at X(0, 0).
    static constexpr int CONT = TRANS ? R : S;       // contiguous extent
    static_assert(THREADS % CONT == 0, "threads must cover whole contiguous rows");
    static constexpr int RPP = THREADS / CONT;       // strided positions per pass
    __device__ __forceinline__ static uint32_t lane_offset(int64_t ld, int tid) {
        return (uint32_t)(((int64_t)(tid / CONT) * ld + tid % CONT) * (int64_t)sizeof(double));
    }
    __device__ __forceinline__ static bool fast_ld(int64_t ld) { return sbase_ld(ld); }
    __device__ __forceinline__ void load_elem_fast(int i, const double* origin, int64_t ld, uint32_t off) {
        v[i] = load_sbase(origin + (int64_t)i * RPP * ld, off);
    }
    __device__ __forceinline__ void store_elem(int i, double* __restrict__ L, int lld, int tid) const {
        int r, s;
        coord(tid + i * THREADS, r, s);
        L[r * lld + s] = v[i];
    }
    __device__ __forceinline__ void store(double* __restrict__ L, int lld, int tid) const {
#pragma unroll
        for (int i = 0; i < N; ++i) store_elem(i, L, lld, tid);
    }
    // X(r, s) from tile-major slabs of 16 columns (row pitch 16, consecutive
    // slabs slab_stride apart): X(r, s) = P[(s / 16) * slab_stride + r * 16 +
    // s % 16] for s < slim (the columns the storage holds; zero-padded up to
    // there), zero beyond.
    __device__ __forceinline__ void load_slabs_elem(int i, const double* __restrict__ P, int64_t slab_stride,
                                                    int64_t slim, int tid) {
        static_assert(!TRANS, "slabs hold rows of 16 consecutive columns");
        int r, s;
        coord(tid + i * THREADS, r, s);
        v[i] = *(s < slim ? P + (int64_t)(s / 16) * slab_stride + r * 16 + s % 16 : &kZeroEntry);   // as in load
    }
    __device__ __forceinline__ void load_slabs(const double* __restrict__ P, int64_t slab_stride, int64_t slim,
                                               int tid) {
#pragma unroll
        for (int i = 0; i < N; ++i) load_slabs_elem(i, P, slab_stride, slim, tid);
    }
};

// Unchecked staging for tiles that lie wholly inside the operand.  Thread tid
// loads elements e = tid + i*THREADS; because THREADS is a multiple of the
// contiguous extent, element i sits at a fixed offset i*step from element 0,
// so one pointer per thread plus a wave-uniform step address every load.
template <int R, int S, int THREADS, bool TRANS>
struct FastStage {
    static constexpr int N = (R * S) / THREADS;
    static constexpr int CONT = TRANS ? R : S;       // contiguous extent
    static_assert(THREADS % CONT == 0, "threads must cover whole contiguous rows");
    static constexpr int ROWS_PER_PASS = THREADS / CONT;
    double v[N];
    const double* p;   // this thread's element 0 for the current slice
    int64_t step;      // distance between consecutive elements i (elements)

    // X(r, s) as in Stage; (r0, s0) is the tile origin.
    __device__ __forceinline__ void init(const double* __restrict__ P, int64_t ld, int64_t r0, int64_t s0, int tid) {
        const int c = tid % CONT, q = tid / CONT;
        if (TRANS) p = P + (s0 + q) * ld + r0 + c;
        else       p = P + (r0 + q) * ld + s0 + c;
        step = (int64_t)ROWS_PER_PASS * ld;
    }
    __device__ __forceinline__ void advance(int64_t delta) { p += delta; }
    __device__ __forceinline__ void load() {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = p[i * step];
    }
    __device__ __forceinline__ void store(double* __restrict__ L, int lld, int tid) const {
        const int c = tid % CONT, q = tid / CONT;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int rr = q + i * ROWS_PER_PASS;  // index along the strided extent
            if (TRANS) L[c * lld + rr] = v[i];
            else       L[rr * lld + c] = v[i];
        }
    }
};

// Predicated staging for any tile: like FastStage (one pointer per thread,
// wave-uniform stride), but each thread knows how many of its N elements lie
// inside the operand (nv) and whether its contiguous coordinate does; the
// others read as zero.  For an interior tile every element is valid.
template <int R, int S, int THREADS, bool TRANS>
struct PStage {
    static constexpr int N = (R * S) / THREADS;
    static constexpr int CONT = TRANS ? R : S;       // contiguous extent
    static_assert(THREADS % CONT == 0, "threads must cover whole contiguous rows");
    static constexpr int RPP = THREADS / CONT;       // strided positions per pass
    double v[N];

    // X(r, s) = P[(r0 + r) * ld + s0 + s] (!TRANS) or P[(s0 + s) * ld + r0 + r]
    // (TRANS); valid where r0 + r < rlim and s0 + s < slim.
    __device__ __forceinline__ void load(const double* __restrict__ P, int64_t ld, int64_t r0, int64_t s0,
                                         int64_t rlim, int64_t slim, int tid) {
        const int c = tid % CONT, q = tid / CONT;
        const int64_t gc = (TRANS ? r0 : s0) + c, lim_c = TRANS ? rlim : slim;
        const int64_t gq = (TRANS ? s0 : r0) + q, lim_q = TRANS ? slim : rlim;
        const int64_t rem = lim_q - gq;
        int nv = rem <= 0 ? 0 : (int)((rem + RPP - 1) / RPP);
        if (nv > N || gc >= lim_c) nv = gc >= lim_c ? 0 : N;
        const double* p = P + gq * ld + gc;
        const int64_t step = (int64_t)RPP * ld;
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = (i < nv) ? p[i * step] : 0.0;
    }
    __device__ __forceinline__ void store(double* __restrict__ L, int lld, int tid) const {
        const int c = tid % CONT, q = tid / CONT;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int rr = q + i * RPP;
            if (TRANS) L[c * lld + rr] = v[i];
            else       L[rr * lld + c] = v[i];
        }
    }
};

// Micro-kernel: acc += A(:, a_k0 : a_k0 + 4*ksteps) * B(b_k0 : ..., :) from LDS.
// A is read from As[m][k] (pitch a_ld), B from Bs[k][n] (pitch b_ld).
template <class CF, int KSTEPS>
__device__ __forceinline__ void mma_lds(const double* __restrict__ As, int a_ld, int a_k0,
                                        const double* __restrict__ Bs, int b_ld, int b_k0,
                                        d4 (&acc)[CF::BM][CF::BN], int wm, int wn, int lane) {
    const int li = lane & 15, lk = lane >> 4;
    const double* ap = As + (wm * CF::WTM + li) * a_ld + a_k0 + lk;
    const double* bp = Bs + (b_k0 + lk) * b_ld + wn * CF::WTN + li;
#pragma unroll
    for (int kk = 0; kk < KSTEPS; ++kk) {
        double a[CF::BM], b[CF::BN];
#pragma unroll
        for (int i = 0; i < CF::BM; ++i) a[i] = ap[i * 16 * a_ld + kk * 4];
#pragma unroll
        for (int j = 0; j < CF::BN; ++j) b[j] = bp[kk * 4 * b_ld + j * 16];
#pragma unroll
        for (int i = 0; i < CF::BM; ++i)
#pragma unroll
            for (int j = 0; j < CF::BN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// The same micro-kernel with the fragments of step kk + 1 read from LDS
// before the MFMAs of step kk are issued (two fragment register sets), so a
// wave waits for LDS once per slice rather than once per 4-deep step.  For
// small wave tiles, whose four MFMAs per step do not cover an LDS read.
// between(kk) runs in step kk, after those reads and before its MFMAs: work
// placed there (staging loads and stores) is spread over the MFMA stream
// instead of stalling it all at once.
template <class CF, int KSTEPS, class Between>
__device__ __forceinline__ void mma_lds_pipe(const double* __restrict__ As, int a_ld, int a_k0,
                                             const double* __restrict__ Bs, int b_ld, int b_k0,
                                             d4 (&acc)[CF::BM][CF::BN], int wm, int wn, int lane,
                                             Between&& between) {
    const int li = lane & 15, lk = lane >> 4;
    const double* ap = As + (wm * CF::WTM + li) * a_ld + a_k0 + lk;
    const double* bp = Bs + (b_k0 + lk) * b_ld + wn * CF::WTN + li;
    double a[2][CF::BM], b[2][CF::BN];
#pragma unroll
    for (int i = 0; i < CF::BM; ++i) a[0][i] = ap[i * 16 * a_ld];
#pragma unroll
    for (int j = 0; j < CF::BN; ++j) b[0][j] = bp[j * 16];
#pragma unroll
    for (int kk = 0; kk < KSTEPS; ++kk) {
        const int cur = kk & 1;
        if (kk + 1 < KSTEPS) {
#pragma unroll
            for (int i = 0; i < CF::BM; ++i) a[cur ^ 1][i] = ap[i * 16 * a_ld + (kk + 1) * 4];
#pragma unroll
            for (int j = 0; j < CF::BN; ++j) b[cur ^ 1][j] = bp[(kk + 1) * 4 * b_ld + j * 16];
        }
        between(kk);
        __builtin_amdgcn_sched_barrier(0);   // keep the next step's reads ahead of these MFMAs
#pragma unroll
        for (int i = 0; i < CF::BM; ++i)
#pragma unroll
            for (int j = 0; j < CF::BN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <class CF>
__device__ __forceinline__ void zero_acc(d4 (&acc)[CF::BM][CF::BN]) {
#pragma unroll
    for (int i = 0; i < CF::BM; ++i)
#pragma unroll
        for (int j = 0; j < CF::BN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

// One entry of the epilogue, alpha * acc + beta * c with the product alpha * acc
// rounded first and beta * c fused into the addition (beta == 0: c is
// ignored).  Every epilogue and the batched k-split reduction use this form,
// so a result written in several passes rounds the same way wherever the
// passes run.
__device__ __forceinline__ double epilogue_value(double alpha, double acc, double beta, double c) {
    const double v = alpha * acc;
    return beta != 0.0 ? __builtin_fma(beta, c, v) : v;
}

// Epilogue: C = alpha * acc + beta * C on the workgroup tile at (m0, n0);
// beta == 0 does not read C.  Sixteen consecutive lanes write one 128-byte row
// segment.
// TRI = 1 (2): store only the entries with row >= col (row <= col), the
// triangle of a symmetric update; TRI = 0 stores the whole tile.
template <class CF, int TRI>
__device__ __forceinline__ void store_c_tri(const d4 (&acc)[CF::BM][CF::BN], double alpha, double beta,
                                        double* __restrict__ C, int64_t ldc, int64_t m0, int64_t n0,
                                        int64_t M, int64_t N, int wm, int wn, int lane) {
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < CF::BM; ++i) {
        // One block row of the wave tile at a time: its C values are all
        // loaded before any is used (an entry outside C reads C[0] and is
        // discarded), so the reads cost one memory latency, not one each.
        double cv[CF::BN][4];
        if (beta != 0.0) {
#pragma unroll
            for (int j = 0; j < CF::BN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + wm * CF::WTM + i * 16 + lk + 4 * r;
                    const int64_t col = n0 + wn * CF::WTN + j * 16 + li;
                    const bool in = row < M && col < N && (TRI == 0 || (TRI == 1 ? row >= col : row <= col));
                    cv[j][r] = C[in ? row * ldc + col : 0];
                }
        }
#pragma unroll
        for (int j = 0; j < CF::BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * CF::WTM + i * 16 + lk + 4 * r;
                const int64_t col = n0 + wn * CF::WTN + j * 16 + li;
                if (row < M && col < N && (TRI == 0 || (TRI == 1 ? row >= col : row <= col)))
                    C[row * ldc + col] = epilogue_value(alpha, acc[i][j][r], beta, beta != 0.0 ? cv[j][r] : 0.0);
            }
    }
}

// The C values the epilogue of the tile at (m0, n0) reads, loaded ahead of
// it so that their latency overlaps MFMAs.  Every lane loads: an entry
// outside C, or every entry when !read (beta = 0, C is not read), comes from
// kZeroEntry.
template <class CF>
__device__ __forceinline__ void load_c(double (&cv)[CF::BM][CF::BN][4], const double* __restrict__ C, int64_t ldc,
                                       int64_t m0, int64_t n0, int64_t M, int64_t N, int wm, int wn, int lane,
                                       bool read) {
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < CF::BM; ++i)
#pragma unroll
        for (int j = 0; j < CF::BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * CF::WTM + i * 16 + lk + 4 * r;
                const int64_t col = n0 + wn * CF::WTN + j * 16 + li;
                cv[i][j][r] = *(read && row < M && col < N ? C + row * ldc + col : &kZeroEntry);
            }
}

// Epilogue with C already loaded (load_c): C = alpha * acc + beta * cv.
template <class CF>
__device__ __forceinline__ void store_c_loaded(const d4 (&acc)[CF::BM][CF::BN], double alpha, double beta,
                                               const double (&cv)[CF::BM][CF::BN][4], double* __restrict__ C,
                                               int64_t ldc, int64_t m0, int64_t n0, int64_t M, int64_t N, int wm,
                                               int wn, int lane) {
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < CF::BM; ++i)
#pragma unroll
        for (int j = 0; j < CF::BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * CF::WTM + i * 16 + lk + 4 * r;
                const int64_t col = n0 + wn * CF::WTN + j * 16 + li;
                if (row < M && col < N) C[row * ldc + col] = epilogue_value(alpha, acc[i][j][r], beta, cv[i][j][r]);
            }
}

// load_c and store_c_loaded for a tile that lies inside C (ldc below 2^24):
// each of a lane's entries is at a wave-uniform address (Cw, the wave's C
// origin, plus a multiple of 16 rows or columns) plus the lane offset coff =
// ((lane / 16) * ldc + lane % 16) * 8 bytes, so no entry needs address
// arithmetic or a bounds test.  With !read every entry loads kZeroEntry.
template <class CF>
__device__ __forceinline__ void load_c_fast(double (&cv)[CF::BM][CF::BN][4], const double* Cw, int64_t ldc,
                                            uint32_t coff, bool read) {
    const uint32_t co = read ? coff : 0u;
#pragma unroll
    for (int i = 0; i < CF::BM; ++i)
#pragma unroll
        for (int j = 0; j < CF::BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                cv[i][j][r] = load_sbase(read ? Cw + (int64_t)(i * 16 + 4 * r) * ldc + j * 16 : &kZeroEntry, co);
}
template <class CF>
__device__ __forceinline__ void store_c_fast(const d4 (&acc)[CF::BM][CF::BN], double alpha, double beta,
                                             const double (&cv)[CF::BM][CF::BN][4], double* Cw, int64_t ldc,
                                             uint32_t coff) {
#pragma unroll
    for (int i = 0; i < CF::BM; ++i)
#pragma unroll
        for (int j = 0; j < CF::BN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                store_sbase(Cw + (int64_t)(i * 16 + 4 * r) * ldc + j * 16, coff,
                            epilogue_value(alpha, acc[i][j][r], beta, cv[i][j][r]));
}

template <class CF>
__device__ __forceinline__ void store_c(const d4 (&acc)[CF::BM][CF::BN], double alpha, double beta,
                                        double* __restrict__ C, int64_t ldc, int64_t m0, int64_t n0,
                                        int64_t M, int64_t N, int wm, int wn, int lane) {
    store_c_tri<CF, 0>(acc, alpha, beta, C, ldc, m0, n0, M, N, wm, wn, lane);
}

// ---------------------------------------------------------------------------
// Register-resident C tile at (m0, n0): acc = the product of its A row panel
// and B column panel over k in [k_begin, k_end), through the double-buffered
// LDS stage.  (tm, tn) only staggers the k start (see below).
template <class CF, bool TA, bool TB, bool FAST_INTERIOR = true>
__device__ __forceinline__ void regc_acc(int64_t M, int64_t N, int64_t k_begin, int64_t k_end,
                                         const double* __restrict__ A, int64_t lda,
                                         const double* __restrict__ B, int64_t ldb, int64_t m0, int64_t n0, int tm,
                                         int tn, double (*As)[CF::MT * CF::A_LD], double (*Bs)[CF::KS * CF::B_LD],
                                         d4 (&acc)[CF::BM][CF::BN]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / CF::WN, wn = wave % CF::WN;

    zero_acc<CF>(acc);
    const int64_t nsl = (k_end - k_begin + CF::KS - 1) / CF::KS;
    // Tiles that share an A row panel (same tm) or a B column panel (same tn)
    // start their k loops a few slices apart and wrap around, so the
    // workgroups of one XCD do not all miss on the same lines at once.
    const int64_t s0 = nsl > 0 ? (int64_t)((tm + tn) & 7) % nsl : 0;
    const bool interior = FAST_INTERIOR && nsl > 0 && (m0 + CF::MT <= M) && (n0 + CF::NT <= N) &&
                          ((k_end - k_begin) % CF::KS == 0);
    if (interior) {
        // Whole tile inside the matrices: no predicates, pointer stepping.
        FastStage<CF::MT, CF::KS, CF::THREADS, TA> fa;
        FastStage<CF::KS, CF::NT, CF::THREADS, TB> fb;
        fa.init(A, lda, m0, k_begin + s0 * CF::KS, tid);
        fb.init(B, ldb, k_begin + s0 * CF::KS, n0, tid);
        const int64_t da = TA ? (int64_t)CF::KS * lda : CF::KS;   // A advances along k
        const int64_t db = TB ? CF::KS : (int64_t)CF::KS * ldb;   // B advances along k
        fa.load();
        fb.load();
        fa.store(As[0], CF::A_LD, tid);
        fb.store(Bs[0], CF::B_LD, tid);
        __syncthreads();
        for (int64_t sl = 0; sl < nsl; ++sl) {
            const int cur = (int)(sl & 1);
            const bool more = sl + 1 < nsl;
            if (more) {
                const bool wrap = (s0 + sl + 1) == nsl;  // next slice index wraps to k_begin
                fa.advance(wrap ? da * (1 - nsl) : da);
                fb.advance(wrap ? db * (1 - nsl) : db);
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
    } else if (nsl > 0) {
        PStage<CF::MT, CF::KS, CF::THREADS, TA> sa;
        PStage<CF::KS, CF::NT, CF::THREADS, TB> sb;
        int64_t kb = k_begin + s0 * CF::KS;
        sa.load(A, lda, m0, kb, M, k_end, tid);
        sb.load(B, ldb, kb, n0, k_end, N, tid);
        sa.store(As[0], CF::A_LD, tid);
        sb.store(Bs[0], CF::B_LD, tid);
        __syncthreads();
        for (int64_t sl = 0; sl < nsl; ++sl) {
            const int cur = (int)(sl & 1);
            const bool more = sl + 1 < nsl;
            if (more) {
                int64_t nx = s0 + sl + 1;
                if (nx >= nsl) nx -= nsl;
                kb = k_begin + nx * CF::KS;
                sa.load(A, lda, m0, kb, M, k_end, tid);
                sb.load(B, ldb, kb, n0, k_end, N, tid);
            }
            mma_lds<CF, CF::KS / 4>(As[cur], CF::A_LD, 0, Bs[cur], CF::B_LD, 0, acc, wm, wn, lane);
            if (more) {
                sa.store(As[cur ^ 1], CF::A_LD, tid);
                sb.store(Bs[cur ^ 1], CF::B_LD, tid);
            }
            __syncthreads();
        }
    }
}

// regc_acc, then C = alpha*acc + beta*C on the tile.  Shared by k_regc, SYRK
// and the persistent batched kernel.
template <class CF, bool TA, bool TB, bool FAST_INTERIOR = true, int TRI = 0>
__device__ __forceinline__ void regc_tile(int64_t M, int64_t N, int64_t k_begin, int64_t k_end, double alpha,
                                          const double* __restrict__ A, int64_t lda,
                                          const double* __restrict__ B, int64_t ldb, double beta,
                                          double* __restrict__ C, int64_t ldc, int64_t m0, int64_t n0, int tm,
                                          int tn, double (*As)[CF::MT * CF::A_LD],
                                          double (*Bs)[CF::KS * CF::B_LD]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    d4 acc[CF::BM][CF::BN];
    regc_acc<CF, TA, TB, FAST_INTERIOR>(M, N, k_begin, k_end, A, lda, B, ldb, m0, n0, tm, tn, As, Bs, acc);
    store_c_tri<CF, TRI>(acc, alpha, beta, C, ldc, m0, n0, M, N, wave / CF::WN, wave % CF::WN, lane);
}

// k_regc: one C granule (MT x NT) per workgroup, accumulated in registers over
// k in [k_begin, k_end); C = alpha*acc + beta*C at the end.
template <class CF, bool TA, bool TB>
__global__ __launch_bounds__(CF::THREADS) __attribute__((amdgpu_waves_per_eu(CF::MT >= 128 ? 2 : 1)))
void k_regc(int64_t M, int64_t N, int64_t k_begin, int64_t k_end, double alpha, const double* __restrict__ A,
            int64_t lda, const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C,
            int64_t ldc, Sched s) {
    __shared__ double As[2][CF::MT * CF::A_LD];
    __shared__ double Bs[2][CF::KS * CF::B_LD];
    int tm, tn;
    decode_tile(s, blockIdx.x, tm, tn);
    const int64_t m0 = s.m_off + (int64_t)tm * CF::MT;
    const int64_t n0 = s.n_off + (int64_t)tn * CF::NT;
    regc_tile<CF, TA, TB>(M, N, k_begin, k_end, alpha, A, lda, B, ldb, beta, C, ldc, m0, n0, tm, tn, As, Bs);
}

// ---------------------------------------------------------------------------
// The A-resident kernel k_a2 loads its A block into LDS once per k chunk and
// then only reads it, so the workgroup synchronises twice per chunk and never
// per slice.  B streams from the L2 (through the vector L1) straight into
// registers, as the Goto loop nest streams its B micro-panels through the L1
// (Sec. 5.2): each wave loads exactly the MFMA fragments it uses, one 32-deep
// slice ahead in a ring of two register sets, one MFMA step's fragments per
// step.  Without a barrier per slice the waves of a workgroup drift apart.
// Two workgroups of one row of four waves share a CU and its SIMDs: a wave
// waiting for memory, or its workgroup refilling its A block at a chunk
// start, leaves the MFMA unit to the other workgroup's waves.

// Fragments of a streamed operand for one wave and one slice: f[kk][x] is the
// operand of MFMA step kk for 16-row (A) or 16-column (B) block x.
template <int KSTEPS, int NX>
struct Frag {
    double f[KSTEPS][NX];
};

// acc += A(:, a_k0 : a_k0 + 4*KSTEPS) * B with A fragments read from LDS
// (As[m][k], pitch a_ld; the reads of step kk + 1 are issued before the MFMAs
// of step kk) and B fragments from registers.  between(kk) runs in step kk
// before its MFMAs (the next slice's loads go there).
template <class CF, int KSTEPS, class Between>
__device__ __forceinline__ void mma_a_lds_b_reg(const double* __restrict__ As, int a_ld, int a_k0,
                                                const double (&bf)[KSTEPS][CF::BN], d4 (&acc)[CF::BM][CF::BN],
                                                int wm, int lane, Between&& between) {
    const int li = lane & 15, lk = lane >> 4;
    const double* ap = As + (wm * CF::WTM + li) * a_ld + a_k0 + lk;
    double a[2][CF::BM];
#pragma unroll
    for (int i = 0; i < CF::BM; ++i) a[0][i] = ap[i * 16 * a_ld];
#pragma unroll
    for (int kk = 0; kk < KSTEPS; ++kk) {
        const int cur = kk & 1;
        if (kk + 1 < KSTEPS) {
#pragma unroll
            for (int i = 0; i < CF::BM; ++i) a[cur ^ 1][i] = ap[i * 16 * a_ld + (kk + 1) * 4];
        }
        between(kk);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < CF::BM; ++i)
#pragma unroll
            for (int j = 0; j < CF::BN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], bf[kk][j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Where a wave's streamed slice lies: its origin, whether all of it is inside
// the operand (then each fragment is a scalar base plus the lane offset), and
// the coordinates of the origin for the predicated form.
struct SlicePlan {
    const double* origin;
    bool interior;
    int64_t k0, x0;
};

// ---------------------------------------------------------------------------
// k_a2: granule = MT rows x (nj * NT) columns.  For each kc chunk of
// [k_begin, k_end) (kc a multiple of KS, at most KC, the depth the LDS block
// is laid out for) the A block (MT x kc) is loaded into LDS once and reused for
// every n-tile of the granule; the B slices stream into registers (above).  C
// is read-modified-written once per chunk: beta applies to the chunk starting
// at k = 0, later chunks accumulate.  With PACKED, B comes from a packed panel
// laid out [n-tile][k][NT] (rows of NT doubles, zero-padded, ldb rows per
// n-tile), whose origin is (pk0, pn0) in B's coordinates; n-tiles are
// numbered from pn0.  With TILED, A is tile-major (128 x 16 slabs; MT divides
// 128).  Registers are capped for two waves per SIMD, so that two four-wave
// workgroups fit a CU.
template <class CF, int KC, bool TA, bool TB, bool PACKED, bool TILED = false>
__global__ __launch_bounds__(CF::THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_a2(int64_t M, int64_t N, int64_t k_begin, int64_t k_end,
                                                    double alpha, const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb, double beta,
                                                    double* __restrict__ C, int64_t ldc, Sched s, int nj,
                                                    int64_t pk0, int64_t pn0, int kc) {
    static_assert(KC % CF::KS == 0, "KC must be a multiple of the slice depth");
    static_assert(!TILED || (CF::KS % 16 == 0 && KC % 16 == 0 && 128 % CF::MT == 0),
                  "tile-major slices start on slab boundaries and blocks sit inside 128-row panels");
    constexpr int AB_LD = KC + 1;
    constexpr int KSTEPS = CF::KS / 4;
    __shared__ double As[CF::MT * AB_LD];
    int tm, tn;
    decode_tile(s, blockIdx.x, tm, tn);
    const int64_t m0 = s.m_off + (int64_t)tm * CF::MT;
    const int64_t nbeg = s.n_off + (int64_t)tn * nj * CF::NT;
    const int64_t nend = (nbeg + (int64_t)nj * CF::NT) < s.n_lim ? (nbeg + (int64_t)nj * CF::NT) : s.n_lim;
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: wave-level addresses stay scalar
    const int wm = wave / CF::WN, wn = wave % CF::WN;
    const int ntiles = (int)((nend - nbeg + CF::NT - 1) / CF::NT);
    const uint32_t coff = (uint32_t)(((int64_t)(lane >> 4) * ldc + (lane & 15)) * 8);
    // every chunk below has at least one step, so no load is conditional
    if (ntiles <= 0) return;

    using SA = Stage<CF::MT, CF::KS, CF::THREADS, TA>;
    const uint32_t aoff = SA::lane_offset(lda, tid);
    // tile-major A: this thread's entry of a 32-deep slice within its two
    // 128 x 16 slabs (element (r, s) of the block at slab s / 16, row r)
    const uint32_t aoff_slab = (uint32_t)((((tid % CF::KS) / 16) * 2048 + (tid / CF::KS) * 16 + tid % 16) * 8);
    // B fragment (kk, x) of a wave's slice: k = 4 kk + lk, n = 16 x + li from
    // the slice origin (column wn * WTN of its n-tile)
    const int64_t ldbs = PACKED ? CF::NT : ldb;
    const int64_t bks = TB ? 1 : ldbs, bxs = TB ? ldbs : 1;   // element strides along k and along n
    const uint32_t blane = (uint32_t)(((int64_t)lk * bks + (int64_t)li * bxs) * 8);
    Frag<KSTEPS, CF::BN> bq[2];
    d4 acc[CF::BM][CF::BN];

    for (int64_t kb = k_begin; kb < k_end; kb += kc) {
        const int64_t kbe = (kb + kc) < k_end ? (kb + kc) : k_end;
        const int nsl = (int)((kbe - kb + CF::KS - 1) / CF::KS);
        const int total = ntiles * nsl;
        auto b_plan = [&](int t) {
            const int j = t / nsl, sl = t - (t / nsl) * nsl;
            SlicePlan p;
            if (PACKED) {
                // panel rows from (kb - pk0 + sl*KS) of n-tile ((nbeg - pn0)/NT + j);
                // ldb is the panel height (kc for a per-chunk pack, the padded
                // k for a tile-major B); rows past it read as zero
                const int64_t row0 = (kb - pk0) + (int64_t)sl * CF::KS;
                p.origin = B + ((nbeg - pn0) / CF::NT + j) * ldb * CF::NT + row0 * CF::NT + wn * CF::WTN;
                p.interior = row0 + CF::KS <= ldb;
                p.k0 = row0;
                p.x0 = 0;
            } else {
                const int64_t k0 = kb + (int64_t)sl * CF::KS, c0 = nbeg + (int64_t)j * CF::NT + wn * CF::WTN;
                p.origin = TB ? B + c0 * ldb + k0 : B + k0 * ldb + c0;
                p.interior = k0 + CF::KS <= kbe && c0 + CF::WTN <= nend && sbase_ld(ldb);
                p.k0 = k0;
                p.x0 = c0;
            }
            return p;
        };
        auto b_load = [&](const SlicePlan& p, int kk, int x) -> double {
            if (p.interior) return load_sbase(p.origin + (int64_t)(4 * kk) * bks + (int64_t)(16 * x) * bxs, blane);
            const int64_t kr = 4 * kk + lk, nc = 16 * x + li;
            const bool ok = PACKED ? p.k0 + kr < ldb : (p.k0 + kr < kbe && p.x0 + nc < nend);
            return *(ok ? p.origin + kr * bks + nc * bxs : &kZeroEntry);
        };
        // The chunk's A block goes to LDS in rounds of slices through two
        // register sets: a round's loads are in flight while the round before
        // it is stored.  The first round is loaded before the barrier that
        // waits for the previous chunk's readers of As.  A chunk whose block
        // lies wholly inside A takes the unchecked loads for every slice, in
        // one round (all of the block's loads in flight at once); an edge
        // chunk takes the checked ones, two slices a round.  Deciding once
        // per chunk keeps the checked path's per-entry addresses out of the
        // fast path's registers.  Tile-major A is zero-padded to whole row
        // panels and slabs, so there every chunk of full slices is interior.
        constexpr int NSL = KC / CF::KS;
        const bool fast = kbe - kb == (int64_t)nsl * CF::KS && (TILED || (m0 + CF::MT <= M && SA::fast_ld(lda)));
        auto rounds = [&](auto kround_tag, auto load_slice) {
            constexpr int KR = decltype(kround_tag)::value;
            auto load_round = [&](SA (&set)[KR], int c0) {
#pragma unroll
                for (int u = 0; u < KR; ++u)
                    if (c0 + u < nsl) load_slice(set[u], c0 + u);
            };
            auto store_round = [&](const SA (&set)[KR], int c0) {
#pragma unroll
                for (int u = 0; u < KR; ++u)
                    if (c0 + u < nsl) set[u].store(As + (c0 + u) * CF::KS, AB_LD, tid);
            };
            SA sq[2][KR];
            load_round(sq[0], 0);
            __syncthreads();  // the previous chunk's readers of As are done
#pragma unroll
            for (int c0 = 0; c0 < NSL; c0 += 2 * KR) {
                if (c0 + KR < NSL) load_round(sq[1], c0 + KR);
                store_round(sq[0], c0);
                if (c0 + 2 * KR < NSL) load_round(sq[0], c0 + 2 * KR);
                if (c0 + KR < NSL) store_round(sq[1], c0 + KR);
            }
        };
        if (fast) {
            rounds(std::integral_constant<int, NSL>{}, [&](SA& st, int c) {
                const int64_t kk = kb + (int64_t)c * CF::KS;
                if constexpr (TILED) {
                    // entry e of this thread: slab row (tid / KS) + e * RPP
                    // of the slabs at kk, column tid % KS (aoff_slab)
                    const double* P = A + ((m0 / 128) * lda + kk / 16) * 2048 + (m0 % 128) * 16;
#pragma unroll
                    for (int e = 0; e < SA::N; ++e) st.v[e] = load_sbase(P + (int64_t)e * SA::RPP * 16, aoff_slab);
                } else {
#pragma unroll
                    for (int e = 0; e < SA::N; ++e)
                        st.load_elem_fast(e, TA ? A + kk * lda + m0 : A + m0 * lda + kk, lda, aoff);
                }
            });
        } else {
            rounds(std::integral_constant<int, 2>{}, [&](SA& st, int c) {
                const int64_t kk = kb + (int64_t)c * CF::KS;
                if constexpr (TILED) {
                    // tile-major A: 128 x 16 slabs, lda = slabs per row panel,
                    // zero beyond the matrix (m0 is a multiple of MT, which
                    // divides 128: the block is rows m0 % 128 .. of its
                    // slabs; a slice starts on a slab boundary)
                    const double* P = A + ((m0 / 128) * lda + kk / 16) * 2048 + (m0 % 128) * 16;
                    st.load_slabs(P, 2048, lda * 16 - kk, tid);
                } else {
                    st.load(A, lda, m0, kk, M, kbe, tid);
                }
            });
        }
        {   // the first B slice, once the A block's registers are free
            const SlicePlan p0 = b_plan(0);
#pragma unroll
            for (int kk = 0; kk < KSTEPS; ++kk)
#pragma unroll
                for (int x = 0; x < CF::BN; ++x) bq[0].f[kk][x] = b_load(p0, kk, x);
        }
        __syncthreads();
        zero_acc<CF>(acc);
        const double beta_eff = (kb == 0) ? beta : 1.0;
        double cv[CF::BM][CF::BN][4];
        // Step t computes slice t (n-tile t / nsl, slice t % nsl) from cur
        // and loads slice t + 1 (clamped to the last) into nxt, spread over
        // its MFMA steps.  A tile's last step is a copy of its own (LAST):
        // it first loads the tile's C values and ends with the epilogue.
        // Every path of a step issues the same loads, so the compiler can
        // count those in flight and wait only for the fragments an MFMA uses.
        auto step = [&](auto last_tag, int t, auto& cur, auto& nxt) {
            constexpr bool LAST = decltype(last_tag)::value;
            const int j = t / nsl, sl = t - j * nsl;
            const int64_t n0 = nbeg + (int64_t)j * CF::NT;
            const bool cin = m0 + CF::MT <= M && n0 + CF::NT <= nend && sbase_ld(ldc);   // tile inside C
            double* Cw = C + (m0 + wm * CF::WTM) * ldc + n0 + wn * CF::WTN;
            if constexpr (LAST) {
                if (cin) load_c_fast<CF>(cv, Cw, ldc, coff, beta_eff != 0.0);
                else     load_c<CF>(cv, C, ldc, m0, n0, M, nend, wm, wn, lane, beta_eff != 0.0);
            }
            const SlicePlan p = b_plan(t + 1 < total ? t + 1 : total - 1);
            mma_a_lds_b_reg<CF, KSTEPS>(As, AB_LD, sl * CF::KS, cur.f, acc, wm, lane, [&](int kk) {
#pragma unroll
                for (int x = 0; x < CF::BN; ++x) nxt.f[kk][x] = b_load(p, kk, x);
            });
            if constexpr (LAST) {
                if (cin) store_c_fast<CF>(acc, alpha, beta_eff, cv, Cw, ldc, coff);
                else     store_c_loaded<CF>(acc, alpha, beta_eff, cv, C, ldc, m0, n0, M, nend, wm, wn, lane);
                zero_acc<CF>(acc);
            }
        };
        auto any_step = [&](int t, auto& cur, auto& nxt) {
            if (t % nsl == nsl - 1) step(std::true_type{}, t, cur, nxt);
            else                    step(std::false_type{}, t, cur, nxt);
        };
        // two steps per iteration (the ring's register sets stay fixed); an
        // odd last step is peeled
        int t = 0;
#pragma unroll 1
        for (; t + 1 < total; t += 2) {
            any_step(t, bq[0], bq[1]);
            any_step(t + 1, bq[1], bq[0]);
        }
        if (t < total) any_step(t, bq[0], bq[1]);
    }
}

// Depth of the register ring that streams k_b2's A slices (a 32-deep slice
// is about 2 us of MFMAs).
constexpr int kRing = 2;

// ---------------------------------------------------------------------------
// k_b2: mirror of k_a2.  Granule = (mi * MT) rows x NT columns; for each KC
// chunk the B block (KC x NT) is resident in LDS and reused for every m-tile.
// Unlike k_a2, the A slices stream through two LDS buffers (a register ring
// of two sets, one slice entry stored and one refilled per MFMA step): each
// wave reading its own A fragments from memory would read 16 rows of 32
// bytes per load, which measured slower.  With TILED, A is tile-major
// (128 x 16 slabs, lda = slabs per row panel) and B comes from tile-major
// 128-column panels (ldb = the padded k; NT divides 128), both zero beyond
// the matrix.
template <class CF, int KC, bool TA, bool TB, bool TILED = false>
__global__ __launch_bounds__(CF::THREADS) void k_b2(int64_t M, int64_t N, int64_t k_begin, int64_t k_end,
                                                    double alpha, const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb, double beta,
                                                    double* __restrict__ C, int64_t ldc, Sched s, int mi) {
    static_assert(KC % CF::KS == 0, "KC must be a multiple of the slice depth");
    static_assert(!TILED || (CF::KS % 16 == 0 && KC % 16 == 0 && 128 % CF::MT == 0 && 128 % CF::NT == 0),
                  "tile-major slices start on slab boundaries and tiles sit inside 128-wide panels");
    __shared__ double Bs[KC * CF::B_LD];
    __shared__ double As[2][CF::MT * CF::A_LD];
    int tm, tn;
    decode_tile(s, blockIdx.x, tm, tn);
    const int64_t mbeg = s.m_off + (int64_t)tm * mi * CF::MT;
    const int64_t mend = (mbeg + (int64_t)mi * CF::MT) < s.m_lim ? (mbeg + (int64_t)mi * CF::MT) : s.m_lim;
    const int64_t n0 = s.n_off + (int64_t)tn * CF::NT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform, as in k_a2
    const int wm = wave / CF::WN, wn = wave % CF::WN;
    const int mtiles = (int)((mend - mbeg + CF::MT - 1) / CF::MT);
    const uint32_t coff = (uint32_t)(((int64_t)(lane >> 4) * ldc + (lane & 15)) * 8);
    if (mtiles <= 0) return;   // as in k_a2: every chunk has a step

    using SA = Stage<CF::MT, CF::KS, CF::THREADS, TA>;
    using SB = Stage<CF::KS, CF::NT, CF::THREADS, TB>;
    SA sa[kRing];
    d4 acc[CF::BM][CF::BN];
    const uint32_t aoff = SA::lane_offset(lda, tid), boff = SB::lane_offset(TILED ? 128 : ldb, tid);
    // tile-major A: lane offset within a slice of 128 x 16 slabs (entry i
    // of a lane is RPP rows further down the same slab)
    const uint32_t aoff_slab = (uint32_t)((((tid % CF::KS) / 16) * 2048 + (tid / CF::KS) * 16 + tid % 16) * 8);

    for (int64_t kb = k_begin; kb < k_end; kb += KC) {
        const int64_t kbe = (kb + KC) < k_end ? (kb + KC) : k_end;
        const int nsl = (int)((kbe - kb + CF::KS - 1) / CF::KS);
        const int total = mtiles * nsl;
        // element e of A slice t of this chunk (m-tile t / nsl, slice t % nsl)
        auto load_a = [&](auto& st, int t, int e) {
            const int i = t / nsl, sl = t - (t / nsl) * nsl;
            const int64_t r0 = mbeg + (int64_t)i * CF::MT, kk = kb + (int64_t)sl * CF::KS;
            if constexpr (TILED) {
                const double* P = A + ((r0 / 128) * lda + kk / 16) * 2048 + (r0 % 128) * 16;
                st.load_slabs_elem(e, P, 2048, lda * 16 - kk, tid);
            } else {
                st.load_elem(e, A, lda, r0, kk, mend, kbe, tid);
            }
        };
        // all of A slice t: the interior form when the slice lies inside A
        // (as load_b_all in k_a2)
        auto a_plan = [&](int t, bool& interior, const double*& origin) {
            const int i = t / nsl, sl = t - (t / nsl) * nsl;
            const int64_t r0 = mbeg + (int64_t)i * CF::MT, kk = kb + (int64_t)sl * CF::KS;
            if constexpr (TILED) {
                origin = A + ((r0 / 128) * lda + kk / 16) * 2048 + (r0 % 128) * 16;
                interior = kk + CF::KS <= lda * 16;
            } else {
                origin = TA ? A + kk * lda + r0 : A + r0 * lda + kk;
                interior = r0 + CF::MT <= mend && kk + CF::KS <= kbe && SA::fast_ld(lda);
            }
        };
        auto load_a_elem = [&](auto& st, int t, int e, bool interior, const double* origin) {
            if (interior) {
                if constexpr (TILED) st.v[e] = load_sbase(origin + (int64_t)e * SA::RPP * 16, aoff_slab);   // RPP rows of 16 further
                else                 st.load_elem_fast(e, origin, lda, aoff);
            } else {
                load_a(st, t, e);
            }
        };
        auto load_a_all = [&](auto& st, int t) {
            bool interior;
            const double* origin;
            a_plan(t, interior, origin);
#pragma unroll
            for (int e = 0; e < SA::N; ++e) load_a_elem(st, t, e, interior, origin);
        };
        // The chunk's B block and its first kRing A slices are all loaded
        // into registers at once, then stored to LDS once the previous
        // chunk's readers are done (as in k_a2).
        SB sq[KC / CF::KS];
#pragma unroll
        for (int c = 0; c < KC / CF::KS; ++c) {
            if (c >= nsl) break;
            const int64_t kk = kb + (int64_t)c * CF::KS;
            if (TILED) {   // 128-column panels of ldb rows, k-major; the block is columns n0 % 128 ..
                const double* P = B + (n0 / 128) * ldb * 128 + n0 % 128;
                if (kk + CF::KS <= ldb) {
#pragma unroll
                    for (int e = 0; e < SB::N; ++e) sq[c].load_elem_fast(e, P + kk * 128, 128, boff);
                } else {
                    sq[c].load(P, 128, kk, 0, ldb, CF::NT, tid);
                }
            } else if (kk + CF::KS <= kbe && n0 + CF::NT <= N && SB::fast_ld(ldb)) {
#pragma unroll
                for (int e = 0; e < SB::N; ++e)
                    sq[c].load_elem_fast(e, TB ? B + n0 * ldb + kk : B + kk * ldb + n0, ldb, boff);
            } else {
                sq[c].load(B, ldb, kk, n0, kbe, N, tid);
            }
        }
        // A slices kRing ahead through a ring of register sets (as the B
        // slices of k_a2)
#pragma unroll
        for (int u = 0; u < kRing; ++u) load_a_all(sa[u], u < total ? u : total - 1);
        __syncthreads();  // previous chunk's readers of As / Bs are done
#pragma unroll
        for (int c = 0; c < KC / CF::KS; ++c) {
            if (c >= nsl) break;
            sq[c].store(Bs + c * CF::KS * CF::B_LD, CF::B_LD, tid);
        }
        sa[0].store(As[0], CF::A_LD, tid);
        __syncthreads();
        zero_acc<CF>(acc);
        const double beta_eff = (kb == 0) ? beta : 1.0;
        double cv[CF::BM][CF::BN][4];
        // the steps of k_a2 with the roles of A and B exchanged
        auto step = [&](int t, auto& reload, auto& ready) {
            const int cur = t & 1;
            const int i = t / nsl, sl = t - i * nsl;
            const int64_t r0 = mbeg + (int64_t)i * CF::MT;
            const bool last = sl == nsl - 1;
            const int tr = t + kRing < total ? t + kRing : total - 1;
            const bool cin = r0 + CF::MT <= mend && n0 + CF::NT <= N && sbase_ld(ldc);   // tile inside C
            double* Cw = C + (r0 + wm * CF::WTM) * ldc + n0 + wn * CF::WTN;
            if (last) {
                if (cin) load_c_fast<CF>(cv, Cw, ldc, coff, beta_eff != 0.0);
                else     load_c<CF>(cv, C, ldc, r0, n0, mend, N, wm, wn, lane, beta_eff != 0.0);
            }
            bool rin;
            const double* rorg;
            a_plan(tr, rin, rorg);
            // as in k_a2: one slice entry stored and one refilled per MFMA step
            mma_lds_pipe<CF, CF::KS / 4>(As[cur], CF::A_LD, 0, Bs, CF::B_LD, sl * CF::KS, acc, wm, wn, lane,
                                         [&](int kq) {
#pragma unroll
                for (int e = kq; e < SA::N; e += CF::KS / 4) {
                    ready.store_elem(e, As[cur ^ 1], CF::A_LD, tid);
                    load_a_elem(reload, tr, e, rin, rorg);
                }
            });
            if (last) {
                if (cin) store_c_fast<CF>(acc, alpha, beta_eff, cv, Cw, ldc, coff);
                else     store_c_loaded<CF>(acc, alpha, beta_eff, cv, C, ldc, r0, n0, mend, N, wm, wn, lane);
                zero_acc<CF>(acc);
            }
            __syncthreads();
        };
        static_assert(kRing == 2, "the unrolled steps below assume a ring of two");
        int t = 0;
#pragma unroll 1
        for (; t + 1 < total; t += 2) {
            step(t, sa[0], sa[1]);
            step(t + 1, sa[1], sa[0]);
        }
        if (t < total) step(t, sa[0], sa[1]);
    }
}

// ---------------------------------------------------------------------------
// Packing (Sec. 5.2-5.3: a block is copied into a contiguous buffer when it
// first becomes resident or guest).  Packs the B panel rows [pk0, pk0+kc),
// columns [pn0, pn0+nc) into P laid out [n-tile j][k row p][NT], zero-padded
// past k and n.  One thread per packed element; writes are contiguous, reads
// contiguous along n (or along k when TB).
template <int NT, bool TB>
__global__ __launch_bounds__(256) void k_pack_b(const double* __restrict__ B, int64_t ldb, int64_t K, int64_t N,
                                                int64_t pk0, int64_t pn0, int kc, int ntiles,
                                                double* __restrict__ P) {
    const int64_t total = (int64_t)ntiles * kc * NT;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / ((int64_t)kc * NT);
        const int64_t rem = e - j * kc * NT;
        const int64_t p = rem / NT, q = rem - (rem / NT) * NT;
        const int64_t gk = pk0 + p, gn = pn0 + j * NT + q;
        P[e] = (gk < K && gn < N) ? (TB ? B[gn * ldb + gk] : B[gk * ldb + gn]) : 0.0;
    }
}

}  // namespace momms

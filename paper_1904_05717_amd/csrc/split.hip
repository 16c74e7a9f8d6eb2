// Split-precision FP64-accurate product on BF16 MFMA (Ozaki-style splitting,
// Ozaki, Ogita, Oishi & Rump, Numer. Algorithms 59 (2012)).  The paper has no
// such method; this is the precision extension of the MOMMS family: the
// slice products run on the register-resident-C loop nest (member C3C0 order)
// with BF16 operands.
//
//   s1 exponent scan : e_i = frexp exponent of max_p |op(A)_ip| (so the row
//                      maximum is < 2^e_i), f_j likewise per column of op(B).
//   s2 slicing       : d_0 = rint(a' 2^w_0), d_s = rint(r_s 2^w_s),
//                      r_{s+1} = r_s - d_s 2^-w_s, a' = a 2^-e_i,
//                      w_s = 8 + 9 s.  |d_0| <= 256, |d_s| <= 256: exact BF16.
//   s3 slice products: for each diagonal d = s + t <= S-1 one launch computes
//                      Q_d = sum_s D^A_s D^B_{d-s} with v_mfma_f32_16x16x32_bf16.
//                      Products are <= 2^16, so FP32 sums of at most 256 of
//                      them are exact integers below 2^24; every 256 products
//                      they are added into FP64 (exact: |Q_d| < 2^53).
//   s4 recombination : V = sum_{d = S-1 .. 0} Q_d 2^-(16 + 9 d) in that order
//                      (each launch adds its term to V), then
//                      C = fl(fl(alpha * V 2^(e_i + f_j)) + fl(beta * C)).
// Steps s1-s3 are exact and s4 has a fixed order, so the result is
// reproducible bit for bit.
//
// INT8 and FP8 E4M3 slices run the same four steps on byte MFMAs (7-bit
// truncated and 4/5-bit rounded slices).  The modular form (Ozaki, Uchino &
// Imamura, "Ozaki scheme II", 2025) replaces s2-s4: the operands are rounded
// to t-bit integers A', B' (per row / column scale 2^(t - e)), each is reduced
// modulo N pairwise coprime moduli p_l <= 256 into int8 residues, one INT8
// product per modulus gives A'B' mod p_l, and the Chinese remainder theorem in
// 128-bit integers recovers X = A'B' exactly (t is chosen so that
// 2 k 4^t < M = prod p_l); X is rounded once to FP64 and scaled back.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "../../include/momms.h"
#include "plan_internal.h"
#include "sched.h"

namespace momms {
namespace split {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));

constexpr int kB0 = 8;       // bits of the first BF16 slice
constexpr int kB = 9;        // bits of every further slice
constexpr int kMT = 128;     // workgroup tile of the slice-product kernel
constexpr int kKS = 64;      // k-slice staged in LDS (bf16 elements)
constexpr int kKPad = 256;   // k padded to a multiple of this (whole fold periods)
constexpr int kExpNone = INT_MIN;   // exponent of an all-zero row/column
// INT8 slices: 7 bits each (truncation keeps |d| <= 127); workgroup tile
// 256 x 128, k-slice 128 bytes.  Every INT32 sum of one diagonal is exact
// while slices * kp * 127^2 < 2^31, i.e. slices * kp <= 2^17.
constexpr int kI8Bits = 7;
constexpr int kI8MT = 256, kI8NT = 256, kI8KS = 128;
constexpr int64_t kI8MaxProducts = (int64_t)1 << 17;
// 8 BF16 slices carry 8 + 7 * 9 = 71 bits and 10 INT8 slices 70: beyond the
// 53 of a double in both cases, so larger counts add nothing.
constexpr int kMaxSlicesBf16 = 8, kMaxSlicesI8 = 10;
// FP8 E4M3 slices: 4 bits, then 5 (round to nearest, |d| <= 16, exact in
// E4M3); products reach 2^8, so FP32 sums are exact while slices * k_p <= 2^16.
constexpr int kF8B0 = 4, kF8B = 5, kMaxSlicesF8 = 12;
constexpr int64_t kF8MaxProducts = (int64_t)1 << 16;
// Modular form: at most 16 moduli (M < 2^126) and t <= 60 bits.
constexpr int kMaxModuli = 16, kMaxCrtBits = 60;
constexpr int kCrtLimbs = 5;   // 12-bit limbs of the t <= 60 bit integer operands

typedef unsigned __int128 u128;

// Everything the residue and reconstruction kernels need, passed by value.
struct CrtParams {
    int n, t;
    int p[kMaxModuli];
    float ipf[kMaxModuli], pf[kMaxModuli];                      // 1/p, p
    float hif[kMaxModuli], lof[kMaxModuli];                     // (p - 1) / 2, -(p / 2): centred range
    float climb[kMaxModuli][5];                                 // 2^(12 i) mod p
    uint32_t w20[kMaxModuli][7];   // CRT weight W_l = (M/p_l) ((M/p_l)^-1 mod p_l) < M in 20-bit digits
    float wf[kMaxModuli];          // W_l / M, rounded
    uint64_t m_lo, m_hi;           // M
};

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

__device__ __forceinline__ int exp_or_zero(int e) { return e == kExpNone ? 0 : e; }

__global__ __launch_bounds__(256) void k_fill_int(int* __restrict__ p, int64_t n, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// frexp exponent of |x| for x != 0 (|x| < 2^e); zero contributes nothing.
__device__ __forceinline__ int exp_of(double x) {
    int e;
    (void)frexp(x, &e);
    return e;
}

// Per stored row r of P (rows x cols, pitch ld): out[r] = max exponent.  One
// wave per (row, column chunk); lanes read consecutive columns.
__global__ __launch_bounds__(256) void k_rowmax_exp(const double* __restrict__ P, int64_t ld, int64_t rows,
                                                    int64_t cols, int64_t chunk, int* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t c1 = c0 + chunk < cols ? c0 + chunk : cols;
    double mx = 0.0;
    for (int64_t c = c0 + lane; c < c1; c += 64) mx = fmax(mx, fabs(P[r * ld + c]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0 && mx != 0.0) atomicMax(out + r, exp_of(mx));
}

// Per stored column c: out[c] = max exponent over a chunk of rows; threads
// walk consecutive columns.
__global__ __launch_bounds__(256) void k_colmax_exp(const double* __restrict__ P, int64_t ld, int64_t rows,
                                                    int64_t cols, int64_t chunk, int* __restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    const int64_t r0 = (int64_t)blockIdx.y * chunk;
    const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
    double mx = 0.0;
    int64_t r = r0;
    for (; r + 8 <= r1; r += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = P[(r + u) * ld + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) mx = fmax(mx, fabs(v[u]));
    }
    for (; r < r1; ++r) mx = fmax(mx, fabs(P[r * ld + c]));
    if (mx != 0.0) atomicMax(out + c, exp_of(mx));
}

// OCP FP8 E4M3 byte (bias 7, 3 mantissa bits) of an integer |d| <= 16.
__device__ __forceinline__ uint32_t e4m3_of_int(int d) {
    if (d == 0) return 0u;
    const uint32_t sgn = d < 0 ? 0x80u : 0u;
    const int a = d < 0 ? -d : d;
    const int e = 31 - __clz(a);                       // a in [2^e, 2^(e+1))
    const uint32_t man = (uint32_t)(((a << 3) >> e) - 8);
    return sgn | ((uint32_t)(e + 7) << 3) | man;
}

// Slices of the logical R x Cc matrix X, X(r, c) = P[r*ld + c] (TRANSPOSED =
// false) or P[c*ld + r] (true), scaled per row by 2^-e[r].  Writes
// out[s][r][c] (pitch Cp, slice stride Rp*Cp) for all r < Rp, c < Cp (zero
// outside X) in the slice type KIND.  64 x 64 tiles go through LDS so that
// global reads and writes are both contiguous.
// KIND: 0 BF16 bit patterns (round to nearest, 8 + 9 s bits), 1 int8 values
// (truncation, 7 (s + 1) bits), 2 FP8 E4M3 bytes (round to nearest, 4 + 5 s).
template <bool TRANSPOSED, int KIND>
__global__ __launch_bounds__(256) void k_slice(const double* __restrict__ P, int64_t ld, int64_t R, int64_t Cc,
                                               const int* __restrict__ e, int S, void* __restrict__ outv,
                                               int64_t Rp, int64_t Cp) {
    __shared__ double tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int idx = tid + 256 * i;
        int rr, cc;
        if (TRANSPOSED) { cc = idx >> 6; rr = idx & 63; }
        else            { rr = idx >> 6; cc = idx & 63; }
        const int64_t gr = r0 + rr, gc = c0 + cc;
        double v = 0.0;
        if (gr < R && gc < Cc) v = TRANSPOSED ? P[gc * ld + gr] : P[gr * ld + gc];
        tile[rr][cc] = v;
    }
    __syncthreads();
    // Thread tid slices 16 consecutive columns of row tid / 4 and stores each
    // slice's 16 values with 16-byte stores (Cp is a multiple of 64).
    const int rr = tid >> 2, cb = (tid & 3) * 16;
    const int64_t gr = r0 + rr;
    if (gr >= Rp) return;
    const int ee = gr < R ? exp_or_zero(e[gr]) : 0;
    double rem[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) rem[j] = ldexp(tile[rr][cb + j], -ee);
    const int64_t slice = Rp * Cp;
    const int64_t o = gr * Cp + c0 + cb;
    for (int s_ = 0; s_ < S; ++s_) {
        if (KIND == 1) {
            const int w = kI8Bits * (s_ + 1);
            const double up = ldexp(1.0, w), down = ldexp(1.0, -w);
            uint32_t word[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t x = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double d = trunc(rem[4 * q + b] * up);            // |d| <= 127
                    rem[4 * q + b] -= d * down;
                    x |= (uint32_t)(uint8_t)(int8_t)d << (8 * b);
                }
                word[q] = x;
            }
            *reinterpret_cast<uint4*>(static_cast<int8_t*>(outv) + o + s_ * slice) =
                make_uint4(word[0], word[1], word[2], word[3]);
        } else if (KIND == 2) {
            const int w = kF8B0 + s_ * kF8B;
            const double up = ldexp(1.0, w), down = ldexp(1.0, -w);
            uint32_t word[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t x = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double d = rint(rem[4 * q + b] * up);             // |d| <= 16
                    rem[4 * q + b] -= d * down;
                    x |= e4m3_of_int((int)d) << (8 * b);
                }
                word[q] = x;
            }
            *reinterpret_cast<uint4*>(static_cast<int8_t*>(outv) + o + s_ * slice) =
                make_uint4(word[0], word[1], word[2], word[3]);
        } else {
            const int w = kB0 + s_ * kB;
            const double up = ldexp(1.0, w), down = ldexp(1.0, -w);
            uint32_t word[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint32_t x = 0;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double d = rint(rem[2 * q + b] * up);             // |d| <= 256
                    rem[2 * q + b] -= d * down;
                    x |= (__float_as_uint((float)d) >> 16) << (16 * b);
                }
                word[q] = x;
            }
            uint4* dst = reinterpret_cast<uint4*>(static_cast<uint16_t*>(outv) + o + s_ * slice);
            dst[0] = make_uint4(word[0], word[1], word[2], word[3]);
            dst[1] = make_uint4(word[4], word[5], word[6], word[7]);
        }
    }
}

// Modular form, operand side: X(r, c) as in k_slice, x = rint(X 2^(t - e[r]))
// (an exact integer, |x| <= 2^t), and for every modulus p_l the centred
// residue x mod p_l in [-128, 127] (odd p_l: [-(p_l-1)/2, (p_l-1)/2]) as
// int8, out[l][r][c] (pitch Cp, a multiple of 128, plane stride Rp*Cp, Rp a
// multiple of 32), zero outside X.
template <bool TRANSPOSED>
__global__ __launch_bounds__(256) void k_residues(const double* __restrict__ P, int64_t ld, int64_t R, int64_t Cc,
                                                  const int* __restrict__ e, CrtParams cp,
                                                  int8_t* __restrict__ out, int64_t Rp, int64_t Cp) {
    // 32 x 128 tiles: each row of a plane gets whole 128-byte lines.  A
    // stored row (TRANSPOSED = false) is already contiguous along c, so a
    // thread reads its 16 values directly (staging them through LDS with
    // lane-contiguous loads measured 13% slower); the transposed side goes
    // through LDS.
    __shared__ double tile[TRANSPOSED ? 32 : 1][129];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 128;
    const int tid = threadIdx.x;
    const int rr = tid >> 3, cb = (tid & 7) * 16;
    const int64_t gr = r0 + rr;
    double v16[16];
    if (TRANSPOSED) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int idx = tid + 256 * i;
            const int cc = idx >> 5, tr = idx & 31;
            const int64_t g_r = r0 + tr, g_c = c0 + cc;
            tile[tr][cc] = (g_r < R && g_c < Cc) ? P[g_c * ld + g_r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) v16[j] = tile[rr][cb + j];
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int64_t g_c = c0 + cb + j;
            v16[j] = (gr < R && g_c < Cc) ? P[gr * ld + g_c] : 0.0;
        }
    }
    if (gr >= Rp) return;
    const int ee = gr < R ? exp_or_zero(e[gr]) : 0;
    // x = sum_i a_i 2^(12 i) with 12-bit limbs a_i of the sign of x
    // (|a_i| <= 2^12), exact in FP32; then x = sum_i a_i c_il (mod p_l) with
    // c_il = 2^(12 i) mod p_l < 256.  Every partial sum is an integer of
    // magnitude below 2^22, so s and s - q p are exact FP32 integers for
    // q = rint(RN(s RN(1/p))); q is the nearest integer to s / p or, within
    // 0.003 of a tie, the next one, which one correction each way repairs.
    float a[16][kCrtLimbs];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        double v = rint(ldexp(v16[j], cp.t - ee));
#pragma unroll
        for (int i = kCrtLimbs - 1; i >= 0; --i) {
            const double hi = trunc(ldexp(v, -12 * i));   // exact: v is an integer below 2^60
            a[j][i] = (float)hi;
            v = fma(-hi, ldexp(1.0, 12 * i), v);
        }
    }
    const int64_t plane = Rp * Cp;
    const int64_t o = gr * Cp + c0 + cb;
    for (int l = 0; l < cp.n; ++l) {
        const float pf = cp.pf[l], ipf = cp.ipf[l], hi = cp.hif[l], lo = cp.lof[l];
        float c[kCrtLimbs];
#pragma unroll
        for (int i = 0; i < kCrtLimbs; ++i) c[i] = cp.climb[l][i];
        uint32_t word[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t w = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = 4 * q + b;
                float sres = a[j][0];
#pragma unroll
                for (int i = 1; i < kCrtLimbs; ++i) sres = fmaf(a[j][i], c[i], sres);
                float r = fmaf(-rintf(sres * ipf), pf, sres);   // within one unit of [-p/2, p/2]
                if (r > hi) r -= pf;
                if (r < lo) r += pf;
                w |= (uint32_t)(uint8_t)(int8_t)(int)r << (8 * b);
            }
            word[q] = w;
        }
        *reinterpret_cast<uint4*>(out + o + l * plane) = make_uint4(word[0], word[1], word[2], word[3]);
    }
}

// Modular form, reconstruction: for each (i, j) the residues r_l = X mod p_l
// of the N INT8 products (uint8 in [0, p_l), R[l][i / 4][j][i % 4]) give
// S = sum_l r_l W_l = X (mod M).  S is summed exactly in seven 20-bit digit
// columns with 24-bit multiplies (16 * 255 * (2^20 - 1) < 2^32) and
// assembled modulo 2^128; q = floor(sum_l r_l RN(W_l / M)) is within one of
// floor(S / M), so S - q M (modulo 2^128, read as signed) lies in [-M, 2M)
// and one correction each way gives S mod M; values above M / 2 stand for
// X - M.  X (|X| < M / 2 < 2^125) is rounded once to FP64 (top 64 bits with
// a sticky bit, then the exact u64 conversion), scaled by 2^(e_i + f_j - 2t),
// and C = fl(fl(alpha T) + fl(beta C)).  A thread takes 4 rows of a column.
__device__ __forceinline__ double i128_to_double_rn(__int128 x) {
    const bool neg = x < 0;
    const u128 u = neg ? (u128)0 - (u128)x : (u128)x;
    const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
    double d;
    if (hi == 0) {
        d = (double)lo;
    } else {
        const int lz = __clzll(hi);
        const u128 v = u << lz;
        const uint64_t top = (uint64_t)(v >> 64) | ((uint64_t)v != 0 ? 1ull : 0ull);
        d = ldexp((double)top, 64 - lz);
    }
    return neg ? -d : d;
}

__global__ __launch_bounds__(256) void k_crt_combine(int64_t M, int64_t N, const uint8_t* __restrict__ Rs,
                                                     int64_t plane, int64_t ldr, const int* __restrict__ ea,
                                                     const int* __restrict__ eb, CrtParams cp, double alpha,
                                                     double beta, double* __restrict__ C, int64_t ldc) {
    const int64_t groups = (M + 3) / 4;
    const u128 Mm = ((u128)cp.m_hi << 64) | cp.m_lo;
    const u128 half = Mm >> 1;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < groups * N;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q4 = g / N, j = g - q4 * N;
        uint32_t acc[4][7];
        float sf[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sf[r] = 0.0f;
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[r][c] = 0u;
        }
        // every plane's word in flight at once (planes past cp.n re-read the
        // last one and are not used)
        uint32_t wl[kMaxModuli];
        const uint8_t* rp = Rs + (q4 * ldr + j) * 4;
#pragma unroll
        for (int l = 0; l < kMaxModuli; ++l)
            wl[l] = *reinterpret_cast<const uint32_t*>(rp + (int64_t)(l < cp.n ? l : cp.n - 1) * plane);
#pragma unroll
        for (int l = 0; l < kMaxModuli; ++l) {
            if (l >= cp.n) break;
            const uint32_t w = wl[l];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t x = (w >> (8 * r)) & 0xffu;
#pragma unroll
                for (int c = 0; c < 7; ++c) acc[r][c] += __umul24(x, cp.w20[l][c]);
                sf[r] = fmaf((float)x, cp.wf[l], sf[r]);
            }
        }
        const int ej = exp_or_zero(eb[j]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = 4 * q4 + r;
            if (i >= M) break;
            u128 S = 0;
#pragma unroll
            for (int c = 0; c < 7; ++c) S += (u128)acc[r][c] << (20 * c);
            const uint64_t q = (uint64_t)floorf(sf[r]);
            __int128 X = (__int128)(S - (u128)q * Mm);
            if (X < 0) X += (__int128)Mm;
            if (X >= (__int128)Mm) X -= (__int128)Mm;
            if ((u128)X > half) X -= (__int128)Mm;
            const double T = ldexp(i128_to_double_rn(X), exp_or_zero(ea[i]) + ej - 2 * cp.t);
            double o = __dmul_rn(alpha, T);
            if (beta != 0.0) o = __dadd_rn(o, __dmul_rn(beta, C[i * ldc + j]));
            C[i * ldc + j] = o;
        }
    }
}

// BF16 slice products and recombination (s3 + s4) for every diagonal in one
// launch.  The workgroup owns a 256 x 128 tile of C and walks the diagonals
// d = S-1 .. 0 (smallest terms first); for each, the pairs s = 0 .. d, and
// for each pair the k range in 64-deep steps:
//   Q_d = sum_{s=0..d} D^A_s D^B_{d-s}   (v_mfma_f32_16x16x32_bf16),
// exact: products are at most 2^16, so an FP32 accumulator stays an exact
// integer for 256 of them (four steps) and is then added into an exact FP64
// sum (a quarter of the accumulators on each step).  At the end of a diagonal the recombination step of s4 runs on the
// tile: V = Q_d 2^-(16+9d) (first diagonal) or V + Q_d 2^-(16+9d), and on
// the last diagonal C = fl(fl(alpha V 2^(e_i+f_j)) + fl(beta C)).  V lives
// in the workspace between diagonals; only this workgroup touches its tile.
//
// Eight waves of 64 x 64 (4 along m, 2 along n; 16 accumulator blocks, 64
// FP32 and 128 FP64 accumulator registers per lane).  Per 64-deep step a
// wave reads 16 KiB of fragments from LDS for 32 MFMAs.  SA is [S][mp][kp],
// SB is [S][np][kp] (B by column), BF16, zero-padded to the tile and to kp.
//
// Staging: global -> LDS directly (global_load_lds_dwordx4, no staging
// registers), three LDS stages of one step each (48 KiB), issued two steps
// ahead.  A stage holds each operand as two 32-deep windows of 64-byte rows;
// the 16-byte chunk q of row r sits in slot q ^ ((r >> 1) & 3), so the
// 16-row fragment reads (row li, chunk lk) are free of bank conflicts.  One
// DMA instruction fills 16 rows of one window (lane L: row L / 4, slot
// L % 4, which holds chunk (L % 4) ^ ((L / 8) & 3)); wave w fills A row
// groups 4w .. 4w+3 and B row groups 2w, 2w+1 of every stage.
namespace bf {
constexpr int kMT = 256, kNT = 128;                     // workgroup tile
constexpr int kWinA = kMT * 64, kWinB = kNT * 64;       // bytes of one 32-deep window
constexpr int kStageA = 2 * kWinA, kStageB = 2 * kWinB; // one 64-deep step
constexpr int kStage = kStageA + kStageB;               // 48 KiB
constexpr int kStages = 3;
static_assert(kStage / 1024 == 6 * 8, "1 KiB per wave instruction: four A and two B per wave");

__device__ __forceinline__ int lds_off(int r, int q) { return r * 64 + 16 * (q ^ ((r >> 1) & 3)); }

typedef __attribute__((address_space(1))) const uint8_t gbyte;
typedef __attribute__((address_space(3))) void lvoid;
}  // namespace bf

// SA and SB are not __restrict__ (see k_split_i8_diag).
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_split_bf16(int64_t M, int64_t N, int64_t kp, int S, const uint16_t* SA, const uint16_t* SB,
                  int64_t sa_stride, int64_t sb_stride, const int* __restrict__ ea, const int* __restrict__ eb,
                  double* __restrict__ V, int64_t ldv, double alpha, double beta, double* __restrict__ C,
                  int64_t ldc, Sched sc) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[bf::kStages * bf::kStage];
    int tm, tn;
    decode_tile(sc, blockIdx.x, tm, tn);
    const int64_t m0 = sc.m_off + (int64_t)tm * bf::kMT, n0 = sc.n_off + (int64_t)tn * bf::kNT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: keeps DMA targets scalar
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 15, lk = lane >> 4;

    // Fragment i of a window starts 16 rows (1 KiB) after fragment i - 1,
    // with the same swizzle, so one offset per operand serves all four.
    const int fa0 = bf::lds_off(wm * 64 + li, lk), fb0 = bf::kStageA + bf::lds_off(wn * 64 + li, lk);

    // DMA sources (byte offsets from the tile's first row at the step's k)
    // and LDS destinations (from the stage's start) of this thread.
    const int dr = lane >> 2, dq = (lane & 3) ^ ((dr >> 1) & 3);
    const int64_t rowb = 2 * kp;   // bytes per slice row
    // 32-bit per-lane offsets that never change, added to a scalar base per
    // step: the DMA then takes the scalar-base form, and no address register
    // of an instruction in flight is ever rewritten
    // Wave w's four A instructions cover row groups 4w .. 4w+3 of one window
    // (16 rows apart: a scalar step), its two B instructions row groups 2w,
    // 2w+1 of one window.
    const int wa = (4 * wave) >> 4, ga0 = (4 * wave) & 15, wb = (2 * wave) >> 3, gb0 = (2 * wave) & 7;
    uint32_t voffa = (uint32_t)((16 * ga0 + dr) * rowb + wa * 64 + dq * 16);
    uint32_t voffb = (uint32_t)((16 * gb0 + dr) * rowb + wb * 64 + dq * 16);
    const int ldsta = wa * bf::kWinA + ga0 * 1024, ldstb = bf::kStageA + wb * bf::kWinB + gb0 * 1024;
    const int64_t grp = 16 * rowb;   // bytes between two row groups

    const int nks = (int)(kp / kKS);
    const int total = S * (S + 1) / 2 * nks;
    const int last = total - 1;
    // Tiles sharing a slice panel start their k loops apart (as in the FP64
    // kernel): step kq of a pair reads k-step (kq + kshift) mod nks.
    const int kshift = ((tm + tn) & 7) % nks;
    bf::gbyte* ga = (bf::gbyte*)reinterpret_cast<const uint8_t*>(SA) + m0 * rowb;
    bf::gbyte* gb = (bf::gbyte*)reinterpret_cast<const uint8_t*>(SB) + n0 * rowb;

    // Coordinates (diagonal, pair, k-step) of the next step to fetch; steps
    // run diagonal by diagonal from d = S-1, pairs s = 0..d, then k.  The
    // coordinates stop at the last step: surplus fetches re-read it into a
    // stage nobody reads again.
    int fd = S - 1, fs = 0, fk = 0, fetched = 0;
#define MOMMS_BF_FETCH(stage_)                                                                       \
    do {                                                                                             \
        int kq_ = fk + kshift;                                                                       \
        if (kq_ >= nks) kq_ -= nks;                                                                  \
        const int64_t kb_ = (int64_t)kq_ * (kKS * 2);                                                \
        bf::gbyte* pa_ = ga + (int64_t)fs * sa_stride * 2 + kb_;                                     \
        bf::gbyte* pb_ = gb + (int64_t)(fd - fs) * sb_stride * 2 + kb_;                              \
        uint8_t* dst_ = lds + (stage_) * bf::kStage;                                                 \
        /* opaque per use: base + offset is not hoisted into a 64-bit register */                    \
        asm volatile("" : "+v"(voffa), "+v"(voffb));                                                 \
        _Pragma("unroll") for (int u = 0; u < 4; ++u) {                                              \
            bf::gbyte* pu_ = pa_ + u * grp;                                                          \
            asm volatile("" : "+s"(pu_));   /* the row-group step stays in the scalar base */        \
            __builtin_amdgcn_global_load_lds(pu_ + voffa, (bf::lvoid*)(dst_ + ldsta + u * 1024), 16, 0, 0); \
        }                                                                                            \
        _Pragma("unroll") for (int u = 0; u < 2; ++u) {                                              \
            bf::gbyte* pu_ = pb_ + u * grp;                                                          \
            asm volatile("" : "+s"(pu_));                                                            \
            __builtin_amdgcn_global_load_lds(pu_ + voffb, (bf::lvoid*)(dst_ + ldstb + u * 1024), 16, 0, 0); \
        }                                                                                            \
        /* advance (branch-free scalar selects; stops at the last step) */                           \
        const int adv_ = fetched < last ? 1 : 0;                                                     \
        fetched += adv_;                                                                             \
        fk += adv_;                                                                                  \
        const int wk_ = fk == nks ? 1 : 0;                                                           \
        fk = wk_ ? 0 : fk;                                                                           \
        fs += wk_;                                                                                   \
        const int ws_ = fs > fd ? 1 : 0;                                                             \
        fs = ws_ ? 0 : fs;                                                                           \
        fd -= ws_;                                                                                   \
    } while (0)

    f4 acc[4][4];
    double q[4][4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 4; ++r) q[i][j][r] = 0.0;
        }

    // Row u of accumulator blocks (acc[u][*]) is added into the exact FP64
    // sums q on step u of every group of four: four steps (256 products,
    // sums <= 2^24) between two folds of any accumulator, and every diagonal
    // ends on a group boundary with all rows folded.  One row per step keeps
    // the conversions and FP64 adds spread out, next to the MFMAs of the
    // other rows.
#define MOMMS_BF_FOLD(u_)                                                                            \
    do {                                                                                             \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                              \
            _Pragma("unroll") for (int r = 0; r < 4; ++r) q[u_][j][r] += (double)acc[u_][j][r];      \
            acc[u_][j] = f4{0.f, 0.f, 0.f, 0.f};                                                     \
        }                                                                                            \
    } while (0)
    // One 32-deep window: four B and four A fragments, rows ia_, ia_ + 1
    // of blocks first, then MID_ (a fold or nothing), then rows ib_, ib_ + 1.
#define MOMMS_BF_LOADB(w_)                                                                           \
    _Pragma("unroll") for (int j = 0; j < 4; ++j)                                                    \
        b[j] = *reinterpret_cast<const bf16x8*>(base + (w_) * bf::kWinB + fb0 + j * 1024)
    // A step that folds row u_: in the second window the pair holding row
    // u_ goes first, so its fold overlaps the other pair's MFMAs.
#define MOMMS_BF_WIN(w_, ia_, ib_, MID_)                                                             \
    do {                                                                                             \
        bf16x8 a[4];                                                                                 \
        _Pragma("unroll") for (int i = 0; i < 4; ++i)                                                \
            a[i] = *reinterpret_cast<const bf16x8*>(base + (w_) * bf::kWinA + fa0 + i * 1024);       \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                                                \
            acc[ia_][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ia_], b[j], acc[ia_][j], 0, 0, 0); \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                                                \
            acc[ia_ + 1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ia_ + 1], b[j], acc[ia_ + 1][j], 0, 0, 0); \
        MID_;                                                                                        \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                                                \
            acc[ib_][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ib_], b[j], acc[ib_][j], 0, 0, 0); \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                                                \
            acc[ib_ + 1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ib_ + 1], b[j], acc[ib_ + 1][j], 0, 0, 0); \
    } while (0)
#define MOMMS_BF_STEP(u_)                                                                            \
    do {                                                                                             \
        constexpr int pf_ = ((u_) / 2) * 2, po_ = 2 - pf_;                                           \
        bf16x8 b[4];                                                                                 \
        MOMMS_BF_LOADB(0);                                                                           \
        MOMMS_BF_WIN(0, 0, 2, (void)0);                                                              \
        MOMMS_BF_LOADB(1);                                                                           \
        MOMMS_BF_WIN(1, pf_, po_, MOMMS_BF_FOLD(u_));                                                \
    } while (0)

    MOMMS_BF_FETCH(0);
    MOMMS_BF_FETCH(1);
    // Four steps at a time (every diagonal is a multiple of four steps:
    // kp is a multiple of 256); step u of a group folds row u.
    int stage = 0, fstage = 2;
#define MOMMS_BF_ONE(u_)                                                                             \
    do {                                                                                             \
        /* this thread's fetches of this step have landed (the next step's  */                       \
        /* six may still be in flight); after the barrier everyone's have,  */                       \
        /* and everyone is done with the previous step's stage, which the   */                       \
        /* fetch below overwrites.  A bare barrier: __syncthreads() would   */                       \
        /* add a workgroup fence, and the fetches in flight count as LDS    */                       \
        /* writes, so it would wait for all of them.                        */                       \
        asm volatile("s_waitcnt vmcnt(6)\n\ts_barrier" ::: "memory");                                 \
        MOMMS_BF_FETCH(fstage);                                                                      \
        const uint8_t* base = lds + stage * bf::kStage;                                              \
        MOMMS_BF_STEP(u_);                                                                           \
        /* steps are not interleaved: that would need more registers */                              \
        __builtin_amdgcn_sched_barrier(0);                                                           \
        stage = stage == 2 ? 0 : stage + 1;                                                          \
        fstage = fstage == 2 ? 0 : fstage + 1;                                                       \
    } while (0)
    for (int cd = S - 1; cd >= 0; --cd) {
        const int clen = (cd + 1) * nks;
        for (int cj = 0; cj < clen; cj += 4) {
            MOMMS_BF_ONE(0);
            MOMMS_BF_ONE(1);
            MOMMS_BF_ONE(2);
            MOMMS_BF_ONE(3);
        }
        // end of the diagonal: the rows folded earlier in the last group
        // into FP64 too (row 3 was folded on the last step)
#pragma unroll
        for (int i = 0; i < 3; ++i) MOMMS_BF_FOLD(i);
        // s4 for diagonal cd: lane (li, lk) holds rows 4 lk + r, column li
        // of each 16 x 16 block.  Addresses are built here from a scalar base
        // and a 32-bit lane offset, both opaque, so that the compiler cannot
        // hoist 64 element addresses out of the main loop (they would not
        // fit beside the accumulators).
        {
            const int shift = 2 * kB0 + cd * kB;
            const bool first = cd == S - 1, lastd = cd == 0;
            const int64_t rb = m0 + wm * 64, cbase = n0 + wn * 64;
            const bool full = rb + 64 <= M && cbase + 64 <= N;
            uint32_t lo_v = (uint32_t)(((int64_t)(4 * lk) * ldv + li) * 8);
            uint32_t lo_c = (uint32_t)(((int64_t)(4 * lk) * ldc + li) * 8);
            bf::gbyte* vb = (bf::gbyte*)reinterpret_cast<const uint8_t*>(V + rb * ldv + cbase);
            bf::gbyte* cb = (bf::gbyte*)reinterpret_cast<const uint8_t*>(C + rb * ldc + cbase);
            int64_t sv = ldv * 8, sc8 = ldc * 8;   // row strides in bytes
            // rows and columns of C left from the wave's corner (at most 64
            // matter), and this lane's first row and column in a block
            int mrem = (int)(M - rb < 64 ? M - rb : 64), nrem = (int)(N - cbase < 64 ? N - cbase : 64);
            int lrow = 4 * lk, lcol = li;
            asm volatile("" : "+v"(lo_v), "+v"(lo_c), "+s"(vb), "+s"(cb), "+s"(sv), "+s"(sc8), "+s"(mrem),
                         "+s"(nrem), "+v"(lrow), "+v"(lcol));
            // one 16 x 16 block at a time, so that the V and C loads in
            // flight need no more registers than the accumulators leave free
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    __builtin_amdgcn_sched_barrier(0);
                    const int64_t col = cbase + j * 16 + li;
                    const bool col_ok = j * 16 + lcol < nrem;
                    const int fcol = lastd && col_ok ? exp_or_zero(eb[col]) : 0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double term = ldexp(q[i][j][r], -shift);
                        q[i][j][r] = 0.0;
                        const int64_t row = rb + i * 16 + 4 * lk + r;
                        __attribute__((address_space(1))) double* pv =
                            (__attribute__((address_space(1))) double*)(vb + (i * 16 + r) * sv + j * 128 + lo_v);
                        __attribute__((address_space(1))) double* pc =
                            (__attribute__((address_space(1))) double*)(cb + (i * 16 + r) * sc8 + j * 128 + lo_c);
                        if (!full && (i * 16 + r + lrow >= mrem || !col_ok)) continue;
                        const double v = first ? term : __dadd_rn(*pv, term);
                        if (lastd) {
                            const double T = ldexp(v, exp_or_zero(ea[row]) + fcol);
                            double o = __dmul_rn(alpha, T);
                            if (beta != 0.0) o = __dadd_rn(o, __dmul_rn(beta, *pc));
                            *pc = o;
                        } else {
                            *pv = v;
                        }
                    }
                }
        }
    }
#undef MOMMS_BF_ONE
    // the surplus fetches must land before the workgroup's LDS is released
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#undef MOMMS_BF_FETCH
#undef MOMMS_BF_FOLD
#undef MOMMS_BF_WIN
#undef MOMMS_BF_LOADB
#undef MOMMS_BF_STEP
}

// INT8 form of one diagonal: Q = sum_{s=0..d} D^A_s D^B_{d-s} with
// v_mfma_i32_16x16x64_i8 into INT32 accumulators (exact, no folding), then
// the same recombination step as the BF16 kernel.  SA is [S][mp][kp] int8,
// SB is [S][np][kp] int8 (B stored column by column), zero-padded.  The
// 256 x 256 workgroup tile is split over 8 waves as 2 (m) x 4 (n), each
// owning 128 x 64: per 128-deep k-step a wave reads 24 KiB of fragments for
// 64 MFMAs, which keeps the LDS (about 205 B/clk for conflict-free 16-byte
// reads, 138 B/clk for writes) below the MFMA time.
//
// LDS holds each k-step as two 64-byte windows per row, unpadded; the
// 16-byte chunk q of row r sits in slot q ^ ((r >> 1) & 3), which makes the
// 16-row fragment reads (row li, chunk lk) free of bank conflicts on gfx950.
// Two LDS stages and one register set: a step's global loads are issued in
// the middle of the step two before it and stored to LDS in the middle of
// the step before it, so the stores overlap MFMAs.
namespace i8 {
constexpr int kWinA = kI8MT * 64, kWinB = kI8NT * 64;     // bytes of one 64-deep window
constexpr int kStageA = 2 * kWinA, kStageB = 2 * kWinB;   // one 128-deep k-step

__device__ __forceinline__ int lds_off(int r, int q) { return r * 64 + 16 * (q ^ ((r >> 1) & 3)); }
}  // namespace i8

#define MOMMS_I8_GLOAD(R, t_)                                                                   \
    do {                                                                                         \
        const int s_ = (t_) / nks;                                                               \
        int kq = (t_) - s_ * nks + kshift;                                                       \
        if (kq >= nks) kq -= nks;                                                                \
        const int64_t kk = (int64_t)kq * kI8KS + gcol;                                           \
        const int8_t* pa = SA + (int64_t)s_ * sa_stride + (m0 + grow) * kp + kk;                 \
        const int8_t* pb = SB + (int64_t)(d - s_) * sb_stride + (n0 + grow) * kp + kk;           \
        R##0 = *reinterpret_cast<const uint4*>(pa);                                              \
        R##1 = *reinterpret_cast<const uint4*>(pa + 64 * kp);                                    \
        R##2 = *reinterpret_cast<const uint4*>(pa + 128 * kp);                                   \
        R##3 = *reinterpret_cast<const uint4*>(pa + 192 * kp);                                   \
        R##4 = *reinterpret_cast<const uint4*>(pb);                                              \
        R##5 = *reinterpret_cast<const uint4*>(pb + 64 * kp);                                    \
        R##6 = *reinterpret_cast<const uint4*>(pb + 128 * kp);                                   \
        R##7 = *reinterpret_cast<const uint4*>(pb + 192 * kp);                                   \
    } while (0)

#define MOMMS_I8_LSTORE(buf_, R)                                                                 \
    do {                                                                                         \
        int8_t* la = As + (buf_) * i8::kStageA + sw;                                             \
        int8_t* lb = Bs + (buf_) * i8::kStageB + sw;                                             \
        *reinterpret_cast<uint4*>(la) = R##0;                                                    \
        *reinterpret_cast<uint4*>(la + 64 * 64) = R##1;                                          \
        *reinterpret_cast<uint4*>(la + 128 * 64) = R##2;                                         \
        *reinterpret_cast<uint4*>(la + 192 * 64) = R##3;                                         \
        *reinterpret_cast<uint4*>(lb) = R##4;                                                    \
        *reinterpret_cast<uint4*>(lb + 64 * 64) = R##5;                                          \
        *reinterpret_cast<uint4*>(lb + 128 * 64) = R##6;                                         \
        *reinterpret_cast<uint4*>(lb + 192 * 64) = R##7;                                         \
    } while (0)

// One 64-deep window of the current stage: 4 B fragments stay, the 8 A
// fragments stream through in pairs, 32 MFMAs.  The next pair is read from
// LDS before the current pair's MFMAs are issued, so a pair's read latency
// is covered by the MFMAs of the pair before it.
#define MOMMS_I8_WINDOW(buf_, w_)                                                                \
    do {                                                                                         \
        const int8_t* la = As + (buf_) * i8::kStageA + (w_) * i8::kWinA;                         \
        const int8_t* lb = Bs + (buf_) * i8::kStageB + (w_) * i8::kWinB;                         \
        i4 bf[4];                                                                                \
        _Pragma("unroll") for (int j = 0; j < 4; ++j)                                            \
            bf[j] = *reinterpret_cast<const i4*>(lb + fb_off[j]);                                \
        i4 ap[2][2];                                                                             \
        ap[0][0] = *reinterpret_cast<const i4*>(la + fa_off[0]);                                 \
        ap[0][1] = *reinterpret_cast<const i4*>(la + fa_off[1]);                                 \
        _Pragma("unroll") for (int i2 = 0; i2 < 8; i2 += 2) {                                    \
            const int c_ = (i2 >> 1) & 1;                                                        \
            if (i2 + 2 < 8) {                                                                    \
                ap[c_ ^ 1][0] = *reinterpret_cast<const i4*>(la + fa_off[i2 + 2]);               \
                ap[c_ ^ 1][1] = *reinterpret_cast<const i4*>(la + fa_off[i2 + 3]);               \
            }                                                                                    \
            __builtin_amdgcn_sched_barrier(0);                                                   \
            _Pragma("unroll") for (int j = 0; j < 4; ++j)                                        \
                acc[i2][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[c_][0], bf[j], acc[i2][j], 0, 0, 0); \
            _Pragma("unroll") for (int j = 0; j < 4; ++j)                                        \
                acc[i2 + 1][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[c_][1], bf[j], acc[i2 + 1][j], 0, 0, 0); \
            __builtin_amdgcn_sched_barrier(0);                                                   \
        }                                                                                        \
    } while (0)

// One k-step t on LDS buffer buf_: run window 0, store step t + 1 (held in
// the register set since the previous step) into the other buffer (last
// read in step t - 1, before the previous barrier), issue the loads of step
// t + 2 into the freed registers, run window 1, synchronise.  The stores
// overlap window 1's MFMAs; each load has a whole step to land.  On the last
// step the store writes a repeat of it that nobody reads: kept
// unconditional, so that the compiler sees the same loads and stores on
// every path and waits only for the loads each store needs.
#define MOMMS_I8_STEP(t_, buf_) MOMMS_I8_STEP_G(t_, buf_, MOMMS_I8_GLOAD)
#define MOMMS_I8_STEP_G(t_, buf_, GLOAD_)                                                        \
    do {                                                                                         \
        MOMMS_I8_WINDOW(buf_, 0);                                                                \
        __builtin_amdgcn_sched_barrier(0);                                                       \
        MOMMS_I8_LSTORE((buf_) ^ 1, g);                                                          \
        __builtin_amdgcn_sched_barrier(0);                                                       \
        GLOAD_(g, (t_) + 2 < last ? (t_) + 2 : last);                                            \
        __builtin_amdgcn_sched_barrier(0);                                                       \
        MOMMS_I8_WINDOW(buf_, 1);                                                                \
        __syncthreads();                                                                         \
    } while (0)

// FP8 form: one v_mfma_f32_16x16x128_f8f6f4 covers both 64-deep windows of a
// k-step.  Only the pairing of A and B k values matters, so lane (li, lk)
// supplies chunk lk of window 0 and chunk lk of window 1 of its row for both
// operands (the conflict-free fragment reads of the INT8 form; checked on the
// device against exact integer products).  Half h runs A fragments 4h..4h+3
// against the 4 B fragments read at the start of the step.
__device__ __forceinline__ i8v frag_f8(const int8_t* p, int win) {
    const i4 lo = *reinterpret_cast<const i4*>(p), hi = *reinterpret_cast<const i4*>(p + win);
    return i8v{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}
#define MOMMS_F8_HALF(buf_, h_)                                                                  \
    do {                                                                                         \
        const int8_t* la = As + (buf_) * i8::kStageA;                                            \
        _Pragma("unroll") for (int i2 = 4 * (h_); i2 < 4 * (h_) + 4; i2 += 2) {                  \
            const i8v a0 = frag_f8(la + fa_off[i2], i8::kWinA);                                  \
            const i8v a1 = frag_f8(la + fa_off[i2 + 1], i8::kWinA);                              \
            _Pragma("unroll") for (int j = 0; j < 4; ++j)                                        \
                acc[i2][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a0, bf8[j], acc[i2][j], 0, 0, 0, 0, 0, 0); \
            _Pragma("unroll") for (int j = 0; j < 4; ++j)                                        \
                acc[i2 + 1][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a1, bf8[j], acc[i2 + 1][j], 0, 0, 0, 0, 0, 0); \
            __builtin_amdgcn_sched_barrier(0);                                                   \
        }                                                                                        \
    } while (0)

#define MOMMS_F8_STEP(t_, buf_)                                                                  \
    do {                                                                                         \
        const int8_t* lb = Bs + (buf_) * i8::kStageB;                                            \
        i8v bf8[4];                                                                              \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) bf8[j] = frag_f8(lb + fb_off[j], i8::kWinB); \
        MOMMS_F8_HALF(buf_, 0);                                                                  \
        __builtin_amdgcn_sched_barrier(0);                                                       \
        if ((t_) + 1 < total) MOMMS_I8_LSTORE((buf_) ^ 1, g);                                    \
        __builtin_amdgcn_sched_barrier(0);                                                       \
        MOMMS_I8_GLOAD(g, (t_) + 2 < last ? (t_) + 2 : last);                                    \
        __builtin_amdgcn_sched_barrier(0);                                                       \
        MOMMS_F8_HALF(buf_, 1);                                                                  \
        __syncthreads();                                                                         \
    } while (0)

// SA and SB are deliberately not __restrict__: as provably unclobbered loads
// the compiler would sink the prefetch past the barrier to its use.  F8: the
// slices are FP8 E4M3 and the accumulators FP32 (exact: every partial sum is
// an integer below 2^24).
template <bool FIRST, bool LAST, bool F8>
__global__ __launch_bounds__(512) void k_split_i8_diag(int64_t M, int64_t N, int64_t kp, int d,
                                                       const int8_t* SA, const int8_t* SB, int64_t sa_stride,
                                                       int64_t sb_stride, int shift, const int* __restrict__ ea,
                                                       const int* __restrict__ eb, double* __restrict__ V,
                                                       int64_t ldv, double alpha, double beta,
                                                       double* __restrict__ C, int64_t ldc, Sched sc) {
    __shared__ __attribute__((aligned(16))) int8_t As[2 * i8::kStageA];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2 * i8::kStageB];
    int tm, tn;
    decode_tile(sc, blockIdx.x, tm, tn);
    const int64_t m0 = sc.m_off + (int64_t)tm * kI8MT, n0 = sc.n_off + (int64_t)tn * kI8NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    const int li = lane & 15, lk = lane >> 4;

    typename std::conditional<F8, f4, i4>::type acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = {0, 0, 0, 0};

    // staging: thread tid moves the 16-byte chunk gq of rows grow, grow + 64,
    // grow + 128, grow + 192 of both operands (8 threads cover one row's 128
    // bytes of a k-step); chunks 0-3 go to window 0, chunks 4-7 to window 1.
    // Rows grow + 64 i share grow's swizzle; A and B windows have equal size.
    const int grow = tid >> 3, gq = tid & 7, gcol = gq * 16;
    const int sw = i8::lds_off(grow, gq & 3) + (gq >> 2) * i8::kWinA;
    int fa_off[8], fb_off[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) fa_off[i] = i8::lds_off(wm * 128 + i * 16 + li, lk);
#pragma unroll
    for (int j = 0; j < 4; ++j) fb_off[j] = i8::lds_off(wn * 64 + j * 16 + li, lk);

    const int nks = (int)(kp / kI8KS);
    const int total = (d + 1) * nks;
    const int last = total - 1;
    const int kshift = ((tm + tn) & 7) % nks;
    uint4 g0, g1, g2, g3, g4, g5, g6, g7;

    // Loads are unconditional (past the end they re-read the last step, in
    // bounds): a conditional load would make every later wait a full one.
    MOMMS_I8_GLOAD(g, 0);
    MOMMS_I8_LSTORE(0, g);
    MOMMS_I8_GLOAD(g, 1 < last ? 1 : last);
    __syncthreads();
    if constexpr (F8) {
        for (int t = 0; t < total; ++t) MOMMS_F8_STEP(t, t & 1);
    } else {
        for (int t = 0; t < total; ++t) MOMMS_I8_STEP(t, t & 1);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the surplus prefetches


#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * 128 + i * 16 + 4 * lk + r;
                const int64_t col = n0 + wn * 64 + j * 16 + li;
                if (row >= M || col >= N) continue;
                const double term = ldexp((double)acc[i][j][r], -shift);
                const double v = FIRST ? term : __dadd_rn(V[row * ldv + col], term);
                if (LAST) {
                    const double T = ldexp(v, exp_or_zero(ea[row]) + exp_or_zero(eb[col]));
                    double o = __dmul_rn(alpha, T);
                    if (beta != 0.0) o = __dadd_rn(o, __dmul_rn(beta, C[row * ldc + col]));
                    C[row * ldc + col] = o;
                } else {
                    V[row * ldv + col] = v;
                }
            }
}
// Modular form, s3: the N INT8 products of the residue planes as one
// persistent launch.  Work items are (modulus l, C tile) in modulus-major
// order; workgroup b takes items b, b + G, b + 2G, ... (G = gridDim.x, a
// multiple of 8 no larger than the item count, so each workgroup's tiles map
// to its own XCD in the grouped order).  The k-steps of a workgroup's items
// form one sequence, so the two-step prefetch runs across item boundaries
// and a tile's epilogue does not drain the pipeline.  Epilogue: acc mod p_l
// (acc = hi 2^16 + lo, s = hi (2^16 mod p) + lo is exact in FP32, one FP32
// quotient estimate, two corrections), four rows of one column per 32-bit
// store into R[l][row / 4][col][row % 4] (pitch ldr columns).
struct CrtOut {
    uint8_t* R;
    int64_t plane, ldr;   // bytes per modulus plane; columns per 4-row group
    int p[kMaxModuli], c16[kMaxModuli];
    float ipf[kMaxModuli];
};

// *(base + off bytes) as 16 bytes for a wave-uniform base and a 32-bit lane
// offset: a global load with a scalar base address and a vector offset, no
// per-lane 64-bit address arithmetic (both operands opaque, or the compiler
// folds the offset in once and steps 64-bit vector addresses).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 gu32x4;
typedef __attribute__((address_space(1))) const uint8_t gbyte_c;
__device__ __forceinline__ uint4 load16_sbase(const int8_t* base, uint32_t off) {
    gbyte_c* b = (gbyte_c*)reinterpret_cast<const uint8_t*>(base);
    asm volatile("" : "+s"(b), "+v"(off));
    const u32x4 v = *reinterpret_cast<gu32x4*>(b + off);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// The loads of the next step to fetch (item f_it, k-step f_s), then the
// fetch state advances unless it is at the last step (the kernel fetches
// steps 0, 1, 2, ... in order and repeats the last).  An item's bases and k
// stagger are computed once per item (f_item), not per step.
#define MOMMS_CRT_GLOAD(R, t_)                                                                   \
    do {                                                                                         \
        int kq = f_s + f_shift;                                                                  \
        if (kq >= nks) kq -= nks;                                                                \
        const int8_t* pa = f_pa + (int64_t)kq * kI8KS;                                           \
        const int8_t* pb = f_pb + (int64_t)kq * kI8KS;                                           \
        R##0 = load16_sbase(pa, goff);                                                           \
        R##1 = load16_sbase(pa + 64 * kp, goff);                                                 \
        R##2 = load16_sbase(pa + 128 * kp, goff);                                                \
        R##3 = load16_sbase(pa + 192 * kp, goff);                                                \
        R##4 = load16_sbase(pb, goff);                                                           \
        R##5 = load16_sbase(pb + 64 * kp, goff);                                                 \
        R##6 = load16_sbase(pb + 128 * kp, goff);                                                \
        R##7 = load16_sbase(pb + 192 * kp, goff);                                                \
        if (f_n < last) {                                                                        \
            ++f_n;                                                                               \
            if (++f_s == nks) {                                                                  \
                f_s = 0;                                                                         \
                ++f_it;                                                                          \
                f_item();                                                                        \
            }                                                                                    \
        }                                                                                        \
    } while (0)

__device__ __forceinline__ uint32_t residue_u8(int a, int p, int c16, float ipf) {
    const int s = (a >> 16) * c16 + (a & 0xffff);   // = a (mod p), |s| < 2^24
    int r = s - (int)floorf((float)s * ipf) * p;    // in [-p, 2p)
    if (r < 0) r += p;
    if (r >= p) r -= p;
    return (uint32_t)r;
}

__global__ __launch_bounds__(512) void k_crt_gemm(int64_t M, int64_t N, int64_t kp, const int8_t* SA,
                                                  const int8_t* SB, int64_t sa_stride, int64_t sb_stride, Sched sc,
                                                  int tiles, int items, CrtOut co) {
    __shared__ __attribute__((aligned(16))) int8_t As[2 * i8::kStageA];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2 * i8::kStageB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    const int li = lane & 15, lk = lane >> 4;
    i4 acc[8][4];
    const int grow = tid >> 3, gq = tid & 7, gcol = gq * 16;
    const int sw = i8::lds_off(grow, gq & 3) + (gq >> 2) * i8::kWinA;
    int fa_off[8], fb_off[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) fa_off[i] = i8::lds_off(wm * 128 + i * 16 + li, lk);
#pragma unroll
    for (int j = 0; j < 4; ++j) fb_off[j] = i8::lds_off(wn * 64 + j * 16 + li, lk);

    const int G = (int)gridDim.x;
    const int nks = (int)(kp / kI8KS);
    const int n_it = (items - (int)blockIdx.x + G - 1) / G;   // >= 1: G <= items
    const int total = n_it * nks;
    const int last = total - 1;
    uint4 g0, g1, g2, g3, g4, g5, g6, g7;
    // fetch state (see MOMMS_CRT_GLOAD): this thread's 16-byte chunk of row
    // grow at a 32-bit offset from the item's scalar bases
    const uint32_t goff = (uint32_t)((int64_t)grow * kp + gcol);
    int f_it = 0, f_s = 0, f_n = 0, f_shift = 0;
    const int8_t *f_pa = SA, *f_pb = SB;
    auto f_item = [&]() {
        const int j_ = (int)blockIdx.x + f_it * G;
        const int l_ = j_ / tiles;
        int tm_, tn_;
        decode_tile(sc, j_ - l_ * tiles, tm_, tn_);
        f_shift = ((tm_ + tn_) & 7) % nks;
        f_pa = SA + (int64_t)l_ * sa_stride + (sc.m_off + (int64_t)tm_ * kI8MT) * kp;
        f_pb = SB + (int64_t)l_ * sb_stride + (sc.n_off + (int64_t)tn_ * kI8NT) * kp;
    };
    f_item();

    MOMMS_CRT_GLOAD(g, 0);
    MOMMS_I8_LSTORE(0, g);
    MOMMS_CRT_GLOAD(g, 1 < last ? 1 : last);
    __syncthreads();
    int t = 0;
    for (int it = 0; it < n_it; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = i4{0, 0, 0, 0};
        for (int s = 0; s < nks; ++s, ++t) MOMMS_I8_STEP_G(t, t & 1, MOMMS_CRT_GLOAD);
        const int jt = (int)blockIdx.x + it * G;
        const int l = jt / tiles;
        int tm, tn;
        decode_tile(sc, jt - l * tiles, tm, tn);
        const int64_t m0 = sc.m_off + (int64_t)tm * kI8MT, n0 = sc.n_off + (int64_t)tn * kI8NT;
        const int p = co.p[l], c16 = co.c16[l];
        const float ipf = co.ipf[l];
        uint8_t* R = co.R + (int64_t)l * co.plane;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row0 = m0 + wm * 128 + i * 16 + 4 * lk;
                const int64_t col = n0 + wn * 64 + j * 16 + li;
                if (row0 >= M || col >= N) continue;
                uint32_t w = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) w |= residue_u8(acc[i][j][r], p, c16, ipf) << (8 * r);
                *reinterpret_cast<uint32_t*>(R + ((row0 >> 2) * co.ldr + col) * 4) = w;
            }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the surplus prefetches
}
#undef MOMMS_CRT_GLOAD
#undef MOMMS_I8_STEP_G

#undef MOMMS_I8_GLOAD
#undef MOMMS_I8_LSTORE
#undef MOMMS_F8_HALF
#undef MOMMS_F8_STEP
#undef MOMMS_I8_WINDOW
#undef MOMMS_I8_STEP

// C = beta * C (beta == 0 writes zeros).
__global__ __launch_bounds__(256) void k_scale(int64_t M, int64_t N, double beta, double* __restrict__ C,
                                               int64_t ldc) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / N, j = e - (e / N) * N;
        C[i * ldc + j] = beta == 0.0 ? 0.0 : beta * C[i * ldc + j];
    }
}

struct Layout {
    int64_t mp, np, kp;
    size_t off_ea, off_eb, off_sa, off_sb, off_v, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// crt: the modular form; the V region then holds the N residue planes of
// the products, uint8 [N][ceil(m/4)][np][4].
static Layout layout(int64_t m, int64_t n, int64_t k, int S, bool bytes, bool crt = false) {
    Layout L;
    const size_t esz = bytes ? sizeof(int8_t) : sizeof(uint16_t);
    L.mp = rup(m > 0 ? m : 1, bytes ? kI8MT : bf::kMT);
    L.np = rup(n > 0 ? n : 1, bytes ? kI8NT : bf::kNT);
    L.kp = rup(k > 0 ? k : 1, bytes ? kI8KS : kKPad);
    size_t o = 0;
    L.off_ea = o; o = align256(o + sizeof(int) * (size_t)m);
    L.off_eb = o; o = align256(o + sizeof(int) * (size_t)n);
    L.off_sa = o; o = align256(o + esz * (size_t)S * L.mp * L.kp);
    L.off_sb = o; o = align256(o + esz * (size_t)S * L.np * L.kp);
    L.off_v = o;
    o = align256(o + (crt ? (size_t)S * (size_t)rup(m, 4) * L.np : S > 1 ? sizeof(double) * (size_t)m * n : 0));
    L.total = o;
    return L;
}

static int gcd_int(int a, int b) {
    while (b != 0) {
        const int r = a % b;
        a = b;
        b = r;
    }
    return a;
}

// The N largest pairwise coprime integers in [2, 256], greedily from 256
// down; M = their product; t = the largest integer <= 60 with 2 k 4^t < M
// (0 when not even t = 1 fits); the CRT weights.  Host only.
static int crt_params(int N, int64_t k, CrtParams* cp) {
    *cp = CrtParams{};
    cp->n = N;
    int got = 0;
    for (int p = 256; p >= 2 && got < N; --p) {
        bool ok = true;
        for (int q = 0; q < got; ++q) ok = ok && gcd_int(p, cp->p[q]) == 1;
        if (ok) cp->p[got++] = p;
    }
    if (got < N) return -1;
    u128 Mm = 1;
    for (int l = 0; l < N; ++l) Mm *= (u128)cp->p[l];
    const u128 kk2 = 2 * (u128)(k > 0 ? k : 1);
    int t = 0;
    for (int c = 1; c <= kMaxCrtBits; ++c)
        if (kk2 <= ((Mm - 1) >> (2 * c))) t = c;   // 2k 4^c <= M - 1
    cp->t = t;
    for (int l = 0; l < N; ++l) {
        const int p = cp->p[l];
        const u128 Ml = Mm / (u128)p;
        const int a = (int)(Ml % (u128)p);
        int inv = 0;
        for (int x = 1; x < p; ++x)
            if ((a * x) % p == 1) {
                inv = x;
                break;
            }
        const u128 W = Ml * (u128)inv;   // < M because inv < p
        cp->ipf[l] = 1.0f / (float)p;
        cp->pf[l] = (float)p;
        cp->hif[l] = (float)((p - 1) / 2);
        cp->lof[l] = -(float)(p / 2);
        for (int i = 0; i < kCrtLimbs; ++i) cp->climb[l][i] = (float)(((u128)1 << (12 * i)) % (u128)p);
        for (int c = 0; c < 7; ++c) cp->w20[l][c] = (uint32_t)(W >> (20 * c)) & 0xfffffu;
        cp->wf[l] = (float)((double)W / (double)Mm);
    }
    cp->m_lo = (uint64_t)Mm;
    cp->m_hi = (uint64_t)(Mm >> 64);
    return 0;
}

template <bool F, bool L, bool F8>
static void launch_i8_diag(dim3 grid, hipStream_t st, int64_t M, int64_t N, int64_t kp, int d, const int8_t* SA,
                           const int8_t* SB, int64_t sas, int64_t sbs, int shift, const int* ea, const int* eb,
                           double* V, int64_t ldv, double alpha, double beta, double* C, int64_t ldc, Sched s) {
    hipLaunchKernelGGL((k_split_i8_diag<F, L, F8>), grid, dim3(512), 0, st, M, N, kp, d, SA, SB, sas, sbs, shift, ea,
                       eb, V, ldv, alpha, beta, C, ldc, s);
}

}  // namespace split
}  // namespace momms

extern "C" {

size_t momms_split_workspace_size(int64_t m, int64_t n, int64_t k, int slices, int slice_type) {
    using namespace momms::split;
    if (m < 0 || n < 0 || k < 0 || slices < 1) return 0;
    const int max_slices = slice_type == MOMMS_SLICE_BF16     ? kMaxSlicesBf16
                           : slice_type == MOMMS_SLICE_INT8     ? kMaxSlicesI8
                           : slice_type == MOMMS_SLICE_FP8      ? kMaxSlicesF8
                           : slice_type == MOMMS_SLICE_INT8_CRT ? kMaxModuli
                                                                : 0;
    if (slices > max_slices) return 0;
    return layout(m, n, k, slices, slice_type != MOMMS_SLICE_BF16, slice_type == MOMMS_SLICE_INT8_CRT).total;
}

int momms_crt_bits(int64_t k, int moduli, int* moduli_out) {
    using namespace momms::split;
    if (k < 0) return -1;
    if (moduli < 1 || moduli > kMaxModuli) return -2;
    CrtParams cp;
    if (crt_params(moduli, k, &cp) != 0) return MOMMS_ERR_INTERNAL;
    if (moduli_out != nullptr)
        for (int l = 0; l < moduli; ++l) moduli_out[l] = cp.p[l];
    return cp.t >= 1 ? cp.t : MOMMS_ERR_INFEASIBLE;
}

int momms_gemm_split(int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int slices,
                     int slice_type, int family_member, void* workspace, size_t ws_bytes,
                     momms_stream_t stream) {
    using namespace momms;
    using namespace momms::split;
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
    if (slice_type != MOMMS_SLICE_BF16 && slice_type != MOMMS_SLICE_INT8 && slice_type != MOMMS_SLICE_FP8 &&
        slice_type != MOMMS_SLICE_INT8_CRT)
        return -15;
    const bool f8 = slice_type == MOMMS_SLICE_FP8;
    const bool crt = slice_type == MOMMS_SLICE_INT8_CRT;
    const bool bytes = slice_type != MOMMS_SLICE_BF16;   // INT8, FP8 and the moduli share the byte layout
    const int max_slices = crt ? kMaxModuli : f8 ? kMaxSlicesF8 : bytes ? kMaxSlicesI8 : kMaxSlicesBf16;
    if (slices < 1 || slices > max_slices) return -14;
    if (family_member != MOMMS_AUTO && family_member != MOMMS_C0 && family_member != MOMMS_C3C0) return -16;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return -17;
    const Layout L = layout(m, n, k, slices, bytes, crt);
    // Every diagonal's sum must stay exact: INT8 in INT32 (slices * kp <=
    // 2^17, products up to 127^2), FP8 in FP32 (slices * kp <= 2^16, products
    // up to 16^2, sums below 2^24).  Moduli: one product each, residues up to
    // 128 in magnitude: kp <= 2^17 (a sum of 2^17 products (-128)^2 wraps in
    // INT32, which only p = 256 can see, and 256 divides 2^32).
    const int64_t exact_limit = f8 ? kF8MaxProducts : kI8MaxProducts;
    if (bytes && reads_ab && (crt ? L.kp : (int64_t)slices * L.kp) > exact_limit) return MOMMS_ERR_INFEASIBLE;
    CrtParams cp{};
    if (crt && reads_ab && (crt_params(slices, k, &cp) != 0 || cp.t < 1)) return MOMMS_ERR_INFEASIBLE;
    if (reads_ab && (workspace == nullptr || ws_bytes < L.total)) return -18;
    if (cdiv(m, kMT) * cdiv(n, kMT) >= (int64_t)INT_MAX / 2) return MOMMS_ERR_INFEASIBLE;

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (m == 0 || n == 0) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;
    if (alpha == 0.0 || k == 0) {
        int grid = (int)cdiv(m * n, 256);
        if (grid > 16384) grid = 16384;
        hipLaunchKernelGGL(k_scale, dim3(grid), dim3(256), 0, st, m, n, beta, C, ldc);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    char* ws = static_cast<char*>(workspace);
    int* ea = reinterpret_cast<int*>(ws + L.off_ea);
    int* eb = reinterpret_cast<int*>(ws + L.off_eb);
    void* SA = ws + L.off_sa;
    void* SB = ws + L.off_sb;
    double* V = reinterpret_cast<double*>(ws + L.off_v);

    // s1: exponents of the rows of op(A) and the columns of op(B)
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, st, ea, m, kExpNone);
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, eb, n, kExpNone);
    const int64_t chunk = 1024, col_chunk = 128;   // column scans: more blocks, fewer rows each
    if (!ta)  // rows of A
        hipLaunchKernelGGL(k_rowmax_exp, dim3((unsigned)cdiv(m, 4), (unsigned)cdiv(k, chunk)), dim3(256), 0, st, A,
                           lda, m, k, chunk, ea);
    else      // A stored k x m: columns
        hipLaunchKernelGGL(k_colmax_exp, dim3((unsigned)cdiv(m, 256), (unsigned)cdiv(k, col_chunk)), dim3(256), 0,
                           st, A, lda, k, m, col_chunk, ea);
    if (!tb)  // B stored k x n: columns
        hipLaunchKernelGGL(k_colmax_exp, dim3((unsigned)cdiv(n, 256), (unsigned)cdiv(k, col_chunk)), dim3(256), 0,
                           st, B, ldb, k, n, col_chunk, eb);
    else      // B stored n x k: rows
        hipLaunchKernelGGL(k_rowmax_exp, dim3((unsigned)cdiv(n, 4), (unsigned)cdiv(k, chunk)), dim3(256), 0, st, B,
                           ldb, n, k, chunk, eb);
    // s2: slices.  A side X = op(A) (m x k); B side X = op(B)^T (n x k).
    {
        const dim3 ga((unsigned)cdiv(L.kp, 64), (unsigned)cdiv(L.mp, 64));
        const dim3 gb((unsigned)cdiv(L.kp, 64), (unsigned)cdiv(L.np, 64));
#define MOMMS_SLICE_LAUNCH(KIND_)                                                                                \
    do {                                                                                                        \
        if (!ta) hipLaunchKernelGGL((k_slice<false, KIND_>), ga, dim3(256), 0, st, A, lda, m, k, ea, slices, SA, L.mp, L.kp); \
        else     hipLaunchKernelGGL((k_slice<true, KIND_>), ga, dim3(256), 0, st, A, lda, m, k, ea, slices, SA, L.mp, L.kp);  \
        if (!tb) hipLaunchKernelGGL((k_slice<true, KIND_>), gb, dim3(256), 0, st, B, ldb, n, k, eb, slices, SB, L.np, L.kp);  \
        else     hipLaunchKernelGGL((k_slice<false, KIND_>), gb, dim3(256), 0, st, B, ldb, n, k, eb, slices, SB, L.np, L.kp); \
    } while (0)
        int8_t* ra = static_cast<int8_t*>(SA);
        int8_t* rb = static_cast<int8_t*>(SB);
        if (crt) {
            const dim3 ra_g((unsigned)(L.kp / 128), (unsigned)(L.mp / 32));
            const dim3 rb_g((unsigned)(L.kp / 128), (unsigned)(L.np / 32));
            if (!ta) hipLaunchKernelGGL((k_residues<false>), ra_g, dim3(256), 0, st, A, lda, m, k, ea, cp, ra, L.mp, L.kp);
            else     hipLaunchKernelGGL((k_residues<true>), ra_g, dim3(256), 0, st, A, lda, m, k, ea, cp, ra, L.mp, L.kp);
            if (!tb) hipLaunchKernelGGL((k_residues<true>), rb_g, dim3(256), 0, st, B, ldb, n, k, eb, cp, rb, L.np, L.kp);
            else     hipLaunchKernelGGL((k_residues<false>), rb_g, dim3(256), 0, st, B, ldb, n, k, eb, cp, rb, L.np, L.kp);
        } else if (f8) {
            MOMMS_SLICE_LAUNCH(2);
        } else if (bytes) {
            MOMMS_SLICE_LAUNCH(1);
        } else {
            MOMMS_SLICE_LAUNCH(0);
        }
#undef MOMMS_SLICE_LAUNCH
    }
    // s3 + s4: one launch per diagonal, smallest first.
    const int tile_m = bytes ? kI8MT : bf::kMT, tile_n = bytes ? kI8NT : bf::kNT;
    Sched s;
    s.m_off = 0;
    s.n_off = 0;
    s.m_lim = m;
    s.n_lim = n;
    s.tiles_m = (int)cdiv(m, tile_m);
    s.tiles_n = (int)cdiv(n, tile_n);
    const bool grouped = family_member != MOMMS_C0;
    const int gm = 4;  // tiles per group along m in the grouped order
    s.group_m = grouped ? (s.tiles_m < gm ? s.tiles_m : gm) : 1;
    s.xcd = grouped ? kXcds : 1;
    const dim3 grid((unsigned)(s.tiles_m * s.tiles_n));
    const int64_t sas = L.mp * L.kp, sbs = L.np * L.kp;
    if (crt) {
        // s3: one INT8 product per modulus, persistent over (modulus, tile) items
        CrtOut co{};
        co.R = reinterpret_cast<uint8_t*>(ws + L.off_v);
        co.ldr = L.np;
        co.plane = rup(m, 4) * L.np;
        for (int l = 0; l < slices; ++l) {
            co.p[l] = cp.p[l];
            co.c16[l] = 65536 % cp.p[l];
            co.ipf[l] = cp.ipf[l];
        }
        const int tiles = s.tiles_m * s.tiles_n;
        const int items = tiles * slices;
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        int G = items < cus ? items : cus;
        if (G >= kXcds) G -= G % kXcds;
        hipLaunchKernelGGL(k_crt_gemm, dim3((unsigned)G), dim3(512), 0, st, m, n, L.kp,
                           static_cast<const int8_t*>(SA), static_cast<const int8_t*>(SB), sas, sbs, s, tiles, items,
                           co);
        // s4: Chinese remainder reconstruction, rounding and the C update
        const int64_t work = cdiv(m, 4) * n;
        int64_t blocks = cdiv(work, 256);
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_crt_combine, dim3((unsigned)blocks), dim3(256), 0, st, m, n, co.R, co.plane, co.ldr, ea,
                           eb, cp, alpha, beta, C, ldc);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    if (bytes) {
        // s3 + s4, byte slices: one launch per diagonal, smallest first
        for (int d = slices - 1; d >= 0; --d) {
            const bool first = d == slices - 1, last = d == 0;
            const int shift = f8 ? 2 * kF8B0 + d * kF8B : 2 * kI8Bits + d * kI8Bits;
            const int8_t* a8 = static_cast<const int8_t*>(SA);
            const int8_t* b8 = static_cast<const int8_t*>(SB);
            decltype(&launch_i8_diag<true, true, false>) launch;
            if (f8) launch = first ? (last ? launch_i8_diag<true, true, true> : launch_i8_diag<true, false, true>)
                                   : (last ? launch_i8_diag<false, true, true> : launch_i8_diag<false, false, true>);
            else    launch = first ? (last ? launch_i8_diag<true, true, false> : launch_i8_diag<true, false, false>)
                                   : (last ? launch_i8_diag<false, true, false> : launch_i8_diag<false, false, false>);
            launch(grid, st, m, n, L.kp, d, a8, b8, sas, sbs, shift, ea, eb, V, n, alpha, beta, C, ldc, s);
        }
    } else {
        // s3 + s4, BF16: every diagonal in one launch
        hipLaunchKernelGGL(k_split_bf16, grid, dim3(512), 0, st, m, n, L.kp, slices,
                           static_cast<const uint16_t*>(SA), static_cast<const uint16_t*>(SB), sas, sbs, ea, eb, V,
                           n, alpha, beta, C, ldc, s);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"

// Workgroup -> tile order shared by the FP64 and split-precision kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace momms {

constexpr int kXcds = 8;  // XCDs on MI355X; workgroup b is dispatched to XCD b % 8

// Workgroup tile: MT x NT of C per workgroup, KS = LDS k-slice depth,
// WM x WN waves of 64 lanes, each owning a (MT/WM) x (NT/WN) sub-tile.
template <int MT_, int NT_, int KS_, int WM_, int WN_>
struct TileCfg {
    static constexpr int MT = MT_, NT = NT_, KS = KS_, WM = WM_, WN = WN_;
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int WTM = MT / WM, WTN = NT / WN;
    static constexpr int BM = WTM / 16, BN = WTN / 16;
    // LDS row pitches (doubles): A slices are stored [m][k], B slices [k][n].
    static constexpr int A_LD = KS + 1;
    static constexpr int B_LD = NT + 2;
    static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be a multiple of 16");
    static_assert(KS % 4 == 0, "k-slice must be a multiple of the MFMA depth 4");
};

// Region of C covered by one launch and the order in which workgroups visit
// its granules.  A granule is the C area one workgroup owns.
struct Sched {
    int64_t m_off, n_off;  // region origin (elements)
    int64_t m_lim, n_lim;  // region end, exclusive, already clipped to (m, n)
    int tiles_m, tiles_n;  // granules in the region
    int group_m;           // grouped order: group_m granule rows are swept
                           // column by column; 1 = row-major, tiles_m = column-major
    int xcd;               // 1: plain order; 8: each XCD takes a contiguous run of the order
};

// Workgroup b -> granule (tm, tn).  With xcd == 8 the run of the tile order
// handed to XCD x is [x*q + min(x, r), ...) where q, r = T / 8, T % 8, so the
// workgroups that share one L2 work on neighbouring granules.
__device__ __forceinline__ void decode_tile(const Sched& s, int b, int& tm, int& tn) {
    const int T = s.tiles_m * s.tiles_n;
    int t = b;
    if (s.xcd > 1) {
        const int x = b % s.xcd, slot = b / s.xcd;
        const int q = T / s.xcd, r = T % s.xcd;
        t = x * q + (x < r ? x : r) + slot;
    }
    const int per_group = s.group_m * s.tiles_n;
    const int g = t / per_group;
    const int first_m = g * s.group_m;
    const int rows = (s.tiles_m - first_m) < s.group_m ? (s.tiles_m - first_m) : s.group_m;
    const int local = t - g * per_group;
    tm = first_m + local % rows;
    tn = local / rows;
}

}  // namespace momms

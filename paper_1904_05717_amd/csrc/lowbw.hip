// Low-bandwidth emulation for the family's bandwidth experiments (Sec. 5,
// "Experimental setup", and the varying-bandwidth comparisons of Goto's
// algorithm with B3A2C0 and C4A2C0 in Sec. 5's L3 and L4 studies).  There the
// rate of I/O was lowered against the rate of computation by running the
// memory with fewer channels and a lower multiplier.  A GPU's memory clock is
// not the user's to set, so here a second kernel takes bandwidth instead: it
// streams a large device buffer on its own stream while a product runs on
// another.
//
// Every workgroup of the streamer asks for all of a compute unit's LDS, so no
// workgroup of the product can share a compute unit with it: the product runs
// on the other compute units, and its HBM bandwidth is what the streamer
// leaves.  Mode 1 runs the same kernel (same registers, same LDS, so the same
// placement) asleep instead of reading: a product beside it runs on the same
// remaining compute units at full bandwidth, and the ratio of the two times
// isolates the bandwidth.  The streamer reads with non-temporal loads, and its
// buffer should exceed the 256 MiB MALL, so its reads reach HBM.
//
// Every workgroup leaves its loop when the stop bit of the flag is set
// (momms_lowbw_stop, enqueued after the product), when its wall-clock budget
// has run out, or after a fixed number of rounds, whichever comes first.
#include <hip/hip_runtime.h>

#include "../../include/momms.h"

namespace momms {
namespace lowbw {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kUnroll = 16;                     // 16-byte loads in flight per lane
constexpr int64_t kRoundVecs = 64 * kUnroll;    // vectors one wave reads per round (16 KiB)
constexpr int kRoundsPerPoll = 8;               // rounds between looks at the flag and the clock
constexpr unsigned long long kStopBit = 1ull << 63;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The flag is polled with an atomic add, not a load: a plain load, even an
// agent-scope atomic one, can keep returning the copy held in this XCD's L2
// after another XCD has set the flag.  One thread per workgroup polls and
// shares the answer through LDS, which keeps the atomics to one per
// workgroup per poll.
//
// rec: four words per wave: rounds done, a checksum of what was read (keeps the
// loads), wall clock at entry, wall clock at exit.
__global__ __launch_bounds__(kThreads) void k_stream(int mode, const u32x4* __restrict__ buf, int64_t rounds_per_wave,
                                                     unsigned long long* flag, uint64_t max_ticks, int64_t max_rounds,
                                                     unsigned long long* rec) {
    extern __shared__ u32x4 reserved[];   // held: it keeps the product off this compute unit
    volatile int* stop_seen = reinterpret_cast<volatile int*>(reserved);
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const u32x4* base = buf + gw * rounds_per_wave * kRoundVecs + lane;
    const uint64_t t0 = wall_clock64();
    u32x4 acc = {0u, 0u, 0u, 0u};
    int64_t r = 0, pos = 0;
    while (r < max_rounds) {
        if (threadIdx.x == 0) {
            const unsigned long long seen = atomicAdd(flag, 1ull);
            *stop_seen = (seen & kStopBit) != 0 || wall_clock64() - t0 > max_ticks;
        }
        __syncthreads();
        const int stop = *stop_seen;
        __syncthreads();   // every wave has read it before thread 0 writes the next
        if (stop) break;
        for (int q = 0; q < kRoundsPerPoll; ++q) {
            if (mode == 0) {
                const u32x4* p = base + pos * kRoundVecs;
                u32x4 v[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(p + u * 64);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) acc ^= v[u];
                if (++pos == rounds_per_wave) pos = 0;
            } else {
                __builtin_amdgcn_s_sleep(32);
            }
        }
        r += kRoundsPerPoll;
    }
    const uint64_t t1 = wall_clock64();
    // xor across the wave so one lane can store it
    unsigned int c = acc.x ^ acc.y ^ acc.z ^ acc.w;
    for (int off = 32; off > 0; off >>= 1) c ^= __shfl_xor(c, off);
    if (lane == 0) {
        rec[4 * gw + 0] = (unsigned long long)r;
        rec[4 * gw + 1] = c;
        rec[4 * gw + 2] = t0;
        rec[4 * gw + 3] = t1;
    }
}

// op 0: only the stamp; 1: clear the flag (before the streamer starts);
// 2: set the stop bit.
__global__ void k_signal(unsigned long long* flag, int op, unsigned long long* stamp) {
    if (threadIdx.x == 0) {
        if (stamp != nullptr) *stamp = wall_clock64();
        if (op == 1) *flag = 0ull;
        if (op == 2) atomicOr(flag, kStopBit);
    }
}

static int launch_signal(unsigned long long* flag, int op, unsigned long long* stamp, hipStream_t st) {
    hipLaunchKernelGGL(k_signal, dim3(1), dim3(64), 0, st, flag, op, stamp);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace lowbw
}  // namespace momms

extern "C" {

size_t momms_lowbw_min_bytes(int workgroups) {
    using namespace momms::lowbw;
    if (workgroups <= 0) return 0;
    return (size_t)workgroups * kWaves * kRoundVecs * 16;
}

size_t momms_lowbw_record_words(int workgroups) {
    using namespace momms::lowbw;
    return workgroups <= 0 ? 0 : (size_t)workgroups * kWaves * 4;
}

int64_t momms_lowbw_round_bytes(void) { return momms::lowbw::kRoundVecs * 16; }

int64_t momms_lowbw_clock_hz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -1;
    return (int64_t)khz * 1000;
}

int momms_lowbw_start(int mode, const void* buf, size_t bytes, int workgroups, unsigned long long* flag, unsigned long long* rec,
                      double max_seconds, int64_t max_rounds, momms_stream_t stream) {
    using namespace momms::lowbw;
    if (mode != 0 && mode != 1) return -1;
    if (mode == 0 && buf == nullptr) return -2;
    if (mode == 0 && (reinterpret_cast<uintptr_t>(buf) & 15) != 0) return -2;
    if (workgroups <= 0) return -4;
    if (mode == 0 && bytes < momms_lowbw_min_bytes(workgroups)) return -3;
    if (flag == nullptr) return -5;
    if (rec == nullptr) return -6;
    if (!(max_seconds > 0.0) || max_seconds > 60.0) return -7;
    if (max_rounds <= 0) return -8;
    int dev = 0, cus = 0, lds = 0, khz = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return (int)e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return (int)e;
    if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return (int)e;
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return (int)e;
    if (workgroups > cus) return -4;   // every streamer workgroup must be resident at once
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stream),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds)) != hipSuccess)
        return (int)e;
    const int64_t rounds_per_wave =
        mode == 0 ? (int64_t)(bytes / (size_t)momms_lowbw_min_bytes(workgroups)) : 1;
    const uint64_t max_ticks = (uint64_t)(max_seconds * (double)khz * 1000.0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc;
    // Clear the flag and wait for the clear on the host, so a stop enqueued
    // on any stream after this call returns cannot be overtaken by it.
    if ((rc = launch_signal(flag, 1, nullptr, st)) != 0) return rc;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_stream, dim3(workgroups), dim3(kThreads), (size_t)lds, st, mode,
                       static_cast<const u32x4*>(buf), rounds_per_wave, flag, max_ticks, max_rounds, rec);
    e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

int momms_lowbw_stop(unsigned long long* flag, unsigned long long* stamp, momms_stream_t stream) {
    if (flag == nullptr) return -1;
    return momms::lowbw::launch_signal(flag, 2, stamp, static_cast<hipStream_t>(stream));
}

int momms_lowbw_stamp(unsigned long long* stamp, momms_stream_t stream) {
    if (stamp == nullptr) return -1;
    return momms::lowbw::launch_signal(nullptr, 0, stamp, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Batched uneven FP64 GEMMs: one persistent launch over a device queue of
// work items, replayed from a hipGraph captured at plan time.
//
// Each problem runs one family member of its own (Sec. 2.3: which operand is
// worth keeping resident depends on the problem's shape), with a 64 x 64 or
// 128 x 128 register tile:
//   C0    : one item per C tile over all of k, tiles in row-major order;
//   C3C0  : the same items in the grouped order (8 tile rows swept column by
//           column), so the tiles running together share A and B panels;
//   B3C0  : k split into k_c3 chunks (the outer loop of the member), one item
//           per (chunk, tile), chunk by chunk, tiles column by column (a
//           chunk's run of items shares a B block);
//   A3C0  : as B3C0 with the tiles row by row (the run shares an A block).
// A k-split item writes its partial tile to the plan's workspace; the item
// that completes a tile's last chunk (an arrival counter per tile) adds the
// partials into C in chunk order, with the rounding of the single-product
// member's per-chunk epilogue, so the result is deterministic and equal bit
// for bit to the single product of the same member and register tile.
// Workgroups take items in order of decreasing work (longest processing time
// first) across all problems, so long items start early and short ones fill
// the tail.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/momms.h"
#include "kernels_f64.hip"
#include "plan_internal.h"

namespace momms {
namespace batch {

using BL = TileCfg<128, 128, 16, 2, 2>;
using BS = TileCfg<64, 64, 16, 2, 2>;

constexpr int64_t kSplitKc = 512;   // k_c3 of the single-product B3C0 / A3C0

struct Prob {
    int64_t m, n, k, lda, ldb, ldc;
    const double* A;
    const double* B;
    double* C;
    double alpha, beta;
    double* P;       // k-split: partial tiles [tile][chunk][t * t]
    unsigned* cnt;   // k-split: arrivals per tile
    int64_t kc;      // k extent of one chunk (k when not split)
    int tile;        // 64 or 128
    int tiles_n;     // tiles per row of C
    int chunks;      // k chunks (1: not split)
    int member;
};

struct Item {
    int prob;
    int tile;    // row-major tile index within the problem
    int chunk;   // k chunk (0 when not split)
    int pad;
};

// The problem table holds device pointers, but a pointer read from memory is
// generic to the compiler, which then emits flat loads and stores.  Flat loads
// also count on the LDS wait counter, so every wait for an LDS read would wait
// for the prefetch in flight too.  Rebuilding each pointer from its address
// as a global-memory pointer lets the compiler emit global instructions (a
// cast of the generic pointer alone is folded away).
template <class T>
__device__ __forceinline__ T* global_ptr(T* p) {
    return (T*)((__attribute__((address_space(1))) T*)(uintptr_t)p);
}

// Start of every replay: the queue counter and every arrival counter to zero
// (a kernel, not a memset node, inside the captured graph).
__global__ __launch_bounds__(256) void k_reset(unsigned* __restrict__ counter, unsigned* __restrict__ cnt,
                                               int64_t ncnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *counter = 0u;
    for (int64_t j = i; j < ncnt; j += (int64_t)gridDim.x * blockDim.x) cnt[j] = 0u;
}

// A k-split item's tile is complete: C = the chunk partials added in chunk
// order, each pass rounded as the single product's epilogue rounds it (first
// chunk with beta, later ones with beta = 1).
template <int T>
__device__ __forceinline__ void reduce_chunks(const Prob& p, int tile, int64_t m0, int64_t n0) {
    const double* P = p.P + (int64_t)tile * p.chunks * T * T;
    const int rows = (int)((p.m - m0) < T ? (p.m - m0) : T), cols = (int)((p.n - n0) < T ? (p.n - n0) : T);
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int r = e / T, c = e - (e / T) * T;
        if (r >= rows || c >= cols) continue;
        double* cp = p.C + (m0 + r) * p.ldc + n0 + c;
        double v = epilogue_value(p.alpha, P[e], p.beta, p.beta != 0.0 ? *cp : 0.0);
        for (int q = 1; q < p.chunks; ++q) v = epilogue_value(p.alpha, P[(int64_t)q * T * T + e], 1.0, v);
        *cp = v;
    }
}

template <class CF>
__device__ __forceinline__ void run_item(const Prob& p, const Item& w, double* lds_a, double* lds_b, int* flag) {
    constexpr int T = CF::MT;
    auto As = reinterpret_cast<double (*)[CF::MT * CF::A_LD]>(lds_a);
    auto Bs = reinterpret_cast<double (*)[CF::KS * CF::B_LD]>(lds_b);
    const int tm = w.tile / p.tiles_n, tn = w.tile - (w.tile / p.tiles_n) * p.tiles_n;
    const int64_t m0 = (int64_t)tm * T, n0 = (int64_t)tn * T;
    const bool split = p.chunks > 1;
    const int64_t kb = (int64_t)w.chunk * p.kc, ke = (kb + p.kc) < p.k ? (kb + p.kc) : p.k;
    d4 acc[CF::BM][CF::BN];
    regc_acc<CF, false, false, false>(p.m, p.n, kb, ke, p.A, p.lda, p.B, p.ldb, m0, n0, tm, tn, As, Bs, acc);
    // one epilogue for both kinds of item: C = alpha acc + beta C on the tile,
    // or the raw partial (alpha 1, beta 0) into the tile's chunk slot
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* dst = split ? p.P + ((int64_t)w.tile * p.chunks + w.chunk) * T * T : p.C;
    store_c<CF>(acc, split ? 1.0 : p.alpha, split ? 0.0 : p.beta, dst, split ? T : p.ldc, split ? 0 : m0,
                split ? 0 : n0, split ? T : p.m, split ? T : p.n, wave / CF::WN, wave % CF::WN, lane);
    if (!split) return;
    // release the partial at device scope, then count the arrival; the
    // workgroup that brings the count to `chunks` acquires and reduces
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *flag = (atomicAdd(p.cnt + w.tile, 1u) == (unsigned)(p.chunks - 1)) ? 1 : 0;
    __syncthreads();
    if (*flag) {
        __threadfence();
        reduce_chunks<T>(p, w.tile, m0, n0);
    }
}

// Persistent workgroups: pop an item from the queue, run it with its
// problem's member and register tile, repeat until the queue is empty.  Every
// workgroup leaves once the counter passes nitems; no item waits for another.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_batch(const Prob* __restrict__ probs, const Item* __restrict__ items, int nitems,
             unsigned* __restrict__ counter) {
    // one flat LDS area per operand, viewed as the two stage buffers of
    // either tile class
    __shared__ double lds_a[2 * BL::MT * BL::A_LD];
    __shared__ double lds_b[2 * BL::KS * BL::B_LD];
    __shared__ int next, last_flag;
    for (;;) {
        if (threadIdx.x == 0) next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = next;
        __syncthreads();  // all threads have read `next` before it is overwritten
        if (it >= nitems) break;
        const Item w = items[it];
        Prob p = probs[w.prob];
        p.A = global_ptr(p.A);
        p.B = global_ptr(p.B);
        p.C = global_ptr(p.C);
        if (p.chunks > 1) {
            p.P = global_ptr(p.P);
            p.cnt = global_ptr(p.cnt);
        }
        if (p.tile == 128) run_item<BL>(p, w, lds_a, lds_b, &last_flag);
        else run_item<BS>(p, w, lds_a, lds_b, &last_flag);
    }
}
static_assert(BS::MT * BS::A_LD <= BL::MT * BL::A_LD, "64-tile A stage must fit the 128-tile area");
static_assert(BS::KS * BS::B_LD <= BL::KS * BL::B_LD, "64-tile B stage must fit the 128-tile area");

// Per-slot rates of the two register tiles and the fixed cost of an item
// (a tile's prologue, epilogue and queue pop).  Defaults: the 128-tile body
// sustains about 66 TFLOP/s over 512 slots; the 64-tile body about 0.55 of
// that per slot (both measured on 512-problem batches).  A measured table
// replaces them through momms_batch_set_rates.
static double g_rate128 = 66e12 / 512.0, g_rate64 = 0.55 * 66e12 / 512.0, g_item_s = 1.5e-6;

static double item_seconds(int t, int64_t k) {
    return 2.0 * t * t * (double)(k > 0 ? k : 1) / (t == 128 ? g_rate128 : g_rate64) + g_item_s;
}

// Register tile of one problem (Sec. 2.3's choice of blocking by shape,
// applied to the level-0 block): both tile classes run in the same resident
// workgroup slots, so a choice costs the slot time of its padded tiles.
static int prior_tile(int64_t m, int64_t n, int64_t k) {
    auto cost = [&](int t) {
        const double tiles = (double)((m + t - 1) / t) * (double)((n + t - 1) / t);
        return tiles * item_seconds(t, k);
    };
    return cost(128) <= cost(64) ? 128 : 64;
}

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace batch
}  // namespace momms

struct momms_batch {
    int count;
    int nitems;
    int grid;
    int64_t ncnt;
    momms::batch::Prob* d_probs;
    momms::batch::Item* d_items;
    unsigned* d_counter;
    unsigned* d_cnt;
    double* d_partials;
    hipGraph_t graph;
    hipGraphExec_t exec;
    std::vector<int> tiles, members, chunks;
    double flops, padded_flops;
};

static void batch_free(momms_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->d_cnt) (void)hipFree(b->d_cnt);
    if (b->d_partials) (void)hipFree(b->d_partials);
    delete b;
}

extern "C" {

int momms_batch_create(momms_batch** out, int count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* const* A, const int64_t* lda, const double* const* B, const int64_t* ldb,
                       double* const* C, const int64_t* ldc, const double* alpha, const double* beta,
                       const int* member_or_auto, const int* tile) {
    using namespace momms;
    using namespace momms::batch;
    if (!out) return -1;
    *out = nullptr;
    if (count < 0) return -2;
    if (count > 0 && (!m || !n || !k)) return !m ? -3 : (!n ? -4 : -5);
    if (count > 0 && (!A || !lda)) return !A ? -6 : -7;
    if (count > 0 && (!B || !ldb)) return !B ? -8 : -9;
    if (count > 0 && (!C || !ldc)) return !C ? -10 : -11;
    if (count > 0 && (!alpha || !beta)) return !alpha ? -12 : -13;
    std::vector<Prob> probs((size_t)count);
    std::vector<int> tiles((size_t)count, 0), members((size_t)count, 0), chunks((size_t)count, 1);
    double flops = 0.0, padded = 0.0, slot_seconds = 0.0;
    // pass 1: validate, pick the register tile, sum the slot time
    for (int i = 0; i < count; ++i) {
        const int64_t mi = m[i], ni = n[i], ki = k[i];
        if (mi < 0) return -3;
        if (ni < 0) return -4;
        if (ki < 0) return -5;
        const bool reads_ab = alpha[i] != 0.0 && ki > 0 && mi > 0 && ni > 0;
        if (reads_ab && !A[i]) return -6;
        if (lda[i] < (ki > 1 ? ki : 1)) return -7;
        if (reads_ab && !B[i]) return -8;
        if (ldb[i] < (ni > 1 ? ni : 1)) return -9;
        if (mi > 0 && ni > 0 && !C[i]) return -10;
        if (ldc[i] < (ni > 1 ? ni : 1)) return -11;
        const int mem = member_or_auto ? member_or_auto[i] : MOMMS_AUTO;
        if (mem != MOMMS_AUTO && mem != MOMMS_C0 && mem != MOMMS_C3C0 && mem != MOMMS_B3C0 && mem != MOMMS_A3C0)
            return -14;
        int t = tile ? tile[i] : 0;
        if (t != 0 && t != 64 && t != 128) return -15;
        if (t == 0) t = prior_tile(mi, ni, ki);
        tiles[(size_t)i] = t;
        members[(size_t)i] = mem;
        Prob& p = probs[(size_t)i];
        p.m = mi;
        p.n = ni;
        // alpha == 0: only C := beta C, so A and B are never read (not even
        // to multiply by zero, which would turn an Inf or NaN into NaN)
        p.k = reads_ab ? ki : 0;
        p.lda = lda[i];
        p.ldb = ldb[i];
        p.ldc = ldc[i];
        p.A = reads_ab ? A[i] : nullptr;
        p.B = reads_ab ? B[i] : nullptr;
        p.C = C[i];
        p.alpha = alpha[i];
        p.beta = beta[i];
        p.tile = t;
        p.tiles_n = (int)cdiv(ni, t);
        p.kc = p.k;
        p.chunks = 1;
        if (mi == 0 || ni == 0) continue;
        const int64_t ntiles = cdiv(mi, t) * cdiv(ni, t);
        if (ntiles > (int64_t)1 << 24) return MOMMS_ERR_INFEASIBLE;
        flops += 2.0 * (double)mi * (double)ni * (double)ki;
        padded += 2.0 * (double)ntiles * t * t * (double)p.k;
        slot_seconds += (double)ntiles * item_seconds(t, p.k);
    }
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    if (e != hipSuccess || cus <= 0) return e != hipSuccess ? (int)e : MOMMS_ERR_NO_DEVICE;
    const int slots = 2 * cus;   // two resident workgroups per CU (<= 256 registers, 68 KiB LDS each)
    // pass 2: members.  AUTO keeps whole-k tiles (C0 / C3C0 by whether the
    // problem has tiles in both directions) unless one tile's item would run
    // longer than a quarter of the mean slot time: then k is split (the k_c3
    // loop of B3C0 when the problem is taller than wide, A3C0 otherwise) into
    // chunks of a quarter of that time, so no item holds up the tail.
    const double target = slot_seconds / slots / 4.0;
    int64_t ncnt = 0, npart = 0;
    std::vector<int64_t> cnt_off((size_t)count, -1), part_off((size_t)count, -1);
    for (int i = 0; i < count; ++i) {
        Prob& p = probs[(size_t)i];
        int& mem = members[(size_t)i];
        const int t = p.tile;
        const int64_t tm = cdiv(p.m, t), tn = cdiv(p.n, t);
        if (mem == MOMMS_AUTO) {
            const double one = item_seconds(t, p.k);
            if (p.k >= 4 * 256 && one > target && target > 0.0) {
                mem = tm >= tn ? MOMMS_B3C0 : MOMMS_A3C0;
                const int64_t pieces = (int64_t)std::ceil(one / target);
                int64_t kc = (cdiv(p.k, pieces) + 255) / 256 * 256;
                p.kc = kc < 256 ? 256 : kc;
            } else {
                mem = (tm > 1 && tn > 1) ? MOMMS_C3C0 : MOMMS_C0;
            }
        } else if ((mem == MOMMS_B3C0 || mem == MOMMS_A3C0) && p.k > kSplitKc) {
            p.kc = kSplitKc;
        }
        p.member = mem;
        if ((mem == MOMMS_B3C0 || mem == MOMMS_A3C0) && p.k > p.kc && p.m > 0 && p.n > 0) {
            p.chunks = (int)cdiv(p.k, p.kc);
            cnt_off[(size_t)i] = ncnt;
            part_off[(size_t)i] = npart;
            ncnt += tm * tn;
            npart += tm * tn * p.chunks * (int64_t)t * t;
        } else {
            p.kc = p.k;
        }
        chunks[(size_t)i] = p.chunks;
    }
    // the queue: per problem in its member's order, then longest work first
    std::vector<Item> items;
    for (int i = 0; i < count; ++i) {
        const Prob& p = probs[(size_t)i];
        if (p.m == 0 || p.n == 0) continue;
        const int tm = (int)cdiv(p.m, p.tile), tn = (int)cdiv(p.n, p.tile);
        for (int c = 0; c < p.chunks; ++c) {
            if (p.member == MOMMS_C3C0) {
                const int gm = tm < 8 ? tm : 8;
                for (int g = 0; g < tm; g += gm)
                    for (int y = 0; y < tn; ++y)
                        for (int x = g; x < g + gm && x < tm; ++x) items.push_back(Item{i, x * tn + y, c, 0});
            } else if (p.member == MOMMS_B3C0) {
                for (int y = 0; y < tn; ++y)
                    for (int x = 0; x < tm; ++x) items.push_back(Item{i, x * tn + y, c, 0});
            } else {
                for (int q = 0; q < tm * tn; ++q) items.push_back(Item{i, q, c, 0});
            }
        }
    }
    if (items.size() > (size_t)1 << 30) return MOMMS_ERR_INFEASIBLE;
    auto work = [&](const Item& w) {
        const Prob& p = probs[(size_t)w.prob];
        const int64_t kb = (int64_t)w.chunk * p.kc;
        const int64_t kl = (p.k - kb) < p.kc ? (p.k - kb) : p.kc;
        return (double)p.tile * p.tile * (double)kl;
    };
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) { return work(a) > work(b); });

    momms_batch* b = new (std::nothrow) momms_batch();
    if (!b) return MOMMS_ERR_INTERNAL;
    b->count = count;
    b->nitems = (int)items.size();
    b->tiles = tiles;
    b->members = members;
    b->chunks = chunks;
    b->flops = flops;
    b->padded_flops = padded;
    b->ncnt = ncnt;
    b->grid = std::min(slots, std::max(b->nitems, 1));   // never more workgroups than items
    hipStream_t cs = nullptr;
#define MOMMS_TRY(x)               \
    do {                           \
        e = (x);                   \
        if (e != hipSuccess) {     \
            if (cs) (void)hipStreamDestroy(cs);                       \
            batch_free(b);         \
            return (int)e;         \
        }                          \
    } while (0)
    MOMMS_TRY(hipMalloc(&b->d_probs, sizeof(Prob) * (size_t)(count > 0 ? count : 1)));
    MOMMS_TRY(hipMalloc(&b->d_items, sizeof(Item) * (items.empty() ? 1 : items.size())));
    MOMMS_TRY(hipMalloc(&b->d_counter, 256));
    MOMMS_TRY(hipMalloc(&b->d_cnt, sizeof(unsigned) * (size_t)(ncnt > 0 ? ncnt : 1)));
    if (npart > 0) MOMMS_TRY(hipMalloc(&b->d_partials, sizeof(double) * (size_t)npart));
    for (int i = 0; i < count; ++i) {
        Prob& p = probs[(size_t)i];
        p.cnt = cnt_off[(size_t)i] >= 0 ? b->d_cnt + cnt_off[(size_t)i] : nullptr;
        p.P = part_off[(size_t)i] >= 0 ? b->d_partials + part_off[(size_t)i] : nullptr;
    }
    if (count > 0) MOMMS_TRY(hipMemcpy(b->d_probs, probs.data(), sizeof(Prob) * (size_t)count, hipMemcpyHostToDevice));
    if (!items.empty())
        MOMMS_TRY(hipMemcpy(b->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    // Capture: the counters are reset by a kernel (no memset node), then the
    // persistent kernel runs.
    const int rgrid = (int)std::min<int64_t>(std::max<int64_t>(cdiv(ncnt, 256), 1), 1024);
    MOMMS_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    MOMMS_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_reset, dim3(rgrid), dim3(256), 0, cs, b->d_counter, b->d_cnt, ncnt);
    hipLaunchKernelGGL(k_batch, dim3(b->grid), dim3(256), 0, cs, b->d_probs, b->d_items, b->nitems, b->d_counter);
    MOMMS_TRY(hipStreamEndCapture(cs, &b->graph));
    MOMMS_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    MOMMS_TRY(hipStreamDestroy(cs));
    cs = nullptr;
#undef MOMMS_TRY
    *out = b;
    return 0;
}

int momms_batch_run(momms_batch* plan, momms_stream_t stream) {
    if (!plan) return -1;
    if (plan->nitems == 0) return 0;
    const hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? 0 : (int)e;
}

int momms_batch_info(const momms_batch* plan, int64_t* items, int64_t* workgroups, double* flops,
                     double* padded_flops, int* members, int* tiles, int* chunks) {
    if (!plan) return -1;
    if (items) *items = plan->nitems;
    if (workgroups) *workgroups = plan->nitems > 0 ? plan->grid : 0;
    if (flops) *flops = plan->flops;
    if (padded_flops) *padded_flops = plan->padded_flops;
    for (int i = 0; i < plan->count; ++i) {
        if (members) members[i] = plan->members[(size_t)i];
        if (tiles) tiles[i] = plan->tiles[(size_t)i];
        if (chunks) chunks[i] = plan->chunks[(size_t)i];
    }
    return 0;
}

int momms_batch_destroy(momms_batch* plan) {
    if (!plan) return -1;
    batch_free(plan);
    return 0;
}

int momms_batch_select_tile(int64_t m, int64_t n, int64_t k) {
    if (m < 0 || n < 0 || k < 0) return -1;
    return momms::batch::prior_tile(m, n, k);
}

int momms_batch_set_rates(double rate128, double rate64, double item_seconds) {
    if (!(rate128 > 0) || !std::isfinite(rate128)) return -1;
    if (!(rate64 > 0) || !std::isfinite(rate64)) return -2;
    if (!(item_seconds >= 0) || !std::isfinite(item_seconds)) return -3;
    momms::batch::g_rate128 = rate128;
    momms::batch::g_rate64 = rate64;
    momms::batch::g_item_s = item_seconds;
    return 0;
}

}  // extern "C"

// Batched uneven FP64 GEMMs: one persistent launch over a device queue of
// (problem, tile) items, replayed from a hipGraph captured at plan time.
//
// Every problem runs the register-resident-C loop nest (member C0: C tile in
// registers over all of k, LDS staging the streamed k-slices) with a 64 x 64
// or 128 x 128 register tile chosen per problem.  Workgroups take items in
// order of decreasing work (longest-processing-time first) across both tile
// classes, so the large tiles start early and the small ones fill the tail.
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

struct Prob {
    int64_t m, n, k, lda, ldb, ldc;
    const double* A;
    const double* B;
    double* C;
    double alpha, beta;
    int tile;     // 64 or 128
    int tiles_n;  // tiles per row of C
};

struct Item {
    int prob;
    int tile;  // row-major tile index within the problem
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

__global__ __launch_bounds__(64) void k_reset(unsigned* __restrict__ counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

// Persistent workgroups: pop an item from the queue (ordered by decreasing
// work over both tile classes), run its tile with that problem's register
// tile, repeat until the queue is empty.  Every workgroup leaves once the
// counter passes nitems.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_batch(const Prob* __restrict__ probs, const Item* __restrict__ items, int nitems,
             unsigned* __restrict__ counter) {
    // one flat LDS area per operand, viewed as the two stage buffers of
    // either tile class
    __shared__ double lds_a[2 * BL::MT * BL::A_LD];
    __shared__ double lds_b[2 * BL::KS * BL::B_LD];
    __shared__ int next;
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
        const int tm = w.tile / p.tiles_n, tn = w.tile - (w.tile / p.tiles_n) * p.tiles_n;
        if (p.tile == 128)
            regc_tile<BL, false, false, false>(p.m, p.n, 0, p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C,
                                               p.ldc, (int64_t)tm * 128, (int64_t)tn * 128, tm, tn,
                                               reinterpret_cast<double (*)[BL::MT * BL::A_LD]>(lds_a),
                                               reinterpret_cast<double (*)[BL::KS * BL::B_LD]>(lds_b));
        else
            regc_tile<BS, false, false, false>(p.m, p.n, 0, p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C,
                                               p.ldc, (int64_t)tm * 64, (int64_t)tn * 64, tm, tn,
                                               reinterpret_cast<double (*)[BS::MT * BS::A_LD]>(lds_a),
                                               reinterpret_cast<double (*)[BS::KS * BS::B_LD]>(lds_b));
    }
}
static_assert(BS::MT * BS::A_LD <= BL::MT * BL::A_LD, "64-tile A stage must fit the 128-tile area");
static_assert(BS::KS * BS::B_LD <= BL::KS * BL::B_LD, "64-tile B stage must fit the 128-tile area");

// Analytic prior for the register tile of one problem (Sec. 2.3's logic of
// choosing the blocking by shape, applied to the level-0 block): both tile
// classes run in the same resident-workgroup slots, so the cost of a choice
// is the slot time of its padded tiles, tiles * (2 t^2 k / R_t + overhead).
// R_128 is the measured per-slot rate of the 128-tile body (66 TFLOP/s over
// 512 slots); the 64-tile body sustains about 0.55 of that per slot
// (measured on 512-problem batches, all-64 against all-128).  The padded
// area decides: small or thin problems take 64, large ones 128.
static int prior_tile(int64_t m, int64_t n, int64_t k) {
    const double r128 = 66e12 / 512.0, r64 = 0.55 * r128, overhead = 1.5e-6;
    auto cost = [&](int t, double rate) {
        const double tiles = (double)((m + t - 1) / t) * (double)((n + t - 1) / t);
        return tiles * (2.0 * t * t * (double)(k > 0 ? k : 1) / rate + overhead);
    };
    return cost(128, r128) <= cost(64, r64) ? 128 : 64;
}

}  // namespace batch
}  // namespace momms

struct momms_batch {
    int count;
    int nitems;
    int grid;
    momms::batch::Prob* d_probs;
    momms::batch::Item* d_items;
    unsigned* d_counter;
    hipGraph_t graph;
    hipGraphExec_t exec;
    std::vector<int> tiles;  // chosen register tile per problem
    double flops;
};

static void batch_free(momms_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

extern "C" {

int momms_batch_create(momms_batch** out, int count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* const* A, const int64_t* lda, const double* const* B, const int64_t* ldb,
                       double* const* C, const int64_t* ldc, const double* alpha, const double* beta,
                       const int* tile) {
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
    std::vector<Item> items;
    std::vector<int> tiles((size_t)count, 0);
    double flops = 0.0;
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
        int t = tile ? tile[i] : 0;
        if (t != 0 && t != 64 && t != 128) return -14;
        if (t == 0) t = prior_tile(mi, ni, ki);
        tiles[(size_t)i] = t;
        Prob& p = probs[(size_t)i];
        p.m = mi;
        p.n = ni;
        p.k = ki;
        p.lda = lda[i];
        p.ldb = ldb[i];
        p.ldc = ldc[i];
        p.A = A[i];
        p.B = B[i];
        p.C = C[i];
        p.alpha = alpha[i];
        // alpha == 0 with k > 0 still runs through the kernel (acc = 0); C is
        // then scaled by beta exactly as the single-GEMM path does.
        p.beta = beta[i];
        p.tile = t;
        const int64_t tmn = (mi + t - 1) / t, tnn = (ni + t - 1) / t;
        p.tiles_n = (int)tnn;
        if (mi == 0 || ni == 0) continue;
        if (tmn * tnn > (int64_t)1 << 24) return MOMMS_ERR_INFEASIBLE;
        for (int64_t q = 0; q < tmn * tnn; ++q) items.push_back(Item{i, (int)q});
        flops += 2.0 * (double)mi * (double)ni * (double)ki;
    }
    if (items.size() > (size_t)1 << 30) return MOMMS_ERR_INFEASIBLE;
    // longest work first (tile area x k), stable in problem order
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
        const Prob& pa = probs[(size_t)a.prob];
        const Prob& pb = probs[(size_t)b.prob];
        return (double)pa.tile * pa.tile * (double)pa.k > (double)pb.tile * pb.tile * (double)pb.k;
    });
    momms_batch* b = new (std::nothrow) momms_batch();
    if (!b) return MOMMS_ERR_INTERNAL;
    b->count = count;
    b->nitems = (int)items.size();
    b->tiles = tiles;
    b->flops = flops;
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    if (e != hipSuccess || cus <= 0) {
        batch_free(b);
        return e != hipSuccess ? (int)e : MOMMS_ERR_NO_DEVICE;
    }
    // two resident workgroups per CU (<= 256 registers, 68 KiB LDS each);
    // never more workgroups than items
    b->grid = std::min(cus * 2, std::max(b->nitems, 1));
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
    if (count > 0) MOMMS_TRY(hipMemcpy(b->d_probs, probs.data(), sizeof(Prob) * (size_t)count, hipMemcpyHostToDevice));
    if (!items.empty())
        MOMMS_TRY(hipMemcpy(b->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
    // Capture: the queue counter is reset by a kernel (no memset node), then
    // the persistent kernel runs.
    MOMMS_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    MOMMS_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, cs, b->d_counter);
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

int momms_batch_info(const momms_batch* plan, int64_t* items, int64_t* workgroups, double* flops, int* tiles) {
    if (!plan) return -1;
    if (items) *items = plan->nitems;
    if (workgroups) *workgroups = plan->nitems > 0 ? plan->grid : 0;
    if (flops) *flops = plan->flops;
    if (tiles)
        for (int i = 0; i < plan->count; ++i) tiles[i] = plan->tiles[(size_t)i];
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

}  // extern "C"

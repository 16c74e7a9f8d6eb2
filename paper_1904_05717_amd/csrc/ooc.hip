// Out-of-core level: host memory as the slow layer below HBM.  The paper
// names the extension of the family to out-of-core computation, where the
// transfers are explicit and overlapped, as future work (Sec. 6); its loop
// structure is the level-by-level one of Sec. 3.2 with one more level:
//
//   level 5 (host memory)  -> level 4 (HBM): Resident C.  C is cut into
//   mb x nb blocks; each block lives in HBM while the k loop streams
//   mb x kb panels of A and kb x nb panels of B over PCIe (C costs a read
//   and a write, so it is the operand to keep, Sec. 2.2).  Host traffic is
//   C: 2mn (mn without the read when beta = 0), A: mk ceil(n/nb),
//   B: kn ceil(m/mb) elements, the Resident C count of Sec. 2.2 with the
//   block in HBM.
//
// Inside HBM each block product is an ordinary family member (momms_gemm_ex).
// Copies run on a copy stream and products on the compute stream; two C
// buffers and two panel slots let the copy of the next panel (and of the
// next C block) overlap the current product, ordered by events:
//   panel slot s: copy -> ready[s] -> product -> free[s] -> next copy into s;
//   C buffer b:   (write-back of block b-2) -> load -> cready[b] -> products
//                 -> cdone[b] -> write-back on the copy stream.
#include <hip/hip_runtime.h>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {
namespace ooc {

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t c[2], a[2], b[2], total;
};

static Layout layout(int64_t mb, int64_t nb, int64_t kb) {
    Layout L;
    size_t o = 0;
    for (int i = 0; i < 2; ++i) {
        L.c[i] = o;
        o = align256(o + sizeof(double) * (size_t)mb * nb);
    }
    for (int i = 0; i < 2; ++i) {
        L.a[i] = o;
        o = align256(o + sizeof(double) * (size_t)mb * kb);
        L.b[i] = o;
        o = align256(o + sizeof(double) * (size_t)kb * nb);
    }
    L.total = o;
    return L;
}

struct Events {
    hipEvent_t ready[2], free_[2], cready[2], cdone[2], end;
    int made = 0;
    bool ok = true;
    hipEvent_t* all[9] = {&ready[0], &ready[1], &free_[0], &free_[1], &cready[0], &cready[1],
                          &cdone[0], &cdone[1], &end};
    Events() {
        for (hipEvent_t* e : all) {
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
                ok = false;
                return;
            }
            ++made;
        }
    }
    ~Events() {
        for (int i = 0; i < made; ++i) (void)hipEventDestroy(*all[i]);   // released once complete
    }
};

}  // namespace ooc
}  // namespace momms

extern "C" {

size_t momms_ooc_workspace_size(int64_t mb, int64_t nb, int64_t kb) {
    if (mb < 1 || nb < 1 || kb < 1) return 0;
    return momms::ooc::layout(mb, nb, kb).total;
}

int momms_gemm_ooc(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda, const double* B,
                   int64_t ldb, double beta, double* C, int64_t ldc, int64_t mb, int64_t nb, int64_t kb,
                   int family_member, void* workspace, size_t ws_bytes, momms_stream_t stream,
                   momms_stream_t copy_stream) {
    using namespace momms;
    using namespace momms::ooc;
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (k < 0) return -3;
    const bool reads_ab = alpha != 0.0 && k > 0 && m > 0 && n > 0;
    if (reads_ab && A == nullptr) return -5;
    if (lda < (k > 1 ? k : 1)) return -6;
    if (reads_ab && B == nullptr) return -7;
    if (ldb < (n > 1 ? n : 1)) return -8;
    if (m > 0 && n > 0 && C == nullptr) return -10;
    if (ldc < (n > 1 ? n : 1)) return -11;
    if (mb < 1) return -12;
    if (nb < 1) return -13;
    if (kb < 1) return -14;
    if (family_member < 0 || family_member >= MOMMS_NUM_MEMBERS) return -15;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return -16;
    const Layout L = layout(mb, nb, kb);
    if (m > 0 && n > 0 && (workspace == nullptr || ws_bytes < L.total)) return -17;
    if (m == 0 || n == 0) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;

    hipStream_t st = static_cast<hipStream_t>(stream);
    hipStream_t cs = static_cast<hipStream_t>(copy_stream);
    Events ev;
    if (!ev.ok) return MOMMS_ERR_INTERNAL;
    char* ws = static_cast<char*>(workspace);
    const bool ab = alpha != 0.0 && k > 0;
    const int64_t panels = ab ? cdiv(k, kb) : 1;   // alpha = 0 or k = 0: one product with k = 0 scales C
    int64_t p = 0;                                  // panel counter over the whole call
    int64_t blk = 0;
    hipError_t e = hipSuccess;
#define MOMMS_OOC_CHECK(x)                     \
    do {                                       \
        e = (x);                               \
        if (e != hipSuccess) return (int)e;    \
    } while (0)
    for (int64_t i0 = 0; i0 < m; i0 += mb) {
        const int64_t mr = m - i0 < mb ? m - i0 : mb;
        for (int64_t j0 = 0; j0 < n; j0 += nb, ++blk) {
            const int64_t nr = n - j0 < nb ? n - j0 : nb;
            const int cb = (int)(blk & 1);
            double* Cd = reinterpret_cast<double*>(ws + L.c[cb]);
            // C block in (row pitch nr); the copy stream already finished the
            // write-back of the block that used this buffer two blocks ago.
            if (beta != 0.0)
                MOMMS_OOC_CHECK(hipMemcpy2DAsync(Cd, sizeof(double) * nr, C + i0 * ldc + j0, sizeof(double) * ldc,
                                                 sizeof(double) * nr, mr, hipMemcpyHostToDevice, cs));
            MOMMS_OOC_CHECK(hipEventRecord(ev.cready[cb], cs));
            MOMMS_OOC_CHECK(hipStreamWaitEvent(st, ev.cready[cb], 0));
            for (int64_t q = 0; q < panels; ++q, ++p) {
                const int s = (int)(p & 1);
                const int64_t p0 = q * kb;
                const int64_t kr = ab ? (k - p0 < kb ? k - p0 : kb) : 0;
                double* Ad = reinterpret_cast<double*>(ws + L.a[s]);
                double* Bd = reinterpret_cast<double*>(ws + L.b[s]);
                if (kr > 0) {
                    MOMMS_OOC_CHECK(hipStreamWaitEvent(cs, ev.free_[s], 0));
                    MOMMS_OOC_CHECK(hipMemcpy2DAsync(Ad, sizeof(double) * kr, A + i0 * lda + p0, sizeof(double) * lda,
                                                     sizeof(double) * kr, mr, hipMemcpyHostToDevice, cs));
                    MOMMS_OOC_CHECK(hipMemcpy2DAsync(Bd, sizeof(double) * nr, B + p0 * ldb + j0, sizeof(double) * ldb,
                                                     sizeof(double) * nr, kr, hipMemcpyHostToDevice, cs));
                    MOMMS_OOC_CHECK(hipEventRecord(ev.ready[s], cs));
                    MOMMS_OOC_CHECK(hipStreamWaitEvent(st, ev.ready[s], 0));
                }
                const double bq = q == 0 ? beta : 1.0;
                const int rc = momms_gemm_ex(0, 0, mr, nr, kr, ab ? alpha : 0.0, Ad, kr > 1 ? kr : 1, Bd, nr, bq, Cd,
                                             nr, family_member, nullptr, 0, st);
                if (rc != 0) return rc;
                MOMMS_OOC_CHECK(hipEventRecord(ev.free_[s], st));
            }
            MOMMS_OOC_CHECK(hipEventRecord(ev.cdone[cb], st));
            MOMMS_OOC_CHECK(hipStreamWaitEvent(cs, ev.cdone[cb], 0));
            MOMMS_OOC_CHECK(hipMemcpy2DAsync(C + i0 * ldc + j0, sizeof(double) * ldc, Cd, sizeof(double) * nr,
                                             sizeof(double) * nr, mr, hipMemcpyDeviceToHost, cs));
        }
    }
    // the caller's stream covers the last write-back
    MOMMS_OOC_CHECK(hipEventRecord(ev.end, cs));
    MOMMS_OOC_CHECK(hipStreamWaitEvent(st, ev.end, 0));
#undef MOMMS_OOC_CHECK
    return 0;
}

}  // extern "C"

/*
 * momms.h - C ABI of the MI355X (gfx950) MOMMS GEMM library.
 *
 * The library computes C := alpha * op(A) * op(B) + beta * C in IEEE binary64
 * with hand-written HIP kernels on FP64 MFMA (v_mfma_f64_16x16x4_f64).  The
 * operation is the ordinary matrix product of Smith & van de Geijn, "The
 * MOMMS Family of Matrix Multiplication Algorithms" (SC19), Sec. 2.1
 * (gamma_ij = sum_p alpha_ip beta_pj) used as the update C += A B of
 * Sec. 2.2.1, with BLAS alpha/beta semantics added.
 *
 * A "family member" fixes the loop order and which operand block is kept
 * resident at each memory level (Sec. 3.2-3.3; naming convention of
 * Sec. 3.3, e.g. B3A2C0 = B resident at level 3, A at level 2, C at level 0).
 * The levels are re-derived for gfx950:
 *     level 0 = VGPR/AGPR register tile of a workgroup (C accumulators),
 *     level 2 = LDS (160 KiB per CU),
 *     level 3 = the 4 MiB L2 of one XCD (8 XCDs, each with its own L2),
 *     level 4 = the 256 MiB Infinity Cache (MALL), shared by the chip.
 * Level 1 (the 32 KiB vector L1) is always skipped, as the paper skips its
 * L1 (Sec. 5.2).
 *
 * Conventions shared by every entry point
 *   - Storage is ROW-MAJOR.  op(A) is m x k, op(B) is k x n, C is m x n.
 *     Without transposition A is stored m x k with leading dimension
 *     lda >= max(1,k); with transA != 0, A is stored k x m (lda >= max(1,m))
 *     and op(A) = A^T.  Likewise B is k x n (ldb >= max(1,n)) or, with
 *     transB != 0, n x k (ldb >= max(1,k)).  ldc >= max(1,n).
 *   - Matrix pointers are DEVICE pointers owned by the caller.  The library
 *     never frees or retains them.  C must not alias A or B (not checked).
 *   - Calls are asynchronous on the given (or the library's current) HIP
 *     stream; nothing inside synchronizes the device or allocates memory,
 *     except momms_batch_create/momms_batch_destroy.
 *   - Quick return (no kernel launched, status 0) when m == 0, n == 0, or
 *     (alpha == 0 or k == 0) and beta == 1.  With alpha == 0 (or k == 0) A
 *     and B are not read.  With beta == 0, C is not read, so NaNs in C do not
 *     propagate.
 *   - Return value: 0 on success.  -i means argument number i (1-based, in
 *     the order of the C prototype) is invalid; this check is done on the
 *     host before any HIP call.  A positive value is a hipError_t reported
 *     by the runtime after a launch.  momms_status_string() describes codes.
 *   - Accuracy: every member returns, per entry, a result within
 *     2 (k+2) 2^-53 (|alpha| (|op(A)||op(B)|)_ij + |beta| |C_ij|) of the
 *     exact value (forward error bound of a k-term dot product in any
 *     summation order).  Integer-valued data whose partial sums stay below
 *     2^53 is reproduced exactly.
 */
#ifndef MOMMS_H
#define MOMMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque HIP stream handle (hipStream_t); NULL is the default stream. */
typedef void *momms_stream_t;

/* Family members.  The loop nests are those of Sec. 3.2 (two loops per
 * level), with blocksizes re-derived for the gfx950 levels listed above. */
enum momms_member {
    MOMMS_AUTO = 0,    /* pick by the analytic model and the tuned table   */
    MOMMS_C0 = 1,      /* C resident in registers over all of k; LDS only
                          stages streamed k-slices; plain tile order        */
    MOMMS_C3C0 = 2,    /* as C0, with the workgroups of one XCD covering one
                          C block (XCD-aware grouped tile order)            */
    MOMMS_B3C0 = 3,    /* B block (kc3 x nc3) resident in one XCD's L2; the
                          XCD sweeps m; C updated once per kc3              */
    MOMMS_A3C0 = 4,    /* A block (mc3 x kc3) resident in one XCD's L2; the
                          XCD sweeps n; C updated once per kc3              */
    MOMMS_A2C0 = 5,    /* Goto's algorithm (Sec. 4.3): A block resident in
                          LDS, B panel streamed, C updated once per kc      */
    MOMMS_B3A2C0 = 6,  /* Sec. 5.2: B block in L2, A block in LDS           */
    MOMMS_A3B2C0 = 7,  /* Sec. 5.4: A block in L2, B block in LDS           */
    MOMMS_C3A2C0 = 8,  /* Sec. 5.4: C block in L2, A block in LDS           */
    MOMMS_C4A2C0 = 9,  /* Sec. 5.3: C block in the MALL, A block in LDS     */
    MOMMS_NUM_MEMBERS = 10
};

/* Status codes besides -i (bad argument i) and positive hipError_t values. */
#define MOMMS_OK 0
#define MOMMS_ERR_INFEASIBLE 1002   /* problem too large for the tile grid   */
#define MOMMS_ERR_NO_DEVICE 1003    /* no gfx950 device / HIP init failed    */
#define MOMMS_ERR_INTERNAL 1004
#define MOMMS_ERR_SCRATCH 1005      /* needs more than the static scratch    */

/* Blocking plan of one member for one problem (host-side description). */
typedef struct momms_plan {
    int member;          /* enum momms_member, never MOMMS_AUTO here        */
    int kernel;          /* 0: register-resident C over a k range;
                            1: A block resident in LDS; 2: B block in LDS   */
    int mt, nt, ks;      /* workgroup C tile and LDS k-slice (kernel 1: mt
                            is the A block's rows, 32 with two workgroups
                            per CU, 64 with one for C3A2C0 on problems
                            whose 64-row tiles fill the chip)               */
    int nj, mi;          /* n-tiles per LDS-resident A block (kernel 1);
                            m-tiles per LDS-resident B block (kernel 2)     */
    int group_m;         /* height (in tiles) of a grouped tile order       */
    int xcd_aware;       /* workgroup -> tile map keeps one XCD's tiles
                            contiguous in the tile order                    */
    int pack;            /* streamed panel packed into the workspace        */
    int64_t kc;          /* k extent of the LDS-resident block              */
    int64_t mc3, nc3, kc3;   /* level-3 (XCD L2) block; for C4A2C0, kc3 is
                                the host's k step (four kc chunks per
                                launch)                                    */
    int64_t mc4, nc4;        /* level-4 (MALL) block                        */
    int64_t nc;              /* outermost n blocksize (Goto's n_c)          */
    int64_t k_range;     /* k extent one workgroup accumulates before it
                            writes C (C traffic = 2mn * ceil(k/k_range))    */
    int64_t launches;    /* kernel launches per call (packing included)     */
    int64_t workgroups;  /* workgroups per call                             */
} momms_plan;

/* Data-movement model of one planned call (Sec. 2.2 counts made exact with
 * ceilings at the margins, Sec. 4.1-4.2 level interactions).  Bytes. */
typedef struct momms_bytes {
    double flops;            /* 2 m n k                                     */
    double compulsory;       /* 8 (mk + kn + mn) + 8 mn if beta != 0        */
    double l2_read;          /* bytes the L2s read from the fabric
                                (MALL/HBM); comparable with FETCH_SIZE      */
    double l2_write;         /* bytes written back past the L2s;
                                comparable with WRITE_SIZE                  */
    double hbm_read;         /* level-4 model: reads that miss the MALL     */
    double hbm_write;        /* level-4 model: writes that reach HBM        */
    double lds_fill;         /* bytes copied global -> LDS                  */
    double pack;             /* bytes read + written by packing kernels     */
    double a_reads, b_reads, c_reads, c_writes;  /* l2_read split by operand
                                (elements x 8)                              */
} momms_bytes;

/* ---------------------------------------------------------------------
 * Plain FP64 GEMM, the family's entry point.  Argument numbers for -i:
 * 1 m, 2 n, 3 k, 4 alpha, 5 A, 6 lda, 7 B, 8 ldb, 9 beta, 10 C, 11 ldc,
 * 12 family_member.  No transposition; runs on the stream set by
 * momms_set_stream (default: NULL stream).  Members that pack a panel run
 * unpacked here (no workspace argument).
 */
int momms_gemm(int64_t m, int64_t n, int64_t k, double alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb,
               double beta, double *C, int64_t ldc, int family_member);

/* Full form: transposition flags (for the backward products
 * dA = dC B^T, dB = A^T dC), explicit workspace and stream.  Argument
 * numbers: 1 transA, 2 transB, 3 m, 4 n, 5 k, 6 alpha, 7 A, 8 lda, 9 B,
 * 10 ldb, 11 beta, 12 C, 13 ldc, 14 family_member, 15 workspace,
 * 16 ws_bytes, 17 stream.  workspace may be NULL (then nothing is packed);
 * if non-NULL it must be 256-byte aligned device memory (else -15) holding
 * at least momms_workspace_size(...) bytes (else -16), not used
 * concurrently by another call. */
int momms_gemm_ex(int transA, int transB, int64_t m, int64_t n, int64_t k,
                  double alpha, const double *A, int64_t lda,
                  const double *B, int64_t ldb, double beta,
                  double *C, int64_t ldc, int family_member,
                  void *workspace, size_t ws_bytes, momms_stream_t stream);

/* Allocation-free form of momms_gemm_ex, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same product, arguments 1-14 as in
 * momms_gemm_ex and 15 stream, with no workspace argument.  A member that
 * packs a panel (A2C0) packs it into a library-owned static device array of
 * MOMMS_STATIC_SCRATCH_BYTES (4 MiB) instead, so the result is bitwise equal
 * to momms_gemm_ex with a workspace; other members use no scratch.  If the
 * member would need more than the array holds the call returns
 * MOMMS_ERR_SCRATCH before any HIP call (no member does at present: Goto's
 * panel is at most 288 x 1024 doubles).  Each GPU has its own array, kept
 * until the process ends and shared by every call on that GPU: calls that
 * overlap in time on one GPU (different streams, or different host threads)
 * race on it and must be serialized by the caller.  Nothing is allocated,
 * freed or synchronized; the first call on a device looks up the array's
 * device address (hipGetSymbolAddress) with that device current. */
#define MOMMS_STATIC_SCRATCH_BYTES ((size_t)4 << 20)
int momms_gemm_static(int transA, int transB, int64_t m, int64_t n, int64_t k,
                      double alpha, const double *A, int64_t lda,
                      const double *B, int64_t ldb, double beta,
                      double *C, int64_t ldc, int family_member,
                      momms_stream_t stream);

/* Workspace bytes the member needs to pack its streamed panel for this
 * shape (0 if it packs nothing).  Host-only. */
size_t momms_workspace_size(int64_t m, int64_t n, int64_t k, int family_member);

/* Stream used by momms_gemm.  Host-only bookkeeping; returns 0. */
int momms_set_stream(momms_stream_t stream);

/* Introspection (host-only, no GPU needed). */
int momms_num_members(void);                  /* MOMMS_NUM_MEMBERS         */
const char *momms_member_name(int member);    /* e.g. "B3A2C0"; NULL if bad */
int momms_member_id(const char *name);        /* inverse; -1 if unknown    */
/* Plan of `member` (MOMMS_AUTO resolves to the chosen member) for the
 * shape.  Argument numbers: 1 member, 2 m, 3 n, 4 k, 5 out. */
int momms_member_plan(int member, int64_t m, int64_t n, int64_t k,
                      momms_plan *out);
/* Model prediction for the member's plan.  1 member, 2 m, 3 n, 4 k,
 * 5 beta, 6 packed (nonzero: count packing traffic), 7 out. */
int momms_model_bytes(int member, int64_t m, int64_t n, int64_t k,
                      double beta, int packed, momms_bytes *out);
/* Member MOMMS_AUTO resolves to for the shape: the measured table entry of
 * the shape's bucket (rounded log2 of m, n and k) if one is set, else the
 * analytic prior: among the members that keep C in registers over all of k,
 * the fewest model bytes, then the lower id.  Host-only. */
int momms_select_member(int64_t m, int64_t n, int64_t k);
/* The analytic prior alone.  Host-only. */
int momms_select_member_prior(int64_t m, int64_t n, int64_t k);
/* Installs the measured table (at most 64 entries; count 0 clears it):
 * entry i maps the bucket (log2_m[i], log2_n[i], log2_k[i]) to member[i].
 * The table is process-wide; calls racing with momms_gemm on other threads
 * must be serialised by the caller.  Argument numbers: 1 count, 2 log2_m,
 * 3 log2_n, 4 log2_k, 5 member.  Host-only. */
int momms_set_member_table(int count, const int *log2_m, const int *log2_n, const int *log2_k,
                           const int *member);

const char *momms_status_string(int status);

/* Element transfers of the resident algorithms of the paper (Sec. 2.2:
 * Resident C with an mc x nc block, Resident A with mc x kc, Resident B with
 * kc x nc), with ceilings at the margins, between a slow and a fast memory.
 * resident is 'A', 'B' or 'C'; (b1, b2) is (mc, nc), (mc, kc) or (kc, nc)
 * respectively.  counts[4] receives {A reads, B reads, C reads, C writes}
 * (elements; beta == 0 skips the first read of C).  Host-only.  Argument
 * numbers: 1 resident, 2 m, 3 n, 4 k, 5 b1, 6 b2, 7 beta, 8 counts. */
int momms_model_resident(int resident, int64_t m, int64_t n, int64_t k, int64_t b1, int64_t b2,
                         double beta, double *counts);
/* Cost-balanced Resident A block for a fast memory of M elements when a B
 * element costs beta_b and a C element beta_c (Sec. 2.4):
 * mc = sqrt(beta_b/beta_c M), kc = sqrt(beta_c/beta_b M).  Host-only. */
int momms_balanced_block(double M, double beta_b, double beta_c, double *mc, double *kc);
/* The planner's level-2 (LDS) block solver (Sec. 2.4 balance within the
 * Sec. 4.1 capacity): for a fast memory of lds_bytes (one workgroup's share
 * of a CU's LDS) holding the resident block (row pitch kc + 1 doubles) plus
 * two streamed k-slices of slice x (tile_other + 2) doubles (none when
 * tile_other is 0: the streamed panel goes straight to registers), the block
 * (rows a multiple of row_step, which is a positive multiple of 16, and kc a
 * multiple of slice) with the most flops per unit of streamed cost, the
 * streamed panel costing beta_stream and C beta_c per element; ties go to the
 * block nearer the continuous optimum (momms_balanced_block), then to fewer
 * rows.  The LDS-resident kernels are built for its answer on gfx950: the
 * A-resident block for 80 KiB (two workgroups per CU) with row_step 32, the
 * B-resident block for 160 KiB with row_step 64.  Returns 0, or -i for a bad
 * argument i (rows and kc are 0 when nothing fits).  Host-only. */
int momms_lds_block(double lds_bytes, int slice, int tile_other, int row_step, double beta_stream, double beta_c,
                    int *rows, int *kc);

/* ---------------------------------------------------------------------
 * Split-precision FP64-accurate product (Ozaki-style error-free splitting;
 * Ozaki, Ogita, Oishi & Rump, Numer. Algorithms 59, 2012 - the paper itself
 * has no such method).  op(A) and op(B) are split per row / per column into
 * `slices` integer slices of 8 (first) and 9 (further) bits, exact in BF16;
 * the slice pairs s + t <= slices-1 are multiplied on BF16 MFMA with exact
 * FP32 accumulation over chunks of at most 256 products, summed exactly in
 * FP64 per diagonal s + t, and recombined smallest diagonal first in FP64:
 *   C := fl(fl(alpha * 2^(e_i+f_j) V_ij) + fl(beta * C_ij)).
 * The result is deterministic (bit-reproducible).  Its error against the
 * exact product is at most about (slices+2) * k * 2^(e_i+f_j) * 2^-(9*slices)
 * + (slices+2) u (|A||B|)_ij, where 2^e_i > max_p |op(A)_ip| and
 * 2^f_j > max_p |op(B)_pj|; 7 slices give FP64-level accuracy for data
 * spanning 16 decades.  Inputs must be finite.
 * MOMMS_SLICE_INT8 uses 7-bit slices cut by truncation (|d| <= 127, exact
 * in int8) multiplied on INT8 MFMA with INT32 accumulation, exact over a
 * whole diagonal while slices * k (k rounded up to 128) <= 2^17; larger k
 * returns MOMMS_ERR_INFEASIBLE.  Its error bound is the BF16 one with
 * 2^-(7 slices) for 2^-(9 slices), so 9 INT8 slices match 7 BF16 ones.
 * MOMMS_SLICE_FP8 uses slices of 4 (first) and 5 (further) bits cut by
 * round to nearest (|d| <= 16, exact in OCP FP8 E4M3) multiplied on FP8
 * MFMA with FP32 accumulation, exact over a whole diagonal while slices * k
 * (k rounded up to 128) <= 2^16; larger k returns MOMMS_ERR_INFEASIBLE.  Its
 * error bound is the BF16 one with 2^-(5 slices) for 2^-(9 slices).
 * MOMMS_SLICE_INT8_CRT is the modular form (Ozaki, Uchino & Imamura,
 * "Ozaki scheme II", 2025); `slices` is then the number N of moduli, the N
 * largest pairwise coprime integers <= 256 (256, 255, 253, 251, 247, ...),
 * with product M.  With t the largest integer <= 60 such that 2 k 4^t < M
 * (MOMMS_ERR_INFEASIBLE if t < 1, or if k rounded up to 128 exceeds 2^17),
 * op(A) and op(B) are rounded to integers A'_ip = rint(A_ip 2^(t-e_i)),
 * B'_pj = rint(B_pj 2^(t-f_j)); the N products of their residues run on
 * INT8 MFMA and the Chinese remainder theorem recovers X = A'B' exactly, so
 *   C := fl(fl(alpha * RN(X_ij) 2^(e_i+f_j-2t)) + fl(beta * C_ij)),
 * bit-reproducible.  Error against the exact product:
 *   <= 2^(e_i-t-1) sum_p |op(B)_pj| + 2^(f_j-t-1) sum_p |op(A)_ip|
 *      + k 2^(e_i+f_j-2t-2) + u |C_ij|.
 * At k = 8192, 14 moduli give t = 48, 15 give t = 51, 16 give t = 55.
 * Argument numbers: 1 transA, 2 transB, 3 m, 4 n, 5 k, 6 alpha, 7 A, 8 lda,
 * 9 B, 10 ldb, 11 beta, 12 C, 13 ldc, 14 slices (1..8 BF16, 1..10 INT8,
 * 1..12 FP8, 1..16 moduli), 15 slice_type (MOMMS_SLICE_BF16, MOMMS_SLICE_FP8,
 * MOMMS_SLICE_INT8 or MOMMS_SLICE_INT8_CRT), 16 family_member (MOMMS_AUTO, MOMMS_C0 or
 * MOMMS_C3C0: tile order of the slice products), 17 workspace (device,
 * 256-byte aligned), 18 ws_bytes (>= momms_split_workspace_size), 19 stream.
 * The workspace holds the exponents, the slices (or residues) and the FP64
 * partial sums (or the residues of the products); it must not be used
 * concurrently by another call.
 */
enum momms_slice_type { MOMMS_SLICE_BF16 = 0, MOMMS_SLICE_FP8 = 1, MOMMS_SLICE_INT8 = 2, MOMMS_SLICE_INT8_CRT = 3 };

size_t momms_split_workspace_size(int64_t m, int64_t n, int64_t k, int slices, int slice_type);

/* Modular form: the bit count t used for inner dimension k with `moduli`
 * moduli (MOMMS_SLICE_INT8_CRT above), or MOMMS_ERR_INFEASIBLE when t < 1;
 * if moduli_out is non-NULL it receives the moduli (host memory, `moduli`
 * ints).  Host-only.  Errors: -1 k < 0, -2 moduli outside 1..16. */
int momms_crt_bits(int64_t k, int moduli, int *moduli_out);

int momms_gemm_split(int transA, int transB, int64_t m, int64_t n, int64_t k,
                     double alpha, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double beta,
                     double *C, int64_t ldc, int slices, int slice_type,
                     int family_member, void *workspace, size_t ws_bytes,
                     momms_stream_t stream);

/* ---------------------------------------------------------------------
 * Batched uneven FP64 GEMMs.  momms_batch_create builds a plan for `count`
 * independent problems C_i := alpha_i A_i B_i + beta_i C_i (row-major, no
 * transposition; all pointer arrays are HOST arrays holding DEVICE
 * pointers).  Each problem runs one family member (Sec. 2.3: the shape
 * decides which operand is worth keeping resident) inside one persistent
 * kernel:
 *   MOMMS_C0    one work item per C tile over all of k, row-major tile order;
 *   MOMMS_C3C0  the same items in a grouped order (8 tile rows swept column by
 *               column), so the items running together share panels;
 *   MOMMS_B3C0  k split into k_c3 = 512 chunks, an item per (chunk, tile),
 *               tiles column by column within a chunk (a run shares a B block);
 *   MOMMS_A3C0  as B3C0 with the tiles row by row (a run shares an A block).
 * A split tile's partials are added into C in chunk order by whichever item
 * completes the tile, rounded as the single product's per-chunk epilogue, so
 * every member's result equals momms_gemm_ex with the same member and
 * register tile bit for bit.  MOMMS_AUTO (member_or_auto NULL, or 0 for a
 * problem) picks per problem: B3C0 (taller than wide) or A3C0 when one
 * whole-k tile would run longer than a quarter of the mean per-slot time
 * (then k is split into chunks of about that length, multiples of 256), else
 * C3C0 when the problem has more than one tile each way, else C0.  The
 * register tile (tile NULL or 0: the slot-time prior of
 * momms_batch_select_tile; else 64 or 128 per problem) is chosen first.
 * The plan uploads a descriptor table and a work queue ordered by
 * decreasing work, allocates the split partials and arrival counters, and
 * captures a hipGraph of a counter-reset kernel and the persistent kernel.
 * The plan owns that device memory (allocated here, freed by
 * momms_batch_destroy) and keeps the caller's matrix pointers: they must
 * stay valid while the plan is used.  With alpha_i == 0 (or k_i == 0) A_i
 * and B_i are not read (they may be NULL): C_i := beta_i C_i; beta_i == 0
 * does not read C_i.  Argument numbers: 1 out, 2 count, 3 m, 4 n, 5 k, 6 A,
 * 7 lda, 8 B, 9 ldb, 10 C, 11 ldc, 12 alpha, 13 beta, 14 member_or_auto
 * (MOMMS_AUTO, MOMMS_C0, MOMMS_C3C0, MOMMS_B3C0 or MOMMS_A3C0 per problem;
 * other members are not batched), 15 tile.  A per-problem argument error
 * returns the number of that array.  Synchronous (copies the tables).
 */
typedef struct momms_batch momms_batch;

int momms_batch_create(momms_batch **out, int count, const int64_t *m, const int64_t *n,
                       const int64_t *k, const double *const *A, const int64_t *lda,
                       const double *const *B, const int64_t *ldb, double *const *C,
                       const int64_t *ldc, const double *alpha, const double *beta,
                       const int *member_or_auto, const int *tile);
/* Replays the captured graph on `stream` (asynchronous).  Runs of one plan
 * must not overlap (they share the queue and arrival counters).  1 plan,
 * 2 stream. */
int momms_batch_run(momms_batch *plan, momms_stream_t stream);
/* Plan facts: queue items, persistent workgroups, total 2mnk flops, the
 * flops of the padded tiles, and per problem (arrays of count entries) the
 * member, the register tile and the number of k chunks.  Any output
 * pointer may be NULL. */
int momms_batch_info(const momms_batch *plan, int64_t *items, int64_t *workgroups, double *flops,
                     double *padded_flops, int *members, int *tiles, int *chunks);
int momms_batch_destroy(momms_batch *plan);
/* The slot-time prior's register tile (64 or 128) for one problem. */
int momms_batch_select_tile(int64_t m, int64_t n, int64_t k);
/* Installs the per-slot rates the prior uses (flop/s of one resident
 * workgroup slot with the 128 and the 64 register tile, and the fixed
 * seconds of one work item), e.g. from a measured table; plans created
 * afterwards use them.  Process-wide.  Errors: -1, -2, -3 for a rate or
 * time that is not positive and finite (the item time may be 0).
 * Host-only. */
int momms_batch_set_rates(double rate128, double rate64, double item_seconds);

/* ---------------------------------------------------------------------
 * Tile-major ("prepacked") storage (Sec. 5.2: matrices stored so that every
 * block the algorithm partitions them into is contiguous, which removes
 * packing and isolates temporal from spatial locality).
 *   op(A), m x k:  [m-tile of 128 rows][k-slab of 16][128][16]
 *   op(B), k x n:  [n-tile of 128 columns][k][128]
 * doubles, zero beyond the matrix (k padded to a multiple of 16, m and n to
 * multiples of 128).  `operand` is 'A' or 'B'; rows x cols is the logical
 * m x k (A) or k x n (B).  Buffers are device memory owned by the caller.
 */
/* Bytes of a tiled operand; 0 for an invalid operand or negative sizes. */
size_t momms_tiled_size(int operand, int64_t rows, int64_t cols);
/* T := tiled op(X), op(X) = X (trans = 0, X rows x cols with pitch ldx) or
 * X^T (trans = 1, X stored cols x rows).  Asynchronous on `stream`.
 * Argument numbers: 1 operand, 2 trans, 3 rows, 4 cols, 5 X, 6 ldx, 7 T. */
int momms_to_tiled(int operand, int trans, int64_t rows, int64_t cols, const double *X, int64_t ldx,
                   double *T, momms_stream_t stream);
/* X := the rows x cols matrix held in tiled T (row-major, pitch ldx).
 * Argument numbers: 1 operand, 2 rows, 3 cols, 4 T, 5 X, 6 ldx. */
int momms_from_tiled(int operand, int64_t rows, int64_t cols, const double *T, double *X, int64_t ldx,
                     momms_stream_t stream);
/* C := alpha At Bt + beta C on tiled operands, C row-major (pitch ldc).
 * family_member: MOMMS_AUTO, MOMMS_C0, MOMMS_C3C0, MOMMS_B3C0, MOMMS_A3C0
 * (the members that keep the C tile in registers), MOMMS_A2C0 (Goto, which
 * reads the tiled B panels in place instead of packing them), or any of the
 * LDS-resident members (MOMMS_B3A2C0, MOMMS_A3B2C0, MOMMS_C3A2C0,
 * MOMMS_C4A2C0).  Loop nests and
 * k stagger are those of momms_gemm_ex, so the result equals that call's bit
 * for bit.  beta = 0 does not read C.  Argument numbers: 1 m, 2 n, 3 k,
 * 4 alpha, 5 At, 6 Bt, 7 beta, 8 C, 9 ldc, 10 family_member, 11 stream. */
int momms_gemm_tiled(int64_t m, int64_t n, int64_t k, double alpha, const double *At, const double *Bt,
                     double beta, double *C, int64_t ldc, int family_member, momms_stream_t stream);

/* ---------------------------------------------------------------------
 * Symmetric rank-k update on the family (the paper names the other level-3
 * BLAS as the next target, Sec. 6): C := alpha op(A) op(A)^T + beta C on the
 * lower (uplo = 'L') or upper ('U') triangle of the n x n row-major C (pitch
 * ldc); op(A) = A (trans = 0, n x k, pitch lda) or A^T (trans = 1, A stored
 * k x n).  The other triangle is neither read nor written.  family_member:
 * MOMMS_AUTO (= MOMMS_C3C0), MOMMS_C0 or MOMMS_C3C0, whose tile orders are
 * kept with the tiles outside the triangle skipped.  beta = 0 does not read C.
 * Argument numbers: 1 uplo, 2 trans, 3 n, 4 k, 5 alpha, 6 A, 7 lda, 8 beta,
 * 9 C, 10 ldc, 11 family_member, 12 stream.
 */
int momms_syrk(int uplo, int trans, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
               double beta, double *C, int64_t ldc, int family_member, momms_stream_t stream);

/* ---------------------------------------------------------------------
 * Triangular multiply and solve (the other level-3 BLAS are the paper's
 * next target, Sec. 6).  T is the lower (uplo 'L') or upper ('U') triangle
 * of the m x m matrix A, with a unit diagonal when diag == 'U' (the
 * diagonal of A is then not read; the other triangle never is); op(T) = T
 * (trans 0) or T^T (trans 1).  B and C are m x n.  All row-major device
 * memory; no workspace.  Both halve the triangle recursively: the
 * off-diagonal blocks are family products (momms_gemm_ex, MOMMS_AUTO) and
 * diagonal blocks of at most 64 rows are solved or multiplied by one
 * substitution kernel (one thread per column of B).
 *   momms_trmm:  C := alpha op(T) B, out of place (C must not overlap A or
 *                B); alpha == 0 writes C = 0 without reading A or B.
 *   momms_trsm:  B := X with op(T) X = alpha B, in place; alpha == 0 sets
 *                B = 0 without reading A.  No singularity check: a zero on a
 *                non-unit diagonal gives infinities or NaNs as IEEE division
 *                does.
 * Errors: -1 uplo, -2 trans, -3 diag, -4 m, -5 n, -7 A, -8 lda (< m),
 * -9 B, -10 ldb (< n), -11 C, -12 ldc (< n); positive HIP errors. */
int momms_trmm(int uplo, int trans, int diag, int64_t m, int64_t n, double alpha, const double *A,
               int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc, momms_stream_t stream);
int momms_trsm(int uplo, int trans, int diag, int64_t m, int64_t n, double alpha, const double *A,
               int64_t lda, double *B, int64_t ldb, momms_stream_t stream);

/* Cholesky factorization A = U^T U (the recursive blocked factorizations
 * the paper names as future work, Sec. 6).  uplo must be 'U': U is written
 * over the upper triangle of the row-major n x n device matrix A (the
 * memory layout of LAPACK's column-major lower factor); the strictly lower
 * triangle is never read or written.  Recursive halving onto momms_trsm and
 * momms_syrk; diagonal blocks of at most 128 rows are factored in registers
 * by one workgroup.  info (device int, may be NULL) is set to 0, or to the 1-based
 * row of the first pivot that is not positive (A not positive definite; the
 * factorization continues with NaNs past it); read it after the stream has
 * drained.  Errors: -1 uplo, -2 n, -3 A, -4 lda (< n); codes of momms_trsm
 * and momms_syrk; positive HIP errors. */
int momms_potrf(int uplo, int64_t n, double *A, int64_t lda, int *info, momms_stream_t stream);

/* ---------------------------------------------------------------------
 * Out-of-core product: host memory as the level below HBM (the paper's
 * out-of-core future work, Sec. 6; the loop levels of Sec. 3.2 with one more
 * level).  C := alpha A B + beta C with A (m x k), B (k x n) and C (m x n)
 * row-major in HOST memory (pinned memory lets the copies overlap the
 * products; pageable memory works, with staged copies).  Resident C at the
 * HBM level: C is processed in mb x nb blocks held in the device workspace
 * while mb x kb panels of A and kb x nb panels of B are copied in; each
 * block product runs `family_member` (MOMMS_AUTO picks per block shape).
 * Host traffic: C 2mn (mn if beta == 0), A mk ceil(n/nb), B kn ceil(m/mb)
 * elements.  Copies go on copy_stream, products on stream, ordered by
 * events (two C buffers and two panel slots); the call returns once all
 * work is enqueued, and C is complete when `stream` has drained.  beta == 0
 * does not read C; alpha == 0 or k == 0 does not read A or B.
 * workspace: device memory, 256-byte aligned, at least
 * momms_ooc_workspace_size(mb, nb, kb) bytes.  Errors: -1 m, -2 n, -3 k,
 * -5 A, -6 lda, -7 B, -8 ldb, -10 C, -11 ldc, -12 mb, -13 nb, -14 kb,
 * -15 family_member, -16 workspace alignment, -17 workspace missing or too
 * small; codes of momms_gemm_ex from a block product; positive HIP errors
 * from the copies. */
size_t momms_ooc_workspace_size(int64_t mb, int64_t nb, int64_t kb);
int momms_gemm_ooc(int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                   int64_t mb, int64_t nb, int64_t kb, int family_member,
                   void *workspace, size_t ws_bytes, momms_stream_t stream, momms_stream_t copy_stream);

/* ---------------------------------------------------------------------
 * Low-bandwidth emulation: the varying-bandwidth experiments of Sec. 5
 * ("Experimental setup"; Goto's algorithm against B3A2C0 and C4A2C0 as the
 * bandwidth to main memory drops).  The paper lowered the memory clock and
 * channel count; here a streaming kernel on its own stream takes HBM bandwidth
 * while a product runs on another stream.
 *
 * momms_lowbw_start enqueues that kernel on `stream`: `workgroups` workgroups
 * of 1024 threads, each holding all of one compute unit's LDS, so no product
 * workgroup shares a compute unit with it (1 <= workgroups <= the number of
 * compute units; multiples of 8 spread it evenly over the XCDs).  mode 0
 * streams `buf` (device memory, 16-byte aligned, at least
 * momms_lowbw_min_bytes(workgroups) bytes, best well above the 256 MiB MALL)
 * with non-temporal 16-byte loads, each wave round after round over its own
 * contiguous share; it never writes `buf`.  mode 1 holds the same compute
 * units asleep and reads nothing (buf may be NULL): the control that leaves
 * the bandwidth and takes the same compute units.  Every workgroup polls
 * *flag (a device 64-bit word, by atomic add: it counts the polls) every 8
 * rounds and leaves its loop when the stop bit (bit 63) is set, when
 * max_seconds (0 < max_seconds <= 60) of wall clock have passed since it
 * started, or after max_rounds rounds (rounded up to a multiple of 8).
 * The call clears *flag on `stream`, waits on the host for that
 * clear and for `stream`'s earlier work, then enqueues the kernel and
 * returns; run the product on another stream, then momms_lowbw_stop.
 * rec (device, momms_lowbw_record_words(workgroups) words) receives, for
 * each wave w, rec[4w] = rounds done (momms_lowbw_round_bytes() bytes each
 * in mode 0), rec[4w+1] = a checksum of what it read, rec[4w+2] and
 * rec[4w+3] = the wall clock (momms_lowbw_clock_hz() ticks per second) when
 * it started and stopped.  Errors: -1 mode, -2 buf (missing or unaligned),
 * -3 bytes too small, -4 workgroups, -5 flag, -6 rec, -7 max_seconds,
 * -8 max_rounds; positive HIP errors. */
size_t momms_lowbw_min_bytes(int workgroups);
size_t momms_lowbw_record_words(int workgroups);
int64_t momms_lowbw_round_bytes(void);
int64_t momms_lowbw_clock_hz(void);
int momms_lowbw_start(int mode, const void *buf, size_t bytes, int workgroups, unsigned long long *flag,
                      unsigned long long *rec, double max_seconds, int64_t max_rounds, momms_stream_t stream);
/* Enqueue on `stream` a one-thread kernel that writes the wall clock to *stamp
 * (device, may be NULL) and then sets the stop bit of *flag by atomic or: the
 * streamer's workgroups see it at their next poll and leave.  Errors: -1
 * flag; positive HIP errors. */
int momms_lowbw_stop(unsigned long long *flag, unsigned long long *stamp, momms_stream_t stream);
/* Enqueue a one-thread kernel that writes the wall clock to *stamp, to mark
 * where a product starts.  Errors: -1 stamp; positive HIP errors. */
int momms_lowbw_stamp(unsigned long long *stamp, momms_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MOMMS_H */

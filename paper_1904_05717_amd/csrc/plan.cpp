// Host-side planner and data-movement model of the MOMMS family on gfx950.
// No HIP calls: everything here runs (and is tested) without a GPU.
//
// Blocksizes are derived from the gfx950 capacities, not from the paper's
// CPU numbers:
//   level 0: a workgroup's register tile of C.  128 x 128 fp64 = 128 KiB held
//            by 4 waves (64 doubles per lane), i.e. sqrt(M0) ~ 128 - the same
//            order as the paper's LDS-class block, because the register file
//            (512 KiB/CU) is larger than the LDS (160 KiB/CU).
//   level 2: LDS.  The resident block is sized by lds_block(): the Sec. 2.4
//            balance between the streamed panel (from the L2) and C (from
//            HBM, read and written), within the Sec. 4.1 capacity, on the
//            MFMA wave grid.  The A-resident kernel streams B through
//            registers, so its block has LDS to itself; two of its
//            workgroups share a CU (one computes while the other refills its
//            block), so each has half: 32 x 288 (72 KiB).  The B-resident
//            kernel keeps two 32-deep A slices beside its block: 160 x 64
//            (80 KiB).
//   level 3: one XCD's 4 MiB L2.  A 512 x 512 resident block (2 MiB) leaves
//            half the L2 for the guest and streamed panels (Sec. 4.1).
//   level 4: the 256 MiB MALL.  A 4096 x 4096 C block (128 MiB) leaves half.
#include <cmath>
#include <cstring>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {

static const char* const kNames[MOMMS_NUM_MEMBERS] = {
    "AUTO", "C0", "C3C0", "B3C0", "A3C0", "A2C0", "B3A2C0", "A3B2C0", "C3A2C0", "C4A2C0"};

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile of the register-resident kernel: 128 x 128 when there are enough
// tiles to give every CU work twice over, else 64 x 64.
static inline int regc_tile(int64_t m, int64_t n) {
    return (cdiv(m, 128) * cdiv(n, 128) >= 2 * kCUs) ? 128 : 64;
}

// Level-2 (LDS) block of the LDS-resident kernels (Sec. 2.4 balance within
// the Sec. 4.1 capacity).  A resident A block of rows x kc, streaming B
// slices (cost beta_stream per element) and updating C (cost beta_c per
// element, covering its read and its write), does 2 rows kc flops per column
// of B for beta_stream kc + beta_c rows of cost; the continuous optimum at a
// capacity of M elements is rows = sqrt(beta_stream / beta_c M), kc =
// sqrt(beta_c / beta_stream M) (momms_balanced_block).  The kernels need rows
// a multiple of row_step (32 per row of 32-row waves: the A-resident kernel
// has one, the B-resident kernel two columns) and kc a multiple of the slice
// depth; the block plus two streamed k-slices of slice x (tile_other + 2)
// must fit lds_doubles with the block's row pitch kc + 1.  tile_other = 0
// means the streamed panel does not pass through LDS at all (the A-resident
// kernel reads its B fragments straight into registers), so the block has
// the whole of it.  The slice depth
// is the kernels' choice (32: enough MFMAs between two barriers), made before
// the block is sized.  Among those blocks the one
// with the most flops per unit cost wins; ties go to the one nearer the
// continuous optimum (in kc / rows), then to fewer rows.  The B-resident
// kernel is the mirror (rows = block columns).
void lds_block(double lds_doubles, int slice, int tile_other, int row_step, double beta_stream, double beta_c,
               int* rows, int* kc) {
    const double stream = tile_other > 0 ? 2.0 * slice * (tile_other + 2) : 0.0;
    const double M = lds_doubles - stream;
    const double ratio_opt = beta_c / beta_stream;   // kc / rows at the optimum
    int best_r = 0, best_k = 0;
    double best_e = -1.0, best_d = 0.0;
    for (int r = row_step; r <= 512; r += row_step) {
        const int kmax = (int)std::floor(M / r) - 1;   // r (kc + 1) <= M
        const int kcand = (kmax / slice) * slice;
        if (kcand < slice) continue;
        const double e = 2.0 * r * kcand / (beta_stream * kcand + beta_c * r);
        const double d = std::fabs(std::log((double)kcand / r / ratio_opt));
        if (e > best_e * (1.0 + 1e-12) || (e > best_e * (1.0 - 1e-12) && d < best_d - 1e-12)) {
            best_e = e;
            best_d = d;
            best_r = r;
            best_k = kcand;
        }
    }
    *rows = best_r;
    *kc = best_k;
}

// gfx950 costs for lds_block: an element of the streamed panel comes from the
// L2 (64 B/clk per CU, 2.4 GHz: 39 TB/s over 256 CUs); an element of C is
// read from and written to HBM (8 TB/s), so it costs 2 x 39 / 8 times more.
constexpr double kLdsDoubles = 160.0 * 1024 / 8;
constexpr double kBetaStream = 1.0, kBetaC = 2.0 * 39.3 / 8.0;

// The LDS-resident kernels are compiled for the solver's answer on gfx950;
// the plan refuses to run if the two ever disagree.
static bool lds_blocks_match() {
    static const bool ok = [] {
        int ra = 0, ka = 0, rb = 0, kb = 0;
        // A block alone in its workgroup's share of LDS; B block beside A
        // slices of kMTb, one workgroup per CU
        int r1 = 0, k1 = 0;
        lds_block(kLdsDoubles / kWGsPerCuA, kKSlds, 0, 32, kBetaStream, kBetaC, &ra, &ka);
        lds_block(kLdsDoubles, kKSlds, 0, 64, kBetaStream, kBetaC, &r1, &k1);   // a CU to itself
        lds_block(kLdsDoubles, kKSlds, kMTb, 64, kBetaStream, kBetaC, &rb, &kb);
        return ra == kMCa && ka == kKCa && r1 == kMCa1 && k1 == kKCa && rb == kNCb && kb == kKC;
    }();
    return ok;
}

// Column tiles per workgroup (the inner loop over the resident block): the
// largest of 4, 2, 1 that still gives 512 workgroups (two rounds on the chip
// of the B-resident kernel, one of the A-resident kernel).
static int tiles_per_wg(int64_t blocks, int64_t tiles_other) {
    for (int j = 4; j > 1; j /= 2)
        if (blocks * cdiv(tiles_other, j) >= 2 * kCUs) return j;
    return 1;
}

int plan_member(int member, int64_t m, int64_t n, int64_t k, momms_plan* p) {
    std::memset(p, 0, sizeof(*p));
    if (!lds_blocks_match()) return -1;
    p->member = member;
    p->ks = 16;
    p->xcd_aware = 0;
    p->group_m = 1;
    p->k_range = k;
    p->launches = 1;
    switch (member) {
        case MOMMS_C0:
        case MOMMS_C3C0:
        case MOMMS_B3C0:
        case MOMMS_A3C0: {
            const int t = regc_tile(m, n);
            p->kernel = 0;
            p->mt = p->nt = t;
            const int64_t tm = cdiv(m, t), tn = cdiv(n, t);
            p->workgroups = tm * tn;
            if (member == MOMMS_C3C0) {
                // Level 3: the workgroups resident on one XCD at a time cover
                // one C block of group_m x (per_xcd / group_m) tiles.  Level
                // 4: one launch covers a C region of as many tiles as the
                // chip holds at once (8 XCD blocks, at most 4 blocks wide),
                // so every launch starts its workgroups together and their k
                // loops stay in step; the host loops over these regions.
                // When the whole problem fits one such region, or k is so
                // short that a launch per region costs more than the
                // lockstep saves, one launch covers everything.
                const int per_xcd = (t >= 128) ? kWGsPerXcd128 : kWGsPerXcd64;
                const int64_t conc = (int64_t)8 * per_xcd;
                p->xcd_aware = 1;
                p->group_m = (int)(tm < 8 ? tm : 8);
                p->mc3 = (int64_t)8 * t;
                p->nc3 = (int64_t)(per_xcd / 8) * t;
                if (tm * tn <= conc || k < 2048) {
                    p->mc4 = tm * t;
                    p->nc4 = tn * t;
                } else {
                    int64_t rn = tn < 4 * (per_xcd / 8) ? tn : 4 * (per_xcd / 8);
                    int64_t rm = conc / rn;
                    if (rm > tm) rm = tm;
                    p->mc4 = rm * t;
                    p->nc4 = rn * t;
                }
                p->launches = cdiv(m, p->mc4) * cdiv(n, p->nc4);
            } else if (member == MOMMS_B3C0 || member == MOMMS_A3C0) {
                p->xcd_aware = 1;
                p->kc3 = 512;
                p->k_range = p->kc3 < k ? p->kc3 : k;
                p->launches = k > 0 ? cdiv(k, p->kc3) : 1;
                p->workgroups *= p->launches;
                // Column-major order (B3): one XCD's run of tiles shares
                // columns, i.e. a B block; row-major (A3): shares an A block.
                p->group_m = (member == MOMMS_B3C0) ? (int)tm : 1;
                if (member == MOMMS_B3C0) { p->nc3 = t; p->mc3 = m; }
                else { p->mc3 = t; p->nc3 = n; }
            }
            break;
        }
        case MOMMS_A2C0: {
            // Goto: n by nc -> k by kc (pack B panel) -> m by 32 (A block
            // in LDS) -> n by 128 across workgroups (the parallel 2nd loop).
            p->kernel = 1;
            p->mt = kMCa;
            p->nt = kNTa;
            p->ks = kKSlds;
            p->kc = kKCa;
            p->nc = kGotoNc;
            p->nj = tiles_per_wg(cdiv(m, p->mt), cdiv(n < p->nc ? n : p->nc, p->nt));
            p->k_range = p->kc < k ? p->kc : k;
            p->pack = 1;
            const int64_t jcs = cdiv(n, p->nc), pcs = k > 0 ? cdiv(k, p->kc) : 1;
            const int64_t ncw = n < p->nc ? n : p->nc;
            p->launches = jcs * pcs * 2;  // pack + compute
            p->workgroups = jcs * pcs * cdiv(m, p->mt) * cdiv(ncw, (int64_t)p->nj * p->nt);
            break;
        }
        case MOMMS_B3A2C0: {
            // n by nc3 -> k by kc3 (B block in one XCD's L2) -> m by 32 (A
            // block in LDS) -> k by kc -> n by 128.  nc3 = nj tiles (at most
            // 512: a 288 x 512 B block is 1.2 MiB of the 4 MiB L2).
            p->kernel = 1;
            p->mt = kMCa;
            p->nt = kNTa;
            p->ks = kKSlds;
            p->kc = kKCa;
            p->kc3 = kKCa;      // one A block per B block: three (864 x 512) would not fit half the L2
            p->nj = tiles_per_wg(cdiv(m, p->mt), cdiv(n, p->nt));
            p->nc3 = (int64_t)p->nj * p->nt;
            p->xcd_aware = 1;
            p->group_m = (int)cdiv(m, p->mt);
            p->k_range = p->kc < k ? p->kc : k;
            p->launches = k > 0 ? cdiv(k, p->kc3) : 1;
            p->workgroups = p->launches * cdiv(m, p->mt) * cdiv(n, p->nc3);
            break;
        }
        case MOMMS_A3B2C0: {
            // m by mc3 -> k by kc3 (A block in one XCD's L2) -> n by 64 (B
            // block in LDS) -> k by kc -> m by 128.  mc3 = mi tiles (at most
            // 512).
            p->kernel = 2;
            p->mt = kMTb;
            p->nt = kNCb;
            p->ks = kKSlds;
            p->kc = kKC;
            p->kc3 = 3 * kKC;   // whole LDS blocks: a ragged last kc would cost a C pass of its own
            p->mi = tiles_per_wg(cdiv(n, p->nt), cdiv(m, p->mt));
            p->mc3 = (int64_t)p->mi * p->mt;
            p->xcd_aware = 1;
            p->group_m = 1;
            p->k_range = p->kc < k ? p->kc : k;
            p->launches = k > 0 ? cdiv(k, p->kc3) : 1;
            p->workgroups = p->launches * cdiv(m, p->mc3) * cdiv(n, p->nt);
            break;
        }
        case MOMMS_C3A2C0: {
            // n, m by a C block per XCD -> k by kc -> m by 64 (A block in
            // LDS) -> n by 128; one launch, every workgroup walks all of k.
            // Sec. 4.1 at level 3: the C block is the tiles one XCD runs at
            // once (32 workgroups, one per CU, so that they stay in step
            // through k: 32 tiles of 64 x 128, 2 MiB, half the L2).  Between two visits of a C tile the XCD also
            // reads one chunk's guests, the A rows (rows x kc) and B columns
            // (kc x cols) of the block, and they must fit the other half.
            // The block's shape (group_m tile rows, swept column by column)
            // minimises rows + cols; kc is then the deepest whole number of
            // slices, up to the LDS block's depth, whose guests fit (8192^2:
            // 8 x 4 tiles = 512 x 512, kc = 256).  When tiles of 64 rows
            // would not give every CU one, the two-per-CU block of 32 rows
            // runs instead: the launch then fits the chip at once, so every
            // workgroup is resident from its start to its end and none can
            // fall behind a round.
            p->kernel = 1;
            const bool fill = cdiv(m, kMCa1) * cdiv(n, kNTa) >= kCUs;
            p->mt = fill ? kMCa1 : kMCa;
            p->nt = kNTa;
            p->ks = kKSlds;
            p->nj = 1;
            p->xcd_aware = 1;
            const int per_xcd = fill ? kWGsPerXcdA1 : 32 * kWGsPerCuA;
            const int64_t tm = cdiv(m, p->mt), tn = cdiv(n, p->nt);
            double best = -1.0;
            for (int g = 1; g <= per_xcd; g *= 2) {
                const int gm = (int)(g < tm ? g : (tm > 0 ? tm : 1));
                const double cols = std::fmin((double)tn, std::ceil((double)per_xcd / gm));
                const double rows = std::fmin((double)tm, std::ceil((double)per_xcd / cols));
                const double edge = rows * p->mt + cols * p->nt;
                if (best < 0.0 || edge < best) {
                    best = edge;
                    p->group_m = gm;
                    p->mc3 = (int64_t)rows * p->mt;
                    p->nc3 = (int64_t)cols * p->nt;
                }
            }
            const int64_t kfit = (int64_t)(0.5 * kL2Bytes / (8.0 * (best > 0.0 ? best : 1.0)));
            p->kc = kfit / kKSlds * kKSlds;
            if (p->kc > kKCa) p->kc = kKCa;
            if (p->kc < kKSlds) p->kc = kKSlds;
            p->k_range = p->kc < k ? p->kc : k;
            p->workgroups = cdiv(m, p->mt) * cdiv(n, p->nt);
            break;
        }
        case MOMMS_C4A2C0: {
            // m, n by a 4096 x 4096 C block (MALL) -> k by kc3 = 4 kc -> k by
            // kc -> m by 32 (A block in LDS) -> n by 128.  One launch walks
            // four chunks: with one, a launch holds two rounds of workgroups
            // and its tail idles the chip; with eight, its A and B panels (72
            // MiB each) and the 128 MiB C block would overflow the 256 MiB
            // MALL (four: 36 MiB each).  Each chunk moves the same data.
            p->kernel = 1;
            p->mt = kMCa;
            p->nt = kNTa;
            p->ks = kKSlds;
            p->kc = kKCa;
            p->kc3 = 4 * kKCa;
            p->mc4 = p->nc4 = 4096;
            p->nj = tiles_per_wg(cdiv(m < p->mc4 ? m : p->mc4, p->mt), cdiv(n < p->nc4 ? n : p->nc4, p->nt));
            p->k_range = p->kc < k ? p->kc : k;
            const int64_t blocks = cdiv(m, p->mc4) * cdiv(n, p->nc4);
            const int64_t pcs = k > 0 ? cdiv(k, p->kc3) : 1;
            p->launches = blocks * pcs;
            const int64_t mw = m < p->mc4 ? m : p->mc4, nw = n < p->nc4 ? n : p->nc4;
            p->workgroups = p->launches * cdiv(mw, p->mt) * cdiv(nw, (int64_t)p->nj * p->nt);
            break;
        }
        default:
            return -1;
    }
    return 0;
}

size_t workspace_bytes(int member, int64_t m, int64_t n, int64_t k) {
    (void)m;
    (void)k;
    if (member != MOMMS_A2C0) return 0;
    const int64_t nc = n < kGotoNc ? n : kGotoNc;
    return (size_t)(kKCa * cdiv(nc, kNTa) * kNTa) * sizeof(double);
}

// Measured table: shape buckets (rounded log2 of m, n, k) whose best member
// was measured on the device by the tuning sweep; consulted before the
// analytic prior.
struct TunedEntry {
    int lm, ln, lk, member;
};
static TunedEntry g_tuned[64];
static int g_ntuned = 0;

static int log2_bucket(int64_t x) {
    if (x <= 1) return 0;
    return (int)std::lround(std::log2((double)x));
}

int set_tuned(int count, const int* lm, const int* ln, const int* lk, const int* member) {
    if (count < 0 || count > 64) return -1;
    for (int i = 0; i < count; ++i)
        if (member[i] < 1 || member[i] >= MOMMS_NUM_MEMBERS) return -5;
    for (int i = 0; i < count; ++i) g_tuned[i] = TunedEntry{lm[i], ln[i], lk[i], member[i]};
    g_ntuned = count;
    return 0;
}

int select_member(int64_t m, int64_t n, int64_t k) {
    const int bm = log2_bucket(m), bn = log2_bucket(n), bk = log2_bucket(k);
    for (int i = 0; i < g_ntuned; ++i)
        if (g_tuned[i].lm == bm && g_tuned[i].ln == bn && g_tuned[i].lk == bk) return g_tuned[i].member;
    return select_member_prior(m, n, k);
}

int select_member_prior(int64_t m, int64_t n, int64_t k) {
    // Analytic prior (Sec. 2.3: resident C needs k large, resident B needs m
    // large, resident A needs n large), then fewest model bytes, then lowest
    // id.  Only members that keep C in registers over all of k are
    // candidates: on gfx950 they dominate the LDS-resident members for every
    // shape the model was evaluated on (C traffic 2mn instead of
    // 2mn * ceil(k/128)).
    int best = MOMMS_C3C0;
    double best_bytes = -1.0;
    const int cand[] = {MOMMS_C3C0, MOMMS_C0, MOMMS_B3C0, MOMMS_A3C0};
    for (int c : cand) {
        momms_bytes b;
        if (model_bytes(c, m, n, k, 1.0, 0, &b) != 0) continue;
        const double tot = b.l2_read + b.l2_write;
        if (best_bytes < 0 || tot < best_bytes * (1.0 - 1e-9)) {
            best = c;
            best_bytes = tot;
        }
    }
    return best;
}

const char* member_name(int member) {
    if (member < 0 || member >= MOMMS_NUM_MEMBERS) return nullptr;
    return kNames[member];
}

int member_id(const char* name) {
    if (!name) return -1;
    for (int i = 0; i < MOMMS_NUM_MEMBERS; ++i)
        if (std::strcmp(name, kNames[i]) == 0) return i;
    return -1;
}

}  // namespace momms

// ---------------------------------------------------------------------------
// C ABI: host-only introspection.
extern "C" {

int momms_num_members(void) { return MOMMS_NUM_MEMBERS; }

const char* momms_member_name(int member) { return momms::member_name(member); }

int momms_member_id(const char* name) { return momms::member_id(name); }

int momms_select_member(int64_t m, int64_t n, int64_t k) {
    if (m < 0 || n < 0 || k < 0) return -1;
    return momms::select_member(m, n, k);
}

int momms_member_plan(int member, int64_t m, int64_t n, int64_t k, momms_plan* out) {
    if (member < 0 || member >= MOMMS_NUM_MEMBERS) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (k < 0) return -4;
    if (!out) return -5;
    if (member == MOMMS_AUTO) member = momms::select_member(m, n, k);
    return momms::plan_member(member, m, n, k, out) == 0 ? 0 : MOMMS_ERR_INTERNAL;
}


int momms_set_member_table(int count, const int* log2_m, const int* log2_n, const int* log2_k, const int* member) {
    if (count < 0 || count > 64) return -1;
    if (count > 0 && !log2_m) return -2;
    if (count > 0 && !log2_n) return -3;
    if (count > 0 && !log2_k) return -4;
    if (count > 0 && !member) return -5;
    return momms::set_tuned(count, log2_m, log2_n, log2_k, member);
}

int momms_select_member_prior(int64_t m, int64_t n, int64_t k) {
    if (m < 0 || n < 0 || k < 0) return -1;
    return momms::select_member_prior(m, n, k);
}

size_t momms_workspace_size(int64_t m, int64_t n, int64_t k, int member) {
    if (m < 0 || n < 0 || k < 0 || member < 0 || member >= MOMMS_NUM_MEMBERS) return 0;
    if (member == MOMMS_AUTO) member = momms::select_member(m, n, k);
    return momms::workspace_bytes(member, m, n, k);
}


int momms_lds_block(double lds_bytes, int slice, int tile_other, int row_step, double beta_stream, double beta_c,
                    int* rows, int* kc) {
    if (!(lds_bytes > 0) || !std::isfinite(lds_bytes)) return -1;
    if (slice < 1) return -2;
    if (tile_other < 0) return -3;
    if (row_step < 16 || row_step % 16 != 0) return -4;
    if (!(beta_stream > 0) || !std::isfinite(beta_stream)) return -5;
    if (!(beta_c > 0) || !std::isfinite(beta_c)) return -6;
    if (!rows) return -7;
    if (!kc) return -8;
    momms::lds_block(lds_bytes / 8.0, slice, tile_other, row_step, beta_stream, beta_c, rows, kc);
    return 0;
}

int momms_balanced_block(double M, double beta_b, double beta_c, double* mc, double* kc) {
    if (!(M > 0)) return -1;
    if (!(beta_b > 0)) return -2;
    if (!(beta_c > 0)) return -3;
    if (!mc) return -4;
    if (!kc) return -5;
    // Resident A with streamed B (cost beta_b per element) and C (beta_c):
    // flops per unit cost 2 mc / beta_b + 2 kc / beta_c is largest, with
    // mc kc = M, at mc = sqrt(beta_b / beta_c * M), kc = sqrt(beta_c / beta_b * M)
    // (Sec. 2.4).
    *mc = std::sqrt(beta_b / beta_c * M);
    *kc = std::sqrt(beta_c / beta_b * M);
    return 0;
}

const char* momms_status_string(int status) {
    if (status == 0) return "success";
    if (status < 0) return "invalid argument (-status is its 1-based position)";
    switch (status) {
        case MOMMS_ERR_INFEASIBLE: return "problem too large for the tile grid";
        case MOMMS_ERR_NO_DEVICE: return "no usable gfx950 device";
        case MOMMS_ERR_INTERNAL: return "internal error";
        case MOMMS_ERR_SCRATCH: return "the member needs more scratch than the static array holds";
        default: return "HIP runtime error (status is the hipError_t value)";
    }
}

}  // extern "C"

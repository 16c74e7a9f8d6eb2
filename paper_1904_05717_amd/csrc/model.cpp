// Data-movement model of the MOMMS family on gfx950 (host only, no HIP
// calls): the element transfers of the Sec. 2.2 resident algorithms, made
// exact with the ceilings the paper keeps at the margins, applied to each
// member's planned loop nest with the Sec. 4.1-4.2 level interactions.  Kept
// apart from the planner: the plans decide what the kernels move, this file
// only predicts it.
#include <cmath>
#include <cstring>

#include "../../include/momms.h"
#include "plan_internal.h"

namespace momms {

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Element transfers of the resident algorithms of Sec. 2.2 between a slow
// and a fast memory, with the ceilings kept at the margins:
//   Resident C (b1 x b2 = mc x nc): A read ceil(n/nc) times, B ceil(m/mc)
//     times, C read and written once.
//   Resident A (b1 x b2 = mc x kc): A read once, B ceil(m/mc) times, C read
//     and written once per kc block of k.
//   Resident B (b1 x b2 = kc x nc): B read once, A ceil(n/nc) times, C read
//     and written once per kc block of k.
// With beta == 0 the first read of each C entry is skipped.  counts = {A
// reads, B reads, C reads, C writes} in elements.
void resident_counts(int resident, int64_t m, int64_t n, int64_t k, int64_t b1, int64_t b2, double beta,
                     double* counts) {
    const double M = (double)m, N = (double)n, K = (double)k;
    double a, b, passes;
    if (resident == 'C') {
        a = M * K * (double)cdiv(n, b2);
        b = K * N * (double)cdiv(m, b1);
        passes = 1.0;
    } else if (resident == 'A') {
        a = M * K;
        b = K * N * (double)cdiv(m, b1);
        passes = k > 0 ? (double)cdiv(k, b2) : 1.0;
    } else {
        a = M * K * (double)cdiv(n, b2);
        b = K * N;
        passes = k > 0 ? (double)cdiv(k, b1) : 1.0;
    }
    counts[0] = a;
    counts[1] = b;
    counts[2] = M * N * (passes - 1.0 + (beta != 0.0 ? 1.0 : 0.0));
    counts[3] = M * N * passes;
}

// ---------------------------------------------------------------------------
// Data-movement model.  Element counts of Sec. 2.2 with the ceilings the
// paper keeps at the margins, applied to the loop nest of each member:
//   an operand block that is resident at a level is read once per pass of the
//   loop that makes it resident; a streamed operand is read once per
//   iteration of the loops around it that do not index it; C is read and
//   written once per pass over its k range (read skipped when beta == 0 on
//   the first pass).
// "L2" figures count what crosses the boundary between the per-XCD L2s and
// the fabric, under ideal residency (Sec. 4.1: the block plus its guest
// panel fit).  For the L2 level the unit that shares a block is "the
// workgroups resident on one XCD at a time" (kWGsPerXcd of them).
// n-granules of width g over n split into panels of width w (the last panel
// may be narrower): sum over the panels of ceil(panel / g).
static int64_t granules(int64_t n, int64_t w, int64_t g) {
    const int64_t full = n / w, rest = n - full * w;
    return full * cdiv(w, g) + (rest > 0 ? cdiv(rest, g) : 0);
}

// Sec. 4.1 at level 3: a block of rows x cols doubles stays in one XCD's
// 4 MiB L2 next to what streams through it when it takes at most half.
static bool fits_l2(int64_t rows, int64_t cols) {
    return 8.0 * (double)rows * (double)cols <= 0.5 * 4.0 * 1024 * 1024;
}

static double c_traffic(int64_t m, int64_t n, int64_t k, int64_t k_range, double beta, double* rd, double* wr) {
    const double passes = (k > 0 && k_range > 0) ? (double)cdiv(k, k_range) : 1.0;
    const double mn = (double)m * (double)n;
    *rd = mn * (passes - 1.0 + (beta != 0.0 ? 1.0 : 0.0));
    *wr = mn * passes;
    return *rd + *wr;
}

int model_bytes(int member, int64_t m, int64_t n, int64_t k, double beta, int packed, momms_bytes* o) {
    momms_plan p;
    if (plan_member(member, m, n, k, &p) != 0) return -1;
    std::memset(o, 0, sizeof(*o));
    const double M = (double)m, N = (double)n, K = (double)k;
    o->flops = 2.0 * M * N * K;
    o->compulsory = 8.0 * (M * K + K * N + M * N + (beta != 0.0 ? M * N : 0.0));
    double a = 0, b = 0, cr = 0, cw = 0;
    c_traffic(m, n, k, p.k_range, beta, &cr, &cw);
    const double t = (double)p.mt;
    const double tm = (double)cdiv(m, p.mt), tn = (double)cdiv(n, p.nt);
    const int per_xcd = (p.mt >= 128) ? kWGsPerXcd128 : kWGsPerXcd64;
    switch (member) {
        case MOMMS_C0: {
            // Plain order: XCD x holds tiles x, x+8, ...; the tiles one XCD
            // runs together span rows R = ceil(per_xcd*8 / tn) of the tile
            // grid and columns C = min(tn, per_xcd*8) / 8 (every 8th).
            const double run = (double)per_xcd * kXcdsH;  // consecutive tiles in flight chip-wide
            const double rows = std::ceil(run / tn) < tm ? std::ceil(run / tn) : tm;
            const double cols = std::ceil((tn < run ? tn : run) / kXcdsH);
            const double tiles_per_round = (double)per_xcd;
            const double rounds = (tm * tn) / (tiles_per_round * kXcdsH);
            // per XCD round: `rows` A panels and `cols` B panels of depth k
            a = rounds * kXcdsH * rows * t * K;
            b = rounds * kXcdsH * cols * t * K;
            if (a > M * K * tn) a = M * K * tn;
            if (b > K * N * tm) b = K * N * tm;
            break;
        }
        case MOMMS_C3C0: {
            // Each launch covers one level-4 region; inside it every XCD
            // holds one level-3 C block (mc3 x nc3) whose workgroups read
            // each A row panel and B column panel of the block once.
            // Summed over blocks: A is read once per block column, B once
            // per block row (ceilings at the margins).
            a = M * K * (double)cdiv(n, p.nc3);
            b = K * N * (double)cdiv(m, p.mc3);
            break;
        }
        case MOMMS_B3C0: {
            // Per kc3 pass, XCD runs walk down tile columns: a B block
            // (kc3 x t) is read once per column; A panels once per tile,
            // unless the pass's whole A panel (m x kc3) fits an XCD's L2
            // (Sec. 4.1), which then reads it once.
            a = fits_l2(m, p.kc3) ? M * K * std::fmin(tn, kXcdsH) : M * K * tn;
            b = K * N;
            break;
        }
        case MOMMS_A3C0: {
            a = M * K;
            b = fits_l2(p.kc3, n) ? K * N * std::fmin(tm, kXcdsH) : K * N * tm;
            break;
        }
        case MOMMS_A2C0: {
            // A block (128 x kc) read once per (jc, pc, ic); B panel once per
            // (jc, pc) per workgroup row group... B slices stream from L2 for
            // every m-block: kn * ceil(m/128) at the LDS boundary, but the
            // panel (kc x nc, <= 4 MiB) is the guest that the skipped L3 may
            // keep: count it once per (jc, pc) from the fabric.
            // A is read once per n-granule of nj tiles, panel by panel (the
            // last n_c panel may be narrower)
            a = M * K * (double)granules(n, p.nc, (int64_t)p.nj * p.nt);
            b = K * N;
            break;
        }
        case MOMMS_B3A2C0: {
            // B block kc3 x nc3 resident in L2: B read once.  A block read
            // once per (jc3, pc3) per m-block (once per XCD when the pass's
            // A panel m x kc3 fits its L2).
            const double jc3 = (double)cdiv(n, p.nc3);
            a = fits_l2(m, p.kc3) ? M * K * std::fmin(jc3, kXcdsH) : M * K * jc3;
            b = K * N;
            break;
        }
        case MOMMS_A3B2C0: {
            const double ic3 = (double)cdiv(m, p.mc3);
            a = M * K;
            b = fits_l2(p.kc3, n) ? K * N * std::fmin(ic3, kXcdsH) : K * N * ic3;
            break;
        }
        case MOMMS_C3A2C0: {
            // One XCD round is 32 workgroups (one per CU; 64 for the
            // two-per-CU block of small problems) in the grouped order
            // (group_m tile rows swept column by column): a C block of cols =
            // min(tn, per_xcd / group_m) tile columns and per_xcd / cols tile
            // rows, which is
            // Resident C for A and B.  Its lines stay in the L2 for reads (C
            // read once), but the L2 writes the updated lines back after
            // every kc pass (measured: the write traffic is C once per pass),
            // so C is written once per pass.
            const double per_xcd = p.mt == kMCa1 ? kWGsPerXcdA1 : 32.0 * kWGsPerCuA;
            const double cols = std::fmin(tn, std::ceil(per_xcd / (double)p.group_m));
            const double rows = std::fmin(tm, std::ceil(per_xcd / cols));
            double cnt[4];
            resident_counts('C', m, n, k, (int64_t)rows * p.mt, (int64_t)cols * p.nt, beta, cnt);
            a = cnt[0];
            b = cnt[1];
            double cr1 = 0, cw1 = 0;
            c_traffic(m, n, k, k, beta, &cr1, &cw1);
            cr = cr1;
            break;
        }
        case MOMMS_C4A2C0: {
            const double bm = (double)cdiv(m, p.mc4);
            a = M * K * (double)granules(n, p.nc4, (int64_t)p.nj * p.nt);
            b = K * N * bm;
            break;
        }
        default:
            return -1;
    }
    o->a_reads = 8.0 * a;
    o->b_reads = 8.0 * b;
    o->c_reads = 8.0 * cr;
    o->c_writes = 8.0 * cw;
    o->l2_read = o->a_reads + o->b_reads + o->c_reads;
    o->l2_write = o->c_writes;
    // Level-4 (MALL, 256 MiB) model: operands that fit the MALL together are
    // read from HBM once; C updates of k-split members hit the MALL when the
    // C region one pass touches fits (C4 block), else go to HBM.
    const double mall = 256.0 * 1024 * 1024;
    const double total_in = 8.0 * (M * K + K * N);
    const double cbytes = 8.0 * M * N;
    if (total_in + cbytes <= mall * 0.75) {
        o->hbm_read = total_in + (beta != 0.0 ? cbytes : 0.0);
        o->hbm_write = cbytes;
    } else {
        o->hbm_read = o->a_reads + o->b_reads;
        if (member == MOMMS_C4A2C0 || member == MOMMS_C3A2C0 || p.k_range >= k) {
            o->hbm_read += (beta != 0.0 ? cbytes : 0.0);
            o->hbm_write = cbytes;
        } else {
            o->hbm_read += o->c_reads;
            o->hbm_write = o->c_writes;
        }
        if (o->hbm_read < total_in) o->hbm_read = total_in;
    }
    // LDS fills: every streamed or resident element copied global -> LDS.
    if (p.kernel == 0) {
        o->lds_fill = 8.0 * (M * K * tn + K * N * tm);
    } else if (p.kernel == 1) {
        o->lds_fill = 8.0 * (M * K * (double)cdiv(n, (int64_t)p.nj * p.nt) + K * N * tm);
    } else {
        o->lds_fill = 8.0 * (M * K * tn + K * N * (double)cdiv(m, (int64_t)p.mi * p.mt));
    }
    if (packed && p.pack) {
        // the packed panel is read once from B and written once (padded)
        const double jcs = (double)cdiv(n, p.nc), pcs = (double)cdiv(k, p.kc);
        const double ncp = (double)(cdiv(p.nc < n ? p.nc : n, 128) * 128);
        o->pack = 8.0 * (K * N + jcs * pcs * (double)p.kc * ncp);
    }
    return 0;
}

}  // namespace momms

extern "C" {

int momms_model_bytes(int member, int64_t m, int64_t n, int64_t k, double beta, int packed, momms_bytes* out) {
    if (member < 0 || member >= MOMMS_NUM_MEMBERS) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (k < 0) return -4;
    if (!std::isfinite(beta)) return -5;
    if (!out) return -7;
    if (member == MOMMS_AUTO) member = momms::select_member(m, n, k);
    return momms::model_bytes(member, m, n, k, beta, packed, out) == 0 ? 0 : MOMMS_ERR_INTERNAL;
}

int momms_model_resident(int resident, int64_t m, int64_t n, int64_t k, int64_t b1, int64_t b2, double beta,
                         double* counts) {
    if (resident != 'A' && resident != 'B' && resident != 'C') return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (k < 0) return -4;
    if (b1 < 1) return -5;
    if (b2 < 1) return -6;
    if (!counts) return -8;
    momms::resident_counts(resident, m, n, k, b1, b2, beta, counts);
    return 0;
}

}  // extern "C"

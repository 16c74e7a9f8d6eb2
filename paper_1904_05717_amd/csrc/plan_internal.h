// Internal planner interface shared by plan.cpp and the launch code.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/momms.h"

namespace momms {

constexpr int kCUs = 256;              // MI355X: 8 XCDs x 32 CUs
constexpr double kXcdsH = 8.0;         // XCD count as a double for the model
// LDS-resident blocks (level 2): A block kMCa x kKCa for the A-resident
// kernel, B block kKC x kNCb for the B-resident kernel; the C tiles they
// update are kMCa x kNTa and kMTb x kNCb.  lds_block() derives these from the
// Sec. 2.4 balance and the Sec. 4.1 capacity: the A-resident kernel streams
// its B slices through registers, so its block has the LDS to itself, shared
// by the kWGsPerCuA workgroups a CU runs at once (while one refills its
// block at a chunk start the other computes); the B-resident kernel keeps
// two A slices beside its block, one workgroup per CU.  C3A2C0 runs the
// A-resident kernel with a CU to itself (block kMCa1 x kKCa): its C block is
// the tiles an XCD runs at once, which stay in the L2 only while those
// workgroups move through k together, and two workgroups on one CU drift
// apart (the older one's instructions issue first).  On problems too small
// to give every CU a 64-row tile it runs the two-per-CU block, and the whole
// launch is resident at once.
constexpr int kKSlds = 32;             // k depth of a streamed slice of the LDS-resident kernels
constexpr int64_t kKCa = 288;          // k depth of the A-resident block
constexpr int64_t kKC = 160;           // k depth of the B-resident block
constexpr int kMCa = 32, kNTa = 128;   // A-resident kernel: block rows, C tile columns
constexpr int kWGsPerCuA = 2;          // A-resident kernel: workgroups per CU
constexpr int kMCa1 = 64;              // its block rows with one workgroup per CU (C3A2C0)
constexpr int kMTb = 128, kNCb = 64;   // B-resident kernel: C tile rows, block columns
constexpr int64_t kGotoNc = 1024;      // Goto's n_c: its packed k_c x n_c panel is 2.25 MiB, about half an XCD's L2
constexpr int kWGsPerXcd128 = 64;      // 128x128 register tile: 2 workgroups per CU
constexpr int kWGsPerXcd64 = 128;      // 64x64 register tile: 4 workgroups per CU (LDS-bound)
constexpr int kWGsPerXcdA1 = 32;      // C3A2C0 with a CU each: workgroups one XCD runs at once
constexpr double kL2Bytes = 4.0 * 1024 * 1024;   // one XCD's L2

// A chunk depth the A-resident kernel can run: a whole number of streamed
// slices within the depth its LDS block is laid out for.
inline bool a2_chunk_ok(int64_t kc) { return kc >= kKSlds && kc <= kKCa && kc % kKSlds == 0; }

int plan_member(int member, int64_t m, int64_t n, int64_t k, momms_plan* p);
void lds_block(double lds_doubles, int slice, int tile_other, int row_step, double beta_stream, double beta_c,
               int* rows, int* kc);
size_t workspace_bytes(int member, int64_t m, int64_t n, int64_t k);
int model_bytes(int member, int64_t m, int64_t n, int64_t k, double beta, int packed, momms_bytes* o);
int select_member(int64_t m, int64_t n, int64_t k);
int select_member_prior(int64_t m, int64_t n, int64_t k);
int set_tuned(int count, const int* lm, const int* ln, const int* lk, const int* member);
void resident_counts(int resident, int64_t m, int64_t n, int64_t k, int64_t b1, int64_t b2, double beta,
                     double* counts);
const char* member_name(int member);
int member_id(const char* name);

}  // namespace momms

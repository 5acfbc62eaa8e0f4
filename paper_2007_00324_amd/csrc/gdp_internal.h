// gdp_internal.h -- shared declarations of the gfx950 refinement library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gdp2d.h"
#include "gdp_exact.h"

namespace gdp {

// Host-side mesh (canonical CDT output of Line 1).
struct HostMesh {
  int32_t nV = 0, nT = 0, nS = 0;
  std::vector<double> xy;      // 2V
  std::vector<int32_t> tv;     // 3T
  std::vector<int32_t> tn;     // 3T
  std::vector<int32_t> ts;     // 3T
  std::vector<int32_t> sv;     // 2S
  std::vector<int32_t> sparent;
};

int host_cdt_build(int32_t nv, const double *xy, int32_t ns, const int32_t *seg, HostMesh &out,
                   std::string &err);

// The same CDT built by kernels (gdp_cdt_dev.hip).  d_xy holds the nv input
// points and room for three more; the canonical triangles go to otv / otn /
// ots in the device mesh layout below.
struct DevCdtStats {
  int32_t dt_rounds = 0, seg_rounds = 0;
};
// Radix sort of (64-bit key, int) pairs on the stream (gdp_cdt_dev.hip); the
// sorted pairs end in (k1, v1); hist: 256 * ceil(n / kSortPairsTile) ints.
constexpr int kSortPairsTile = 2048;
hipError_t sort_pairs_u64(hipStream_t stream, uint64_t *k0, int *v0, uint64_t *k1, int *v1, int n, int *hist);
// A reusable workspace for repeated builds (a long-lived caller such as the
// server's Line-1 thread): device scratch that grows to the largest build
// seen, and one pinned counter block.  Without one, a build allocates and
// frees its own.
struct DevCdtWork {
  void *mem = nullptr;
  size_t bytes = 0;
  void *hctr = nullptr;
};
void dev_cdt_work_free(DevCdtWork &ws);
int dev_cdt_build(hipStream_t stream, int32_t nv, double2 *d_xy, int32_t ns, const int2 *d_seg, int4 *otv,
                  int4 *otn, int4 *ots, int32_t cap_out, int32_t *n_tri, DevCdtStats *stats, std::string &err,
                  DevCdtWork *ws = nullptr);

// ---- device mesh --------------------------------------------------------------
// Triangle t: tv[t] = (v0, v1, v2, subsegment-edge mask), tn[t] = (n0, n1, n2, 0),
// ts[t] = (s0, s1, s2, 0); edge i = (v_i, v_{i+1 mod 3}).
struct DevMesh {
  int32_t capV = 0, capT = 0, capS = 0;
  int32_t nV = 0, nT = 0, nS = 0, n_input_v = 0, n_input_s = 0, rounds = 0;
  double2 *vxy = nullptr;
  int32_t *vkind = nullptr;
  int4 *tv = nullptr, *tn = nullptr, *ts = nullptr;
  int2 *sv = nullptr;
  int32_t *spar = nullptr;
  int32_t *spend = nullptr;
};

// Device counters of one round.  Atomics on one 128-byte line are serialised
// by the memory side (about 12 ns each on MI355X), so the two append counters
// of the collection sit on different lines and the statistics are summed in
// striped lines (StatLine) folded in at the end of the round.
struct DevCounters {
  // line 0
  int32_t ncc;        // circumcenter candidates (bad triangles kept)
  int32_t pool_used;  // cavity pool entries allocated
  int32_t fan_used;   // fan records allocated
  int32_t n_enc;      // subsegments flagged by the scan (pending or encroached apex)
  int32_t nbig;       // cavities routed to the cooperative path
  int32_t err;        // error bits (kErr*)
  int32_t nwin_mid, nwin_cc, fresh_total;
  int32_t n_blocked, n_coincident, n_enc_reject, n_unsplittable, n_fan_invalid;
  int32_t n_lost_mark, n_dep_drop;
  int32_t n_kept_mid, n_kept_cc;
  int32_t cav_max;
  int32_t n_mid_cand;  // midpoint candidates that reached the cavity step
  int64_t cav_tri_total;
  int32_t dbg_set;     // first failing insertion record: set flag
  int32_t dbg[6];      // class, element, cavity size, expected fan size, found fan size, round-local index
  int32_t n_f1_drop, n_f2_drop;
  int32_t nwin;        // winners of the round
  // line 1
  int32_t nmk;          // midpoint candidates (flagged subsegments)
  int32_t nwin1;        // nwin + 1 (scan length)
  int32_t abort;        // the round was abandoned before any mesh write (capacity)
  int32_t nmk0;         // midpoint candidates after the collection (R4/R5 add more)
  int32_t fan_total;    // total of the fresh-count scan (fbase[nwin] is what is used)
  int32_t nhuge;        // cavities continued in device memory (beyond the LDS list)
  int64_t cav_len[2];   // per-thread cavities [midpoints, circumcenters]: triangles grown
  int64_t cav_bnd[2];   // ... and their boundary edges
  int64_t n_in_tests;   // incircle evaluations of cavity growth and the dependency test
  int64_t n_or_tests;   // orient2d evaluations of the walk and the fan check
  int64_t n_exact[4];   // exact-stage evaluations (ExactStage: orient, dot, incircle B, incircle C)
  // winners of the round (what a sequential insertion of the same points touches)
  int64_t win_cav;      // sum of cavity sizes |C|
  int64_t win_bnd;      // sum of boundary (fan) edges b
  int64_t win_steps;    // walk steps of the circumcenter winners
  int64_t win_cc_cav;   // |C| and b of the circumcenter winners alone
  int64_t win_cc_bnd;
  int64_t n_marks[2];   // priority marks placed (atomicMax): midpoint, circumcenter cavities
  // Flip-Flop rounds (Section 4.3, Line 8)
  int64_t ff_points;    // points of S added
  int64_t ff_iters;     // CDTs examined for redundant points
  int64_t ff_flips;     // 2-2 flips
  int64_t ff_passes;    // flip passes
  int64_t ff_removals;  // redundant points taken out
  int64_t ff_rm_passes; // removal passes
};
static_assert(sizeof(DevCounters) % 8 == 0, "DevCounters is copied as 32-bit words");
static_assert(offsetof(DevCounters, nmk) == 128, "the midpoint append counter starts the second line");

// Statistics of a round, summed per wave into one of kStatStripes lines (the
// wave's global index picks the line) and folded into DevCounters at the end
// of the round, which also clears the lines.
// The exact predicates count their slow-path evaluations into words
// kTally0.. of the same lines (gdp_exact.h).
enum StatField {
  kStCavTri, kStCavLen0, kStCavLen1, kStCavBnd0, kStCavBnd1, kStEncReject, kStFanInvalid, kStUnsplittable,
  kStMidCand, kStLostMark, kStDepDrop, kStBlocked, kStCoincident, kStCavMax, kStInTests, kStOrTests,
  kStExact0, kStExact3 = kStExact0 + 3,
  kStWinCav, kStWinBnd, kStWinSteps, kStWinCcCav, kStWinCcBnd, kStMarks0, kStMarks1, kStFields
};
struct StatLine {
  uint64_t v[32];
};
constexpr int kStatStripes = 64;
static_assert(kStFields <= 32 && sizeof(StatLine) == 256, "one stat line: two cache lines");
static_assert(kStExact0 == kTally0 && kTallyStride == 32 && kTallyStripes == kStatStripes,
              "the exact predicates' counters live in the stat lines");

// Mesh counts and round control in device memory, so that several rounds
// can be queued without the host looking at any count in between.
struct DevState {
  int32_t nV, nT, nS;    // live counts (advanced at the end of every completed round)
  int32_t wT, wS;        // bitmap words covering nT / nS (nT / 32 + 1)
  int32_t rounds;        // rounds completed on the mesh
  int32_t serial;        // slot stamp of the running round
  int32_t prev_ncc, prev_nmk, prev_fan;  // list lengths of the last completed round
  int32_t halt;          // kHalt*: nonzero makes every later round kernel return at once
  int32_t nhist;         // rounds recorded in the history since the host last read it
  int32_t done_blocks;   // arrival counter of k_finish's workgroups
  int32_t full;          // the next round collects over the whole mesh (single-workgroup engine)
  int32_t pad[2];
};

constexpr int kHaltDone = 1;   // nothing left to refine
constexpr int kHaltCap = 2;    // round cap reached with work left
constexpr int kHaltAbort = 3;  // a buffer was short: the round wrote nothing and must run again
constexpr int kHaltError = 4;  // walk / input / cavity error (bits in the round counters)
constexpr int kHaltStall = 5;  // candidates but no winner

constexpr int kErrWalk = 1;
constexpr int kErrCavity = 2;
constexpr int kErrPool = 4;
constexpr int kErrHuge = 16;  // a cavity outgrew the LDS list in a round run without the device-memory path
constexpr int kErrInput = 8;

// Candidate state bits.
constexpr int kStFound = 1;     // located (circumcenters) / has seeds (midpoints)
constexpr int kStAlive = 2;     // cavity grown and valid
constexpr int kStW0 = 4;        // holds every mark of its cavity
constexpr int kStWin = 8;       // survives the dependency test
constexpr int kStBig = 16;      // cavity goes to the cooperative path
constexpr int kStDone = 32;     // cavity step finished (alive or dropped)
constexpr int kStHuge = 128;    // cavity continues in device memory (beyond the LDS list)

struct CandSet {
  int32_t *elem;     // triangle slot (circumcenters) or subsegment id (midpoints)
  uint64_t *key;
  double2 *p;
  int32_t *loc;      // located triangle (circumcenters)
  int32_t *state;
  int32_t *off;      // cavity pool offset
  int32_t *len;      // cavity size
};

}  // namespace gdp

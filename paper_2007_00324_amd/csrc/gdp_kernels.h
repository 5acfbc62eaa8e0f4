// gdp_kernels.h -- kernel interface of one refinement round.
#pragma once

#include "gdp_ff_core.h"
#include "gdp_internal.h"

namespace gdp {

constexpr int kStSkip = 64;  // left out by the candidate cap this round

struct FanRec {
  int32_t slot, u, v, o, jn, ts;
};

// Device pointers of the per-round workspace (passed by value to kernels).
struct Work {
  DevState *st;        // counts and round control
  DevCounters *cnt;    // counters of the running round
  DevCounters *hist;   // [hist_cap] counters of completed rounds, read by the host
  int32_t hist_cap;
  uint64_t *mark;      // [capT] max key of the cavities containing the slot
  int32_t *sadj;       // [2*capS] t*4+edge of the triangle on each side (-1 none)
  uint32_t *mflag;     // [capS] subsegment flagged as a midpoint candidate
  CandSet cc, mid;
  uint32_t *w0_t, *w0_s, *win_t, *win_s;  // element bitmaps
  int32_t *rank_t, *rank_s;               // exclusive prefix of bitmap popcounts (per tile)
  int32_t *tiles_t, *tiles_s, *tiles_f;   // tile prefixes of the three scans
  int32_t *win_ref;    // [nwin] winner -> (class bit 31 set for midpoints) | candidate
  int32_t *fbase;      // [nwin+1] exclusive prefix of fresh-slot counts
  int32_t *fcount;     // [nwin] fresh slots per winner (1 or 2)
  int32_t *fan_off;    // [nwin]
  int32_t win_cap;     // length of win_ref / fbase / fcount / fan_off
  int32_t *repl;       // [4*capT] new slot that replaces (old slot, edge)
  int32_t *pool;
  int32_t pool_cap;
  FanRec *fan;
  int32_t fan_cap;
  int32_t *big;
  int32_t big_cap;
  int32_t *hvis;       // [hcap] visited flags of the device-memory cavity path (zero between uses)
  int32_t *hlist;      // [hcap] its cavity list (from the bottom) and rejected slots (from the top)
  int32_t hcap;        // >= capT
  int32_t huge_ok;     // 1: cavities beyond the LDS list continue in device memory this round
  // previous round's lists (incremental collection) and slot stamps
  int32_t *prev_cc_elem;
  uint64_t *prev_cc_key;
  double2 *prev_cc_p;
  int32_t *prev_mid_elem;
  int32_t *tstamp;     // [capT] serial of the round that last wrote the slot
  int32_t *cidx_t;     // [capT] candidate index of a bad triangle in this round's list
  int32_t *cidx_s;     // [capS] candidate index of a flagged subsegment
  uint64_t *keys;      // [capT+capS] scratch for the candidate cap
  int32_t *rhist;      // [256] digit histogram of the radix select (zero between uses)
  StatLine *stat;      // [kStatStripes] statistics of the running round
  uint64_t *tally;     // = stat as 64-bit words: exact-stage counters of the predicates
  double L2;           // edge-length bound l^2 (0: off)
  int32_t enc_mode;    // 0: diametric circle, 1: diametric lens
  int32_t split_mode;  // 0: midpoints, 1: concentric shells
  uint64_t *sel;       // [3] radix select: key prefix, prefix mask, keys still to take
  int32_t pm;
};

// One exclusive scan (see k_scan_tiles).
struct ScanJob {
  const int32_t *in;
  int32_t *out;
  const int32_t *n_dev;  // length in device memory
  int32_t *tiles;        // per-tile totals, then their exclusive prefix
  int32_t *total;
  int mode;              // 0: counts, 1: popcounts of 32-bit words
};

// Every round kernel returns at once when st->halt is set; lengths come from
// device memory, and the grids only bound the parallelism (grid-stride loops).
__global__ void k_scan(DevMesh m, Work w, double B2, int pm);
__global__ void k_collect(DevMesh m, Work w, double B2, int pm);
__global__ void k_pending(DevMesh m, Work w);
__global__ void k_gate(Work w, int max_rounds);
__global__ void k_gather_keys(DevMesh m, Work w, int pm);
__global__ void k_radix_hist(Work w, int shift);
__global__ void k_radix_pick(Work w, int shift, int K);
__global__ void k_apply_cap(Work w);
__global__ void k_locate(DevMesh m, Work w);
__global__ void k_prefilter(DevMesh m, Work w, int mode, int n);
constexpr int kApproxMaxN = 16;
constexpr int kCavCapDefault = 39;  // per-thread cavity slots of the grid kernel (LDS per 128-thread block)
template <int IS_CC, int CAP>
__global__ void k_cavity(DevMesh m, Work w);
__global__ void k_cavity_big(DevMesh m, Work w, int phase);
__global__ void k_cavity_huge(DevMesh m, Work w, int phase);
__global__ void k_own(Work w);
__global__ void k_dep(DevMesh m, Work w);
__global__ void k_scan_tiles(ScanJob a, ScanJob b, const int32_t *halt);
__global__ void k_scan_sums(ScanJob a, ScanJob b, const int32_t *halt);
__global__ void k_winners(Work w);
__global__ void k_record(DevMesh m, Work w);
__global__ void k_write(DevMesh m, Work w);
__global__ void k_finish(DevMesh m, Work w);
// Mesh quality: bad triangles and their area (per-block partials, then one
// fixed-order sum).
constexpr int kQualBlocks = 512;
__global__ void k_quality(DevMesh m, double B2, double L2, unsigned long long *n_part, double *a_part);
__global__ void k_quality_sum(int n_part, const unsigned long long *n_in, const double *a_in,
                              unsigned long long *n_out, double *a_out);
// Scatter of packed uploads: entry e copies bytes[e] (a multiple of 4) from
// src + src_off[e] to dst[e], one workgroup per entry (grid-stride).
struct CopyEnt {
  int64_t src_off;
  int32_t *dst;
  int64_t bytes;
};
__global__ void k_scatter_copy(const int32_t *src, const CopyEnt *ents, int n);

// The exact predicates on a list of queries (kind 0 orient2d, 1 incircle,
// 2 indiametral, 3 lens encroachment; 6 or 8 doubles per query).
__global__ void k_predicates(int kind, int n, const double *pts, int32_t *out, uint64_t *tally);

// Random-slot 64-bit atomicMax throughput (the marks' access pattern).
__global__ void k_atomic_max_bench(uint64_t *table, uint64_t n_slots, int64_t n_ops, uint64_t seed);

// One mesh of the single-workgroup engine.
struct EngDesc {
  DevMesh m;
  Work w[2];  // workspaces of the rounds with an even / odd serial
  double B2;
  int32_t pm, K, f1, approx_n, max_rounds, pad;
};
constexpr int kEngBlock = 1024;
__global__ void k_engine(const EngDesc *descs, int n_mesh, int32_t *head, int round_limit);

// Round-boundary batching (the serving form's shared rounds): one launch per
// phase for a set of meshes.  Workgroup (x, y) works on mesh y, with the
// grid-stride loops of the single-mesh kernels over x; each mesh takes its
// round's workspace from its own serial, its halt code stops its part of
// every launch, and the first round of a mesh (DevState.full) is a full
// collection.  Semantic parameters come from each mesh's descriptor.
struct GangDesc {
  EngDesc e;
  ScanJob js, jt, jf;  // the round's scans (subsegment and triangle winner bitmaps, fresh-slot counts)
};
__global__ void kg_collect(const GangDesc *G);
__global__ void kg_pending(const GangDesc *G);
__global__ void kg_gate(const GangDesc *G);
__global__ void kg_gather_keys(const GangDesc *G);
__global__ void kg_radix_hist(const GangDesc *G, int shift);
__global__ void kg_radix_pick(const GangDesc *G, int shift);
__global__ void kg_apply_cap(const GangDesc *G);
__global__ void kg_locate(const GangDesc *G);
__global__ void kg_prefilter(const GangDesc *G, int mode);
template <int IS_CC>
__global__ void kg_cavity(const GangDesc *G);
__global__ void kg_cavity_big(const GangDesc *G, int phase);
__global__ void kg_cavity_huge(const GangDesc *G, int phase);
__global__ void kg_own(const GangDesc *G);
__global__ void kg_dep(const GangDesc *G);
__global__ void kg_scan_tiles(const GangDesc *G, int which);
__global__ void kg_scan_sums(const GangDesc *G, int which);
__global__ void kg_winners(const GangDesc *G);
__global__ void kg_record(const GangDesc *G);
__global__ void kg_write(const GangDesc *G);
__global__ void kg_finish(const GangDesc *G);
// Copies each mesh's DevState, running counters and first `rounds` history
// records to out + y * stride_words (32-bit words), for one host read.
__global__ void kg_status(const GangDesc *G, int rounds, int32_t *out, int stride_words);

// Flip-Flop insertion (Section 4.3, Line 8; gdp_ff_core.h).  Line 6 of such
// a round: every located circumcenter and midpoint claims the triangles it
// would split with atomicMax of its key (a circumcenter on a subsegment
// flags it instead); a point that holds all its claims goes to S as the pair
// (~key, reference) for the sort into decreasing key order; kf_gather then
// lays S out by rank.  The round ends with kf_round_end (one workgroup).
__global__ void kf_claim_cc(DevMesh m, Work w);
__global__ void kf_claim_mid(DevMesh m, Work w);
__global__ void kf_own(Work w, FfCount *f, uint64_t *skey, int32_t *sref);
__global__ void kf_clear_marks(Work w);
__global__ void kf_gather(DevMesh m, Work w, FfView V, const int32_t *sref);
__global__ void kf_round_end(Work w, const FfCount *f, int32_t nT_new, int32_t nwin, int32_t nwin_mid);
// ... and the steps themselves (gdp_ff.hip): grid-stride loops over the
// elements, counts read from device memory where they change on the device.
__global__ void kf_split(FfView V, int split_stamp, int wst, int tst);
__global__ void kf_split_fix(FfView V, int split_stamp);
__global__ void kf_ctl(FfCount *c, int op, int arg);
__global__ void kf_flip_check(FfView V, int in_stamp, uint64_t pass);
__global__ void kf_flip_apply(FfView V, int wst, int tst);
__global__ void kf_vtri(FfView V);
__global__ void kf_detect(FfView V);
__global__ void kf_rm_mark(FfView V, uint64_t pbase);
__global__ void kf_rm_decide(FfView V, uint64_t pbase);
__global__ void kf_rm_apply(FfView V, int wst, int tst);
__global__ void kf_nwin_mid(FfView V);  // after the scan of alive into newid
__global__ void kf_final_point(FfView V);
__global__ void kf_final_tri(FfView V);
__global__ void kf_final_mid(FfView V);
__global__ void kf_final_flag(FfView V);
__global__ void kf_final_flag_clear(FfView V);
__global__ void kf_compact_list(FfView V, int n_alloc, int n_live);
__global__ void kf_compact_move(FfView V);
__global__ void kf_compact_fix(FfView V, int n_live);
__global__ void kf_rotate(FfView V, int n);
__global__ void kf_all_slots(FfView V, int n, int wst);  // every slot onto the worklist

constexpr int kCavBlockSize = 128;
constexpr int kBigBlockSize = 256;
constexpr int kHugeBlock = 1024;
constexpr int kScanTileSize = 256 * 8;

}  // namespace gdp

// gdp_api.hip -- C ABI (include/gdp2d.h): contexts, meshes in device memory
// and the host loop that issues one refinement round after another
// (Algorithm 1, "repeat ... until L is empty").
#include <algorithm>
#include <array>
#include <atomic>
#include <memory>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "gdp_kernels.h"

using namespace gdp;

// ---- static scratch of the allocation-free entry point ---------------------
// gdp_mesh_quality_noalloc keeps its per-workgroup partial sums here instead
// of in memory it allocates.  Each device holds its own copy, at its own
// address, resolved once per device when a context is created on it; host
// code uses only that resolved address (the symbol's host-side name is not a
// device address).  Calls that overlap on one device share the array and race.
namespace {
constexpr size_t kScratchBytes = 16384;
static_assert((size_t)kQualBlocks * (sizeof(unsigned long long) + sizeof(double)) <= kScratchBytes,
              "the quality partials fit in the scratch array");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
// With `device` current: resolves the device address of the scratch array once.
void resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[device] = ptr;
}
void *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

struct gdp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
};

// Device memory shared by the meshes of one batch (freed with the last one).
struct gdp_arena {
  void *base = nullptr;
  int refs = 0;
  std::function<void()> release;  // set: the memory is a server job region, handed back on release
};

void arena_release(gdp_arena *a) {
  if (--a->refs > 0) return;
  if (a->release) a->release();
  else if (a->base) (void)hipFree(a->base);
  delete a;
}

// Device buffers of the Flip-Flop rounds (insert_mode 1), allocated by the
// first such round and grown with the mesh.
struct FfBufs {
  int32_t capP = 0;   // points of S
  int32_t capK = 0;   // candidates (sort input)
  int32_t capT = 0, capV = 0, capS = 0;
  int64_t pool_cap = 0;
  uint64_t *skey0 = nullptr, *skey1 = nullptr;
  int32_t *sref0 = nullptr, *sref1 = nullptr, *shist = nullptr;
  double2 *pt = nullptr;
  int4 *pinfo = nullptr, *pslots = nullptr;
  int2 *pab = nullptr;
  int32_t *alive = nullptr, *red = nullptr, *vtri = nullptr, *newid = nullptr;
  int4 *grp = nullptr, *fc0 = nullptr, *fc1 = nullptr;
  int32_t *sstamp = nullptr, *wstamp = nullptr, *tstamp = nullptr, *moved = nullptr;
  uint64_t *claim = nullptr, *fprio = nullptr, *vmark = nullptr;
  int32_t *list[2] = {nullptr, nullptr};
  int32_t *touched = nullptr, *dead = nullptr, *hole = nullptr, *mover = nullptr;
  int32_t *ntiles = nullptr;  // tile totals of the rank scan
  int32_t *sflag = nullptr, *mid_rank = nullptr, *pool = nullptr;
  FfCount *d_c = nullptr, *h_c = nullptr;
  int32_t stamp = 0;   // last slot stamp handed out (splits, worklists, touched list)
  uint64_t pass = 0;   // last pass number (flip claims, removal marks)
};

struct gdp_mesh {
  gdp_ctx *ctx = nullptr;
  gdp_arena *arena = nullptr;  // non-null: the device arrays below live in a batch arena
  DevMesh m;
  // Two rounds (parity p, then the other) captured as one HIP graph, for
  // groups of small rounds; rebuilt when a buffer, a parameter or the grid
  // estimate changes.
  struct RoundGraph {
    hipGraphExec_t exec = nullptr;
    uint64_t key = 0;
    int64_t est = 0;
  } graph[2];
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  EngDesc *d_eng = nullptr;          // descriptor of this mesh for the single-workgroup engine
  EngDesc *h_eng = nullptr;          // pinned
  int32_t *d_head = nullptr;         // the engine's queue head
  DevCounters *d_cnt = nullptr;
  DevCounters *h_cnt = nullptr;  // pinned
  StatLine *d_stat = nullptr;    // [kStatStripes] statistics of the running round
  uint64_t *mark = nullptr;
  int32_t *sadj = nullptr;
  uint32_t *mflag = nullptr;
  CandSet cc{}, mid{};
  uint32_t *w0_t = nullptr, *w0_s = nullptr, *win_t = nullptr, *win_s = nullptr;
  int32_t *rank_t = nullptr, *rank_s = nullptr;
  int32_t *win_ref = nullptr, *fbase = nullptr, *fcount = nullptr, *fan_off = nullptr;
  int32_t *repl = nullptr;
  int32_t *pool = nullptr;
  int32_t pool_cap = 0;
  FanRec *fan = nullptr;
  int32_t fan_cap = 0;
  int32_t *big = nullptr;
  int32_t *hvis = nullptr, *hlist = nullptr;  // [capT] cavities beyond the LDS list (device-memory path)
  bool huge_mode = false;  // launch the device-memory cavity path (set once a round needed it)
  bool engine_off = false; // a single-workgroup engine round met a cavity beyond its LDS list
  int32_t *prev_cc_elem = nullptr;
  uint64_t *prev_cc_key = nullptr;
  double2 *prev_cc_p = nullptr;
  int32_t *prev_mid_elem = nullptr;
  int32_t *tstamp = nullptr;
  int32_t cdt_rounds[2] = {0, 0};  // rounds of the device CDT builder (points, segments)
  int32_t *cidx_t = nullptr, *cidx_s = nullptr;
  // cc.elem/key/p, mid.elem and the prev_* arrays form two list buffers; a
  // round with an odd serial uses them the other way round
  int32_t serial = 0;  // rounds ever executed on this mesh object (slot stamps)
  uint64_t *keys = nullptr;
  int32_t *rhist = nullptr;
  uint64_t *sel = nullptr;
  int32_t *tiles_t = nullptr, *tiles_s = nullptr, *tiles_f = nullptr;  // tile prefixes of the three scans
  int32_t tiles_cap = 0;
  DevState *d_st = nullptr;
  DevState *h_st = nullptr;       // pinned
  DevCounters *d_hist = nullptr;  // counters of the rounds completed since the last sync
  DevCounters *h_hist = nullptr;  // pinned
  int32_t wT = 0, wS = 0;      // workspace capacities (triangles, subsegments)
  std::vector<gdp_round_stats> stats;
  double last_ms = 0.0;
  // optional per-kernel timing (HIP events around every launch)
  bool prof = false;
  struct ProfRec {
    int id;
    hipEvent_t a, b;
    int round;  // index of the round within its group
    int64_t items, bytes;
  };
  int cur_round = 0;
  std::vector<ProfRec> prof_pending;
  double prof_ms[16] = {};
  int64_t prof_launches[16] = {}, prof_items[16] = {}, prof_bytes[16] = {};
  FfBufs *ff = nullptr;  // Flip-Flop rounds
};

namespace {
enum ProfId {
  P_SCAN = 0, P_CAP, P_LOCATE, P_CAV_CC, P_CAV_MID, P_CAV_BIG, P_PREFILTER, P_OWN, P_DEP, P_PREFIX,
  P_WINNERS, P_RECORD, P_WRITE, P_FINISH, P_ENGINE, P_NUM
};
const char *kProfNames[P_NUM] = {"k_scan", "k_cap", "k_locate", "k_cavity_cc", "k_cavity_mid", "k_cavity_big",
                                  "k_prefilter", "k_own", "k_dep", "k_prefix_sum", "k_winners", "k_record", "k_write",
                                  "k_finish", "k_engine"};
// Records HIP events around the launches issued in its scope (if enabled);
// items and algorithmic bytes are filled in once the round's counts are read.
struct Prof {
  gdp_mesh *M;
  int id;
  hipEvent_t a = nullptr;
  Prof(gdp_mesh *M_, int id_) : M(M_), id(id_) {
    if (M->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, M->ctx->stream);
  }
  ~Prof() {
    if (!M->prof || !a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, M->ctx->stream);
    M->prof_pending.push_back({id, a, b, M->cur_round, 0, 0});
  }
};
}  // namespace

namespace {

thread_local std::string g_noctx_err;

gdp_status fail(gdp_ctx *ctx, gdp_status s, const std::string &msg) {
  if (ctx) ctx->err = msg; else g_noctx_err = msg;
  return s;
}

#define HIPCHECK(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, GDP_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_));   \
  } while (0)

template <class T>
hipError_t dalloc(T **p, size_t n) {
  return hipMalloc((void **)p, sizeof(T) * std::max<size_t>(n, 1));
}

// Grows a device array from old_n to new_n elements, keeping the first keep_n
// elements and filling the new tail with `fill` bytes.
template <class T>
hipError_t dgrow(T **p, size_t old_n, size_t new_n, size_t keep_n, int fill, hipStream_t s) {
  T *q = nullptr;
  hipError_t e = hipMalloc((void **)&q, sizeof(T) * std::max<size_t>(new_n, 1));
  if (e != hipSuccess) return e;
  if (!*p) keep_n = 0;  // nothing to keep: initialise everything
  if (*p && keep_n) {
    e = hipMemcpyAsync(q, *p, sizeof(T) * keep_n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  if (new_n > keep_n) {
    e = hipMemsetAsync(q + keep_n, fill, sizeof(T) * (new_n - keep_n), s);
    if (e != hipSuccess) return e;
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (*p) (void)hipFree(*p);
  *p = q;
  (void)old_n;
  return hipSuccess;
}

inline int words(int n) { return n / 32 + 1; }

// A mesh whose arrays live in a batch or server region moves them into
// allocations of its own before any of them grows (defined below).
gdp_status detach(gdp_mesh *M);

gdp_status grow_tri(gdp_mesh *M, int32_t need) {
  gdp_ctx *ctx = M->ctx;
  if (need <= M->m.capT) return GDP_OK;
  if (M->arena) {
    gdp_status d = detach(M);
    if (d != GDP_OK) return d;
  }
  hipStream_t s = ctx->stream;
  int32_t oc = M->m.capT;
  int64_t nc64 = std::max<int64_t>(need, (int64_t)oc + oc / 2 + 1024);
  if (nc64 > (1 << 29)) return fail(ctx, GDP_E_NOMEM, "triangle capacity limit exceeded");
  int32_t nc = (int32_t)nc64;
  HIPCHECK(dgrow(&M->m.tv, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->m.tn, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->m.ts, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->mark, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.elem, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.key, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.p, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.loc, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.state, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.off, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->cc.len, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->w0_t, words(oc), words(nc), words(oc), 0, s));
  HIPCHECK(dgrow(&M->win_t, words(oc), words(nc), words(oc), 0, s));
  HIPCHECK(dgrow(&M->rank_t, words(oc), words(nc), words(oc), 0, s));
  HIPCHECK(dgrow(&M->repl, 4 * (size_t)oc, 4 * (size_t)nc, 0, 0xff, s));
  HIPCHECK(dgrow(&M->prev_cc_elem, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->prev_cc_key, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->prev_cc_p, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->tstamp, oc, nc, oc, 0xff, s));
  HIPCHECK(dgrow(&M->cidx_t, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->hvis, oc, nc, 0, 0, s));
  HIPCHECK(dgrow(&M->hlist, oc, nc, 0, 0, s));
  M->m.capT = nc;
  return GDP_OK;
}

gdp_status grow_seg(gdp_mesh *M, int32_t need) {
  gdp_ctx *ctx = M->ctx;
  if (need <= M->m.capS) return GDP_OK;
  if (M->arena) {
    gdp_status d = detach(M);
    if (d != GDP_OK) return d;
  }
  hipStream_t s = ctx->stream;
  int32_t oc = M->m.capS;
  int64_t nc64 = std::max<int64_t>(need, (int64_t)oc + oc / 2 + 1024);
  if (nc64 > (1 << 28)) return fail(ctx, GDP_E_NOMEM, "subsegment capacity limit exceeded");
  int32_t nc = (int32_t)nc64;
  HIPCHECK(dgrow(&M->m.sv, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->m.spar, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->m.spend, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->sadj, 2 * (size_t)oc, 2 * (size_t)nc, 2 * (size_t)oc, 0xff, s));
  HIPCHECK(dgrow(&M->mflag, oc, nc, oc, 0, s));
  size_t om = 2 * (size_t)oc, nm = 2 * (size_t)nc;  // a flagged subsegment can appear twice
  HIPCHECK(dgrow(&M->mid.elem, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->mid.key, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->mid.p, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->mid.loc, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->mid.state, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->mid.off, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->mid.len, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->prev_mid_elem, om, nm, om, 0, s));
  HIPCHECK(dgrow(&M->cidx_s, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->w0_s, words(oc), words(nc), words(oc), 0, s));
  HIPCHECK(dgrow(&M->win_s, words(oc), words(nc), words(oc), 0, s));
  HIPCHECK(dgrow(&M->rank_s, words(oc), words(nc), words(oc), 0, s));
  M->m.capS = nc;
  return GDP_OK;
}

gdp_status grow_vtx(gdp_mesh *M, int32_t need) {
  gdp_ctx *ctx = M->ctx;
  if (need <= M->m.capV) return GDP_OK;
  if (M->arena) {
    gdp_status d = detach(M);
    if (d != GDP_OK) return d;
  }
  hipStream_t s = ctx->stream;
  int32_t oc = M->m.capV;
  int64_t nc64 = std::max<int64_t>(need, (int64_t)oc + oc / 2 + 1024);
  if (nc64 > (1 << 29)) return fail(ctx, GDP_E_NOMEM, "vertex capacity limit exceeded");
  int32_t nc = (int32_t)nc64;
  HIPCHECK(dgrow(&M->m.vxy, oc, nc, oc, 0, s));
  HIPCHECK(dgrow(&M->m.vkind, oc, nc, oc, 0, s));
  M->m.capV = nc;
  return GDP_OK;
}

// Arrays sized by the candidate count (circumcenters + midpoints).
gdp_status grow_cand(gdp_mesh *M) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  int64_t need = (int64_t)M->m.capT + 2 * (int64_t)M->m.capS + 2;
  if (need <= M->wT) return GDP_OK;
  if (M->arena) {
    gdp_status d = detach(M);
    if (d != GDP_OK) return d;
  }
  int64_t nc = std::max<int64_t>(need, (int64_t)M->wT + M->wT / 2);
  // called between k_winners and k_record: keep what is already written
  size_t keep = (size_t)M->wT;
  HIPCHECK(dgrow(&M->win_ref, keep, nc, keep, 0, s));
  HIPCHECK(dgrow(&M->fbase, keep, nc, keep, 0, s));
  HIPCHECK(dgrow(&M->fcount, keep, nc, keep, 0, s));
  HIPCHECK(dgrow(&M->fan_off, keep, nc, keep, 0, s));
  HIPCHECK(dgrow(&M->big, keep, nc, keep, 0, s));
  HIPCHECK(dgrow(&M->keys, keep, nc, keep, 0, s));
  int64_t nt = nc / kScanTileSize + 2;
  HIPCHECK(dgrow(&M->tiles_t, 0, nt, 0, 0, s));
  HIPCHECK(dgrow(&M->tiles_s, 0, nt, 0, 0, s));
  HIPCHECK(dgrow(&M->tiles_f, 0, nt, 0, 0, s));
  M->tiles_cap = (int32_t)nt;
  M->wT = (int32_t)nc;
  return GDP_OK;
}

constexpr int kHistCap = 64;  // rounds queued between two host synchronisations, at most
constexpr int64_t kEngineDefaultMax = 1024;  // candidates per round run by the single-workgroup engine
// The engine grows its large (cooperative) cavities one after the other, the
// grid kernels side by side: a mesh whose last round had more of them stays
// on the grid kernels for the next round (rounded-cocircular inputs give
// hundreds per round; perf only, the rounds are the same either way).
constexpr int64_t kEngineBigMax = 8;

// Workspace pointers of a round; the two list buffers swap roles with the
// parity of the round's serial.
Work make_work(gdp_mesh *M, const gdp_params *P, int parity) {
  const int pm = P->priority_mode;
  Work w;
  memset(&w, 0, sizeof w);  // no stray padding bytes (graph keys hash the struct)
  w.L2 = P->max_edge_len_sq;
  w.enc_mode = P->encroach_mode;
  w.split_mode = P->split_mode;
  w.st = M->d_st;
  w.cnt = M->d_cnt;
  w.stat = M->d_stat;
  w.tally = (uint64_t *)M->d_stat;
  w.hist = M->d_hist;
  w.hist_cap = kHistCap;
  w.mark = M->mark;
  w.sadj = M->sadj;
  w.mflag = M->mflag;
  w.cc = M->cc;
  w.mid = M->mid;
  w.prev_cc_elem = M->prev_cc_elem; w.prev_cc_key = M->prev_cc_key; w.prev_cc_p = M->prev_cc_p;
  w.prev_mid_elem = M->prev_mid_elem;
  if (parity & 1) {
    std::swap(w.cc.elem, w.prev_cc_elem);
    std::swap(w.cc.key, w.prev_cc_key);
    std::swap(w.cc.p, w.prev_cc_p);
    std::swap(w.mid.elem, w.prev_mid_elem);
  }
  w.w0_t = M->w0_t; w.w0_s = M->w0_s; w.win_t = M->win_t; w.win_s = M->win_s;
  w.rank_t = M->rank_t; w.rank_s = M->rank_s;
  w.tiles_t = M->tiles_t; w.tiles_s = M->tiles_s; w.tiles_f = M->tiles_f;
  w.win_ref = M->win_ref; w.fbase = M->fbase; w.fcount = M->fcount; w.fan_off = M->fan_off;
  w.win_cap = M->wT;
  w.repl = M->repl;
  w.pool = M->pool; w.pool_cap = M->pool_cap;
  w.fan = M->fan; w.fan_cap = M->fan_cap;
  w.big = M->big; w.big_cap = M->wT;
  w.hvis = M->hvis; w.hlist = M->hlist; w.hcap = M->m.capT;
  w.huge_ok = M->huge_mode ? 1 : 0;
  w.tstamp = M->tstamp;
  w.cidx_t = M->cidx_t; w.cidx_s = M->cidx_s;
  w.keys = M->keys; w.rhist = M->rhist; w.sel = M->sel;
  w.pm = pm;
  return w;
}

// FNV-1a over raw bytes.
uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = (const unsigned char *)p;
  for (size_t i = 0; i < n; i++) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// Grid for a grid-stride kernel over about n items.
inline unsigned stride_grid(int64_t n, int bs) {
  return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + bs - 1) / bs), 8192);
}

// Exclusive scans of one or two jobs (b.in == nullptr: one); n_bound bounds
// the lengths (in device memory) and sizes the grid.
gdp_status scan(gdp_mesh *M, const ScanJob &a, const ScanJob &b, int64_t n_bound) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  int64_t ntiles = std::max<int64_t>(1, (n_bound + kScanTileSize - 1) / kScanTileSize);
  if (ntiles > M->tiles_cap) return fail(ctx, GDP_E_NOMEM, "scan tile buffer too small");
  const int32_t *halt = &M->d_st->halt;
  Prof pr(M, P_PREFIX);
  unsigned g = (unsigned)std::min<int64_t>((b.in ? 2 : 1) * ntiles, 2048);
  hipLaunchKernelGGL(k_scan_tiles, dim3(g), dim3(256), 0, s, a, b, halt);
  hipLaunchKernelGGL(k_scan_sums, dim3(b.in ? 2 : 1), dim3(256), 0, s, a, b, halt);
  HIPCHECK(hipGetLastError());
  return GDP_OK;
}

// Small device buffers and their pinned host mirrors.
gdp_status alloc_control(gdp_mesh *M) {
  gdp_ctx *ctx = M->ctx;
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  if (!ok(dalloc(&M->d_cnt, 1)) || !ok(hipHostMalloc((void **)&M->h_cnt, sizeof(DevCounters))) ||
      !ok(dalloc(&M->d_stat, kStatStripes)) ||
      !ok(dalloc(&M->d_st, 1)) || !ok(hipHostMalloc((void **)&M->h_st, sizeof(DevState))) ||
      !ok(dalloc(&M->d_hist, kHistCap)) || !ok(hipHostMalloc((void **)&M->h_hist, sizeof(DevCounters) * kHistCap)) ||
      !ok(dalloc(&M->rhist, 256)) || !ok(dalloc(&M->sel, 4)))
    return fail(ctx, GDP_E_NOMEM, "allocation failed");
  HIPCHECK(hipMemsetAsync(M->d_cnt, 0, sizeof(DevCounters), ctx->stream));
  HIPCHECK(hipMemsetAsync(M->d_stat, 0, sizeof(StatLine) * kStatStripes, ctx->stream));
  HIPCHECK(hipMemsetAsync(M->d_st, 0, sizeof(DevState), ctx->stream));
  HIPCHECK(hipMemsetAsync(M->rhist, 0, 256 * sizeof(int32_t), ctx->stream));
  HIPCHECK(hipMemsetAsync(M->sel, 0, 4 * sizeof(uint64_t), ctx->stream));
  return GDP_OK;
}

void free_extras(gdp_mesh *M);

void free_mesh_arrays(gdp_mesh *M) {
  if (M->arena) {
    free_extras(M);
    arena_release(M->arena);
    M->arena = nullptr;
    return;
  }
  void *ptrs[] = {M->m.vxy, M->m.vkind, M->m.tv, M->m.tn, M->m.ts, M->m.sv, M->m.spar, M->m.spend,
                  M->d_cnt, M->d_stat, M->mark, M->sadj, M->mflag,
                  M->cc.elem, M->cc.key, M->cc.p, M->cc.loc, M->cc.state, M->cc.off, M->cc.len,
                  M->mid.elem, M->mid.key, M->mid.p, M->mid.loc, M->mid.state, M->mid.off, M->mid.len,
                  M->w0_t, M->w0_s, M->win_t, M->win_s, M->rank_t, M->rank_s, M->win_ref, M->fbase,
                  M->fcount, M->fan_off, M->repl, M->pool, M->fan, M->big, M->keys, M->rhist, M->sel,
                  M->d_st, M->d_hist, M->tiles_t, M->tiles_s, M->tiles_f, M->prev_cc_elem, M->prev_cc_key, M->prev_cc_p, M->prev_mid_elem, M->tstamp,
                  M->cidx_t, M->cidx_s, M->hvis, M->hlist};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  free_extras(M);
}

// Allocations a mesh owns even inside a batch arena: pinned host mirrors,
// captured graphs, the engine descriptor.
void free_extras(gdp_mesh *M) {
  if (M->ff) {
    FfBufs *F = M->ff;
    void *ptrs[] = {F->skey0, F->skey1, F->sref0, F->sref1, F->shist, F->pt, F->pinfo, F->pslots, F->pab,
                    F->alive, F->red, F->vtri, F->newid, F->grp, F->fc0, F->fc1, F->sstamp, F->wstamp,
                    F->tstamp, F->moved, F->claim, F->fprio, F->vmark, F->list[0], F->list[1], F->touched,
                    F->dead, F->hole, F->mover, F->ntiles, F->sflag, F->mid_rank, F->pool, F->d_c};
    for (void *q : ptrs)
      if (q) (void)hipFree(q);
    if (F->h_c) (void)hipHostFree(F->h_c);
    delete F;
    M->ff = nullptr;
  }
  if (M->h_cnt) (void)hipHostFree(M->h_cnt);
  if (M->h_st) (void)hipHostFree(M->h_st);
  if (M->h_hist) (void)hipHostFree(M->h_hist);
  for (auto &g : M->graph)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (M->d_eng) (void)hipFree(M->d_eng);
  if (M->d_head) (void)hipFree(M->d_head);
  if (M->h_eng) (void)hipHostFree(M->h_eng);
  if (M->cap_stream) (void)hipStreamDestroy(M->cap_stream);
}

// Allocates a device mesh with room for the given counts (arrays not filled).
gdp_status mesh_new(gdp_ctx *ctx, int32_t nV, int32_t nIV, int32_t nT, int32_t nS, int32_t nIS, int32_t rounds,
                    gdp_mesh **out) {
  gdp_mesh *M = new gdp_mesh();
  M->ctx = ctx;
  auto bail = [&](gdp_status st) {
    free_mesh_arrays(M);
    delete M;
    return st;
  };
  M->m.nV = nV; M->m.nT = nT; M->m.nS = nS;
  M->m.n_input_v = nIV; M->m.n_input_s = nIS; M->m.rounds = rounds;
  // room for the refined mesh from the start (about 2.5x the input vertices
  // at B = sqrt(2)): growing later costs allocations, copies and a device
  // synchronisation per array
  const int64_t cV = std::max<int64_t>(3 * (int64_t)nV + 1024, nV);
  const int64_t cT = std::max<int64_t>(2 * cV + 2048, nT);
  const int64_t cS = std::max<int64_t>(16 * (int64_t)nS + 1024, nS);
  if (cT > (1 << 29) || cS > (1 << 28)) return bail(fail(ctx, GDP_E_NOMEM, "mesh too large"));
  M->m.capV = 0; M->m.capT = 0; M->m.capS = 0;
  gdp_status st;
  if ((st = grow_vtx(M, (int32_t)cV)) != GDP_OK) return bail(st);
  if ((st = grow_tri(M, (int32_t)cT)) != GDP_OK) return bail(st);
  if ((st = grow_seg(M, (int32_t)cS)) != GDP_OK) return bail(st);
  if ((st = grow_cand(M)) != GDP_OK) return bail(st);
  if ((st = alloc_control(M)) != GDP_OK) return bail(st);
  M->pool_cap = std::max(1 << 16, 2 * M->m.capT + 65536);
  if (dalloc(&M->pool, M->pool_cap) != hipSuccess) return bail(fail(ctx, GDP_E_NOMEM, "allocation failed"));
  M->fan_cap = std::max(1 << 16, 2 * M->m.capT);
  if (dalloc(&M->fan, M->fan_cap) != hipSuccess) return bail(fail(ctx, GDP_E_NOMEM, "allocation failed"));
  *out = M;
  return GDP_OK;
}

void mesh_delete(gdp_mesh *M) {
  free_mesh_arrays(M);
  delete M;
}

// Allocates a device mesh with room for the given counts and uploads it.
gdp_status upload(gdp_ctx *ctx, int32_t nV, int32_t nIV, const double *xy, const int32_t *vkind,
                  int32_t nT, const int32_t *tv, const int32_t *tn, const int32_t *ts, int32_t nS,
                  int32_t nIS, const int32_t *sv, const int32_t *spar, const uint8_t *spend,
                  int32_t rounds, gdp_mesh **out) {
  hipStream_t s = ctx->stream;
  gdp_mesh *M = nullptr;
  gdp_status st = mesh_new(ctx, nV, nIV, nT, nS, nIS, rounds, &M);
  if (st != GDP_OK) return st;
  std::vector<double2> hv(nV);
  for (int i = 0; i < nV; i++) hv[i] = make_double2(xy[2 * i], xy[2 * i + 1]);
  std::vector<int4> htv(nT), htn(nT), hts(nT);
  for (int t = 0; t < nT; t++) {
    int mask = (ts[3 * t] >= 0 ? 1 : 0) | (ts[3 * t + 1] >= 0 ? 2 : 0) | (ts[3 * t + 2] >= 0 ? 4 : 0);
    htv[t] = make_int4(tv[3 * t], tv[3 * t + 1], tv[3 * t + 2], mask);
    htn[t] = make_int4(tn[3 * t], tn[3 * t + 1], tn[3 * t + 2], 0);
    hts[t] = make_int4(ts[3 * t], ts[3 * t + 1], ts[3 * t + 2], 0);
  }
  std::vector<int2> hsv(nS);
  std::vector<int32_t> hsp(nS), hpend(nS);
  for (int k = 0; k < nS; k++) {
    hsv[k] = make_int2(sv[2 * k], sv[2 * k + 1]);
    hsp[k] = spar[k];
    hpend[k] = spend ? spend[k] : 0;
  }
  std::vector<int32_t> hk(nV, 0);
  if (vkind) hk.assign(vkind, vkind + nV);
  auto chk = [&](hipError_t e, const char *what) {
    if (e != hipSuccess) { fail(ctx, GDP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)); return false; }
    return true;
  };
  if (!chk(hipMemcpyAsync(M->m.vxy, hv.data(), sizeof(double2) * nV, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.vkind, hk.data(), sizeof(int32_t) * nV, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.tv, htv.data(), sizeof(int4) * nT, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.tn, htn.data(), sizeof(int4) * nT, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.ts, hts.data(), sizeof(int4) * nT, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.sv, hsv.data(), sizeof(int2) * nS, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.spar, hsp.data(), sizeof(int32_t) * nS, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipMemcpyAsync(M->m.spend, hpend.data(), sizeof(int32_t) * nS, hipMemcpyHostToDevice, s), "upload") ||
      !chk(hipStreamSynchronize(s), "sync")) {
    mesh_delete(M);
    return GDP_E_DEVICE;
  }
  *out = M;
  return GDP_OK;
}

// After an abandoned round: grow what the device-side check found short.
// The fan records of the previous round are still needed (they list the
// slots to re-test), so the first keep_fan records survive a regrowth.
gdp_status grow_after_abort(gdp_mesh *M, const DevCounters &c, int keep_fan) {
  gdp_ctx *ctx = M->ctx;
  const DevMesh &m = M->m;
  gdp_status st;
  int nwin = c.nwin;
  if ((st = grow_vtx(M, m.nV + nwin + 1024))) return st;
  if ((st = grow_tri(M, m.nT + std::max(c.fresh_total, 2 * nwin) + 2048))) return st;
  if ((st = grow_seg(M, m.nS + c.nwin_mid + 1024))) return st;
  if ((st = grow_cand(M))) return st;
  if (c.err & kErrPool) {
    int64_t nc = std::max<int64_t>((int64_t)c.pool_used * 2, (int64_t)M->pool_cap * 2);
    if (nc > (1LL << 30)) return fail(ctx, GDP_E_NOMEM, "cavity pool limit exceeded");
    if (M->arena && (st = detach(M))) return st;
    HIPCHECK(dgrow(&M->pool, M->pool_cap, nc, 0, 0, ctx->stream));
    M->pool_cap = (int32_t)nc;
  }
  int64_t fan_need = (int64_t)std::max(c.pool_used, M->pool_cap) + 2 * (int64_t)nwin + 1024;
  if (fan_need > M->fan_cap) {
    if (fan_need > (1LL << 30)) return fail(ctx, GDP_E_NOMEM, "fan buffer limit exceeded");
    if (M->arena && (st = detach(M))) return st;
    HIPCHECK(dgrow(&M->fan, M->fan_cap, fan_need, keep_fan, 0, ctx->stream));
    M->fan_cap = (int32_t)fan_need;
  }
  return GDP_OK;
}

// Queues Lines 3-7 of a round (collection, gate, candidate cap, walk,
// optional prefilters) with workspace w; returns the candidate bound that
// sizes the later grids.
int64_t enqueue_select(gdp_mesh *M, double B2, const gdp_params *P, bool full, int64_t est, const Work &w) {
  hipStream_t s = M->ctx->stream;
  const DevMesh &m = M->m;
  const int bs = P->block_size;
  const int pm = P->priority_mode;
  // ---- R1 collection ----
  {
    Prof pr(M, P_SCAN);
    if (full)
      hipLaunchKernelGGL(k_scan, dim3(stride_grid(std::max(m.nT, m.nS), bs)), dim3(bs), 0, s, m, w, B2, pm);
    else {
      hipLaunchKernelGGL(k_collect, dim3(stride_grid(3 * est, bs)), dim3(bs), 0, s, m, w, B2, pm);
      hipLaunchKernelGGL(k_pending, dim3(stride_grid(est / 4, bs)), dim3(bs), 0, s, m, w);
    }
  }
  hipLaunchKernelGGL(k_gate, dim3(1), dim3(256), 0, s, w, P->max_rounds);
  const int64_t ncand = full ? (int64_t)m.nT + m.nS : 2 * est;
  // ---- R3: candidate cap ----
  if (P->cand_cap_K > 0) {
    Prof pr(M, P_CAP);
    hipLaunchKernelGGL(k_gather_keys, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w, pm);
    const unsigned g = std::min<unsigned>(grid_for(ncand, 256), 1024);
    for (int shift = 56; shift >= 0; shift -= 8) {
      hipLaunchKernelGGL(k_radix_hist, dim3(g), dim3(256), 0, s, w, shift);
      hipLaunchKernelGGL(k_radix_pick, dim3(1), dim3(256), 0, s, w, shift, P->cand_cap_K);
    }
    hipLaunchKernelGGL(k_apply_cap, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, w);
  }
  // ---- R4: locate ----
  {
    Prof pr(M, P_LOCATE);
    hipLaunchKernelGGL(k_locate, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w);
  }
  // ---- optional prefilters F1 / F2 on located circumcenters ----
  if (P->prefilter_f1 || P->cavity_approx_n > 0) {
    Prof pr(M, P_PREFILTER);
    if (P->prefilter_f1)
      for (int mode = 0; mode < 3; mode++)
        hipLaunchKernelGGL(k_prefilter, dim3(stride_grid(ncand, 128)), dim3(128), 0, s, m, w, mode, 0);
    if (P->cavity_approx_n > 0)
      for (int mode = 3; mode < 6; mode++)
        hipLaunchKernelGGL(k_prefilter, dim3(stride_grid(ncand, 128)), dim3(128), 0, s, m, w, mode,
                           P->cavity_approx_n);
  }
  return ncand;
}

// Queues one round (Algorithm 1, Lines 3-9) on the stream.  Every length
// comes from device memory; `est` (an estimate of the candidates) only sizes
// the grids.  `full` selects the full collection (first round of a call).
gdp_status enqueue_round(gdp_mesh *M, double B2, const gdp_params *P, bool full, int parity, int64_t est,
                         int group_index) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  const DevMesh &m = M->m;
  const int bs = P->block_size;
  Work w = make_work(M, P, parity);
  est = std::max<int64_t>(est, 1);
  M->cur_round = group_index;
  const int64_t ncand = enqueue_select(M, B2, P, full, est, w);
  // ---- R5/R6 cavities (marks placed as each valid cavity completes) ----
  {
    Prof pr(M, P_CAV_CC);
    const unsigned g = stride_grid(ncand, kCavBlockSize);
    if (P->cavity_thread_cap == 12) hipLaunchKernelGGL((k_cavity<1, 12>), dim3(g), dim3(kCavBlockSize), 0, s, m, w);
    else if (P->cavity_thread_cap == 24) hipLaunchKernelGGL((k_cavity<1, 24>), dim3(g), dim3(kCavBlockSize), 0, s, m, w);
    else hipLaunchKernelGGL((k_cavity<1, kCavCapDefault>), dim3(g), dim3(kCavBlockSize), 0, s, m, w);
  }
  {
    Prof pr(M, P_CAV_BIG);
    hipLaunchKernelGGL(k_cavity_big, dim3(256), dim3(kBigBlockSize), 0, s, m, w, 0);
    if (M->huge_mode) hipLaunchKernelGGL(k_cavity_huge, dim3(1), dim3(kHugeBlock), 0, s, m, w, 0);
  }
  {
    Prof pr(M, P_CAV_MID);
    const unsigned g = stride_grid(ncand / 4, kCavBlockSize);
    if (P->cavity_thread_cap == 12) hipLaunchKernelGGL((k_cavity<0, 12>), dim3(g), dim3(kCavBlockSize), 0, s, m, w);
    else if (P->cavity_thread_cap == 24) hipLaunchKernelGGL((k_cavity<0, 24>), dim3(g), dim3(kCavBlockSize), 0, s, m, w);
    else hipLaunchKernelGGL((k_cavity<0, kCavCapDefault>), dim3(g), dim3(kCavBlockSize), 0, s, m, w);
  }
  {
    Prof pr(M, P_CAV_BIG);
    hipLaunchKernelGGL(k_cavity_big, dim3(256), dim3(kBigBlockSize), 0, s, m, w, 1);
    if (M->huge_mode) hipLaunchKernelGGL(k_cavity_huge, dim3(1), dim3(kHugeBlock), 0, s, m, w, 1);
  }
  // ---- R8 ownership, R9 dependency ----
  {
    Prof pr(M, P_OWN);
    hipLaunchKernelGGL(k_own, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, w);
  }
  {
    Prof pr(M, P_DEP);
    hipLaunchKernelGGL(k_dep, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w);
  }
  // ---- R10: ranks, fresh slots, capacity check, insertion ----
  gdp_status st;
  const ScanJob js{(const int32_t *)M->win_s, M->rank_s, &M->d_st->wS, M->tiles_s, &M->d_cnt->nwin_mid, 1};
  const ScanJob jt{(const int32_t *)M->win_t, M->rank_t, &M->d_st->wT, M->tiles_t, &M->d_cnt->nwin_cc, 1};
  const ScanJob jf{M->fcount, M->fbase, &M->d_cnt->nwin1, M->tiles_f, &M->d_cnt->fan_total, 0};
  const ScanJob none{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
  if ((st = scan(M, js, jt, std::max(words(m.capS), words(m.capT))))) return st;
  {
    Prof pr(M, P_WINNERS);
    hipLaunchKernelGGL(k_winners, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, w);
  }
  if ((st = scan(M, jf, none, std::min<int64_t>(ncand + 1, M->wT)))) return st;
  {
    Prof pr(M, P_RECORD);
    hipLaunchKernelGGL(k_record, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w);
  }
  {
    Prof pr(M, P_WRITE);
    hipLaunchKernelGGL(k_write, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w);
  }
  {
    Prof pr(M, P_FINISH);
    // at most 256 workgroups: each one arrives on one counter at its end
    // (atomics on one address are serialised, ~12 ns each)
    hipLaunchKernelGGL(k_finish, dim3(std::min(stride_grid(ncand, bs), 256u)), dim3(bs), 0, s, m, w);
  }
  HIPCHECK(hipGetLastError());
  return GDP_OK;
}

gdp_round_stats round_stats_of(const DevCounters &c, const gdp_params *P) {
  gdp_round_stats rs;
  memset(&rs, 0, sizeof rs);
  rs.n_bad = c.ncc;
  rs.n_enc = c.nmk0;
  rs.n_kept_cc = P->cand_cap_K > 0 ? c.n_kept_cc : c.ncc;
  rs.n_kept_mid = P->cand_cap_K > 0 ? c.n_kept_mid : c.nmk0;
  rs.n_blocked = c.n_blocked;
  rs.n_coincident = c.n_coincident;
  rs.n_enc_reject = c.n_enc_reject;
  rs.n_unsplittable = c.n_unsplittable;
  rs.n_fan_invalid = c.n_fan_invalid;
  rs.n_lost_mark = c.n_lost_mark;
  rs.n_dep_drop = c.n_dep_drop;
  rs.n_ins_mid = c.nwin_mid;
  rs.n_ins_cc = c.nwin_cc;
  rs.cav_tri_total = c.cav_tri_total;
  rs.cav_max = c.cav_max;
  rs.n_big_cavities = c.nbig;
  rs.n_mid_cand = c.n_mid_cand;
  rs.n_f1_drop = c.n_f1_drop;
  rs.n_f2_drop = c.n_f2_drop;
  rs.n_incircle_tests = c.n_in_tests;
  rs.n_orient_tests = c.n_or_tests + c.cav_bnd[0] + c.cav_bnd[1];
  rs.n_exact_orient = c.n_exact[kExOrient];
  rs.n_exact_dot = c.n_exact[kExDot];
  rs.n_exact_incircle_b = c.n_exact[kExInB];
  rs.n_exact_incircle_c = c.n_exact[kExInC];
  rs.win_cav_tri = c.win_cav;
  rs.win_fan_edges = c.win_bnd;
  rs.win_walk_steps = c.win_steps;
  rs.win_cc_cav_tri = c.win_cc_cav;
  rs.win_cc_fan_edges = c.win_cc_bnd;
  rs.n_huge_cavities = c.nhuge;
  rs.n_marks_mid = c.n_marks[0];
  rs.n_marks_cc = c.n_marks[1];
  rs.n_ff_points = c.ff_points;
  rs.n_ff_iters = c.ff_iters;
  rs.n_flips = c.ff_flips;
  rs.n_flip_passes = c.ff_passes;
  rs.n_removals = c.ff_removals;
  rs.n_removal_passes = c.ff_rm_passes;
  return rs;
}

// Work items of a profiled launch (round counters c; previous round's list
// lengths pc / pmk / pf; full = full collection over nT slots).
int64_t prof_items(int id, const DevCounters &c, int64_t nT, int64_t pc, int64_t pmk, int64_t pf, bool full) {
  switch (id) {
    case P_SCAN: return full ? nT : pc + pf + pmk;
    case P_CAP: return (int64_t)c.ncc + c.nmk0;
    case P_LOCATE: case P_CAV_CC: return c.ncc;
    case P_CAV_MID: return c.nmk;
    case P_CAV_BIG: return c.nbig;
    case P_RECORD: case P_WRITE: return c.nwin;
    case P_PREFIX: return 0;
    case P_ENGINE: return (int64_t)c.ncc + c.nmk;
    default: return (int64_t)c.ncc + c.nmk;
  }
}

// Algorithmic bytes of a profiled launch (same arguments).
//   Collection, full: every triangle record (16 B) and vertex (16 B) once,
//   both sides of every subsegment (ts record 16 B + side slot 4 B each),
//   pending flags (4 B), the bad records written (elem 4 + key 8 + point 16
//   + state 4 B) and the flagged subsegments (flag 4 + list entry 8 B).
//   Incremental: carried records (elem 4 + key 8 + point 16 read and
//   written, stamp 4), each rewritten slot (fan slot 4 + record 16 + three
//   vertices 48) and the previous flagged list (entry 4 + pending flag 4),
//   plus the new records / flags.
//   Circumcenter cavities: what a sequential insertion of the same points
//   touches for them, counted over the winners only (the cavities of points
//   that lose are waste): per cavity triangle its record (36 B) and its
//   priority mark (8 B read-modify-write + 8 B read), per boundary edge the
//   incircle test of the triangle outside (12 B of vertex ids + 16 B for the
//   far vertex).
int64_t alg_bytes(int id, const DevCounters &c, int64_t nT, int64_t nV, int64_t nS, int64_t pc, int64_t pmk,
                  int64_t pf, bool full) {
  if (id == P_SCAN)
    return full ? 16 * nT + 16 * nV + 40 * nS + 4 * nS + 32LL * c.ncc + 12LL * c.nmk0
                : 64 * pc + 68 * pf + 8 * pmk + 32LL * c.ncc + 12LL * c.nmk0;
  if (id == P_CAV_CC) return 52 * c.win_cc_cav + 28 * c.win_cc_bnd;
  return 0;
}

// Grows what a group of R rounds may need, from the candidate count of the
// last round (a loose bound: the device-side check abandons a round that
// does not fit, and the host grows and runs it again).
gdp_status reserve_group(gdp_mesh *M, int64_t last_cand, int R) {
  gdp_ctx *ctx = M->ctx;
  const DevMesh &m = M->m;
  int64_t wins = std::min<int64_t>(last_cand * R + 64, 1 << 28);
  gdp_status st;
  if ((st = grow_vtx(M, (int32_t)std::min<int64_t>(m.nV + wins, 1 << 29)))) return st;
  if ((st = grow_tri(M, (int32_t)std::min<int64_t>(m.nT + 2 * wins, 1 << 29)))) return st;
  if ((st = grow_seg(M, (int32_t)std::min<int64_t>(m.nS + wins, 1 << 28)))) return st;
  if ((st = grow_cand(M))) return st;
  int64_t pool_need = 6 * last_cand + 4096;
  if (pool_need > M->pool_cap) {
    int64_t nc = std::max<int64_t>(pool_need, (int64_t)M->pool_cap * 3 / 2);
    if (nc > (1LL << 30)) return fail(ctx, GDP_E_NOMEM, "cavity pool limit exceeded");
    if (M->arena && (st = detach(M))) return st;
    HIPCHECK(dgrow(&M->pool, M->pool_cap, nc, 0, 0, ctx->stream));
    M->pool_cap = (int32_t)nc;
  }
  return GDP_OK;
}

// Everything a captured pair of rounds depends on besides device memory.
uint64_t graph_key(gdp_mesh *M, double B2, const gdp_params *P, int64_t est) {
  DevMesh m = M->m;
  m.nV = m.nT = m.nS = m.rounds = 0;  // counts are read from device memory
  Work w = make_work(M, P, 0);
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, &m, sizeof m);
  h = fnv(h, &w, sizeof w);
  h = fnv(h, &B2, sizeof B2);
  h = fnv(h, P, sizeof *P);
  h = fnv(h, &est, sizeof est);
  h = fnv(h, &M->tiles_cap, sizeof M->tiles_cap);
  return h;
}

// Queues `pairs` x (round of parity p, round of parity p ^ 1) as replays of
// a captured graph, capturing it first if needed.
gdp_status launch_pairs(gdp_mesh *M, double B2, const gdp_params *P, int p, int pairs, int64_t est) {
  gdp_ctx *ctx = M->ctx;
  // grids are sized for a power of two at or above the estimate, and kept
  // while the estimate stays within a factor 64 below it
  int64_t cap = 256;
  while (cap < est) cap <<= 1;
  gdp_mesh::RoundGraph &g = M->graph[p];
  if (g.exec && (est > g.est || est * 64 < g.est)) {
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
  int64_t use = g.exec ? g.est : cap;
  uint64_t key = graph_key(M, B2, P, use);
  if (g.exec && g.key != key) {
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    use = cap;
    key = graph_key(M, B2, P, use);
  }
  if (!g.exec) {
    if (!M->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&M->cap_stream, hipStreamNonBlocking));
    hipStream_t user = ctx->stream;
    ctx->stream = M->cap_stream;
    HIPCHECK(hipStreamBeginCapture(M->cap_stream, hipStreamCaptureModeThreadLocal));
    gdp_status st = enqueue_round(M, B2, P, false, p, use, 0);
    if (st == GDP_OK) st = enqueue_round(M, B2, P, false, p ^ 1, use, 1);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(M->cap_stream, &graph);
    ctx->stream = user;
    if (st != GDP_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    HIPCHECK(e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHECK(e);
    g.exec = exec;
    g.key = key;
    g.est = use;
  }
  for (int i = 0; i < pairs; i++) HIPCHECK(hipGraphLaunch(g.exec, ctx->stream));
  return GDP_OK;
}

// Queues up to `rounds` rounds of the single-workgroup engine.
gdp_status launch_engine(gdp_mesh *M, double B2, const gdp_params *P, int rounds) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  if (!M->d_eng) {
    HIPCHECK(dalloc(&M->d_eng, 1));
    HIPCHECK(dalloc(&M->d_head, 1));
    HIPCHECK(hipHostMalloc((void **)&M->h_eng, sizeof(EngDesc)));
  }
  // the previous launch has finished (the host synchronised since), so the
  // pinned descriptor can be rewritten
  EngDesc &d = *M->h_eng;
  memset(&d, 0, sizeof d);
  d.m = M->m;
  d.w[0] = make_work(M, P, 0);
  d.w[1] = make_work(M, P, 1);
  d.B2 = B2;
  d.pm = P->priority_mode;
  d.K = P->cand_cap_K;
  d.f1 = P->prefilter_f1;
  d.approx_n = P->cavity_approx_n;
  d.max_rounds = P->max_rounds;
  HIPCHECK(hipMemcpyAsync(M->d_eng, &d, sizeof d, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemsetAsync(M->d_head, 0, sizeof(int32_t), s));
  M->cur_round = 0;
  {
    Prof pr(M, P_ENGINE);
    hipLaunchKernelGGL(k_engine, dim3(1), dim3(kEngBlock), 0, s, M->d_eng, 1, M->d_head, rounds);
  }
  HIPCHECK(hipGetLastError());
  return GDP_OK;
}


// ---- batched form: many meshes in one arena, one persistent launch ---------
struct Caps {
  int64_t V, T, S, W, tiles, pool, fan;
};

Caps caps_of(const gdp_mesh *M) {
  return {M->m.capV, M->m.capT, M->m.capS, M->wT, M->tiles_cap, M->pool_cap, M->fan_cap};
}

// Every device array of a mesh: f(pointer, element bytes, length, fill byte).
// The lengths match the grow_* functions for the same capacities.
template <class F>
void for_each_array(gdp_mesh *M, const Caps &c, F f) {
  const int64_t wT = c.T / 32 + 1, wS = c.S / 32 + 1;
  f((void **)&M->m.vxy, sizeof(double2), c.V, 0);
  f((void **)&M->m.vkind, 4, c.V, 0);
  f((void **)&M->m.tv, sizeof(int4), c.T, 0);
  f((void **)&M->m.tn, sizeof(int4), c.T, 0);
  f((void **)&M->m.ts, sizeof(int4), c.T, 0);
  f((void **)&M->m.sv, sizeof(int2), c.S, 0);
  f((void **)&M->m.spar, 4, c.S, 0);
  f((void **)&M->m.spend, 4, c.S, 0);
  f((void **)&M->mark, 8, c.T, 0);
  f((void **)&M->sadj, 4, 2 * c.S, 0xff);
  f((void **)&M->mflag, 4, c.S, 0);
  CandSet *sets[2] = {&M->cc, &M->mid};
  for (int k = 0; k < 2; k++) {
    const int64_t n = k == 0 ? c.T : 2 * c.S;
    CandSet &cs = *sets[k];
    f((void **)&cs.elem, 4, n, 0);
    f((void **)&cs.key, 8, n, 0);
    f((void **)&cs.p, sizeof(double2), n, 0);
    f((void **)&cs.loc, 4, n, 0);
    f((void **)&cs.state, 4, n, 0);
    f((void **)&cs.off, 4, n, 0);
    f((void **)&cs.len, 4, n, 0);
  }
  f((void **)&M->prev_cc_elem, 4, c.T, 0);
  f((void **)&M->prev_cc_key, 8, c.T, 0);
  f((void **)&M->prev_cc_p, sizeof(double2), c.T, 0);
  f((void **)&M->prev_mid_elem, 4, 2 * c.S, 0);
  f((void **)&M->w0_t, 4, wT, 0);
  f((void **)&M->win_t, 4, wT, 0);
  f((void **)&M->rank_t, 4, wT, 0);
  f((void **)&M->w0_s, 4, wS, 0);
  f((void **)&M->win_s, 4, wS, 0);
  f((void **)&M->rank_s, 4, wS, 0);
  f((void **)&M->repl, 4, 4 * c.T, 0xff);
  f((void **)&M->tstamp, 4, c.T, 0xff);
  f((void **)&M->cidx_t, 4, c.T, 0);
  f((void **)&M->hvis, 4, c.T, 0);
  f((void **)&M->hlist, 4, c.T, 0);
  f((void **)&M->cidx_s, 4, c.S, 0);
  f((void **)&M->win_ref, 4, c.W, 0);
  f((void **)&M->fbase, 4, c.W, 0);
  f((void **)&M->fcount, 4, c.W, 0);
  f((void **)&M->fan_off, 4, c.W, 0);
  f((void **)&M->big, 4, c.W, 0);
  f((void **)&M->keys, 8, c.W, 0);
  f((void **)&M->tiles_t, 4, c.tiles, 0);
  f((void **)&M->tiles_s, 4, c.tiles, 0);
  f((void **)&M->tiles_f, 4, c.tiles, 0);
  f((void **)&M->pool, 4, c.pool, 0);
  f((void **)&M->fan, sizeof(FanRec), c.fan, 0);
  f((void **)&M->d_stat, sizeof(StatLine), kStatStripes, 0);
  f((void **)&M->d_cnt, sizeof(DevCounters), 1, 0);
  f((void **)&M->d_st, sizeof(DevState), 1, 0);
  f((void **)&M->d_hist, sizeof(DevCounters), kHistCap, 0);
  f((void **)&M->rhist, 4, 256, 0);
  f((void **)&M->sel, 8, 4, 0);
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Pinned host mirrors of a mesh's control block (a batch member gets them
// when it is first refined on its own).
gdp_status alloc_host_mirrors(gdp_mesh *M) {
  gdp_ctx *ctx = M->ctx;
  if (!M->h_cnt && hipHostMalloc((void **)&M->h_cnt, sizeof(DevCounters)) != hipSuccess)
    return fail(ctx, GDP_E_NOMEM, "pinned allocation failed");
  if (!M->h_st && hipHostMalloc((void **)&M->h_st, sizeof(DevState)) != hipSuccess)
    return fail(ctx, GDP_E_NOMEM, "pinned allocation failed");
  if (!M->h_hist && hipHostMalloc((void **)&M->h_hist, sizeof(DevCounters) * kHistCap) != hipSuccess)
    return fail(ctx, GDP_E_NOMEM, "pinned allocation failed");
  return GDP_OK;
}

// A batch member that is refined or overwritten on its own first moves its
// arrays out of the shared arena into allocations of its own.
gdp_status detach(gdp_mesh *M) {
  if (!M->arena) return GDP_OK;
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  std::vector<void **> slot;
  std::vector<size_t> bytes;
  for_each_array(M, caps_of(M), [&](void **pp, size_t es, int64_t n, int) {
    slot.push_back(pp);
    bytes.push_back(es * (size_t)std::max<int64_t>(n, 1));
  });
  std::vector<void *> fresh(slot.size(), nullptr);
  for (size_t i = 0; i < slot.size(); i++) {
    if (hipMalloc(&fresh[i], bytes[i]) != hipSuccess) {
      for (void *q : fresh)
        if (q) (void)hipFree(q);
      return fail(ctx, GDP_E_NOMEM, "device allocation failed");
    }
    HIPCHECK(hipMemcpyAsync(fresh[i], *slot[i], bytes[i], hipMemcpyDeviceToDevice, s));
  }
  HIPCHECK(hipStreamSynchronize(s));
  for (size_t i = 0; i < slot.size(); i++) *slot[i] = fresh[i];
  arena_release(M->arena);
  M->arena = nullptr;
  return alloc_host_mirrors(M);
}

gdp_status status_of_halt(gdp_ctx *ctx, const DevState &d, const DevCounters &c) {
  switch (d.halt) {
    case kHaltDone: return GDP_OK;
    case kHaltCap: return fail(ctx, GDP_E_NOTERM, "round cap reached");
    case kHaltStall: return fail(ctx, GDP_E_STALL, "round had candidates but inserted nothing");
    case kHaltError:
      if (c.err & kErrWalk) return fail(ctx, GDP_E_WALK, "locate walk exceeded its step cap");
      if (c.err & kErrInput) return fail(ctx, GDP_E_INPUT, "a walk left the mesh through a hull edge that is not a subsegment");
      return fail(ctx, GDP_E_CAVITY, "cavity error");
    default: return fail(ctx, GDP_E_DEVICE, "mesh did not finish");
  }
}

// ---- shared rounds: the rounds of several meshes in one launch per phase ----
// (Rule 4 of Section 2.)  Used by the serving form for its active jobs and
// by the batched form for its largest meshes.
struct GangItem {
  gdp_mesh *M;
  const gdp_params *P;
  double B2;
  int64_t last_cand;  // candidates of the last completed round (sizes the grids)
  int aborts;         // consecutive abandoned rounds
  bool full;          // its next round is its first (a full collection)
  void *tag;          // the owner's handle
};

// Device and pinned buffers of a shared-rounds runner (up to cap meshes).
struct GangBufs {
  GangDesc *d_desc = nullptr, *h_desc = nullptr;
  int32_t *d_status = nullptr, *h_status = nullptr;
  int stride_words = 0;  // words of one mesh's status record
  int cap = 0;
};
constexpr int kGangRounds = 2;     // default rounds between two host reads of the meshes' states
constexpr int kGangRoundsMax = 8;

bool gang_bufs_alloc(GangBufs &B, int cap) {
  B.cap = cap;
  B.stride_words = (int)((sizeof(DevState) + (1 + kGangRoundsMax) * sizeof(DevCounters)) / 4);
  return dalloc(&B.d_desc, cap) == hipSuccess &&
         hipHostMalloc((void **)&B.h_desc, sizeof(GangDesc) * cap) == hipSuccess &&
         dalloc(&B.d_status, (size_t)B.stride_words * cap) == hipSuccess &&
         hipHostMalloc((void **)&B.h_status, sizeof(int32_t) * B.stride_words * cap) == hipSuccess;
}

void gang_bufs_free(GangBufs &B) {
  if (B.d_desc) (void)hipFree(B.d_desc);
  if (B.d_status) (void)hipFree(B.d_status);
  if (B.h_desc) (void)hipHostFree(B.h_desc);
  if (B.h_status) (void)hipHostFree(B.h_status);
  B = GangBufs();
}

GangItem gang_item(gdp_mesh *M, const gdp_params *P, double B2, void *tag) {
  return GangItem{M, P, B2, (int64_t)M->m.nT + M->m.nS, 0, true, tag};
}

GangDesc gang_desc(gdp_mesh *M, const gdp_params *P, double B2) {
  GangDesc g;
  memset(&g, 0, sizeof g);
  EngDesc &d = g.e;
  d.m = M->m;
  d.w[0] = make_work(M, P, 0);
  d.w[1] = make_work(M, P, 1);
  // one workgroup runs the device-memory cavity path per mesh and launch
  d.w[0].huge_ok = d.w[1].huge_ok = 1;
  d.B2 = B2;
  d.pm = P->priority_mode;
  d.K = P->cand_cap_K;
  d.f1 = P->prefilter_f1;
  d.approx_n = P->cavity_approx_n;
  d.max_rounds = P->max_rounds;
  g.js = ScanJob{(const int32_t *)M->win_s, M->rank_s, &M->d_st->wS, M->tiles_s, &M->d_cnt->nwin_mid, 1};
  g.jt = ScanJob{(const int32_t *)M->win_t, M->rank_t, &M->d_st->wT, M->tiles_t, &M->d_cnt->nwin_cc, 1};
  g.jf = ScanJob{M->fcount, M->fbase, &M->d_cnt->nwin1, M->tiles_f, &M->d_cnt->fan_total, 0};
  return g;
}

// One round of every job in the descriptors (grids sized for the largest).
void gang_round(hipStream_t s, const GangDesc *D, unsigned n, int64_t max_full, int64_t max_est,
                int64_t max_ncand, int64_t max_words, bool any_cap, bool any_pre) {
  const int bs = 256;
  const unsigned gc = std::max(stride_grid(max_full, bs), stride_grid(3 * max_est, bs));
  hipLaunchKernelGGL(kg_collect, dim3(gc, n), dim3(bs), 0, s, D);
  hipLaunchKernelGGL(kg_pending, dim3(stride_grid(max_est / 4, bs), n), dim3(bs), 0, s, D);
  hipLaunchKernelGGL(kg_gate, dim3(1, n), dim3(256), 0, s, D);
  if (any_cap) {
    hipLaunchKernelGGL(kg_gather_keys, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
    const unsigned g = std::min<unsigned>(grid_for(max_ncand, 256), 1024);
    for (int shift = 56; shift >= 0; shift -= 8) {
      hipLaunchKernelGGL(kg_radix_hist, dim3(g, n), dim3(256), 0, s, D, shift);
      hipLaunchKernelGGL(kg_radix_pick, dim3(1, n), dim3(256), 0, s, D, shift);
    }
    hipLaunchKernelGGL(kg_apply_cap, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  }
  hipLaunchKernelGGL(kg_locate, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  if (any_pre)
    for (int mode = 0; mode < 6; mode++)
      hipLaunchKernelGGL(kg_prefilter, dim3(stride_grid(max_ncand, 128), n), dim3(128), 0, s, D, mode);
  hipLaunchKernelGGL(kg_cavity<1>, dim3(stride_grid(max_ncand, kCavBlockSize), n), dim3(kCavBlockSize), 0, s, D);
  hipLaunchKernelGGL(kg_cavity_big, dim3(256, n), dim3(kBigBlockSize), 0, s, D, 0);
  hipLaunchKernelGGL(kg_cavity_huge, dim3(1, n), dim3(kHugeBlock), 0, s, D, 0);
  hipLaunchKernelGGL(kg_cavity<0>, dim3(stride_grid(max_ncand / 4, kCavBlockSize), n), dim3(kCavBlockSize), 0, s, D);
  hipLaunchKernelGGL(kg_cavity_big, dim3(256, n), dim3(kBigBlockSize), 0, s, D, 1);
  hipLaunchKernelGGL(kg_cavity_huge, dim3(1, n), dim3(kHugeBlock), 0, s, D, 1);
  hipLaunchKernelGGL(kg_own, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  hipLaunchKernelGGL(kg_dep, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  const int64_t tiles_w = std::max<int64_t>(1, (max_words + kScanTileSize - 1) / kScanTileSize);
  hipLaunchKernelGGL(kg_scan_tiles, dim3((unsigned)std::min<int64_t>(2 * tiles_w, 2048), n), dim3(256), 0, s, D, 0);
  hipLaunchKernelGGL(kg_scan_sums, dim3(2, n), dim3(256), 0, s, D, 0);
  hipLaunchKernelGGL(kg_winners, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  const int64_t tiles_f = std::max<int64_t>(1, (max_ncand + 1 + kScanTileSize - 1) / kScanTileSize);
  hipLaunchKernelGGL(kg_scan_tiles, dim3((unsigned)std::min<int64_t>(tiles_f, 2048), n), dim3(256), 0, s, D, 1);
  hipLaunchKernelGGL(kg_scan_sums, dim3(1, n), dim3(256), 0, s, D, 1);
  hipLaunchKernelGGL(kg_record, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  hipLaunchKernelGGL(kg_write, dim3(stride_grid(max_ncand, bs), n), dim3(bs), 0, s, D);
  hipLaunchKernelGGL(kg_finish, dim3(std::min(stride_grid(max_ncand, bs), 256u), n), dim3(bs), 0, s, D);
}

// One group of R shared rounds of every active mesh (at most B.cap), then
// one read of all their states.  Meshes whose refinement ended (done, round
// cap, error) move to `finished` with their status; a mesh whose round found
// a buffer short has that buffer grown and runs the round again, as in the
// plain loop, so each mesh is the plain loop's.  Returns an error only if
// the group itself could not run (then every mesh is finished with it).
void gang_group(gdp_ctx *ctx, GangBufs &B, std::vector<GangItem> &active, int R,
                std::vector<std::pair<GangItem, gdp_status>> &finished) {
  hipStream_t s = ctx->stream;
  const int ns = (int)(sizeof(DevState) / 4), nc = (int)(sizeof(DevCounters) / 4);
  int64_t max_full = 0, max_est = 1, max_ncand = 1, max_words = 1;
  bool any_cap = false, any_pre = false;
  for (size_t q = 0; q < active.size();) {
    GangItem &A = active[q];
    gdp_mesh *M = A.M;
    gdp_status st = reserve_group(M, A.last_cand, R);
    if (st != GDP_OK) {
      finished.push_back({A, st});
      active.erase(active.begin() + q);
      continue;
    }
    const DevMesh &m = M->m;
    // grids sized for the largest mesh's work this round (a full collection
    // for a mesh's first round, the candidate lists after it)
    if (A.full) max_full = std::max<int64_t>(max_full, std::max(m.nT, m.nS));
    else max_est = std::max<int64_t>(max_est, A.last_cand);
    max_ncand = std::max<int64_t>(max_ncand, A.full ? (int64_t)m.nT + m.nS : 2 * A.last_cand);
    max_words = std::max<int64_t>(max_words, std::max(words(m.capS), words(m.capT)));
    any_cap = any_cap || A.P->cand_cap_K > 0;
    any_pre = any_pre || A.P->prefilter_f1 || A.P->cavity_approx_n > 0;
    B.h_desc[q] = gang_desc(M, A.P, A.B2);
    q++;
  }
  const unsigned n = (unsigned)active.size();
  if (n == 0) return;
  bool ok = hipMemcpyAsync(B.d_desc, B.h_desc, sizeof(GangDesc) * n, hipMemcpyHostToDevice, s) == hipSuccess;
  for (int r = 0; ok && r < R; r++)
    gang_round(s, B.d_desc, n, max_full, max_est, max_ncand, max_words, any_cap, any_pre);
  if (ok) {
    hipLaunchKernelGGL(kg_status, dim3(1, n), dim3(256), 0, s, B.d_desc, R, B.d_status, B.stride_words);
    ok = hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(B.h_status, B.d_status, sizeof(int32_t) * B.stride_words * n, hipMemcpyDeviceToHost, s) ==
             hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
  }
  std::vector<GangItem> keep;
  for (unsigned q = 0; q < n; q++) {
    GangItem A = active[q];
    gdp_mesh *M = A.M;
    if (!ok) {
      finished.push_back({A, fail(ctx, GDP_E_DEVICE, "shared round launch failed")});
      continue;
    }
    const int32_t *rec = B.h_status + (size_t)q * B.stride_words;
    DevState d;
    DevCounters c;
    memcpy(&d, rec, sizeof d);
    memcpy(&c, rec + ns, sizeof c);
    const DevCounters *h = (const DevCounters *)(rec + ns + nc);
    const int done = std::min(d.nhist, R);
    for (int i = 0; i < done; i++) {
      M->stats.push_back(round_stats_of(h[i], A.P));
      A.last_cand = (int64_t)h[i].ncc + h[i].nmk;
    }
    M->m.nV = d.nV; M->m.nT = d.nT; M->m.nS = d.nS; M->m.rounds = d.rounds;
    M->serial = d.serial;
    if (done > 0) {
      A.aborts = 0;
      A.full = false;
    }
    gdp_status st = GDP_OK;
    bool over = false;
    if (d.halt == kHaltAbort) {
      // nothing was written: grow and run the same round again
      if (++A.aborts > 16) {
        st = fail(ctx, GDP_E_NOMEM, "round keeps exceeding its buffers");
        over = true;
      } else if ((st = grow_after_abort(M, c, d.full ? 0 : d.prev_fan)) != GDP_OK) {
        over = true;
      } else if (hipMemsetAsync(M->d_cnt, 0, sizeof(DevCounters), s) != hipSuccess ||
                 hipMemsetAsync(M->d_stat, 0, sizeof(StatLine) * kStatStripes, s) != hipSuccess) {
        st = fail(ctx, GDP_E_DEVICE, "reset after an abandoned round failed");
        over = true;
      }
    } else if (d.halt != 0) {
      st = status_of_halt(ctx, d, c);
      over = true;
    }
    if (!over && hipMemsetAsync(&M->d_st->halt, 0, 2 * sizeof(int32_t), s) != hipSuccess) {  // halt, nhist
      st = fail(ctx, GDP_E_DEVICE, "round state reset failed");
      over = true;
    }
    if (over) finished.push_back({A, st});
    else keep.push_back(A);
  }
  active.swap(keep);
}

constexpr size_t kBatchGangMax = 256;  // batched meshes in one group of shared rounds, at most
constexpr int32_t kBatchLine1DevThreads = 8;  // device Line-1 builders of a batch, each on its own stream

// The checks of the device builder's caller (gdp_mesh_create_device).
gdp_status check_pslg_for_device(const gdp_pslg *pslg, std::string &e) {
  const int32_t nv = pslg->n_vertices, ns = pslg->n_segments;
  if (nv < 3 || !pslg->xy || ns < 0 || (ns > 0 && !pslg->seg)) { e = "bad arguments"; return GDP_E_ARG; }
  if (nv > (1 << 28) - 8) { e = "mesh too large"; return GDP_E_NOMEM; }
  for (int64_t i = 0; i < 2 * (int64_t)nv; i++) {
    const double a = std::fabs(pslg->xy[i]);
    if (!std::isfinite(pslg->xy[i]) || a > 0x1p20 || (a != 0.0 && a < 0x1p-100)) {
      e = "coordinate not finite, or nonzero with magnitude outside [2^-100, 2^20]";
      return GDP_E_INPUT;
    }
  }
  for (int32_t k = 0; k < ns; k++) {
    const int32_t a = pslg->seg[2 * k], b = pslg->seg[2 * k + 1];
    if (a < 0 || b < 0 || a >= nv || b >= nv || a == b) {
      e = "segment endpoint out of range or zero length";
      return GDP_E_INPUT;
    }
  }
  return GDP_OK;
}

// Line 1 of one batched input by the device builder, into its arena slot M
// (zeroed and filled beforehand): the input goes up, the canonical CDT is
// written in place, then the mesh's device state.  nT receives the
// triangle count.
int batch_line1_device(hipStream_t st, DevCdtWork &ws, const gdp_pslg &q, gdp_mesh *M, int32_t &nT,
                       std::string &err) {
  const int32_t nv = q.n_vertices, ns = q.n_segments;
  std::vector<int32_t> spar(ns);
  for (int32_t k = 0; k < ns; k++) spar[k] = k;
  if (hipMemcpyAsync(M->m.vxy, q.xy, sizeof(double) * 2 * nv, hipMemcpyHostToDevice, st) != hipSuccess ||
      (ns > 0 && hipMemcpyAsync(M->m.sv, q.seg, sizeof(int32_t) * 2 * ns, hipMemcpyHostToDevice, st) != hipSuccess) ||
      (ns > 0 && hipMemcpyAsync(M->m.spar, spar.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st) != hipSuccess)) {
    err = "upload failed";
    return GDP_E_DEVICE;
  }
  DevCdtStats cs;
  int32_t nt = 0;
  const int rc = dev_cdt_build(st, nv, M->m.vxy, ns, M->m.sv, M->m.tv, M->m.tn, M->m.ts, M->m.capT, &nt, &cs, err, &ws);
  if (rc != GDP_OK) return rc;
  M->cdt_rounds[0] = cs.dt_rounds;
  M->cdt_rounds[1] = cs.seg_rounds;
  DevState ds;
  memset(&ds, 0, sizeof ds);
  ds.nV = nv; ds.nT = nt; ds.nS = ns;
  ds.wT = words(nt); ds.wS = words(ns);
  ds.full = 1;
  if (hipMemcpyAsync(M->d_st, &ds, sizeof ds, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {  // ds and spar are locals
    err = "upload failed";
    return GDP_E_DEVICE;
  }
  nT = nt;
  return GDP_OK;
}
// The batched form (Algorithm 1 for many independent PSLGs): Line 1 on the
// host for every input (in parallel), one arena holding every mesh and its
// workspace, then all of Lines 2-9 in one launch of the single-workgroup
// engine whose workgroups take meshes from a queue, largest first.  A mesh
// whose estimated room runs out is refined again on its own (same result).
gdp_status refine_batch(gdp_ctx *ctx, const gdp_pslg *pslgs, const double *bsq, const gdp_params *P,
                        int32_t count, gdp_mesh **outs, gdp_status *status, double *elapsed_ms) {
  hipStream_t s = ctx->stream;
  for (int32_t i = 0; i < count; i++) {
    outs[i] = nullptr;
    if (status) status[i] = GDP_OK;
  }
  // Line 1.  Inputs with at least batch_line1_device_min_v vertices are
  // triangulated by the device builder (threads with a stream each, writing
  // into the arena), the others on host threads, both at once.  The arena is
  // sized before Line 1 from the input counts (a CDT of V vertices has at
  // most 2V triangles and keeps the input segments), with the device-built
  // meshes last in every array region so that the host-built ones are
  // uploaded as one prefix of each region.
  const int64_t dev_min = P->batch_line1_device_min_v;
  std::vector<int> rc(count, GDP_OK);
  std::vector<std::string> errs(count);
  std::vector<int32_t> ok, ok_dev;
  for (int32_t i = 0; i < count; i++) {
    const gdp_pslg &q = pslgs[i];
    if (q.n_vertices < 3 || !q.xy || q.n_segments < 0 || (q.n_segments > 0 && !q.seg)) {
      rc[i] = GDP_E_ARG;
      errs[i] = "bad arguments";
    } else if (dev_min > 0 && q.n_vertices >= dev_min) {
      rc[i] = check_pslg_for_device(&q, errs[i]);
      if (rc[i] == GDP_OK) ok_dev.push_back(i);
    } else {
      ok.push_back(i);
    }
    if (rc[i] != GDP_OK && status) status[i] = (gdp_status)rc[i];
  }
  const int32_t n_host = (int32_t)ok.size();
  ok.insert(ok.end(), ok_dev.begin(), ok_dev.end());
  if (elapsed_ms) *elapsed_ms = 0.0;
  if (ok.empty()) return GDP_OK;
  // capacities: room for the refined mesh (about 2.5x the input vertices at
  // B = sqrt(2), more for tiny inputs); a mesh that outgrows it falls back
  const int32_t n = (int32_t)ok.size();
  std::vector<gdp_mesh *> mesh(n);
  std::vector<Caps> caps(n);
  std::vector<int32_t> nT0(n, 0);  // triangles of each initial CDT
  gdp_arena *arena = new gdp_arena();
  for (int32_t k = 0; k < n; k++) {
    const int64_t nv = pslgs[ok[k]].n_vertices, ns = pslgs[ok[k]].n_segments;
    Caps c;
    c.V = 3 * nv + 256;
    c.T = std::max<int64_t>(2 * c.V + 256, 2 * nv);
    c.S = 16 * ns + 64;
    c.W = c.T + 2 * c.S + 2;
    c.tiles = c.W / kScanTileSize + 2;
    c.pool = 2 * c.T + 4096;
    c.fan = 2 * c.T + 4096;
    caps[k] = c;
    gdp_mesh *M = new gdp_mesh();
    M->ctx = ctx;
    M->arena = arena;
    arena->refs++;
    mesh[k] = M;
  }
  // arena: one region per array kind, each mesh's array 256-byte aligned in it
  std::vector<size_t> region;
  for (int32_t k = 0; k < n; k++) {
    size_t j = 0;
    for_each_array(mesh[k], caps[k], [&](void **, size_t es, int64_t len, int) {
      if (region.size() <= j) region.push_back(0);
      region[j++] += align256(es * (size_t)std::max<int64_t>(len, 1));
    });
  }
  std::vector<size_t> region_off(region.size());
  size_t total = 0;
  for (size_t j = 0; j < region.size(); j++) {
    region_off[j] = total;
    total += region[j];
  }
  auto bail = [&](gdp_status st) {
    for (gdp_mesh *M : mesh) {
      if (!M) continue;
      M->arena = nullptr;
      delete M;
    }
    if (arena->base) (void)hipFree(arena->base);
    delete arena;
    return st;
  };
  if (hipMalloc(&arena->base, total) != hipSuccess) return bail(fail(ctx, GDP_E_NOMEM, "batch arena allocation failed"));
  char *base = (char *)arena->base;
  std::vector<size_t> run(region.size(), 0);
  std::vector<int> fills(region.size(), 0);
  std::vector<std::vector<size_t>> off(n, std::vector<size_t>(region.size()));
  for (int32_t k = 0; k < n; k++) {
    size_t j = 0;
    for_each_array(mesh[k], caps[k], [&](void **pp, size_t es, int64_t len, int fill) {
      off[k][j] = run[j];
      *pp = base + region_off[j] + run[j];
      fills[j] = fill;
      run[j] += align256(es * (size_t)std::max<int64_t>(len, 1));
      j++;
    });
    const Caps &c = caps[k];
    gdp_mesh *M = mesh[k];
    M->m.capV = (int32_t)c.V; M->m.capT = (int32_t)c.T; M->m.capS = (int32_t)c.S;
    M->wT = (int32_t)c.W; M->tiles_cap = (int32_t)c.tiles;
    M->pool_cap = (int32_t)c.pool; M->fan_cap = (int32_t)c.fan;
  }
  if (hipMemsetAsync(base, 0, total, s) != hipSuccess) return bail(fail(ctx, GDP_E_DEVICE, "arena fill failed"));
  for (size_t j = 0; j < region.size(); j++)
    if (fills[j] && hipMemsetAsync(base + region_off[j], fills[j], region[j], s) != hipSuccess)
      return bail(fail(ctx, GDP_E_DEVICE, "arena fill failed"));
  if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(ctx, GDP_E_DEVICE, "arena fill failed"));
  // the host-built meshes go up packed: per mesh its points, the three
  // triangle arrays (room for the 2V triangles a CDT can have), segments,
  // segment parents and device state, each chunk 16-byte aligned, written by
  // the thread that built the mesh; one copy, then a device scatter into the
  // arena (the arena's room beyond each mesh is already zero)
  enum { C_VXY, C_TV, C_TN, C_TS, C_SV, C_SPAR, C_ST, C_N };
  std::vector<std::array<int64_t, C_N>> pk(n_host);
  int64_t pk_total = 0;
  for (int32_t k = 0; k < n_host; k++) {
    const int64_t nv = pslgs[ok[k]].n_vertices, ns = pslgs[ok[k]].n_segments;
    const int64_t sz[C_N] = {16 * nv, 32 * nv, 32 * nv, 32 * nv, 8 * ns, 4 * ns, (int64_t)sizeof(DevState)};
    for (int c = 0; c < C_N; c++) {
      pk[k][c] = pk_total;
      pk_total += (sz[c] + 15) & ~(int64_t)15;
    }
  }
  std::unique_ptr<char[]> packed(new (std::nothrow) char[std::max<int64_t>(pk_total, 16)]);
  if (!packed) return bail(fail(ctx, GDP_E_NOMEM, "batch staging allocation failed"));
  auto pack = [&](int32_t k, const HostMesh &h) {
    char *b = packed.get();
    memcpy(b + pk[k][C_VXY], h.xy.data(), sizeof(double) * 2 * h.nV);
    int4 *tv = (int4 *)(b + pk[k][C_TV]), *tn = (int4 *)(b + pk[k][C_TN]), *ts = (int4 *)(b + pk[k][C_TS]);
    for (int32_t t = 0; t < h.nT; t++) {
      const int w = (h.ts[3 * t] >= 0 ? 1 : 0) | (h.ts[3 * t + 1] >= 0 ? 2 : 0) | (h.ts[3 * t + 2] >= 0 ? 4 : 0);
      tv[t] = make_int4(h.tv[3 * t], h.tv[3 * t + 1], h.tv[3 * t + 2], w);
      tn[t] = make_int4(h.tn[3 * t], h.tn[3 * t + 1], h.tn[3 * t + 2], 0);
      ts[t] = make_int4(h.ts[3 * t], h.ts[3 * t + 1], h.ts[3 * t + 2], 0);
    }
    if (h.nS) {
      memcpy(b + pk[k][C_SV], h.sv.data(), sizeof(int32_t) * 2 * h.nS);
      memcpy(b + pk[k][C_SPAR], h.sparent.data(), sizeof(int32_t) * h.nS);
    }
    DevState ds;
    memset(&ds, 0, sizeof ds);
    ds.nV = h.nV; ds.nT = h.nT; ds.nS = h.nS;
    ds.wT = words(h.nT); ds.wS = words(h.nS);
    ds.full = 1;
    memcpy(b + pk[k][C_ST], &ds, sizeof ds);
  };
  {
    std::atomic<int32_t> next_h(0), next_d(0);
    const int32_t n_dev = n - n_host;
    unsigned nth = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16));
    nth = std::min<unsigned>(nth, (unsigned)std::max(n_host, 1));
    const unsigned ndt = (unsigned)std::min<int32_t>(n_dev, kBatchLine1DevThreads);
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth && n_host > 0; t++)
      pool.emplace_back([&]() {
        for (int32_t k; (k = next_h.fetch_add(1)) < n_host;) {
          const int32_t i = ok[k];
          HostMesh h;
          rc[i] = host_cdt_build(pslgs[i].n_vertices, pslgs[i].xy, pslgs[i].n_segments, pslgs[i].seg, h, errs[i]);
          if (rc[i] == GDP_OK && (h.nV != pslgs[i].n_vertices || h.nS != pslgs[i].n_segments ||
                                  (int64_t)h.nT > 2 * (int64_t)h.nV)) {
            rc[i] = GDP_E_DEVICE;
            errs[i] = "initial CDT outside the batch's room";
          }
          if (rc[i] == GDP_OK) {
            nT0[k] = h.nT;
            pack(k, h);
          }
        }
      });
    for (unsigned t = 0; t < ndt; t++)
      pool.emplace_back([&]() {
        (void)hipSetDevice(ctx->device);
        hipStream_t ds = nullptr;
        DevCdtWork ws;
        if (hipStreamCreateWithFlags(&ds, hipStreamNonBlocking) != hipSuccess) ds = nullptr;
        for (int32_t q; (q = next_d.fetch_add(1)) < n_dev;) {
          const int32_t k = n_host + q, i = ok[k];
          if (!ds) {
            rc[i] = GDP_E_DEVICE;
            errs[i] = "stream creation failed";
            continue;
          }
          rc[i] = batch_line1_device(ds, ws, pslgs[i], mesh[k], nT0[k], errs[i]);
        }
        if (ds) {
          (void)hipStreamSynchronize(ds);
          (void)hipStreamDestroy(ds);
        }
        dev_cdt_work_free(ws);
      });
    for (auto &th : pool) th.join();
  }
  // meshes whose Line 1 failed leave the batch (their arena room stays unused)
  std::vector<bool> live(n, true);
  for (int32_t k = 0; k < n; k++) {
    const int32_t i = ok[k];
    if (rc[i] == GDP_OK) continue;
    live[k] = false;
    if (status) status[i] = (gdp_status)rc[i];
    arena->refs--;
    mesh[k]->arena = nullptr;
    delete mesh[k];
    mesh[k] = nullptr;
  }
  {
    std::vector<CopyEnt> ents;
    for (int32_t k = 0; k < n_host; k++) {
      if (!live[k]) continue;
      const gdp_mesh *M = mesh[k];
      const int64_t nv = pslgs[ok[k]].n_vertices, ns = pslgs[ok[k]].n_segments, nt = nT0[k];
      int32_t *dst[C_N] = {(int32_t *)M->m.vxy, (int32_t *)M->m.tv, (int32_t *)M->m.tn, (int32_t *)M->m.ts,
                           (int32_t *)M->m.sv, M->m.spar, (int32_t *)M->d_st};
      const int64_t sz[C_N] = {16 * nv, 16 * nt, 16 * nt, 16 * nt, 8 * ns, 4 * ns, (int64_t)sizeof(DevState)};
      for (int c = 0; c < C_N; c++)
        if (sz[c] > 0) ents.push_back(CopyEnt{pk[k][c], dst[c], sz[c]});
    }
    if (!ents.empty()) {
      int32_t *d_pk = nullptr;
      CopyEnt *d_ents = nullptr;
      bool up = hipMalloc(&d_pk, pk_total) == hipSuccess &&
                hipMalloc(&d_ents, sizeof(CopyEnt) * ents.size()) == hipSuccess &&
                hipMemcpy(d_pk, packed.get(), pk_total, hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(d_ents, ents.data(), sizeof(CopyEnt) * ents.size(), hipMemcpyHostToDevice) == hipSuccess;
      if (up) {
        hipLaunchKernelGGL(k_scatter_copy, dim3((unsigned)std::min<size_t>(ents.size(), 8192)), dim3(256), 0, s,
                           d_pk, d_ents, (int)ents.size());
        up = hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
      }
      if (d_pk) (void)hipFree(d_pk);
      if (d_ents) (void)hipFree(d_ents);
      if (!up) return bail(fail(ctx, GDP_E_DEVICE, "batch upload failed"));
    }
    packed.reset();
  }
  const int R_ST = (int)region.size() - 4;  // d_st (then d_hist, rhist, sel)
  for (int32_t k = 0; k < n; k++) {
    if (!live[k]) continue;
    gdp_mesh *M = mesh[k];
    const int32_t nv = pslgs[ok[k]].n_vertices, ns = pslgs[ok[k]].n_segments;
    M->m.nV = nv; M->m.nT = nT0[k]; M->m.nS = ns;
    M->m.n_input_v = nv; M->m.n_input_s = ns; M->m.rounds = 0;
  }
  // Meshes with more input vertices than the split run in shared rounds
  // (every phase one launch for all of them, the whole chip per round), the
  // others one workgroup each in the engine launch.  Either way each mesh is
  // the plain loop's.
  const int64_t split = P->batch_engine_max_v > 0 ? P->batch_engine_max_v : (int64_t)1 << 40;
  std::vector<int32_t> order, gang_k;
  for (int32_t k = 0; k < n; k++)
    if (live[k]) (pslgs[ok[k]].n_vertices > split ? gang_k : order).push_back(k);
  // Queue order.  Largest first keeps the makespan short, but the engines on
  // one XCD share its 4 MB L2, and large meshes side by side evict each
  // other's working sets (measured: each runs many times slower than alone).
  // So the largest quarter, in size order, is spread out: every fourth entry,
  // the others (largest first) in between.  The order changes no mesh.
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return nT0[a] > nT0[b]; });
  const int32_t ne = (int32_t)order.size();
  {
    const int32_t n = ne;
    const int32_t nbig = (n + 3) / 4;
    std::vector<int32_t> spread;
    spread.reserve(n);
    int32_t bi = 0, ri = nbig;
    while ((int32_t)spread.size() < n) {
      const bool take_big = bi < nbig && (spread.size() % 4 == 0 || ri >= n);
      spread.push_back(take_big ? order[bi++] : order[ri++]);
    }
    order.swap(spread);
  }
  std::vector<EngDesc> desc(std::max(ne, 1));
  for (int32_t q = 0; q < ne; q++) {
    const int32_t k = order[q];
    EngDesc &d = desc[q];
    memset(&d, 0, sizeof d);
    d.m = mesh[k]->m;
    d.w[0] = make_work(mesh[k], P, 0);
    d.w[1] = make_work(mesh[k], P, 1);
    d.B2 = bsq[ok[k]];
    d.pm = P->priority_mode;
    d.K = P->cand_cap_K;
    d.f1 = P->prefilter_f1;
    d.approx_n = P->cavity_approx_n;
    d.max_rounds = P->max_rounds;
  }
  EngDesc *d_desc = nullptr;
  int32_t *d_head = nullptr;
  GangBufs gb;
  const int gcap = (int)std::min<size_t>(gang_k.size(), kBatchGangMax);
  if (dalloc(&d_desc, std::max(ne, 1)) != hipSuccess || dalloc(&d_head, 1) != hipSuccess ||
      (gcap > 0 && !gang_bufs_alloc(gb, gcap))) {
    if (d_desc) (void)hipFree(d_desc);
    if (d_head) (void)hipFree(d_head);
    gang_bufs_free(gb);
    return bail(fail(ctx, GDP_E_NOMEM, "descriptor allocation failed"));
  }
  auto free_tmp = [&]() {
    (void)hipFree(d_desc);
    (void)hipFree(d_head);
    gang_bufs_free(gb);
  };
  int cus = 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool ok_run = (ne == 0 || hipMemcpy(d_desc, desc.data(), sizeof(EngDesc) * ne, hipMemcpyHostToDevice) == hipSuccess) &&
                hipMemsetAsync(d_head, 0, sizeof(int32_t), s) == hipSuccess && hipEventCreate(&ev0) == hipSuccess &&
                hipEventCreate(&ev1) == hipSuccess && hipEventRecord(ev0, s) == hipSuccess;
  // the large meshes first, in shared rounds over the whole chip (largest
  // first, at most kBatchGangMax at a time), then the engine launch
  std::vector<gdp_status> gang_st(n, GDP_OK);
  if (ok_run && !gang_k.empty()) {
    std::stable_sort(gang_k.begin(), gang_k.end(), [&](int32_t a, int32_t b) { return nT0[a] > nT0[b]; });
    std::vector<GangItem> active;
    size_t next = 0;
    const int R = P->rounds_per_sync > 0 ? std::min(P->rounds_per_sync, kGangRoundsMax) : kGangRounds;
    while (next < gang_k.size() || !active.empty()) {
      while (next < gang_k.size() && (int)active.size() < gcap) {
        const int32_t k = gang_k[next++];
        active.push_back(gang_item(mesh[k], P, bsq[ok[k]], (void *)(intptr_t)k));
      }
      std::vector<std::pair<GangItem, gdp_status>> finished;
      gang_group(ctx, gb, active, R, finished);
      for (auto &f : finished) gang_st[(int32_t)(intptr_t)f.first.tag] = f.second;
    }
  }
  if (ok_run && ne > 0) {
    hipLaunchKernelGGL(k_engine, dim3((unsigned)std::min(ne, cus)), dim3(kEngBlock), 0, s, d_desc, ne, d_head,
                       1 << 30);
    ok_run = hipGetLastError() == hipSuccess;
  }
  ok_run = ok_run && hipEventRecord(ev1, s) == hipSuccess && hipEventSynchronize(ev1) == hipSuccess;
  float ms = 0.f;
  if (ok_run) (void)hipEventElapsedTime(&ms, ev0, ev1);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  free_tmp();
  if (!ok_run) return bail(fail(ctx, GDP_E_DEVICE, "batch launch failed"));
  if (elapsed_ms) *elapsed_ms = ms;
  // the engine's: device states, counters and per-round histories
  const int R_CNT = R_ST - 1;  // d_cnt precedes d_st
  std::vector<char> hst(region[R_ST]), hcnt(region[R_CNT]), hhist(region[R_ST + 1]);
  if (ne > 0 &&
      (hipMemcpy(hst.data(), base + region_off[R_ST], region[R_ST], hipMemcpyDeviceToHost) != hipSuccess ||
       hipMemcpy(hcnt.data(), base + region_off[R_CNT], region[R_CNT], hipMemcpyDeviceToHost) != hipSuccess ||
       hipMemcpy(hhist.data(), base + region_off[R_ST + 1], region[R_ST + 1], hipMemcpyDeviceToHost) != hipSuccess))
    return bail(fail(ctx, GDP_E_DEVICE, "batch download failed"));
  for (int32_t k : order) {
    gdp_mesh *M = mesh[k];
    const int32_t i = ok[k];
    DevState d;
    DevCounters c;
    memcpy(&d, hst.data() + off[k][R_ST], sizeof d);
    memcpy(&c, hcnt.data() + off[k][R_CNT], sizeof c);
    M->m.nV = d.nV; M->m.nT = d.nT; M->m.nS = d.nS; M->m.rounds = d.rounds;
    M->serial = d.serial;
    M->last_ms = ms;
    const DevCounters *h = (const DevCounters *)(hhist.data() + off[k][R_ST + 1]);
    for (int r = 0; r < std::min(d.nhist, kHistCap); r++) M->stats.push_back(round_stats_of(h[r], P));
    if (d.halt == kHaltAbort) {
      // out of its estimated room: the same refinement on its own
      gdp_mesh_free(M);
      mesh[k] = nullptr;
      gdp_status r = gdp_refine(ctx, &pslgs[i], bsq[i], P, &outs[i]);
      if (status) status[i] = r;
      continue;
    }
    gdp_status r = status_of_halt(ctx, d, c);
    if (status) status[i] = r;
    if (r == GDP_OK || r == GDP_E_NOTERM) {
      outs[i] = M;
    } else {
      gdp_mesh_free(M);
      mesh[k] = nullptr;
    }
  }
  // the shared-rounds meshes are complete
  for (int32_t k : gang_k) {
    gdp_mesh *M = mesh[k];
    const int32_t i = ok[k];
    M->last_ms = ms;
    gdp_status r = gang_st[k];
    if (status) status[i] = r;
    if (r == GDP_OK || r == GDP_E_NOTERM) {
      if (r == GDP_OK && !M->arena && alloc_host_mirrors(M) != GDP_OK) r = GDP_E_NOMEM;
    }
    if (r == GDP_OK || r == GDP_E_NOTERM) {
      outs[i] = M;
    } else {
      if (status) status[i] = r;
      gdp_mesh_free(M);
      mesh[k] = nullptr;
    }
  }
  return GDP_OK;
}

// ---- serving form: continuous batching over the single-workgroup engine ----
// Device memory of a server: one allocation split into job regions by a
// first-fit allocator; it is freed once the server is gone and every region
// (held by a finished mesh the caller still owns) has come back.
struct ServerMem {
  void *base = nullptr;
  size_t size = 0;
  std::mutex mu;
  std::map<size_t, size_t> free_ranges;  // offset -> length
  int live = 0;
  bool closed = false;

  bool take(size_t n, size_t *off) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      size_t rest = it->second - n, o = it->first + n;
      free_ranges.erase(it);
      if (rest) free_ranges[o] = rest;
      live++;
      return true;
    }
    return false;
  }
  // returns true when the whole allocation can go
  bool give(size_t off, size_t n) {
    auto nx = free_ranges.lower_bound(off);
    if (nx != free_ranges.end() && off + n == nx->first) {
      n += nx->second;
      free_ranges.erase(nx);
    }
    auto pv = free_ranges.lower_bound(off);
    if (pv != free_ranges.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        off = pv->first;
        n += pv->second;
        free_ranges.erase(pv);
      }
    }
    free_ranges[off] = n;
    return --live == 0 && closed;
  }
};

void server_mem_release(ServerMem *sm, size_t off, size_t n) {
  bool last;
  {
    std::lock_guard<std::mutex> g(sm->mu);
    last = sm->give(off, n);
  }
  if (last) {
    (void)hipFree(sm->base);
    delete sm;
  }
}

struct Job {
  uint64_t id = 0;
  std::vector<double> xy;    // the input, kept for a fallback refinement on its own
  std::vector<int32_t> seg;
  HostMesh hm;               // Line 1 output
  std::vector<int4> tv, tn, ts;
  double B2 = 2.0;
  gdp_params P;
  Caps caps;
  size_t bytes = 0, off = 0;
  gdp_mesh *mesh = nullptr;
  enum { PREPARED, LINE1, QUEUED, ACTIVE, DONE } state = PREPARED;
  gdp_status status = GDP_OK;
  double t_submit = 0, t_line1 = 0, t_admit = 0, t_done = 0;
  bool grid_only = false;  // outgrew its region in a batched launch: the slots refine it
  int32_t nv_in = 0;       // input vertices
  bool raw = false;        // Line 1 has not run: it runs in the server after arrival
  bool resident = false;   // Line 1 ran on the device, into the job's region
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// One worker per slot: its own stream (so that the jobs of different slots
// overlap on the device) and pinned mirrors lent to the mesh it refines.
// A slot's own stream, pinned mirrors and engine descriptor, lent to each job
// it runs: nothing is allocated or freed per job (hipFree and hipHostFree
// wait for the whole device, which would stall every other slot).
struct ServerWorker {
  gdp_ctx ctx;
  DevCounters *h_cnt = nullptr;
  DevState *h_st = nullptr;
  DevCounters *h_hist = nullptr;
  EngDesc *d_eng = nullptr;
  int32_t *d_head = nullptr;
  EngDesc *h_eng = nullptr;
  std::thread th;
};

// Batched launches for small jobs: every arrived job with at most
// engine_max_v input vertices is refined in one launch of the
// single-workgroup engine together with the other such jobs (one workgroup
// per job, largest first), so that a small job costs one workgroup for its
// whole refinement instead of ~17 launches per round on a slot's stream.
constexpr int kSrvEngMax = 512;  // jobs per batched launch
// Off by default: measured on mixed job streams, a batched launch (as long as
// its slowest job on one compute unit) holds one of the few hardware queues
// that the slots' streams share, which delays their rounds more than the
// launches it saves.
constexpr int32_t kSrvEngineDefaultMaxV = 0;
struct ServerEngine {
  gdp_ctx ctx;
  EngDesc *d_desc = nullptr, *h_desc = nullptr;  // [kSrvEngMax]
  int32_t *d_head = nullptr;
  DevState *h_st = nullptr;                      // [kSrvEngMax]
  DevCounters *h_cnt = nullptr;                  // [kSrvEngMax]
  DevCounters *h_hist = nullptr;                 // [kSrvEngMax * kHistCap]
  int cus = 256;
  std::thread th;
};

// Shared rounds (Rule 4 of Section 2, the default mode): one driver thread
// runs the rounds of every active job together, one launch per phase for all
// of them; jobs join and leave between groups of rounds.
struct ServerGang {
  gdp_ctx ctx;     // the driver's own stream
  GangBufs bufs;   // for max_slots jobs
  std::thread th;
};

// Line 1 in the server (gdp_server_line1): host threads build the CDTs of
// arrived jobs; one more thread builds those of large jobs on the device, on
// its own stream, directly into the job's region.
struct ServerLine1Dev {
  gdp_ctx ctx;
  DevCdtWork ws;
  std::thread th;
};

struct gdp_server {
  gdp_ctx *user = nullptr;  // the caller's context: finished meshes are handed over to it
  ServerMem *mem = nullptr;
  int max_slots = 0;
  int32_t mode = 0;          // 0: shared rounds; 1: a stream and a thread per slot
  int32_t gang_rounds = kGangRounds;  // shared rounds between two host reads
  int32_t engine_max_v = 0;  // 0: no job in the single-workgroup engine launches
  ServerEngine *eng = nullptr;
  ServerGang *gang = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::map<uint64_t, Job *> jobs;
  std::deque<Job *> queue;
  int running = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::vector<ServerWorker *> workers;
  std::chrono::steady_clock::time_point t0;
  int32_t l1_threads = 0;    // > 0: Line 1 runs in the server, after arrival
  int32_t l1_dev_min_v = 0;  // jobs with at least this many input vertices build on the device (0: none)
  std::deque<Job *> l1_host, l1_dev;
  std::vector<std::thread> l1_workers;
  ServerLine1Dev *l1dev = nullptr;
};

namespace {

// The mesh of job J laid out in its region (J->off, J->bytes, J->caps), with
// the byte ranges that must be filled before use (offset, (bytes, fill byte));
// run receives the bytes used.
gdp_mesh *region_mesh(gdp_server *S, Job *J, gdp_ctx *ctx, std::vector<std::pair<size_t, std::pair<size_t, int>>> &fills,
                      size_t &run) {
  gdp_mesh *M = new gdp_mesh();
  M->ctx = ctx;
  gdp_arena *a = new gdp_arena();
  ServerMem *sm = S->mem;
  const size_t off = J->off, n = J->bytes;
  a->base = (char *)sm->base + off;
  a->refs = 1;
  a->release = [sm, off, n]() { server_mem_release(sm, off, n); };
  M->arena = a;
  char *p = (char *)a->base;
  run = 0;
  for_each_array(M, J->caps, [&](void **pp, size_t es, int64_t len, int fill) {
    size_t b = align256(es * (size_t)std::max<int64_t>(len, 1));
    *pp = p + run;
    if (fill) fills.push_back({run, {b, fill}});
    run += b;
  });
  const Caps &c = J->caps;
  M->m.capV = (int32_t)c.V; M->m.capT = (int32_t)c.T; M->m.capS = (int32_t)c.S;
  M->wT = (int32_t)c.W; M->tiles_cap = (int32_t)c.tiles;
  M->pool_cap = (int32_t)c.pool; M->fan_cap = (int32_t)c.fan;
  return M;
}

// Places a prepared job in its region and uploads its initial mesh.
gdp_status admit_job(gdp_server *S, Job *J, gdp_ctx *ctx) {
  hipStream_t st = ctx->stream;
  std::vector<std::pair<size_t, std::pair<size_t, int>>> fills;
  size_t run = 0;
  gdp_mesh *M = region_mesh(S, J, ctx, fills, run);
  char *p = (char *)M->arena->base;
  const HostMesh &h = J->hm;
  M->m.nV = h.nV; M->m.nT = h.nT; M->m.nS = h.nS;
  M->m.n_input_v = h.nV; M->m.n_input_s = h.nS;
  J->mesh = M;
  DevState ds;
  memset(&ds, 0, sizeof ds);
  ds.nV = h.nV; ds.nT = h.nT; ds.nS = h.nS;
  ds.wT = words(h.nT); ds.wS = words(h.nS);
  ds.full = 1;
  HIPCHECK(hipMemsetAsync(p, 0, run, st));
  for (auto &f : fills) HIPCHECK(hipMemsetAsync(p + f.first, f.second.second, f.second.first, st));
  HIPCHECK(hipMemcpyAsync(M->m.vxy, h.xy.data(), sizeof(double) * 2 * h.nV, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(M->m.tv, J->tv.data(), sizeof(int4) * h.nT, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(M->m.tn, J->tn.data(), sizeof(int4) * h.nT, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(M->m.ts, J->ts.data(), sizeof(int4) * h.nT, hipMemcpyHostToDevice, st));
  if (h.nS) {
    HIPCHECK(hipMemcpyAsync(M->m.sv, h.sv.data(), sizeof(int32_t) * 2 * h.nS, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(M->m.spar, h.sparent.data(), sizeof(int32_t) * h.nS, hipMemcpyHostToDevice, st));
  }
  HIPCHECK(hipMemcpyAsync(M->d_st, &ds, sizeof ds, hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));  // the host arrays above are pageable
  return GDP_OK;
}

gdp_status refine_loop(gdp_mesh *M, double B2, const gdp_params *P);

void complete_job(gdp_server *S, Job *J, gdp_status st) {
  std::lock_guard<std::mutex> g(S->mu);
  J->status = st;
  J->t_done = ms_since(S->t0);
  J->state = Job::DONE;
  S->running--;
  S->cv.notify_all();
}

// A worker: takes the oldest arrived job once its region fits, uploads it,
// refines it to the end on its own stream (the plain refinement, whose
// small final rounds run in the single-workgroup engine), hands it over.
void free_server_engine(ServerEngine *E) {
  if (!E) return;
  if (E->ctx.stream) (void)hipStreamDestroy(E->ctx.stream);
  if (E->d_desc) (void)hipFree(E->d_desc);
  if (E->d_head) (void)hipFree(E->d_head);
  if (E->h_desc) (void)hipHostFree(E->h_desc);
  if (E->h_st) (void)hipHostFree(E->h_st);
  if (E->h_cnt) (void)hipHostFree(E->h_cnt);
  if (E->h_hist) (void)hipHostFree(E->h_hist);
  delete E;
}

bool for_engine(const gdp_server *S, const Job *J) {
  return S->engine_max_v > 0 && !J->grid_only && !J->resident && J->nv_in <= S->engine_max_v;
}
bool for_slots(const gdp_server *S, const Job *J) { return !J->resident && S->mode == 1 && !for_engine(S, J); }
// (a job whose CDT was built in its region joins the shared rounds in any mode)
bool for_gang(const gdp_server *S, const Job *J) { return J->resident || (S->mode == 0 && !for_engine(S, J)); }

// One batched launch over jobs already taken from the queue (regions held).
void engine_batch(gdp_server *S, ServerEngine *E, std::vector<Job *> &B) {
  hipStream_t s = E->ctx.stream;
  std::vector<Job *> run;
  for (Job *J : B) {
    gdp_status st = admit_job(S, J, &E->ctx);
    if (st != GDP_OK) {
      if (J->mesh) gdp_mesh_free(J->mesh);
      J->mesh = nullptr;
      complete_job(S, J, st);
      continue;
    }
    run.push_back(J);
  }
  if (run.empty()) return;
  std::stable_sort(run.begin(), run.end(), [](const Job *a, const Job *b) { return a->hm.nT > b->hm.nT; });
  const int n = (int)run.size();
  for (int q = 0; q < n; q++) {
    gdp_mesh *M = run[q]->mesh;
    const gdp_params *P = &run[q]->P;
    EngDesc &d = E->h_desc[q];
    memset(&d, 0, sizeof d);
    d.m = M->m;
    d.w[0] = make_work(M, P, 0);
    d.w[1] = make_work(M, P, 1);
    d.B2 = run[q]->B2;
    d.pm = P->priority_mode;
    d.K = P->cand_cap_K;
    d.f1 = P->prefilter_f1;
    d.approx_n = P->cavity_approx_n;
    d.max_rounds = P->max_rounds;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
            hipMemcpyAsync(E->d_desc, E->h_desc, sizeof(EngDesc) * n, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemsetAsync(E->d_head, 0, sizeof(int32_t), s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(k_engine, dim3((unsigned)std::min(n, E->cus)), dim3(kEngBlock), 0, s, E->d_desc, n,
                       E->d_head, 1 << 30);
    ok = hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess;
  }
  for (int q = 0; ok && q < n; q++) {
    gdp_mesh *M = run[q]->mesh;
    ok = hipMemcpyAsync(&E->h_st[q], M->d_st, sizeof(DevState), hipMemcpyDeviceToHost, s) == hipSuccess &&
         hipMemcpyAsync(&E->h_cnt[q], M->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s) == hipSuccess &&
         hipMemcpyAsync(&E->h_hist[(size_t)q * kHistCap], M->d_hist, sizeof(DevCounters) * kHistCap,
                        hipMemcpyDeviceToHost, s) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  float ms = 0.f;
  if (ok) (void)hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int q = 0; q < n; q++) {
    Job *J = run[q];
    gdp_mesh *M = J->mesh;
    if (!ok) {
      gdp_mesh_free(M);
      J->mesh = nullptr;
      complete_job(S, J, fail(&E->ctx, GDP_E_DEVICE, "batched launch failed"));
      continue;
    }
    const DevState &d = E->h_st[q];
    M->m.nV = d.nV; M->m.nT = d.nT; M->m.nS = d.nS; M->m.rounds = d.rounds;
    M->serial = d.serial;
    M->last_ms = ms;
    const DevCounters *h = &E->h_hist[(size_t)q * kHistCap];
    for (int r = 0; r < std::min(d.nhist, kHistCap); r++) M->stats.push_back(round_stats_of(h[r], &J->P));
    if (d.halt == kHaltAbort) {
      // out of its region's room: a slot refines it from the start
      gdp_mesh_free(M);
      J->mesh = nullptr;
      std::lock_guard<std::mutex> g(S->mu);
      J->grid_only = true;
      J->state = Job::QUEUED;
      S->running--;
      S->queue.push_front(J);
      S->cv.notify_all();
      continue;
    }
    gdp_status st = status_of_halt(&E->ctx, d, E->h_cnt[q]);
    if (st != GDP_OK && st != GDP_E_NOTERM) {
      gdp_mesh_free(M);
      J->mesh = nullptr;
    }
    complete_job(S, J, st);
  }
}

// Takes every arrived small job whose region fits (first come, first
// served), up to kSrvEngMax, and runs them in one batched launch.
void engine_dispatcher(gdp_server *S, ServerEngine *E) {
  (void)hipSetDevice(E->ctx.device);
  for (;;) {
    std::vector<Job *> B;
    {
      std::unique_lock<std::mutex> g(S->mu);
      for (;;) {
        for (auto it = S->queue.begin(); it != S->queue.end() && (int)B.size() < kSrvEngMax;) {
          Job *Q = *it;
          if (!for_engine(S, Q)) {
            ++it;
            continue;
          }
          size_t off;
          bool got;
          {
            std::lock_guard<std::mutex> gm(S->mem->mu);
            got = S->mem->take(Q->bytes, &off);
          }
          if (!got) break;
          Q->off = off;
          Q->state = Job::ACTIVE;
          Q->t_admit = ms_since(S->t0);
          S->running++;
          B.push_back(Q);
          it = S->queue.erase(it);
        }
        if (!B.empty()) break;
        if (S->stop) {
          bool any = false;
          for (Job *Q : S->queue) any = any || for_engine(S, Q);
          if (!any) return;  // what is left is the slots'
          if (S->running == 0) {
            // closing, and the room is held by meshes the caller owns
            for (auto it = S->queue.begin(); it != S->queue.end();) {
              if (!for_engine(S, *it)) {
                ++it;
                continue;
              }
              (*it)->status = GDP_E_NOMEM;
              (*it)->t_done = ms_since(S->t0);
              (*it)->state = Job::DONE;
              it = S->queue.erase(it);
            }
            S->cv.notify_all();
            return;
          }
        }
        S->cv.wait_for(g, std::chrono::milliseconds(1));
      }
    }
    engine_batch(S, E, B);
  }
}


// ---- serving form: shared rounds ------------------------------------------
// The driver: admits arrived jobs (first come, first served) while a slot
// and room are free, runs a group of shared rounds of every active job,
// and retires the jobs that finished.
void gang_driver(gdp_server *S, ServerGang *Gn) {
  (void)hipSetDevice(Gn->ctx.device);
  gdp_ctx *ctx = &Gn->ctx;
  std::vector<GangItem> active;
  for (;;) {
    std::vector<Job *> fresh;
    int R = kGangRounds;
    {
      std::unique_lock<std::mutex> g(S->mu);
      for (;;) {
        for (auto it = S->queue.begin();
             it != S->queue.end() && (int)(active.size() + fresh.size()) < S->max_slots;) {
          Job *Q = *it;
          if (!for_gang(S, Q)) {
            ++it;
            continue;
          }
          if (!Q->resident) {
            size_t off;
            bool got;
            {
              std::lock_guard<std::mutex> gm(S->mem->mu);
              got = S->mem->take(Q->bytes, &off);
            }
            if (!got) break;  // first come, first served: wait for room
            Q->off = off;
          }
          Q->state = Job::ACTIVE;
          Q->t_admit = ms_since(S->t0);
          S->running++;
          fresh.push_back(Q);
          it = S->queue.erase(it);
        }
        if (!fresh.empty() || !active.empty()) break;
        bool mine = false;
        for (Job *Q : S->queue) mine = mine || for_gang(S, Q);
        if (S->stop && !mine) return;
        if (S->stop && mine && S->running == 0) {
          // closing, and the room is held by meshes the caller owns
          for (auto q = S->queue.begin(); q != S->queue.end();) {
            if (!for_gang(S, *q)) {
              ++q;
              continue;
            }
            (*q)->status = GDP_E_NOMEM;
            (*q)->t_done = ms_since(S->t0);
            (*q)->state = Job::DONE;
            q = S->queue.erase(q);
          }
          S->cv.notify_all();
          continue;
        }
        S->cv.wait_for(g, std::chrono::milliseconds(1));
      }
      R = S->gang_rounds;
    }
    for (Job *J : fresh) {
      gdp_status st = GDP_OK;
      if (J->resident) J->mesh->ctx = ctx;  // built on the Line-1 thread's stream, which has finished
      else st = admit_job(S, J, ctx);
      if (st != GDP_OK) {
        if (J->mesh) gdp_mesh_free(J->mesh);
        J->mesh = nullptr;
        complete_job(S, J, st);
        continue;
      }
      active.push_back(gang_item(J->mesh, &J->P, J->B2, J));
    }
    if (active.empty()) continue;
    std::vector<std::pair<GangItem, gdp_status>> finished;
    gang_group(ctx, Gn->bufs, active, R, finished);
    for (auto &f : finished) {
      Job *J = (Job *)f.first.tag;
      gdp_mesh *M = J->mesh;
      gdp_status st = f.second;
      if (st == GDP_OK && !M->arena) st = alloc_host_mirrors(M);
      if (st != GDP_OK && st != GDP_E_NOTERM) {
        gdp_mesh_free(M);
        J->mesh = nullptr;
      }
      complete_job(S, J, st);
    }
  }
}

void free_server_gang(ServerGang *Gn) {
  if (!Gn) return;
  if (Gn->ctx.stream) (void)hipStreamDestroy(Gn->ctx.stream);
  gang_bufs_free(Gn->bufs);
  delete Gn;
}

void server_worker(gdp_server *S, ServerWorker *W) {
  (void)hipSetDevice(W->ctx.device);
  for (;;) {
    Job *J = nullptr;
    {
      std::unique_lock<std::mutex> g(S->mu);
      for (;;) {
        auto it = S->queue.begin();
        while (it != S->queue.end() && !for_slots(S, *it)) ++it;
        if (it != S->queue.end()) {
          Job *Q = *it;
          size_t off;
          bool got;
          {
            std::lock_guard<std::mutex> gm(S->mem->mu);
            got = S->mem->take(Q->bytes, &off);
          }
          if (got) {
            Q->off = off;
            S->queue.erase(it);
            Q->state = Job::ACTIVE;
            Q->t_admit = ms_since(S->t0);
            S->running++;
            J = Q;
            break;
          }
          if (S->stop && S->running == 0) {
            // closing, and the room is held by meshes the caller owns
            for (auto q = S->queue.begin(); q != S->queue.end();) {
              if (!for_slots(S, *q)) {
                ++q;
                continue;
              }
              (*q)->status = GDP_E_NOMEM;
              (*q)->t_done = ms_since(S->t0);
              (*q)->state = Job::DONE;
              q = S->queue.erase(q);
            }
            S->cv.notify_all();
          }
        }
        bool mine = false;
        for (Job *Q : S->queue) mine = mine || for_slots(S, Q);
        if (S->stop && !mine) return;
        // first come, first served: wait for an arrival or for room
        S->cv.wait_for(g, std::chrono::milliseconds(2));
      }
    }
    gdp_status st = admit_job(S, J, &W->ctx);
    gdp_mesh *M = J->mesh;
    if (st == GDP_OK) {
      M->h_cnt = W->h_cnt;
      M->h_st = W->h_st;
      M->h_hist = W->h_hist;
      M->d_eng = W->d_eng;
      M->d_head = W->d_head;
      M->h_eng = W->h_eng;
      st = refine_loop(M, J->B2, &J->P);
      M->h_cnt = nullptr;  // give the lent buffers back; a mesh that left its region gets its own mirrors
      M->h_st = nullptr;
      M->h_hist = nullptr;
      M->d_eng = nullptr;
      M->d_head = nullptr;
      M->h_eng = nullptr;
      if (!M->arena && st == GDP_OK) st = alloc_host_mirrors(M);
    }
    if (st != GDP_OK && st != GDP_E_NOTERM && M) {
      gdp_mesh_free(M);
      J->mesh = nullptr;
    }
    complete_job(S, J, st);
  }
}

// Region sizes of a job from its initial CDT's counts.
void job_caps(gdp_server *S, Job *J, int64_t nV, int64_t nT, int64_t nS) {
  Caps c;
  c.V = 3 * nV + 256;
  c.T = std::max<int64_t>(2 * c.V + 256, nT);
  c.S = 16 * nS + 64;
  c.W = c.T + 2 * c.S + 2;
  c.tiles = c.W / kScanTileSize + 2;
  c.pool = 2 * c.T + 4096;
  c.fan = 2 * c.T + 4096;
  J->caps = c;
  gdp_mesh tmp;
  size_t b = 0;
  for_each_array(&tmp, c, [&](void **, size_t es, int64_t len, int) { b += align256(es * (size_t)std::max<int64_t>(len, 1)); });
  J->bytes = b;
}

// Line 1 of a job on the host, and the arrays and region size it needs.
gdp_status job_line1_host(gdp_server *S, Job *J, std::string &e) {
  int rc = host_cdt_build((int32_t)(J->xy.size() / 2), J->xy.data(), (int32_t)(J->seg.size() / 2), J->seg.data(),
                          J->hm, e);
  if (rc != GDP_OK) return (gdp_status)rc;
  const HostMesh &h = J->hm;
  J->tv.resize(h.nT);
  J->tn.resize(h.nT);
  J->ts.resize(h.nT);
  for (int32_t t = 0; t < h.nT; t++) {
    int w = (h.ts[3 * t] >= 0 ? 1 : 0) | (h.ts[3 * t + 1] >= 0 ? 2 : 0) | (h.ts[3 * t + 2] >= 0 ? 4 : 0);
    J->tv[t] = make_int4(h.tv[3 * t], h.tv[3 * t + 1], h.tv[3 * t + 2], w);
    J->tn[t] = make_int4(h.tn[3 * t], h.tn[3 * t + 1], h.tn[3 * t + 2], 0);
    J->ts[t] = make_int4(h.ts[3 * t], h.ts[3 * t + 1], h.ts[3 * t + 2], 0);
  }
  job_caps(S, J, h.nV, h.nT, h.nS);
  if (J->bytes > S->mem->size) {
    e = "job larger than the server's memory budget";
    return GDP_E_NOMEM;
  }
  return GDP_OK;
}

// Everything a job needs before it arrives: its input and parameters, and
// (unless Line 1 runs in the server) Line 1 on the host.
gdp_status prepare_job(gdp_server *S, const gdp_pslg *pslg, double B2, const gdp_params *P, Job *J) {
  gdp_ctx *ctx = S->user;
  J->B2 = B2;
  J->P = *P;
  // a host synchronisation per round: the other slots keep the device busy
  if (J->P.rounds_per_sync == 0) J->P.rounds_per_sync = 1;
  std::string e;
  gdp_status st;
  if (S->l1_threads > 0 && (st = check_pslg_for_device(pslg, e))) return fail(ctx, st, e);
  J->xy.assign(pslg->xy, pslg->xy + 2 * (size_t)pslg->n_vertices);
  J->seg.assign(pslg->seg, pslg->seg + 2 * (size_t)pslg->n_segments);
  J->nv_in = pslg->n_vertices;
  if (S->l1_threads > 0) {
    J->raw = true;
    return GDP_OK;
  }
  if ((st = job_line1_host(S, J, e))) return fail(ctx, st, e);
  return GDP_OK;
}

// Line 1 of job J has finished in the server with status st: the job joins
// the admission queue, or ends.
void line1_done(gdp_server *S, Job *J, gdp_status st) {
  std::lock_guard<std::mutex> g(S->mu);
  J->t_line1 = ms_since(S->t0);
  if (st != GDP_OK) {
    J->status = st;
    J->t_done = J->t_line1;
    J->state = Job::DONE;
  } else {
    J->state = Job::QUEUED;
    S->queue.push_back(J);
  }
  S->cv.notify_all();
}

// Takes the next job of a Line-1 queue (nullptr once the server stops).
Job *line1_next(gdp_server *S, std::deque<Job *> &q) {
  std::unique_lock<std::mutex> g(S->mu);
  S->cv.wait(g, [&] { return S->stop || !q.empty(); });
  if (S->stop) return nullptr;
  Job *J = q.front();
  q.pop_front();
  return J;
}

void line1_host_worker(gdp_server *S) {
  for (;;) {
    Job *J = line1_next(S, S->l1_host);
    if (!J) return;
    std::string e;
    line1_done(S, J, job_line1_host(S, J, e));
  }
}

// Line 1 of a large job by kernels, into its region: the region is taken
// here (sized from the input: a CDT has at most 2 V triangles), the input
// is uploaded and the device builder writes the canonical CDT in place.
gdp_status job_line1_device(gdp_server *S, ServerLine1Dev *D, Job *J) {
  const int32_t nv = J->nv_in, ns = (int32_t)(J->seg.size() / 2);
  job_caps(S, J, nv, 2 * (int64_t)nv, ns);
  if (J->bytes > S->mem->size) return GDP_E_NOMEM;
  for (;;) {
    {
      std::lock_guard<std::mutex> gm(S->mem->mu);
      if (S->mem->take(J->bytes, &J->off)) break;
    }
    std::unique_lock<std::mutex> g(S->mu);
    if (S->stop) return GDP_E_NOMEM;
    S->cv.wait_for(g, std::chrono::milliseconds(1));
  }
  gdp_ctx *ctx = &D->ctx;
  hipStream_t st = ctx->stream;
  std::vector<std::pair<size_t, std::pair<size_t, int>>> fills;
  size_t run = 0;
  gdp_mesh *M = region_mesh(S, J, ctx, fills, run);
  J->mesh = M;
  char *p = (char *)M->arena->base;
  std::vector<int32_t> spar(ns);
  for (int32_t k = 0; k < ns; k++) spar[k] = k;
  HIPCHECK(hipMemsetAsync(p, 0, run, st));
  for (auto &f : fills) HIPCHECK(hipMemsetAsync(p + f.first, f.second.second, f.second.first, st));
  HIPCHECK(hipMemcpyAsync(M->m.vxy, J->xy.data(), sizeof(double) * 2 * nv, hipMemcpyHostToDevice, st));
  if (ns) {
    HIPCHECK(hipMemcpyAsync(M->m.sv, J->seg.data(), sizeof(int32_t) * 2 * ns, hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(M->m.spar, spar.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
  }
  std::string e;
  int32_t nt = 0;
  DevCdtStats cs;
  const int rc = dev_cdt_build(st, nv, M->m.vxy, ns, M->m.sv, M->m.tv, M->m.tn, M->m.ts, M->m.capT, &nt, &cs, e,
                               &D->ws);
  if (rc != GDP_OK) return (gdp_status)rc;
  M->m.nV = nv; M->m.nT = nt; M->m.nS = ns;
  M->m.n_input_v = nv; M->m.n_input_s = ns;
  M->cdt_rounds[0] = cs.dt_rounds;
  M->cdt_rounds[1] = cs.seg_rounds;
  DevState ds;
  memset(&ds, 0, sizeof ds);
  ds.nV = nv; ds.nT = nt; ds.nS = ns;
  ds.wT = words(nt); ds.wS = words(ns);
  ds.full = 1;
  HIPCHECK(hipMemcpyAsync(M->d_st, &ds, sizeof ds, hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));  // ds and spar are host locals
  J->resident = true;
  return GDP_OK;
}

void line1_dev_worker(gdp_server *S, ServerLine1Dev *D) {
  (void)hipSetDevice(D->ctx.device);
  for (;;) {
    Job *J = line1_next(S, S->l1_dev);
    if (!J) return;
    gdp_status st = job_line1_device(S, D, J);
    if (st != GDP_OK && J->mesh) {
      gdp_mesh_free(J->mesh);
      J->mesh = nullptr;
    }
    line1_done(S, J, st);
  }
}

// Queues up to this many rounds before the next host synchronisation.
// Groups of two or more rounds are queued as graph replays, in pairs.
int rounds_for(const gdp_params *P, int64_t last_cand, bool engine) {
  if (engine) return kHistCap;
  int r;
  if (P->rounds_per_sync > 0) r = std::min(P->rounds_per_sync, kHistCap);
  else if (last_cand > 65536) r = 1;
  else if (last_cand > 8192) r = 4;
  else r = 16;
  // approaching the engine's threshold: end the group about when the
  // candidates fall below it (they shrink by roughly a quarter per round at
  // the end of a refinement), so that the engine takes over in time
  const int64_t eng_max = P->tail_engine_max == 0 ? kEngineDefaultMax : P->tail_engine_max;
  if (P->rounds_per_sync == 0 && eng_max > 0 && r > 2) {
    int k = 0;
    for (double c = (double)last_cand; c > (double)eng_max && k < 16; c *= 0.75) k++;
    r = std::max(2, std::min(r, k));
  }
  return r >= 2 ? r & ~1 : r;
}

// One refinement call: rounds until nothing is left (Algorithm 1, "repeat
// ... until L is empty").  Rounds are queued in groups; the host reads the
// device state once per group.  A round that finds a buffer short writes
// nothing and halts the group; the host grows the buffers and runs it again.
// ---------------------------------------------------------------------------
// Flip-Flop rounds (insert_mode 1; steps in gdp_ff_core.h, kernels in
// gdp_ff.hip).  Every round: Lines 3-7 as in a cavity round (full
// collection), the Line 6 claims, S sorted into decreasing key order, the
// splits, flip passes to the CDT, then detection and removal of redundant
// points until none is left, final ids, compaction, the round's record.
// The host reads the device counters between the phases.
// ---------------------------------------------------------------------------
inline unsigned ff_grid(int64_t n) { return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

gdp_status ff_reserve(gdp_mesh *M, int32_t np) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  if (!M->ff) {
    M->ff = new FfBufs();
    HIPCHECK(dalloc(&M->ff->d_c, 1));
    HIPCHECK(hipHostMalloc((void **)&M->ff->h_c, sizeof(FfCount)));
  }
  FfBufs &F = *M->ff;
  const DevMesh &m = M->m;
  const int64_t needK = (int64_t)m.capT + 2 * (int64_t)m.capS + 2;
  if (needK > F.capK) {
    // the claims' output (skey0, sref0) may already hold S: keep it
    const size_t n = (size_t)needK, o = (size_t)F.capK;
    HIPCHECK(dgrow(&F.skey0, o, n, o, 0, s));
    HIPCHECK(dgrow(&F.skey1, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.sref0, o, n, o, 0, s));
    HIPCHECK(dgrow(&F.sref1, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.shist, 0, 256 * ((n + kSortPairsTile - 1) / kSortPairsTile), 0, 0, s));
    F.capK = (int32_t)needK;
  }
  if (np + 1 > F.capP) {
    const size_t n = (size_t)std::max<int64_t>({(int64_t)np + 1, (int64_t)F.capP * 3 / 2, 1024});
    HIPCHECK(dgrow(&F.pt, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.pinfo, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.pslots, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.pab, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.alive, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.red, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.vtri, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.newid, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.ntiles, 0, n / kFfScanTile + 2, 0, 0, s));
    F.capP = (int32_t)n;
  }
  if (m.capT > F.capT) {
    const size_t n = (size_t)m.capT, o = (size_t)F.capT;
    // stamps and claims keep their values (they are compared with newer ones)
    HIPCHECK(dgrow(&F.sstamp, o, n, o, 0, s));
    HIPCHECK(dgrow(&F.wstamp, o, n, o, 0, s));
    HIPCHECK(dgrow(&F.tstamp, o, n, o, 0, s));
    HIPCHECK(dgrow(&F.claim, o, n, o, 0, s));
    HIPCHECK(dgrow(&F.grp, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.moved, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.fc0, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.fc1, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.fprio, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.list[0], 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.list[1], 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.touched, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.dead, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.hole, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.mover, 0, n, 0, 0, s));
    F.capT = (int32_t)n;
  }
  const int64_t need_pool = std::max<int64_t>(1 << 20, 4 * (int64_t)m.capT);
  if (need_pool > F.pool_cap) {
    HIPCHECK(dgrow(&F.pool, 0, (size_t)need_pool, 0, 0, s));
    F.pool_cap = need_pool;
  }
  if (m.capV > F.capV) {
    HIPCHECK(dgrow(&F.vmark, (size_t)F.capV, (size_t)m.capV, (size_t)F.capV, 0, s));
    F.capV = m.capV;
  }
  if ((int64_t)m.capS + F.capP > F.capS) {
    // cleared by every round's last kernels: no contents to keep
    const size_t n = (size_t)m.capS + (size_t)F.capP;
    HIPCHECK(dgrow(&F.sflag, 0, n, 0, 0, s));
    HIPCHECK(dgrow(&F.mid_rank, 0, n, 0, 0, s));
    F.capS = (int32_t)n;
  }
  return GDP_OK;
}

// A fresh slot stamp / pass number (the stamp arrays, claims and vertex
// marks are cleared when the counters would overflow their fields).
gdp_status ff_next_stamp(gdp_mesh *M, int &out) {
  gdp_ctx *ctx = M->ctx;
  FfBufs &F = *M->ff;
  if (F.stamp >= (1 << 30)) {
    HIPCHECK(hipMemsetAsync(F.sstamp, 0, sizeof(int32_t) * F.capT, ctx->stream));
    HIPCHECK(hipMemsetAsync(F.wstamp, 0, sizeof(int32_t) * F.capT, ctx->stream));
    HIPCHECK(hipMemsetAsync(F.tstamp, 0, sizeof(int32_t) * F.capT, ctx->stream));
    F.stamp = 0;
  }
  out = ++F.stamp;
  return GDP_OK;
}
gdp_status ff_next_pass(gdp_mesh *M, uint64_t &out) {
  gdp_ctx *ctx = M->ctx;
  FfBufs &F = *M->ff;
  if (F.pass >= (1ull << 23)) {
    HIPCHECK(hipMemsetAsync(F.claim, 0, sizeof(uint64_t) * F.capT, ctx->stream));
    HIPCHECK(hipMemsetAsync(F.vmark, 0, sizeof(uint64_t) * F.capV, ctx->stream));
    F.pass = 0;
  }
  out = ++F.pass;
  return GDP_OK;
}

FfView ff_view(gdp_mesh *M, const gdp_params *P, int32_t nmk) {
  FfBufs &F = *M->ff;
  const DevMesh &m = M->m;
  FfView V;
  memset(&V, 0, sizeof V);
  V.vxy = m.vxy; V.vkind = m.vkind; V.tv = m.tv; V.tn = m.tn; V.ts = m.ts;
  V.sv = m.sv; V.spar = m.spar; V.spend = m.spend; V.mflag = M->mflag;
  V.nV = m.nV; V.nT = m.nT; V.nS = m.nS; V.enc_mode = P->encroach_mode;
  V.pt = F.pt; V.pinfo = F.pinfo; V.pab = F.pab; V.pslots = F.pslots;
  V.alive = F.alive; V.red = F.red; V.vtri = F.vtri; V.newid = F.newid;
  V.grp = F.grp; V.sstamp = F.sstamp; V.wstamp = F.wstamp; V.tstamp = F.tstamp; V.moved = F.moved;
  V.claim = F.claim;
  V.list_in = F.list[1]; V.list_out = F.list[0];
  V.touched = F.touched; V.dead = F.dead; V.hole = F.hole; V.mover = F.mover;
  V.newid_tiles = F.ntiles;
  V.fc0 = F.fc0; V.fc1 = F.fc1; V.fprio = F.fprio; V.cand_cap = F.capT;
  V.vmark = F.vmark; V.sflag = F.sflag; V.mid_rank = F.mid_rank;
  V.mid_elem = M->mid.elem; V.mid_state = M->mid.state; V.nmk = nmk;
  V.pool = F.pool; V.pool_cap = F.pool_cap;
  V.c = F.d_c;
  return V;
}

// Writers of the next flip worklist (splits, removals) append to list[out].
void ff_target(gdp_mesh *M, FfView &V, int out) {
  FfBufs &F = *M->ff;
  V.list_out = F.list[out];
  V.n_out = &F.d_c->n_list[out];
}

gdp_status ff_read(gdp_mesh *M, FfCount &c) {
  gdp_ctx *ctx = M->ctx;
  FfBufs &F = *M->ff;
  HIPCHECK(hipMemcpyAsync(F.h_c, F.d_c, sizeof(FfCount), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  c = *F.h_c;
  if (c.err) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "Flip-Flop step found an inconsistent mesh (site %d; round %d, |S| %d of which %d midpoints, "
             "%lld CDTs, %lld flips in %lld passes, %lld removals, %d slots allocated, %d freed)",
             c.err, M->m.rounds + 1, c.np, c.nmid, (long long)c.iters, (long long)c.flips, (long long)c.passes,
             (long long)c.removals, c.n_alloc, c.n_dead);
    return fail(ctx, GDP_E_CAVITY, buf);
  }
  return GDP_OK;
}

// Flip passes until no edge is left to check.  The first input list is
// F.list[cur] (length n_list[cur]), written with stamp in_stamp; est sizes
// the grids.  A pass is two launches; the host reads the counters after
// batches of 4, 8, then 16 passes.
gdp_status ff_lawson(gdp_mesh *M, FfView &V, int &cur, int &in_stamp, int tst, int64_t est) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  FfBufs &F = *M->ff;
  gdp_status st;
  int batch = 4;
  hipLaunchKernelGGL(kf_ctl, dim3(1), dim3(64), 0, s, F.d_c, 0, cur ^ 1);  // candidate counts start at 0
  for (int64_t done = 0; done < (1 << 15);) {
    for (int q = 0; q < batch; q++, done++) {
      int wst;
      uint64_t pass;
      if ((st = ff_next_stamp(M, wst)) || (st = ff_next_pass(M, pass))) return st;
      V.list_in = F.list[cur];
      V.list_out = F.list[cur ^ 1];
      V.n_in = &F.d_c->n_list[cur];
      V.n_out = &F.d_c->n_list[cur ^ 1];
      V.n_cand = &F.d_c->n_cnd[pass & 1];
      V.n_cand_next = &F.d_c->n_cnd[(pass + 1) & 1];
      hipLaunchKernelGGL(kf_flip_check, dim3(ff_grid(est)), dim3(256), 0, s, V, in_stamp, pass);
      hipLaunchKernelGGL(kf_flip_apply, dim3(ff_grid(est)), dim3(256), 0, s, V, wst, tst);
      in_stamp = wst;
      cur ^= 1;
    }
    FfCount c;
    if ((st = ff_read(M, c))) return st;
    if (c.n_list[cur] == 0) return GDP_OK;
    est = c.n_list[cur];
    batch = std::min(batch * 2, 16);
  }
  return fail(ctx, GDP_E_CAVITY, "flip passes did not converge");
}

// Resets the round counters of the Flip-Flop steps (slot allocation from nT).
gdp_status ff_reset(gdp_mesh *M) {
  gdp_ctx *ctx = M->ctx;
  FfBufs &F = *M->ff;
  memset(F.h_c, 0, sizeof(FfCount));
  F.h_c->n_alloc = M->m.nT;
  HIPCHECK(hipMemcpyAsync(F.d_c, F.h_c, sizeof(FfCount), hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  return GDP_OK;
}

// The mesh as the CDT under the symbolic perturbation, each triangle rotated
// so its smallest vertex comes first (the state Flip-Flop rounds keep).
gdp_status ff_canonical(gdp_mesh *M, const gdp_params *P) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  gdp_status st;
  if ((st = ff_reserve(M, 0)) || (st = ff_reset(M))) return st;
  FfBufs &F = *M->ff;
  FfView V = ff_view(M, P, 0);
  const int nT = M->m.nT;
  hipLaunchKernelGGL(kf_rotate, dim3(ff_grid(nT)), dim3(256), 0, s, V, nT);
  int wst, tst;
  if ((st = ff_next_stamp(M, wst)) || (st = ff_next_stamp(M, tst))) return st;
  ff_target(M, V, 0);
  hipLaunchKernelGGL(kf_all_slots, dim3(ff_grid(nT)), dim3(256), 0, s, V, nT, wst);
  int cur = 0, in_stamp = wst;
  if ((st = ff_lawson(M, V, cur, in_stamp, tst, nT))) return st;
  return ff_reset(M);
}

// One Flip-Flop round after the Line 3-7 kernels and the claims have run and
// the host has read the counts.  *recorded: the round was completed and
// recorded; *stall: it inserted nothing and flagged nothing.
gdp_status ff_line8(gdp_mesh *M, const gdp_params *P, int32_t np, int32_t nmid, int32_t nmk, bool *stall) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  FfBufs &F = *M->ff;
  gdp_status st;
  *stall = false;
  const DevMesh &m = M->m;
  // room: np vertices, 2 np slots, nmid subsegments (provisional second halves)
  if ((st = grow_vtx(M, m.nV + np + 16)) || (st = grow_tri(M, m.nT + 2 * np + 16)) ||
      (st = grow_seg(M, m.nS + nmid + 16)) || (st = grow_cand(M)) || (st = ff_reserve(M, np)))
    return st;
  Work w = make_work(M, P, 0);
  FfView V = ff_view(M, P, nmk);
  // S in decreasing key order (the keys were stored complemented)
  if (np > 0) HIPCHECK(sort_pairs_u64(s, F.skey0, F.sref0, F.skey1, F.sref1, np, F.shist));
  hipLaunchKernelGGL(kf_gather, dim3(ff_grid(np)), dim3(256), 0, s, M->m, w, V, (const int32_t *)F.sref1);
  int wst, tst, split_stamp;
  if ((st = ff_next_stamp(M, wst)) || (st = ff_next_stamp(M, tst)) || (st = ff_next_stamp(M, split_stamp)))
    return st;
  ff_target(M, V, 0);
  hipLaunchKernelGGL(kf_split, dim3(ff_grid(np)), dim3(256), 0, s, V, split_stamp, wst, tst);
  hipLaunchKernelGGL(kf_split_fix, dim3(ff_grid(np)), dim3(256), 0, s, V, split_stamp);
  int cur = 0, in_stamp = wst;
  if ((st = ff_lawson(M, V, cur, in_stamp, tst, 3 * (int64_t)np))) return st;
  FfCount c;
  for (int it = 0;; it++) {
    if (it > (1 << 16)) return fail(ctx, GDP_E_CAVITY, "redundant points keep appearing");
    if ((st = ff_read(M, c))) return st;
    hipLaunchKernelGGL(kf_ctl, dim3(1), dim3(64), 0, s, F.d_c, 2, 0);
    hipLaunchKernelGGL(kf_vtri, dim3(ff_grid(c.n_touched)), dim3(256), 0, s, V);
    hipLaunchKernelGGL(kf_detect, dim3(ff_grid(np)), dim3(256), 0, s, V);
    if ((st = ff_read(M, c))) return st;
    if (c.n_red == 0) break;
    // removal passes; their triangles form the next flip worklist
    if ((st = ff_next_stamp(M, wst))) return st;
    ff_target(M, V, cur);
    hipLaunchKernelGGL(kf_ctl, dim3(1), dim3(64), 0, s, F.d_c, 0, cur);
    for (int pass_i = 0;; pass_i++) {
      if (pass_i > (1 << 16)) return fail(ctx, GDP_E_CAVITY, "removal passes did not finish");
      uint64_t pass;
      if ((st = ff_next_pass(M, pass))) return st;
      const uint64_t pbase = pass << 32;
      hipLaunchKernelGGL(kf_ctl, dim3(1), dim3(64), 0, s, F.d_c, 1, 0);
      hipLaunchKernelGGL(kf_rm_mark, dim3(ff_grid(np)), dim3(256), 0, s, V, pbase);
      hipLaunchKernelGGL(kf_rm_decide, dim3(ff_grid(np)), dim3(256), 0, s, V, pbase);
      hipLaunchKernelGGL(kf_rm_apply, dim3(ff_grid(np)), dim3(256), 0, s, V, wst, tst);
      if ((st = ff_read(M, c))) return st;
      if (c.n_left == 0) break;
      if (c.pool_short) {
        // a removal found no room in the pool: grow it (nothing is in flight)
        const int64_t nc = F.pool_cap * 2;
        HIPCHECK(dgrow(&F.pool, 0, (size_t)nc, 0, 0, s));
        F.pool_cap = nc;
        V.pool = F.pool;
        V.pool_cap = nc;
      }
    }
    in_stamp = wst;
    if ((st = ff_lawson(M, V, cur, in_stamp, tst, c.n_list[cur]))) return st;
  }
  // final ids, renumbering, pending flags
  // ranks of the kept points: a tiled exclusive scan of alive (newid holds
  // the in-tile prefix, ntiles the tile prefixes), then the kept midpoints
  {
    const int32_t *no_halt = &F.d_c->err;  // the scan kernels stop on a nonzero word; err is 0 here
    const ScanJob j{V.alive, V.newid, &F.d_c->np, F.ntiles, &F.d_c->nwin, 0};
    const ScanJob none{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (np + kFfScanTile - 1) / kFfScanTile), 2048);
    hipLaunchKernelGGL(k_scan_tiles, dim3(g), dim3(256), 0, s, j, none, no_halt);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, j, none, no_halt);
    hipLaunchKernelGGL(kf_nwin_mid, dim3(1), dim3(64), 0, s, V);
  }
  hipLaunchKernelGGL(kf_final_point, dim3(ff_grid(np)), dim3(256), 0, s, V);
  hipLaunchKernelGGL(kf_final_tri, dim3(ff_grid(c.n_touched)), dim3(256), 0, s, V);
  hipLaunchKernelGGL(kf_final_mid, dim3(ff_grid(nmk)), dim3(256), 0, s, V);
  hipLaunchKernelGGL(kf_final_flag, dim3(ff_grid(m.nS)), dim3(256), 0, s, V);
  hipLaunchKernelGGL(kf_final_flag_clear, dim3(ff_grid(nmid)), dim3(256), 0, s, V);
  if ((st = ff_read(M, c))) return st;
  // compaction: live triangles above the final count fill the holes
  const int n_alloc = c.n_alloc, n_live = c.n_alloc - c.n_dead;
  hipLaunchKernelGGL(kf_ctl, dim3(1), dim3(64), 0, s, F.d_c, 4, 0);
  hipLaunchKernelGGL(kf_compact_list, dim3(ff_grid(c.n_dead)), dim3(256), 0, s, V, n_alloc, n_live);
  hipLaunchKernelGGL(kf_compact_move, dim3(ff_grid(c.n_dead)), dim3(256), 0, s, V);
  hipLaunchKernelGGL(kf_compact_fix, dim3(ff_grid(c.n_dead)), dim3(256), 0, s, V, n_live);
  if (c.nwin == 0 && c.flags == 0) {
    *stall = true;
    return GDP_OK;
  }
  hipLaunchKernelGGL(kf_round_end, dim3(1), dim3(256), 0, s, w, (const FfCount *)F.d_c, n_live, c.nwin, c.nwin_mid);
  HIPCHECK(hipGetLastError());
  return GDP_OK;
}

gdp_status ff_loop(gdp_mesh *M, double B2, const gdp_params *P) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  DevMesh &m = M->m;
  gdp_status st;
  if ((st = ff_canonical(M, P))) return st;
  for (;;) {
    if (m.nV >= (1 << 22)) return fail(ctx, GDP_E_INPUT, "priority mode 2 keys hold vertex ids below 2^22");
    if ((st = ff_reserve(M, 0)) || (st = ff_reset(M))) return st;
    FfBufs &F = *M->ff;
    Work w = make_work(M, P, 0);
    const int bs = P->block_size;
    const int64_t ncand = enqueue_select(M, B2, P, true, m.nT, w);
    hipLaunchKernelGGL(kf_claim_cc, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w);
    hipLaunchKernelGGL(kf_claim_mid, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, m, w);
    hipLaunchKernelGGL(kf_own, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, w, F.d_c, F.skey0, F.sref0);
    hipLaunchKernelGGL(kf_clear_marks, dim3(stride_grid(ncand, bs)), dim3(bs), 0, s, w);
    HIPCHECK(hipMemcpyAsync(M->h_st, M->d_st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(M->h_cnt, M->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    FfCount c;
    if ((st = ff_read(M, c))) return st;
    const DevState d = *M->h_st;
    const DevCounters &dc = *M->h_cnt;
    if (d.halt == kHaltDone) return GDP_OK;
    if (d.halt == kHaltCap) return fail(ctx, GDP_E_NOTERM, "round cap reached");
    if (dc.err & kErrWalk) return fail(ctx, GDP_E_WALK, "locate walk exceeded its step cap");
    if (dc.err & kErrInput)
      return fail(ctx, GDP_E_INPUT, "a walk left the mesh through a hull edge that is not a subsegment");
    if (c.np == 0) return fail(ctx, GDP_E_STALL, "round had candidates but inserted nothing");
    bool stall = false;
    if ((st = ff_line8(M, P, c.np, c.nmid, dc.nmk, &stall))) return st;
    if (stall) {
      // the mesh is whole (the points were all taken out again); nothing
      // was recorded
      HIPCHECK(hipStreamSynchronize(s));
      return fail(ctx, GDP_E_STALL, "round had candidates but inserted nothing");
    }
    HIPCHECK(hipMemcpyAsync(M->h_st, M->d_st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(M->h_hist, M->d_hist, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const DevState e = *M->h_st;
    M->stats.push_back(round_stats_of(M->h_hist[0], P));
    m.nV = e.nV; m.nT = e.nT; m.nS = e.nS; m.rounds = e.rounds;
    M->serial = e.serial;
    HIPCHECK(hipMemsetAsync(&M->d_st->halt, 0, 2 * sizeof(int32_t), s));  // halt, nhist
  }
}

gdp_status refine_loop(gdp_mesh *M, double B2, const gdp_params *P) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  DevMesh &m = M->m;
  M->stats.clear();
  M->prof = P->profile_kernels != 0;
  for (int i = 0; i < 16; i++) { M->prof_ms[i] = 0; M->prof_launches[i] = M->prof_items[i] = M->prof_bytes[i] = 0; }
  M->prof_pending.clear();
  hipEvent_t ev0, ev1;
  HIPCHECK(hipEventCreate(&ev0));
  HIPCHECK(hipEventCreate(&ev1));
  HIPCHECK(hipEventRecord(ev0, s));
  // device state from the host's copy of the counts
  DevState &hs = *M->h_st;
  memset(&hs, 0, sizeof hs);
  hs.nV = m.nV; hs.nT = m.nT; hs.nS = m.nS;
  hs.wT = words(m.nT); hs.wS = words(m.nS);
  hs.rounds = m.rounds;
  hs.serial = M->serial;
  HIPCHECK(hipMemcpyAsync(M->d_st, &hs, sizeof(DevState), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemsetAsync(M->d_cnt, 0, sizeof(DevCounters), s));
  HIPCHECK(hipMemsetAsync(M->d_stat, 0, sizeof(StatLine) * kStatStripes, s));
  gdp_status result = GDP_OK;
  // The first round of a call tests every element; later rounds carry the
  // previous bad list over and re-test only the slots the last round wrote.
  bool full = true;
  int64_t last_cand = (int64_t)m.nT + m.nS;
  int64_t last_big = 0;  // cooperative cavities of the last round
  int64_t prev_ncc = 0, prev_nmk = 0, prev_fan = 0;
  int aborts = 0;
  if (P->insert_mode == 1) result = ff_loop(M, B2, P);
  else for (;;) {
    // small rounds run in the single-workgroup engine
    const int64_t eng_max = P->tail_engine_max == 0 ? kEngineDefaultMax : P->tail_engine_max;
    const bool engine = !full && !M->engine_off && eng_max > 0 && last_cand <= eng_max && last_big <= kEngineBigMax;
    const int R = full ? 1 : rounds_for(P, last_cand, engine);
    gdp_status st;
    if (P->reserve_mode == 0 && !full && (st = reserve_group(M, last_cand, engine ? 4 : R))) return st;
    const int serial0 = M->serial;
    const size_t prof0 = M->prof_pending.size();
    if (engine) {
      if ((st = launch_engine(M, B2, P, R))) return st;
    } else if (R >= 2 && !full && !M->prof) {
      // small rounds: replays of a captured pair of rounds
      if ((st = launch_pairs(M, B2, P, serial0 & 1, R / 2, last_cand))) return st;
    } else {
      for (int i = 0; i < R; i++) {
        if ((st = enqueue_round(M, B2, P, full && i == 0, serial0 + i, full ? (int64_t)m.nT : last_cand, i)))
          return st;
      }
    }
    HIPCHECK(hipMemcpyAsync(M->h_st, M->d_st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(M->h_hist, M->d_hist, sizeof(DevCounters) * std::min(R, kHistCap),
                            hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(M->h_cnt, M->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const DevState d = *M->h_st;
    const int done = std::min(d.nhist, R);
    // profiled launches: items and algorithmic bytes of each completed round
    for (size_t k = prof0; k < M->prof_pending.size(); k++) {
      auto &r = M->prof_pending[k];
      if (r.id == P_ENGINE) {  // one launch for the whole group
        for (int i = 0; i < done; i++) r.items += (int64_t)M->h_hist[i].ncc + M->h_hist[i].nmk;
      } else if (r.round < done) {
        const DevCounters &c = M->h_hist[r.round];
        const bool f = full && r.round == 0;
        int64_t pc = prev_ncc, pmk = prev_nmk, pf = prev_fan;
        if (r.round > 0) {
          const DevCounters &q = M->h_hist[r.round - 1];
          pc = q.ncc;
          pmk = q.nmk;
          pf = q.fan_used;
        }
        // (a full collection is only ever the first round of a group)
        r.items = prof_items(r.id, c, m.nT, pc, pmk, pf, f);
        r.bytes = alg_bytes(r.id, c, m.nT, m.nV, m.nS, pc, pmk, pf, f);
      }
    }
    for (int i = 0; i < done; i++) {
      const DevCounters &c = M->h_hist[i];
      M->stats.push_back(round_stats_of(c, P));
      last_cand = (int64_t)c.ncc + c.nmk;
      last_big = c.nbig;
      prev_ncc = c.ncc;
      prev_nmk = c.nmk;
      prev_fan = c.fan_used;
    }
    if (M->prof && d.halt && M->prof_pending.size() > prof0) {
      // completed rounds stay; of the round that halted, the collection (it
      // ran) or everything it ran before it was abandoned; later rounds of
      // the group did nothing
      std::vector<gdp_mesh::ProfRec> keep(M->prof_pending.begin(), M->prof_pending.begin() + prof0);
      for (size_t k = prof0; k < M->prof_pending.size(); k++) {
        auto &r = M->prof_pending[k];
        bool ran = r.id == P_ENGINE || r.round < done ||
                   (r.round == done && (r.id == P_SCAN || d.halt == kHaltAbort));
        if (ran) keep.push_back(r);
        else { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
      }
      M->prof_pending.swap(keep);
    }
    m.nV = d.nV; m.nT = d.nT; m.nS = d.nS; m.rounds = d.rounds;
    M->serial = d.serial;
    if (done > 0) full = false;
    // restart the group bookkeeping for the next group
    HIPCHECK(hipMemsetAsync(&M->d_st->halt, 0, 2 * sizeof(int32_t), s));  // halt, nhist
    if (d.halt == 0) { aborts = 0; continue; }
    const DevCounters &c = *M->h_cnt;
    if (d.halt == kHaltDone) break;
    if (d.halt == kHaltCap) { result = fail(ctx, GDP_E_NOTERM, "round cap reached"); break; }
    if (d.halt == kHaltError) {
      if (c.err & kErrWalk) { result = fail(ctx, GDP_E_WALK, "locate walk exceeded its step cap"); break; }
      if (c.err & kErrInput) {
        result = fail(ctx, GDP_E_INPUT, "a walk left the mesh through a hull edge that is not a subsegment");
        break;
      }
      char buf[256];
      if (c.dbg_set)
        snprintf(buf, sizeof buf, "fan boundary mismatch (cc=%d elem=%d cavity=%d expected=%d found=%d state=%d)",
                 c.dbg[0], c.dbg[1], c.dbg[2], c.dbg[3], c.dbg[4], c.dbg[5]);
      else
        snprintf(buf, sizeof buf, "cavity step failed");
      result = fail(ctx, GDP_E_CAVITY, buf);
      break;
    }
    if (d.halt == kHaltStall) { result = fail(ctx, GDP_E_STALL, "round had candidates but inserted nothing"); break; }
    // kHaltAbort: nothing was written; grow and run the same round again
    if (++aborts > 16) return fail(ctx, GDP_E_NOMEM, "round keeps exceeding its buffers");
    if (c.err & kErrHuge) {  // rerun with the device-memory cavity path, on the grid kernels
      M->huge_mode = true;
      if (engine) M->engine_off = true;
    }
    if ((st = grow_after_abort(M, c, full ? 0 : d.prev_fan))) return st;
    HIPCHECK(hipMemsetAsync(M->d_cnt, 0, sizeof(DevCounters), s));
    HIPCHECK(hipMemsetAsync(M->d_stat, 0, sizeof(StatLine) * kStatStripes, s));
  }
  HIPCHECK(hipEventRecord(ev1, s));
  HIPCHECK(hipEventSynchronize(ev1));
  float ms = 0.f;
  HIPCHECK(hipEventElapsedTime(&ms, ev0, ev1));
  M->last_ms = ms;
  for (auto &r : M->prof_pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      M->prof_ms[r.id] += t;
      M->prof_launches[r.id] += 1;
      M->prof_items[r.id] += r.items;
      M->prof_bytes[r.id] += r.bytes;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  M->prof_pending.clear();
  M->prof = false;
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  return result;
}

}  // namespace

extern "C" {

void gdp_params_default(gdp_params *p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->block_size = 256;
}

const char *gdp_status_str(gdp_status s) {
  switch (s) {
    case GDP_OK: return "ok";
    case GDP_E_ARG: return "invalid argument";
    case GDP_E_INPUT: return "invalid input PSLG";
    case GDP_E_NOMEM: return "out of memory";
    case GDP_E_DEVICE: return "device error";
    case GDP_E_NOTERM: return "round cap reached";
    case GDP_E_STALL: return "refinement stalled";
    case GDP_E_BUSY: return "busy";
    case GDP_E_WALK: return "walk step cap exceeded";
    case GDP_E_CAVITY: return "cavity too large";
  }
  return "unknown status";
}

gdp_status gdp_ctx_create(int device, void *hip_stream, gdp_ctx **out) {
  if (!out) return GDP_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    g_noctx_err = "no such HIP device";
    return GDP_E_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_noctx_err = "hipSetDevice failed";
    return GDP_E_DEVICE;
  }
  resolve_scratch(device);
  gdp_ctx *c = new gdp_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return GDP_OK;
}

void gdp_ctx_destroy(gdp_ctx *ctx) { delete ctx; }

const char *gdp_last_error(const gdp_ctx *ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

gdp_status gdp_cdt_host(const gdp_pslg *pslg, int32_t *n_tri, int32_t cap_tri, int32_t *tri, int32_t *nbr,
                        int32_t *seg, char *err, int32_t err_len) {
  if (err && err_len > 0) err[0] = 0;
  if (!pslg || !n_tri) return GDP_E_ARG;
  HostMesh hm;
  std::string e;
  int rc = host_cdt_build(pslg->n_vertices, pslg->xy, pslg->n_segments, pslg->seg, hm, e);
  if (rc != GDP_OK) {
    if (err && err_len > 0) snprintf(err, (size_t)err_len, "%s", e.c_str());
    return (gdp_status)rc;
  }
  *n_tri = hm.nT;
  if (cap_tri >= hm.nT) {
    if (tri) memcpy(tri, hm.tv.data(), sizeof(int32_t) * 3 * hm.nT);
    if (nbr) memcpy(nbr, hm.tn.data(), sizeof(int32_t) * 3 * hm.nT);
    if (seg) memcpy(seg, hm.ts.data(), sizeof(int32_t) * 3 * hm.nT);
  }
  return GDP_OK;
}

gdp_status gdp_mesh_create(gdp_ctx *ctx, const gdp_pslg *pslg, gdp_mesh **out) {
  if (!ctx || !pslg || !out) return GDP_E_ARG;
  *out = nullptr;
  HostMesh hm;
  std::string e;
  int rc = host_cdt_build(pslg->n_vertices, pslg->xy, pslg->n_segments, pslg->seg, hm, e);
  if (rc != GDP_OK) return fail(ctx, (gdp_status)rc, e);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  std::vector<uint8_t> pend(hm.nS, 0);
  return upload(ctx, hm.nV, hm.nV, hm.xy.data(), nullptr, hm.nT, hm.tv.data(), hm.tn.data(), hm.ts.data(), hm.nS,
                hm.nS, hm.sv.data(), hm.sparent.data(), pend.data(), 0, out);
}

gdp_status gdp_mesh_create_device(gdp_ctx *ctx, const gdp_pslg *pslg, gdp_mesh **out) {
  if (!ctx || !pslg || !out) return GDP_E_ARG;
  *out = nullptr;
  const int32_t nv = pslg->n_vertices, ns = pslg->n_segments;
  const double *xy = pslg->xy;
  const int32_t *seg = pslg->seg;
  if (nv < 3 || !xy || ns < 0 || (ns > 0 && !seg)) return fail(ctx, GDP_E_ARG, "bad arguments");
  if (nv > (1 << 28) - 8) return fail(ctx, GDP_E_NOMEM, "mesh too large");
  // the checks of the host builder that need no sort; duplicate points and
  // repeated segments are found by the kernels
  for (int64_t i = 0; i < 2 * (int64_t)nv; i++) {
    const double a = std::fabs(xy[i]);
    if (!std::isfinite(xy[i]) || a > 0x1p20 || (a != 0.0 && a < 0x1p-100))
      return fail(ctx, GDP_E_INPUT, "coordinate not finite, or nonzero with magnitude outside [2^-100, 2^20]");
  }
  for (int32_t k = 0; k < ns; k++) {
    const int32_t a = seg[2 * k], b = seg[2 * k + 1];
    if (a < 0 || b < 0 || a >= nv || b >= nv || a == b)
      return fail(ctx, GDP_E_INPUT, "segment endpoint out of range or zero length");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  gdp_mesh *M = nullptr;
  gdp_status st = mesh_new(ctx, nv, nv, 0, ns, ns, 0, &M);
  if (st != GDP_OK) return st;
  hipStream_t s = ctx->stream;
  std::vector<int32_t> spar(ns);
  for (int32_t k = 0; k < ns; k++) spar[k] = k;
  if (hipMemcpyAsync(M->m.vxy, xy, sizeof(double2) * nv, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(M->m.vkind, 0, sizeof(int32_t) * nv, s) != hipSuccess ||
      (ns > 0 && hipMemcpyAsync(M->m.sv, seg, sizeof(int2) * ns, hipMemcpyHostToDevice, s) != hipSuccess) ||
      (ns > 0 && hipMemcpyAsync(M->m.spar, spar.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s) != hipSuccess) ||
      (ns > 0 && hipMemsetAsync(M->m.spend, 0, sizeof(int32_t) * ns, s) != hipSuccess)) {
    mesh_delete(M);
    return fail(ctx, GDP_E_DEVICE, "upload failed");
  }
  std::string e;
  int32_t nt = 0;
  DevCdtStats cs;
  const int rc = dev_cdt_build(s, nv, M->m.vxy, ns, M->m.sv, M->m.tv, M->m.tn, M->m.ts, M->m.capT, &nt, &cs, e);
  if (rc != GDP_OK) {
    mesh_delete(M);
    return fail(ctx, (gdp_status)rc, e);
  }
  M->m.nT = nt;
  M->cdt_rounds[0] = cs.dt_rounds;
  M->cdt_rounds[1] = cs.seg_rounds;
  *out = M;
  return GDP_OK;
}

gdp_status gdp_mesh_upload(gdp_ctx *ctx, int32_t n_v, int32_t n_input_v, const double *xy, const int32_t *vkind,
                           int32_t n_t, const int32_t *tri, const int32_t *nbr, const int32_t *sub_on_edge,
                           int32_t n_s, int32_t n_input_s, const int32_t *sub_v, const int32_t *sub_parent,
                           const uint8_t *sub_pending, int32_t rounds, gdp_mesh **out) {
  if (!ctx || !out) return GDP_E_ARG;
  *out = nullptr;
  if (n_v < 3 || n_t < 1 || n_s < 0 || !xy || !tri || !nbr || !sub_on_edge || (n_s > 0 && (!sub_v || !sub_parent)) ||
      n_input_v > n_v || n_input_s > n_s || rounds < 0)
    return fail(ctx, GDP_E_ARG, "bad mesh arrays");
  for (int64_t i = 0; i < 3 * (int64_t)n_t; i++) {
    if (tri[i] < 0 || tri[i] >= n_v || nbr[i] < -1 || nbr[i] >= n_t || sub_on_edge[i] < -1 || sub_on_edge[i] >= n_s)
      return fail(ctx, GDP_E_ARG, "mesh index out of range");
  }
  for (int64_t i = 0; i < 2 * (int64_t)n_s; i++)
    if (sub_v[i] < 0 || sub_v[i] >= n_v) return fail(ctx, GDP_E_ARG, "subsegment vertex out of range");
  for (int64_t i = 0; i < 2 * (int64_t)n_v; i++) {
    double a = fabs(xy[i]);
    if (!std::isfinite(xy[i]) || a > 0x1p20 || (a != 0.0 && a < 0x1p-100))
      return fail(ctx, GDP_E_ARG, "coordinate out of range");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  return upload(ctx, n_v, n_input_v, xy, vkind, n_t, tri, nbr, sub_on_edge, n_s, n_input_s, sub_v, sub_parent,
                sub_pending, rounds, out);
}

static gdp_status check_params(gdp_ctx *ctx, const gdp_params *params, gdp_params &P) {
  if (params) P = *params; else gdp_params_default(&P);
  if (P.block_size == 0) P.block_size = 256;
  if (P.prefilter_f1 != 0 && P.prefilter_f1 != 1) return fail(ctx, GDP_E_ARG, "prefilter_f1 must be 0 or 1");
  if (P.cavity_approx_n < 0 || P.cavity_approx_n > kApproxMaxN)
    return fail(ctx, GDP_E_ARG, "cavity_approx_n must be in [0, 16]");
  if (P.cand_cap_K < 0 || P.max_rounds < 0 || P.priority_mode < 0 || P.priority_mode > 2)
    return fail(ctx, GDP_E_ARG, "bad parameter");
  if (P.insert_mode != 0 && P.insert_mode != 1) return fail(ctx, GDP_E_ARG, "insert_mode must be 0 or 1");
  if (P.insert_mode == 1 && P.priority_mode != 2)
    return fail(ctx, GDP_E_ARG, "Flip-Flop insertion needs priority_mode 2 (keys independent of slots)");
  // the cavity kernels recover a mark's owner from the perm32 tie-break in
  // the low half of its key, which mode 2 keys do not carry
  if (P.insert_mode == 0 && P.priority_mode == 2)
    return fail(ctx, GDP_E_ARG, "priority_mode 2 is for Flip-Flop insertion (insert_mode 1)");
  if (P.block_size < 64 || P.block_size > 1024 || P.block_size % 64) return fail(ctx, GDP_E_ARG, "bad block size");
  if (P.reserve_mode != 0 && P.reserve_mode != 1) return fail(ctx, GDP_E_ARG, "bad reserve mode");
  if (P.rounds_per_sync < 0 || P.rounds_per_sync > kHistCap)
    return fail(ctx, GDP_E_ARG, "rounds_per_sync must be in [0, 64]");
  if (P.encroach_mode != 0 && P.encroach_mode != 1) return fail(ctx, GDP_E_ARG, "encroach_mode must be 0 or 1");
  if (P.split_mode != 0 && P.split_mode != 1) return fail(ctx, GDP_E_ARG, "split_mode must be 0 or 1");
  if (!(P.max_edge_len_sq >= 0.0) || !std::isfinite(P.max_edge_len_sq))
    return fail(ctx, GDP_E_ARG, "max_edge_len_sq must be finite and >= 0");
  if (P.batch_engine_max_v < 0) return fail(ctx, GDP_E_ARG, "batch_engine_max_v must be >= 0");
  if (P.cavity_thread_cap != 0 && P.cavity_thread_cap != 12 && P.cavity_thread_cap != 24 &&
      P.cavity_thread_cap != kCavCapDefault)
    return fail(ctx, GDP_E_ARG, "cavity_thread_cap must be 0, 12, 24 or 39");
  return GDP_OK;
}

gdp_status gdp_mesh_refine(gdp_ctx *ctx, gdp_mesh *mesh, double ratio_bound_sq, const gdp_params *params) {
  if (!ctx || !mesh || mesh->ctx != ctx) return GDP_E_ARG;
  gdp_params P;
  gdp_status st;
  if ((st = check_params(ctx, params, P))) return st;
  if (!(ratio_bound_sq > 0.0) || !std::isfinite(ratio_bound_sq)) return fail(ctx, GDP_E_ARG, "bad ratio bound");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  if ((st = detach(mesh))) return st;
  return refine_loop(mesh, ratio_bound_sq, &P);
}

gdp_status gdp_refine_batch(gdp_ctx *ctx, const gdp_pslg *pslgs, const double *ratio_bound_sq,
                            const gdp_params *params, int32_t count, gdp_mesh **outs, gdp_status *status,
                            double *elapsed_ms) {
  if (!ctx || count < 0 || (count > 0 && (!pslgs || !ratio_bound_sq || !outs))) return GDP_E_ARG;
  gdp_params P;
  gdp_status st;
  if ((st = check_params(ctx, params, P))) return st;
  if (P.insert_mode != 0) return fail(ctx, GDP_E_ARG, "the batched form runs cavity insertion only");
  for (int32_t i = 0; i < count; i++)
    if (!(ratio_bound_sq[i] > 0.0) || !std::isfinite(ratio_bound_sq[i])) return fail(ctx, GDP_E_ARG, "bad ratio bound");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  return refine_batch(ctx, pslgs, ratio_bound_sq, &P, count, outs, status, elapsed_ms);
}

gdp_status gdp_refine(gdp_ctx *ctx, const gdp_pslg *pslg, double ratio_bound_sq, const gdp_params *params,
                      gdp_mesh **out) {
  if (!out) return GDP_E_ARG;
  *out = nullptr;
  gdp_mesh *m = nullptr;
  gdp_status st = gdp_mesh_create(ctx, pslg, &m);
  if (st != GDP_OK) return st;
  st = gdp_mesh_refine(ctx, m, ratio_bound_sq, params);
  if (st != GDP_OK && st != GDP_E_NOTERM) {
    gdp_mesh_free(m);
    return st;
  }
  *out = m;
  return st;
}

gdp_status gdp_mesh_info_get(const gdp_mesh *mesh, gdp_mesh_info *info) {
  if (!mesh || !info) return GDP_E_ARG;
  info->n_vertices = mesh->m.nV;
  info->n_triangles = mesh->m.nT;
  info->n_subsegments = mesh->m.nS;
  info->n_input_vertices = mesh->m.n_input_v;
  info->n_input_segments = mesh->m.n_input_s;
  info->rounds = mesh->m.rounds;
  info->cdt_point_rounds = mesh->cdt_rounds[0];
  info->cdt_segment_rounds = mesh->cdt_rounds[1];
  int64_t fb = 0;
  for (const gdp_round_stats &r : mesh->stats)
    fb += r.n_exact_orient + r.n_exact_dot + r.n_exact_incircle_b + r.n_exact_incircle_c;
  info->fallbacks = fb;
  return GDP_OK;
}

gdp_status gdp_mesh_device_views(const gdp_mesh *mesh, gdp_device_views *out) {
  if (!mesh || !out) return GDP_E_ARG;
  const DevMesh &m = mesh->m;
  out->n_vertices = m.nV;
  out->n_triangles = m.nT;
  out->n_subsegments = m.nS;
  out->tri_stride = 4;
  out->xy = (const double *)m.vxy;
  out->vkind = m.vkind;
  out->tri = (const int32_t *)m.tv;
  out->nbr = (const int32_t *)m.tn;
  out->sub_on_edge = (const int32_t *)m.ts;
  out->sub_v = (const int32_t *)m.sv;
  out->sub_parent = m.spar;
  out->sub_pending = m.spend;
  return GDP_OK;
}

gdp_status gdp_bench_atomic_max(gdp_ctx *ctx, int64_t n_slots, int64_t n_ops, double *ms) {
  if (!ctx || n_slots <= 0 || n_ops <= 0 || !ms) return ctx ? fail(ctx, GDP_E_ARG, "bad atomic benchmark size") : GDP_E_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = ctx->stream;
  uint64_t *table = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipMalloc((void **)&table, sizeof(uint64_t) * (size_t)n_slots) != hipSuccess)
    return fail(ctx, GDP_E_NOMEM, "atomic benchmark table");
  hipError_t e = hipMemsetAsync(table, 0, sizeof(uint64_t) * (size_t)n_slots, s);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  // one launch warms the table and the code object, the second is timed
  const unsigned grid = 256 * 32;
  for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
    if (rep == 1) e = hipEventRecord(a, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_atomic_max_bench, dim3(grid), dim3(256), 0, s, table, (uint64_t)n_slots, n_ops,
                         (uint64_t)(rep + 1) * 0x2545f4914f6cdd1dull);
      e = hipGetLastError();
    }
    if (rep == 1 && e == hipSuccess) e = hipEventRecord(b, s);
  }
  float t = 0.f;
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(table);
  if (e != hipSuccess) return fail(ctx, GDP_E_DEVICE, std::string("atomic benchmark: ") + hipGetErrorString(e));
  *ms = t;
  return GDP_OK;
}

gdp_status gdp_predicates_eval(gdp_ctx *ctx, int32_t kind, int32_t n, const double *pts, int32_t *signs,
                               int64_t *stage_counts) {
  if (kind < 0 || kind > 3 || n < 0 || (n > 0 && (!pts || !signs))) return ctx ? fail(ctx, GDP_E_ARG, "bad predicate query") : GDP_E_ARG;
  const int w = kind == 1 ? 8 : 6;
  if (!ctx) {
    uint64_t tally[kTallyStride] = {};
    for (int32_t i = 0; i < n; i++) {
      const double *q = pts + (size_t)i * w;
      int r;
      if (kind == 0) r = orient2d(q[0], q[1], q[2], q[3], q[4], q[5], tally);
      else if (kind == 1) r = incircle(q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], tally);
      else if (kind == 2) r = indiametral(q[0], q[1], q[2], q[3], q[4], q[5], tally);
      else r = encroaches(1, q[0], q[1], q[2], q[3], q[4], q[5], tally) ? 1 : 0;
      signs[i] = r;
    }
    if (stage_counts)
      for (int e = 0; e < kExStages; e++) stage_counts[e] = (int64_t)tally[kTally0 + e];
    return GDP_OK;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = ctx->stream;
  const size_t tally_words = (size_t)kTallyStripes * kTallyStride;
  double *d_pts = nullptr;
  int32_t *d_out = nullptr;
  uint64_t *d_tally = nullptr;
  std::vector<uint64_t> h_tally(tally_words);
  hipError_t e = hipMalloc((void **)&d_pts, sizeof(double) * std::max<size_t>(1, (size_t)n * w));
  if (e == hipSuccess) e = hipMalloc((void **)&d_out, sizeof(int32_t) * std::max<int32_t>(1, n));
  if (e == hipSuccess) e = hipMalloc((void **)&d_tally, sizeof(uint64_t) * tally_words);
  if (e == hipSuccess && n > 0)
    e = hipMemcpyAsync(d_pts, pts, sizeof(double) * (size_t)n * w, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(d_tally, 0, sizeof(uint64_t) * tally_words, s);
  if (e == hipSuccess && n > 0) {
    hipLaunchKernelGGL(k_predicates, dim3((n + 255) / 256), dim3(256), 0, s, (int)kind, (int)n,
                       (const double *)d_pts, d_out, d_tally);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(signs, d_out, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_tally.data(), d_tally, sizeof(uint64_t) * tally_words, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_pts);
  (void)hipFree(d_out);
  (void)hipFree(d_tally);
  if (e != hipSuccess) return fail(ctx, GDP_E_DEVICE, std::string("predicate evaluation: ") + hipGetErrorString(e));
  if (stage_counts)
    for (int x = 0; x < kExStages; x++) {
      int64_t sum = 0;
      for (int i = 0; i < kTallyStripes; i++) sum += (int64_t)h_tally[(size_t)i * kTallyStride + kTally0 + x];
      stage_counts[x] = sum;
    }
  return GDP_OK;
}

gdp_status gdp_mesh_quality_noalloc(gdp_ctx *ctx, const gdp_mesh *mesh, double ratio_bound_sq,
                                    double max_edge_len_sq, unsigned long long *d_n_bad, double *d_bad_area) {
  if (!ctx || !mesh || mesh->ctx != ctx || !d_n_bad || !d_bad_area) return GDP_E_ARG;
  if (!(ratio_bound_sq > 0.0) || !std::isfinite(ratio_bound_sq) || !(max_edge_len_sq >= 0.0) ||
      !std::isfinite(max_edge_len_sq))
    return fail(ctx, GDP_E_ARG, "bad quality bound");
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kQualBlocks, ((int64_t)mesh->m.nT + 255) / 256));
  const size_t need = (size_t)g * (sizeof(unsigned long long) + sizeof(double));
  if (need > kScratchBytes) return fail(ctx, GDP_E_ARG, "quality partials exceed the static scratch buffer");
  void *base = scratch_ptr(ctx->device);
  if (!base) return fail(ctx, GDP_E_DEVICE, "static scratch buffer address not resolved for this device");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = ctx->stream;
  // the partials are written by every workgroup before they are read: nothing to clear
  auto *n_part = (unsigned long long *)base;
  auto *a_part = (double *)((char *)base + sizeof(unsigned long long) * kQualBlocks);
  hipLaunchKernelGGL(k_quality, dim3(g), dim3(256), 0, s, mesh->m, ratio_bound_sq, max_edge_len_sq, n_part, a_part);
  hipLaunchKernelGGL(k_quality_sum, dim3(1), dim3(64), 0, s, (int)g, n_part, a_part, d_n_bad, d_bad_area);
  if (hipGetLastError() != hipSuccess) return fail(ctx, GDP_E_DEVICE, "quality kernels failed to launch");
  return GDP_OK;
}

gdp_status gdp_mesh_quality(gdp_ctx *ctx, const gdp_mesh *mesh, double ratio_bound_sq, double max_edge_len_sq,
                            int64_t *n_bad, double *bad_area) {
  if (!ctx || !mesh || mesh->ctx != ctx || !n_bad || !bad_area) return GDP_E_ARG;
  if (!(ratio_bound_sq > 0.0) || !std::isfinite(ratio_bound_sq) || !(max_edge_len_sq >= 0.0) ||
      !std::isfinite(max_edge_len_sq))
    return fail(ctx, GDP_E_ARG, "bad quality bound");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  hipStream_t s = ctx->stream;
  // partials [kQualBlocks] and the totals, then a copy back
  const size_t bytes = (size_t)(kQualBlocks + 1) * (sizeof(unsigned long long) + sizeof(double));
  char *buf = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return fail(ctx, GDP_E_NOMEM, "allocation failed");
  auto *n_part = (unsigned long long *)buf;
  auto *a_part = (double *)(buf + sizeof(unsigned long long) * (kQualBlocks + 1));
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kQualBlocks, ((int64_t)mesh->m.nT + 255) / 256));
  hipLaunchKernelGGL(k_quality, dim3(g), dim3(256), 0, s, mesh->m, ratio_bound_sq, max_edge_len_sq, n_part, a_part);
  hipLaunchKernelGGL(k_quality_sum, dim3(1), dim3(64), 0, s, (int)g, n_part, a_part, n_part + kQualBlocks,
                     a_part + kQualBlocks);
  unsigned long long hn = 0;
  double ha = 0.0;
  bool ok = hipGetLastError() == hipSuccess &&
            hipMemcpyAsync(&hn, n_part + kQualBlocks, sizeof hn, hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipMemcpyAsync(&ha, a_part + kQualBlocks, sizeof ha, hipMemcpyDeviceToHost, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;
  (void)hipFree(buf);
  if (!ok) return fail(ctx, GDP_E_DEVICE, "quality kernels failed");
  *n_bad = (int64_t)hn;
  *bad_area = ha;
  return GDP_OK;
}

gdp_status gdp_mesh_download(gdp_ctx *ctx, const gdp_mesh *mesh, double *xy, int32_t *vkind, int32_t *tri,
                             int32_t *nbr, int32_t *sub_on_edge, int32_t *sub_v, int32_t *sub_parent,
                             uint8_t *sub_pending) {
  if (!ctx || !mesh) return GDP_E_ARG;
  hipStream_t s = ctx->stream;
  const DevMesh &m = mesh->m;
  if (xy) {
    std::vector<double2> h(m.nV);
    HIPCHECK(hipMemcpyAsync(h.data(), m.vxy, sizeof(double2) * m.nV, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int i = 0; i < m.nV; i++) { xy[2 * i] = h[i].x; xy[2 * i + 1] = h[i].y; }
  }
  if (vkind) {
    HIPCHECK(hipMemcpyAsync(vkind, m.vkind, sizeof(int32_t) * m.nV, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  int4 *arrs[3] = {m.tv, m.tn, m.ts};
  int32_t *outs[3] = {tri, nbr, sub_on_edge};
  for (int a = 0; a < 3; a++) {
    if (!outs[a]) continue;
    std::vector<int4> h(m.nT);
    HIPCHECK(hipMemcpyAsync(h.data(), arrs[a], sizeof(int4) * m.nT, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int t = 0; t < m.nT; t++) {
      outs[a][3 * t] = h[t].x;
      outs[a][3 * t + 1] = h[t].y;
      outs[a][3 * t + 2] = h[t].z;
    }
  }
  if (sub_v) {
    HIPCHECK(hipMemcpyAsync(sub_v, m.sv, sizeof(int2) * m.nS, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  if (sub_parent) {
    HIPCHECK(hipMemcpyAsync(sub_parent, m.spar, sizeof(int32_t) * m.nS, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  if (sub_pending) {
    std::vector<int32_t> h(m.nS);
    HIPCHECK(hipMemcpyAsync(h.data(), m.spend, sizeof(int32_t) * m.nS, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int k = 0; k < m.nS; k++) sub_pending[k] = (uint8_t)h[k];
  }
  return GDP_OK;
}

gdp_status gdp_mesh_round_stats(const gdp_mesh *mesh, gdp_round_stats *stats, int32_t cap, int32_t *n) {
  if (!mesh || !n) return GDP_E_ARG;
  int32_t k = (int32_t)mesh->stats.size();
  *n = k;
  if (stats)
    for (int32_t i = 0; i < std::min(k, cap); i++) stats[i] = mesh->stats[i];
  return GDP_OK;
}

gdp_status gdp_mesh_last_refine_ms(const gdp_mesh *mesh, double *ms) {
  if (!mesh || !ms) return GDP_E_ARG;
  *ms = mesh->last_ms;
  return GDP_OK;
}

gdp_status gdp_mesh_kernel_profile(const gdp_mesh *mesh, gdp_kernel_prof *out, int32_t cap, int32_t *n) {
  if (!mesh || !n) return GDP_E_ARG;
  *n = P_NUM;
  if (out)
    for (int i = 0; i < std::min<int>(cap, P_NUM); i++) {
      memset(&out[i], 0, sizeof out[i]);
      snprintf(out[i].name, sizeof out[i].name, "%s", kProfNames[i]);
      out[i].launches = mesh->prof_launches[i];
      out[i].total_ms = mesh->prof_ms[i];
      out[i].items = mesh->prof_items[i];
      out[i].alg_bytes = mesh->prof_bytes[i];
    }
  return GDP_OK;
}

gdp_status gdp_mesh_assign(gdp_ctx *ctx, gdp_mesh *dst, const gdp_mesh *src) {
  if (!ctx || !dst || !src || dst->ctx != ctx || src->ctx != ctx || dst == src) return GDP_E_ARG;
  gdp_status st;
  if ((st = detach(dst))) return st;
  const DevMesh &a = src->m;
  if ((st = grow_vtx(dst, a.nV))) return st;
  if ((st = grow_tri(dst, a.nT))) return st;
  if ((st = grow_seg(dst, a.nS))) return st;
  if ((st = grow_cand(dst))) return st;
  DevMesh &b = dst->m;
  hipStream_t s = ctx->stream;
  HIPCHECK(hipMemcpyAsync(b.vxy, a.vxy, sizeof(double2) * a.nV, hipMemcpyDeviceToDevice, s));
  HIPCHECK(hipMemcpyAsync(b.vkind, a.vkind, sizeof(int32_t) * a.nV, hipMemcpyDeviceToDevice, s));
  HIPCHECK(hipMemcpyAsync(b.tv, a.tv, sizeof(int4) * a.nT, hipMemcpyDeviceToDevice, s));
  HIPCHECK(hipMemcpyAsync(b.tn, a.tn, sizeof(int4) * a.nT, hipMemcpyDeviceToDevice, s));
  HIPCHECK(hipMemcpyAsync(b.ts, a.ts, sizeof(int4) * a.nT, hipMemcpyDeviceToDevice, s));
  if (a.nS) {
    HIPCHECK(hipMemcpyAsync(b.sv, a.sv, sizeof(int2) * a.nS, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(b.spar, a.spar, sizeof(int32_t) * a.nS, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(b.spend, a.spend, sizeof(int32_t) * a.nS, hipMemcpyDeviceToDevice, s));
  }
  // per-round workspace back to its between-rounds state
  HIPCHECK(hipMemsetAsync(dst->mark, 0, sizeof(uint64_t) * b.capT, s));
  HIPCHECK(hipMemsetAsync(dst->mflag, 0, sizeof(uint32_t) * b.capS, s));
  HIPCHECK(hipMemsetAsync(dst->sadj, 0xff, sizeof(int32_t) * 2 * (size_t)b.capS, s));
  HIPCHECK(hipMemsetAsync(dst->w0_t, 0, sizeof(uint32_t) * words(b.capT), s));
  HIPCHECK(hipMemsetAsync(dst->win_t, 0, sizeof(uint32_t) * words(b.capT), s));
  HIPCHECK(hipMemsetAsync(dst->w0_s, 0, sizeof(uint32_t) * words(b.capS), s));
  HIPCHECK(hipMemsetAsync(dst->win_s, 0, sizeof(uint32_t) * words(b.capS), s));
  b.nV = a.nV; b.nT = a.nT; b.nS = a.nS;
  b.n_input_v = a.n_input_v; b.n_input_s = a.n_input_s; b.rounds = a.rounds;
  HIPCHECK(hipStreamSynchronize(s));
  return GDP_OK;
}

gdp_status gdp_mesh_clone(gdp_ctx *ctx, const gdp_mesh *src, gdp_mesh **out) {
  if (!ctx || !src || !out || src->ctx != ctx) return GDP_E_ARG;
  *out = nullptr;
  gdp_mesh *M = new gdp_mesh();
  M->ctx = ctx;
  gdp_status st;
  auto chk = [&](hipError_t e) { return e == hipSuccess; };
  if ((st = grow_vtx(M, src->m.capV)) || (st = grow_tri(M, src->m.capT)) || (st = grow_seg(M, src->m.capS)) ||
      (st = grow_cand(M))) {
    free_mesh_arrays(M);
    delete M;
    return st;
  }
  if ((st = alloc_control(M))) {
    free_mesh_arrays(M);
    delete M;
    return st;
  }
  M->pool_cap = src->pool_cap;
  M->fan_cap = src->fan_cap;
  if (!chk(dalloc(&M->pool, M->pool_cap)) || !chk(dalloc(&M->fan, M->fan_cap))) {
    free_mesh_arrays(M);
    delete M;
    return fail(ctx, GDP_E_NOMEM, "allocation failed");
  }
  if ((st = gdp_mesh_assign(ctx, M, src))) {
    free_mesh_arrays(M);
    delete M;
    return st;
  }
  *out = M;
  return GDP_OK;
}

void gdp_mesh_free(gdp_mesh *mesh) {
  if (!mesh) return;
  free_mesh_arrays(mesh);
  delete mesh;
}


gdp_status gdp_server_create(gdp_ctx *ctx, size_t hbm_budget, int32_t max_slots, gdp_server **out) {
  if (!ctx || !out || max_slots < 1 || hbm_budget < (1u << 20)) return GDP_E_ARG;
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  gdp_server *S = new gdp_server();
  S->user = ctx;
  S->max_slots = max_slots;
  S->t0 = std::chrono::steady_clock::now();
  S->mem = new ServerMem();
  S->mem->size = hbm_budget;
  bool ok = hipMalloc(&S->mem->base, hbm_budget) == hipSuccess;
  if (ok) S->mem->free_ranges[0] = hbm_budget;
  for (int i = 0; ok && i < max_slots; i++) {
    ServerWorker *W = new ServerWorker();
    W->ctx.device = ctx->device;
    S->workers.push_back(W);
    ok = hipStreamCreateWithFlags(&W->ctx.stream, hipStreamNonBlocking) == hipSuccess &&
         hipHostMalloc((void **)&W->h_cnt, sizeof(DevCounters)) == hipSuccess &&
         hipHostMalloc((void **)&W->h_st, sizeof(DevState)) == hipSuccess &&
         hipHostMalloc((void **)&W->h_hist, sizeof(DevCounters) * kHistCap) == hipSuccess &&
         dalloc(&W->d_eng, 1) == hipSuccess && dalloc(&W->d_head, 1) == hipSuccess &&
         hipHostMalloc((void **)&W->h_eng, sizeof(EngDesc)) == hipSuccess;
  }
  if (!ok) {
    for (ServerWorker *W : S->workers) {
      if (W->ctx.stream) (void)hipStreamDestroy(W->ctx.stream);
      if (W->h_cnt) (void)hipHostFree(W->h_cnt);
      if (W->h_st) (void)hipHostFree(W->h_st);
      if (W->h_hist) (void)hipHostFree(W->h_hist);
      if (W->d_eng) (void)hipFree(W->d_eng);
      if (W->d_head) (void)hipFree(W->d_head);
      if (W->h_eng) (void)hipHostFree(W->h_eng);
      delete W;
    }
    if (S->mem->base) (void)hipFree(S->mem->base);
    delete S->mem;
    delete S;
    return fail(ctx, GDP_E_NOMEM, "server allocation failed");
  }
  ServerEngine *E = ok ? new ServerEngine() : nullptr;
  if (E) {
    S->eng = E;
    E->ctx.device = ctx->device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
      E->cus = prop.multiProcessorCount;
    ok = hipStreamCreateWithFlags(&E->ctx.stream, hipStreamNonBlocking) == hipSuccess &&
         dalloc(&E->d_desc, kSrvEngMax) == hipSuccess && dalloc(&E->d_head, 1) == hipSuccess &&
         hipHostMalloc((void **)&E->h_desc, sizeof(EngDesc) * kSrvEngMax) == hipSuccess &&
         hipHostMalloc((void **)&E->h_st, sizeof(DevState) * kSrvEngMax) == hipSuccess &&
         hipHostMalloc((void **)&E->h_cnt, sizeof(DevCounters) * kSrvEngMax) == hipSuccess &&
         hipHostMalloc((void **)&E->h_hist, sizeof(DevCounters) * kHistCap * kSrvEngMax) == hipSuccess;
  }
  if (!ok) {
    free_server_engine(E);
    for (ServerWorker *W : S->workers) {
      (void)hipStreamDestroy(W->ctx.stream);
      (void)hipHostFree(W->h_cnt);
      (void)hipHostFree(W->h_st);
      (void)hipHostFree(W->h_hist);
      (void)hipFree(W->d_eng);
      (void)hipFree(W->d_head);
      (void)hipHostFree(W->h_eng);
      delete W;
    }
    (void)hipFree(S->mem->base);
    delete S->mem;
    delete S;
    return fail(ctx, GDP_E_NOMEM, "server allocation failed");
  }
  ServerGang *Gn = new ServerGang();
  Gn->ctx.device = ctx->device;
  ok = hipStreamCreateWithFlags(&Gn->ctx.stream, hipStreamNonBlocking) == hipSuccess &&
       gang_bufs_alloc(Gn->bufs, max_slots);
  if (!ok) {
    free_server_gang(Gn);
    free_server_engine(E);
    for (ServerWorker *W : S->workers) {
      (void)hipStreamDestroy(W->ctx.stream);
      (void)hipHostFree(W->h_cnt);
      (void)hipHostFree(W->h_st);
      (void)hipHostFree(W->h_hist);
      (void)hipFree(W->d_eng);
      (void)hipFree(W->d_head);
      (void)hipHostFree(W->h_eng);
      delete W;
    }
    (void)hipFree(S->mem->base);
    delete S->mem;
    delete S;
    return fail(ctx, GDP_E_NOMEM, "server allocation failed");
  }
  S->gang = Gn;
  S->engine_max_v = kSrvEngineDefaultMaxV;
  for (ServerWorker *W : S->workers) W->th = std::thread(server_worker, S, W);
  E->th = std::thread(engine_dispatcher, S, E);
  Gn->th = std::thread(gang_driver, S, Gn);
  *out = S;
  return GDP_OK;
}

gdp_status gdp_server_mode(gdp_server *srv, int32_t mode, int32_t rounds_per_group) {
  if (!srv || mode < 0 || mode > 1 || rounds_per_group < 0 || rounds_per_group > kGangRoundsMax) return GDP_E_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  srv->mode = mode;
  srv->gang_rounds = rounds_per_group ? rounds_per_group : kGangRounds;
  srv->cv.notify_all();
  return GDP_OK;
}

gdp_status gdp_server_engine_jobs(gdp_server *srv, int32_t max_input_vertices) {
  if (!srv || max_input_vertices < 0) return GDP_E_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  srv->engine_max_v = max_input_vertices;
  srv->cv.notify_all();
  return GDP_OK;
}

gdp_status gdp_server_prepare(gdp_server *srv, const gdp_pslg *pslg, double ratio_bound_sq, const gdp_params *params,
                              uint64_t *job) {
  if (!srv || !pslg || !job) return GDP_E_ARG;
  gdp_params P;
  gdp_status st;
  if ((st = check_params(srv->user, params, P))) return st;
  if (P.insert_mode != 0) return fail(srv->user, GDP_E_ARG, "the serving form runs cavity insertion only");
  if (!(ratio_bound_sq > 0.0) || !std::isfinite(ratio_bound_sq)) return fail(srv->user, GDP_E_ARG, "bad ratio bound");
  Job *J = new Job();
  if ((st = prepare_job(srv, pslg, ratio_bound_sq, &P, J))) {
    delete J;
    return st;
  }
  std::lock_guard<std::mutex> g(srv->mu);
  J->id = srv->next_id++;
  srv->jobs[J->id] = J;
  *job = J->id;
  return GDP_OK;
}

gdp_status gdp_server_arrive(gdp_server *srv, uint64_t job) {
  if (!srv) return GDP_E_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->jobs.find(job);
  if (it == srv->jobs.end() || it->second->state != Job::PREPARED) return GDP_E_ARG;
  Job *J = it->second;
  J->t_submit = ms_since(srv->t0);
  if (J->raw) {
    J->state = Job::LINE1;
    const bool dev = srv->l1dev && srv->l1_dev_min_v > 0 && J->nv_in >= srv->l1_dev_min_v && srv->mode == 0 &&
                     !for_engine(srv, J);
    (dev ? srv->l1_dev : srv->l1_host).push_back(J);
  } else {
    J->state = Job::QUEUED;
    srv->queue.push_back(J);
  }
  srv->cv.notify_all();
  return GDP_OK;
}

gdp_status gdp_server_line1(gdp_server *srv, int32_t host_threads, int32_t device_min_vertices) {
  if (!srv || host_threads < 1 || host_threads > 64 || device_min_vertices < 0) return GDP_E_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->l1_threads > 0 || !srv->jobs.empty()) return fail(srv->user, GDP_E_BUSY, "Line 1 is set before the first job");
  if (device_min_vertices > 0) {
    ServerLine1Dev *D = new ServerLine1Dev();
    D->ctx.device = srv->user->device;
    if (hipSetDevice(D->ctx.device) != hipSuccess ||
        hipStreamCreateWithFlags(&D->ctx.stream, hipStreamNonBlocking) != hipSuccess) {
      delete D;
      return fail(srv->user, GDP_E_DEVICE, "stream creation failed");
    }
    srv->l1dev = D;
    srv->l1_dev_min_v = device_min_vertices;
    D->th = std::thread(line1_dev_worker, srv, D);
  }
  srv->l1_threads = host_threads;
  for (int i = 0; i < host_threads; i++) srv->l1_workers.emplace_back(line1_host_worker, srv);
  return GDP_OK;
}

gdp_status gdp_server_submit(gdp_server *srv, const gdp_pslg *pslg, double ratio_bound_sq, const gdp_params *params,
                             uint64_t *job) {
  gdp_status st = gdp_server_prepare(srv, pslg, ratio_bound_sq, params, job);
  if (st != GDP_OK) return st;
  return gdp_server_arrive(srv, *job);
}

static gdp_status server_take(gdp_server *srv, uint64_t job, gdp_mesh **out, gdp_job_times *times, bool wait) {
  if (!srv) return GDP_E_ARG;
  if (out) *out = nullptr;
  std::unique_lock<std::mutex> g(srv->mu);
  auto it = srv->jobs.find(job);
  if (it == srv->jobs.end()) return GDP_E_ARG;
  Job *J = it->second;
  if (wait) srv->cv.wait(g, [&] { return J->state == Job::DONE || srv->stop; });
  if (times) {
    times->submit_ms = J->t_submit;
    times->line1_ms = J->t_line1;
    times->admit_ms = J->t_admit;
    times->done_ms = J->t_done;
  }
  if (J->state != Job::DONE) return GDP_E_BUSY;
  gdp_status st = J->status;
  if (J->mesh) {
    J->mesh->ctx = srv->user;
    if (out) *out = J->mesh;
    else gdp_mesh_free(J->mesh);
  }
  srv->jobs.erase(it);
  delete J;
  return st;
}

gdp_status gdp_server_poll(gdp_server *srv, uint64_t job, gdp_mesh **out, gdp_job_times *times) {
  return server_take(srv, job, out, times, false);
}

gdp_status gdp_server_wait(gdp_server *srv, uint64_t job, gdp_mesh **out, gdp_job_times *times) {
  return server_take(srv, job, out, times, true);
}

void gdp_server_destroy(gdp_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv.notify_all();
  }
  for (std::thread &t : srv->l1_workers) t.join();
  if (srv->l1dev) {
    srv->l1dev->th.join();
    (void)hipStreamDestroy(srv->l1dev->ctx.stream);
    dev_cdt_work_free(srv->l1dev->ws);
    delete srv->l1dev;
  }
  for (ServerWorker *W : srv->workers) W->th.join();
  if (srv->eng) srv->eng->th.join();
  if (srv->gang) srv->gang->th.join();
  free_server_engine(srv->eng);
  free_server_gang(srv->gang);
  for (auto &kv : srv->jobs) {
    if (kv.second->mesh) gdp_mesh_free(kv.second->mesh);
    delete kv.second;
  }
  for (ServerWorker *W : srv->workers) {
    (void)hipStreamDestroy(W->ctx.stream);
    (void)hipHostFree(W->h_cnt);
    (void)hipHostFree(W->h_st);
    (void)hipHostFree(W->h_hist);
    (void)hipFree(W->d_eng);
    (void)hipFree(W->d_head);
    (void)hipHostFree(W->h_eng);
    delete W;
  }
  ServerMem *sm = srv->mem;
  bool last;
  {
    std::lock_guard<std::mutex> g(sm->mu);
    sm->closed = true;
    last = sm->live == 0;
  }
  if (last) {
    (void)hipFree(sm->base);
    delete sm;
  }
  delete srv;
}
}  // extern "C"

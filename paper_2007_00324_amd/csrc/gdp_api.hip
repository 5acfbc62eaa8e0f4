// gdp_api.hip -- C ABI (include/gdp2d.h): contexts, meshes in device memory
// and the host loop that issues one refinement round after another
// (Algorithm 1, "repeat ... until L is empty").
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gdp_kernels.h"

using namespace gdp;

struct gdp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
};

struct gdp_mesh {
  gdp_ctx *ctx = nullptr;
  DevMesh m;
  DevCounters *d_cnt = nullptr;
  DevCounters *h_cnt = nullptr;  // pinned
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
  int32_t *prev_cc_elem = nullptr;
  uint64_t *prev_cc_key = nullptr;
  double2 *prev_cc_p = nullptr;
  int32_t *prev_mid_elem = nullptr;
  int32_t *tstamp = nullptr;
  int32_t *cidx_t = nullptr, *cidx_s = nullptr;
  int32_t serial = 0;  // rounds ever executed on this mesh object (slot stamps)
  uint64_t *keys = nullptr;
  int32_t *hist = nullptr;
  uint64_t *thresh = nullptr;
  int32_t *tiles = nullptr;
  int32_t tiles_cap = 0;
  int32_t *h_small = nullptr;  // pinned scratch for small reads
  int32_t wT = 0, wS = 0;      // workspace capacities (triangles, subsegments)
  std::vector<gdp_round_stats> stats;
  double last_ms = 0.0;
  // optional per-kernel timing (HIP events around every launch)
  bool prof = false;
  struct ProfRec {
    int id;
    hipEvent_t a, b;
    int64_t items, bytes;
  };
  std::vector<ProfRec> prof_pending;
  double prof_ms[16] = {};
  int64_t prof_launches[16] = {}, prof_items[16] = {}, prof_bytes[16] = {};
};

namespace {
enum ProfId {
  P_SCAN = 0, P_CAP, P_LOCATE, P_CAV_CC, P_CAV_MID, P_CAV_BIG, P_MARK, P_OWN, P_DEP, P_PREFIX,
  P_WINNERS, P_RECORD, P_WRITE, P_FINISH, P_NUM
};
const char *kProfNames[P_NUM] = {"k_scan", "k_cap", "k_locate", "k_cavity_cc", "k_cavity_mid", "k_cavity_big",
                                  "k_mark", "k_own", "k_dep", "k_prefix_sum", "k_winners", "k_record", "k_write",
                                  "k_finish"};
// Records HIP events around the launches issued in its scope (if enabled).
struct Prof {
  gdp_mesh *M;
  int id;
  hipEvent_t a = nullptr;
  int64_t items, bytes;
  Prof(gdp_mesh *M_, int id_, int64_t items_ = 0, int64_t bytes_ = 0) : M(M_), id(id_), items(items_), bytes(bytes_) {
    if (M->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, M->ctx->stream);
  }
  ~Prof() {
    if (!M->prof || !a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, M->ctx->stream);
    M->prof_pending.push_back({id, a, b, items, bytes});
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

gdp_status grow_tri(gdp_mesh *M, int32_t need) {
  gdp_ctx *ctx = M->ctx;
  if (need <= M->m.capT) return GDP_OK;
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
  M->m.capT = nc;
  return GDP_OK;
}

gdp_status grow_seg(gdp_mesh *M, int32_t need) {
  gdp_ctx *ctx = M->ctx;
  if (need <= M->m.capS) return GDP_OK;
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
  HIPCHECK(dgrow(&M->tiles, 0, nt, 0, 0, s));
  M->tiles_cap = (int32_t)nt;
  M->wT = (int32_t)nc;
  return GDP_OK;
}

Work make_work(gdp_mesh *M, int pm) {
  Work w;
  w.cnt = M->d_cnt;
  w.mark = M->mark;
  w.sadj = M->sadj;
  w.mflag = M->mflag;
  w.cc = M->cc;
  w.mid = M->mid;
  w.w0_t = M->w0_t; w.w0_s = M->w0_s; w.win_t = M->win_t; w.win_s = M->win_s;
  w.rank_t = M->rank_t; w.rank_s = M->rank_s;
  w.win_ref = M->win_ref; w.fbase = M->fbase; w.fcount = M->fcount; w.fan_off = M->fan_off;
  w.win_cap = M->wT;
  w.repl = M->repl;
  w.pool = M->pool; w.pool_cap = M->pool_cap;
  w.fan = M->fan; w.fan_cap = M->fan_cap;
  w.big = M->big; w.big_cap = M->wT;
  w.prev_cc_elem = M->prev_cc_elem; w.prev_cc_key = M->prev_cc_key; w.prev_cc_p = M->prev_cc_p;
  w.prev_mid_elem = M->prev_mid_elem; w.tstamp = M->tstamp;
  w.cidx_t = M->cidx_t; w.cidx_s = M->cidx_s;
  w.keys = M->keys; w.hist = M->hist; w.thresh = M->thresh;
  w.pm = pm;
  return w;
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// Exclusive scan of n entries (mode 0: counts, mode 1: popcounts of words);
// the total is written to *d_total.
// Exclusive scan (mode 0: counts, mode 1: popcounts of words).  n is the
// length, or an upper bound when n_dev points to the length in device memory;
// the total goes to *d_total.
gdp_status scan(gdp_mesh *M, const int32_t *in, int32_t *out, int n, int32_t *d_total, int mode,
                const int32_t *n_dev = nullptr) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  int ntiles = (n + kScanTileSize - 1) / kScanTileSize;
  if (ntiles < 1) ntiles = 1;
  if (ntiles > M->tiles_cap) return fail(ctx, GDP_E_NOMEM, "scan tile buffer too small");
  Prof pr(M, P_PREFIX, n);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, in, out, n, M->tiles, mode, n_dev);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, M->tiles, ntiles, d_total, n_dev);
  hipLaunchKernelGGL(k_scan_add, dim3(std::min<unsigned>(grid_for(std::max(n, 1), 256), 4096)), dim3(256), 0, s,
                     out, n, M->tiles, n_dev);
  HIPCHECK(hipGetLastError());
  return GDP_OK;
}

gdp_status read_counters(gdp_mesh *M) {
  gdp_ctx *ctx = M->ctx;
  HIPCHECK(hipMemcpyAsync(M->h_cnt, M->d_cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  return GDP_OK;
}

void free_mesh_arrays(gdp_mesh *M) {
  void *ptrs[] = {M->m.vxy, M->m.vkind, M->m.tv, M->m.tn, M->m.ts, M->m.sv, M->m.spar, M->m.spend,
                  M->d_cnt, M->mark, M->sadj, M->mflag,
                  M->cc.elem, M->cc.key, M->cc.p, M->cc.loc, M->cc.state, M->cc.off, M->cc.len,
                  M->mid.elem, M->mid.key, M->mid.p, M->mid.loc, M->mid.state, M->mid.off, M->mid.len,
                  M->w0_t, M->w0_s, M->win_t, M->win_s, M->rank_t, M->rank_s, M->win_ref, M->fbase,
                  M->fcount, M->fan_off, M->repl, M->pool, M->fan, M->big, M->keys, M->hist, M->thresh,
                  M->tiles, M->prev_cc_elem, M->prev_cc_key, M->prev_cc_p, M->prev_mid_elem, M->tstamp,
                  M->cidx_t, M->cidx_s};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (M->h_cnt) (void)hipHostFree(M->h_cnt);
  if (M->h_small) (void)hipHostFree(M->h_small);
}

// Allocates a device mesh with room for the given counts and uploads it.
gdp_status upload(gdp_ctx *ctx, int32_t nV, int32_t nIV, const double *xy, const int32_t *vkind,
                  int32_t nT, const int32_t *tv, const int32_t *tn, const int32_t *ts, int32_t nS,
                  int32_t nIS, const int32_t *sv, const int32_t *spar, const uint8_t *spend,
                  int32_t rounds, gdp_mesh **out) {
  hipStream_t s = ctx->stream;
  gdp_mesh *M = new gdp_mesh();
  M->ctx = ctx;
  auto bail = [&](gdp_status st) {
    free_mesh_arrays(M);
    delete M;
    return st;
  };
  M->m.nV = nV; M->m.nT = nT; M->m.nS = nS;
  M->m.n_input_v = nIV; M->m.n_input_s = nIS; M->m.rounds = rounds;
  int32_t capV = std::max(1024, nV * 2), capT = std::max(2048, nT * 2), capS = std::max(1024, nS * 2);
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
  M->m.capV = 0; M->m.capT = 0; M->m.capS = 0;
  gdp_status st;
  if ((st = grow_vtx(M, capV)) != GDP_OK) return bail(st);
  if ((st = grow_tri(M, capT)) != GDP_OK) return bail(st);
  if ((st = grow_seg(M, capS)) != GDP_OK) return bail(st);
  if ((st = grow_cand(M)) != GDP_OK) return bail(st);
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
      !chk(hipMemcpyAsync(M->m.spend, hpend.data(), sizeof(int32_t) * nS, hipMemcpyHostToDevice, s), "upload"))
    return bail(GDP_E_DEVICE);
  if (!chk(dalloc(&M->d_cnt, 1), "alloc") || !chk(hipHostMalloc((void **)&M->h_cnt, sizeof(DevCounters)), "alloc") ||
      !chk(hipHostMalloc((void **)&M->h_small, 1024 * sizeof(int32_t)), "alloc") ||
      !chk(dalloc(&M->hist, 256), "alloc") || !chk(dalloc(&M->thresh, 1), "alloc"))
    return bail(GDP_E_DEVICE);
  M->pool_cap = std::max(1 << 16, 8 * capT);
  if (!chk(dalloc(&M->pool, M->pool_cap), "alloc")) return bail(GDP_E_DEVICE);
  M->fan_cap = std::max(1 << 16, 2 * capT);
  if (!chk(dalloc(&M->fan, M->fan_cap), "alloc")) return bail(GDP_E_DEVICE);
  if (!chk(hipStreamSynchronize(s), "sync")) return bail(GDP_E_DEVICE);
  *out = M;
  return GDP_OK;
}

// Grid for a grid-stride kernel over at most n items.
inline unsigned stride_grid(int64_t n, int bs) {
  return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + bs - 1) / bs), 8192);
}

// Ensures the buffers a round may need, given the scan's counts (a loose
// bound; the device-side check abandons the round if it is not enough).
gdp_status reserve_round(gdp_mesh *M, int ncc, int nmk) {
  gdp_ctx *ctx = M->ctx;
  const DevMesh &m = M->m;
  int64_t wins = (int64_t)ncc + nmk + (ncc >> 3) + 64;
  gdp_status st;
  if ((st = grow_vtx(M, (int32_t)std::min<int64_t>(m.nV + wins, 1 << 29)))) return st;
  if ((st = grow_tri(M, (int32_t)std::min<int64_t>(m.nT + 2 * wins, 1 << 29)))) return st;
  if ((st = grow_seg(M, (int32_t)std::min<int64_t>(m.nS + nmk + (ncc >> 3) + 64, 1 << 28)))) return st;
  if ((st = grow_cand(M))) return st;
  int64_t pool_need = 6 * ((int64_t)ncc + nmk) + 4096;
  if (pool_need > M->pool_cap) {
    int64_t nc = std::max<int64_t>(pool_need, (int64_t)M->pool_cap * 3 / 2);
    if (nc > (1LL << 30)) return fail(ctx, GDP_E_NOMEM, "cavity pool limit exceeded");
    HIPCHECK(dgrow(&M->pool, M->pool_cap, nc, 0, 0, ctx->stream));
    M->pool_cap = (int32_t)nc;
  }
  int64_t fan_need = std::min<int64_t>(M->pool_cap, pool_need) + 2 * wins;
  if (fan_need > M->fan_cap) {
    int64_t nc = std::max<int64_t>(fan_need, (int64_t)M->fan_cap * 3 / 2);
    if (nc > (1LL << 30)) return fail(ctx, GDP_E_NOMEM, "fan buffer limit exceeded");
    HIPCHECK(dgrow(&M->fan, M->fan_cap, nc, 0, 0, ctx->stream));
    M->fan_cap = (int32_t)nc;
  }
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
    HIPCHECK(dgrow(&M->pool, M->pool_cap, nc, 0, 0, ctx->stream));
    M->pool_cap = (int32_t)nc;
  }
  int64_t fan_need = (int64_t)std::max(c.pool_used, M->pool_cap) + 2 * (int64_t)nwin + 1024;
  if (fan_need > M->fan_cap) {
    if (fan_need > (1LL << 30)) return fail(ctx, GDP_E_NOMEM, "fan buffer limit exceeded");
    HIPCHECK(dgrow(&M->fan, M->fan_cap, fan_need, keep_fan, 0, ctx->stream));
    M->fan_cap = (int32_t)fan_need;
  }
  return GDP_OK;
}

// One refinement call: rounds until nothing is left (Algorithm 1, "repeat
// ... until L is empty").  Each round has two host synchronisations: after
// the collection (termination, capacity, candidate cap) and at its end.
gdp_status refine_loop(gdp_mesh *M, double B2, const gdp_params *P) {
  gdp_ctx *ctx = M->ctx;
  hipStream_t s = ctx->stream;
  const int bs = P->block_size;
  const int pm = P->priority_mode;
  M->stats.clear();
  M->prof = P->profile_kernels != 0;
  for (int i = 0; i < 16; i++) { M->prof_ms[i] = 0; M->prof_launches[i] = M->prof_items[i] = M->prof_bytes[i] = 0; }
  M->prof_pending.clear();
  hipEvent_t ev0, ev1;
  HIPCHECK(hipEventCreate(&ev0));
  HIPCHECK(hipEventCreate(&ev1));
  HIPCHECK(hipEventRecord(ev0, s));
  gdp_status result = GDP_OK;
  // The first round of a call tests every element; later rounds carry the
  // previous bad list over and re-test only the slots the last round wrote.
  bool full_scan = true;
  int prev_ncc = 0, prev_nmk = 0, prev_fan = 0;
  int aborts = 0;
  for (;;) {
    DevMesh &m = M->m;
    gdp_status st;
    HIPCHECK(hipMemsetAsync(M->d_cnt, 0, sizeof(DevCounters), s));
    Work w = make_work(M, pm);
    size_t scan_rec = M->prof_pending.size();
    if (full_scan) {
      Prof pr(M, P_SCAN, m.nT);
      hipLaunchKernelGGL(k_scan, dim3(grid_for(std::max(m.nT, m.nS), bs)), dim3(bs), 0, s, m, w, B2, pm);
    } else {
      Prof pr(M, P_SCAN, (int64_t)prev_ncc + prev_fan + prev_nmk);
      hipLaunchKernelGGL(k_carry, dim3(grid_for(prev_ncc, bs)), dim3(bs), 0, s, w, prev_ncc, M->serial - 1);
      hipLaunchKernelGGL(k_scan_dirty, dim3(grid_for(prev_fan, bs)), dim3(bs), 0, s, m, w, prev_fan, B2, pm);
      hipLaunchKernelGGL(k_pending, dim3(grid_for(prev_nmk, bs)), dim3(bs), 0, s, m, w, prev_nmk);
    }
    HIPCHECK(hipGetLastError());
    if ((st = read_counters(M))) return st;  // sync 1
    const int ncc = M->h_cnt->ncc;
    const int nmk0 = M->h_cnt->nmk;
    if (M->prof && scan_rec < M->prof_pending.size())
      // algorithmic bytes of the collection.  Full: every triangle record
      // (16 B) and vertex (16 B) once, both sides of every subsegment (ts
      // record 16 B + side slot 4 B each), pending flags (4 B), the bad records
      // written (elem 4 + key 8 + point 16 + state 4 B) and the flagged
      // subsegments (flag 4 + list entry 8 B).  Incremental: carried records
      // (elem 4 + key 8 + point 16 read and written, stamp 4), each rewritten
      // slot (fan slot 4 + record 16 + three vertices 48) and the previous
      // flagged list (entry 4 + pending flag 4), plus the new records / flags.
      M->prof_pending[scan_rec].bytes =
          full_scan ? 16LL * m.nT + 16LL * m.nV + 40LL * m.nS + 4LL * m.nS + 32LL * ncc + 12LL * nmk0
                    : 64LL * prev_ncc + 68LL * prev_fan + 8LL * prev_nmk + 32LL * ncc + 12LL * nmk0;
    gdp_round_stats rs;
    memset(&rs, 0, sizeof rs);
    rs.n_bad = ncc;
    rs.n_enc = nmk0;
    if (ncc == 0 && nmk0 == 0) break;
    if (P->max_rounds > 0 && m.rounds >= P->max_rounds) {
      hipLaunchKernelGGL(k_unflag, dim3(grid_for(nmk0, bs)), dim3(bs), 0, s, w, nmk0);
      HIPCHECK(hipGetLastError());
      result = fail(ctx, GDP_E_NOTERM, "round cap reached");
      break;
    }
    if (P->reserve_mode == 0 && (st = reserve_round(M, ncc, nmk0))) return st;
    w = make_work(M, pm);
    // ---- R3: candidate cap ----
    bool capped = P->cand_cap_K > 0 && ncc + nmk0 > P->cand_cap_K;
    if (capped) {
      int n = ncc + nmk0;
      Prof pr(M, P_CAP, n);
      hipLaunchKernelGGL(k_gather_keys, dim3(grid_for(n, bs)), dim3(bs), 0, s, m, w, ncc, nmk0, pm);
      uint64_t prefix = 0, pmask = 0;
      int64_t remaining = P->cand_cap_K;
      for (int shift = 56; shift >= 0; shift -= 8) {
        HIPCHECK(hipMemsetAsync(M->hist, 0, 256 * sizeof(int32_t), s));
        hipLaunchKernelGGL(k_radix_hist, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0, s, w, n,
                           shift, prefix, pmask);
        HIPCHECK(hipMemcpyAsync(M->h_small, M->hist, 256 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        int64_t cum = 0;
        int d = 255;
        for (; d > 0; d--) {
          if (cum + M->h_small[d] >= remaining) break;
          cum += M->h_small[d];
        }
        remaining -= cum;
        prefix |= (uint64_t)d << shift;
        pmask |= (uint64_t)0xff << shift;
      }
      HIPCHECK(hipMemcpyAsync(M->thresh, &prefix, sizeof(uint64_t), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_apply_cap, dim3(grid_for(n, bs)), dim3(bs), 0, s, w, ncc, nmk0);
      HIPCHECK(hipGetLastError());
    } else {
      rs.n_kept_cc = ncc;
      rs.n_kept_mid = nmk0;
    }
    // Bound on the midpoint list after R4/R5 (each list entry is a distinct
    // subsegment, twice at most with the cap).
    const int nmk_bound = (int)std::min<int64_t>(2LL * m.nS, (int64_t)nmk0 + ncc + (int64_t)m.nS);
    const int ncand_bound = ncc + nmk_bound;
    // ---- R4: locate ----
    {
      Prof pr(M, P_LOCATE, ncc);
      hipLaunchKernelGGL(k_locate, dim3(grid_for(ncc, bs)), dim3(bs), 0, s, m, w, ncc);
    }
    // ---- optional prefilters F1 / F2 on located circumcenters ----
    if (P->prefilter_f1)
      for (int mode = 0; mode < 3; mode++)
        hipLaunchKernelGGL(k_prefilter, dim3(grid_for(ncc, 128)), dim3(128), 0, s, m, w, ncc, mode, 0);
    if (P->cavity_approx_n > 0)
      for (int mode = 3; mode < 6; mode++)
        hipLaunchKernelGGL(k_prefilter, dim3(grid_for(ncc, 128)), dim3(128), 0, s, m, w, ncc, mode,
                           P->cavity_approx_n);
    // ---- R5/R6 cavities (marks placed as each valid cavity completes) ----
    {
      Prof pr(M, P_CAV_CC, ncc);
      hipLaunchKernelGGL(k_cavity, dim3(grid_for(ncc, kCavBlockSize)), dim3(kCavBlockSize), 0, s, m, w, ncc, 1);
    }
    {
      Prof pr(M, P_CAV_BIG, 0);
      hipLaunchKernelGGL(k_cavity_big, dim3(256), dim3(kBigBlockSize), 0, s, m, w, 0);
    }
    {
      Prof pr(M, P_CAV_MID, nmk0);
      hipLaunchKernelGGL(k_cavity, dim3(stride_grid(nmk_bound, kCavBlockSize)), dim3(kCavBlockSize), 0, s, m, w,
                         0, 0);
    }
    {
      Prof pr(M, P_CAV_BIG, 0);
      hipLaunchKernelGGL(k_cavity_big, dim3(256), dim3(kBigBlockSize), 0, s, m, w, 1);
    }
    // ---- R8 ownership, R9 dependency ----
    {
      Prof pr(M, P_OWN, ncand_bound);
      hipLaunchKernelGGL(k_own, dim3(stride_grid(ncand_bound, bs)), dim3(bs), 0, s, w, ncc);
    }
    {
      Prof pr(M, P_DEP, ncand_bound);
      hipLaunchKernelGGL(k_dep, dim3(stride_grid(ncand_bound, bs)), dim3(bs), 0, s, m, w, ncc);
    }
    // ---- R10: ranks, fresh slots, capacity check, insertion ----
    if ((st = scan(M, (const int32_t *)M->win_s, M->rank_s, words(m.nS), &M->d_cnt->nwin_mid, 1))) return st;
    if ((st = scan(M, (const int32_t *)M->win_t, M->rank_t, words(m.nT), &M->d_cnt->nwin_cc, 1))) return st;
    hipLaunchKernelGGL(k_nwin, dim3(1), dim3(64), 0, s, w);
    {
      Prof pr(M, P_WINNERS, ncand_bound);
      hipLaunchKernelGGL(k_winners, dim3(stride_grid(ncand_bound, bs)), dim3(bs), 0, s, w, ncc);
    }
    if ((st = scan(M, M->fcount, M->fbase, ncand_bound + 1, &M->d_cnt->pad[0], 0, &M->d_cnt->nwin1))) return st;
    hipLaunchKernelGGL(k_check_capacity, dim3(1), dim3(64), 0, s, m, w);
    {
      Prof pr(M, P_RECORD, ncand_bound);
      hipLaunchKernelGGL(k_record, dim3(stride_grid(ncand_bound, bs)), dim3(bs), 0, s, m, w);
    }
    {
      Prof pr(M, P_WRITE, ncand_bound);
      hipLaunchKernelGGL(k_write, dim3(stride_grid(ncand_bound, bs)), dim3(bs), 0, s, m, w, M->serial);
    }
    {
      Prof pr(M, P_FINISH, ncand_bound);
      hipLaunchKernelGGL(k_finish, dim3(stride_grid(ncand_bound, bs)), dim3(bs), 0, s, m, w, ncc);
    }
    HIPCHECK(hipGetLastError());
    if ((st = read_counters(M))) return st;  // sync 2
    DevCounters &c = *M->h_cnt;
    if (c.err & kErrWalk) { result = fail(ctx, GDP_E_WALK, "locate walk exceeded its step cap"); break; }
    if (c.err & kErrInput) {
      result = fail(ctx, GDP_E_INPUT, "a walk left the mesh through a hull edge that is not a subsegment");
      break;
    }
    if (c.err & kErrCavity) {
      char buf[256];
      if (c.dbg_set)
        snprintf(buf, sizeof buf, "fan boundary mismatch (cc=%d elem=%d cavity=%d expected=%d found=%d state=%d)",
                 c.dbg[0], c.dbg[1], c.dbg[2], c.dbg[3], c.dbg[4], c.dbg[5]);
      else
        snprintf(buf, sizeof buf, "cavity exceeded the cooperative-path capacity");
      result = fail(ctx, GDP_E_CAVITY, buf);
      break;
    }
    if (c.abort) {
      // nothing was written: grow and run the same round again
      if (++aborts > 16) return fail(ctx, GDP_E_NOMEM, "round keeps exceeding its buffers");
      DevCounters cc = c;
      if ((st = grow_after_abort(M, cc, full_scan ? 0 : prev_fan))) return st;
      continue;
    }
    aborts = 0;
    const int nmk = c.nmk, nwin_mid = c.nwin_mid, nwin_cc = c.nwin_cc, nwin = c.nwin, fresh = c.fresh_total;
    if (nwin == 0) { result = fail(ctx, GDP_E_STALL, "round had candidates but inserted nothing"); break; }
    if (capped) {
      rs.n_kept_cc = c.n_kept_cc;
      rs.n_kept_mid = c.n_kept_mid;
    }
    rs.n_blocked = c.n_blocked;
    rs.n_coincident = c.n_coincident;
    rs.n_enc_reject = c.n_enc_reject;
    rs.n_unsplittable = c.n_unsplittable;
    rs.n_fan_invalid = c.n_fan_invalid;
    rs.n_lost_mark = c.n_lost_mark;
    rs.n_dep_drop = c.n_dep_drop;
    rs.n_ins_mid = nwin_mid;
    rs.n_ins_cc = nwin_cc;
    rs.cav_tri_total = c.cav_tri_total;
    rs.cav_max = c.cav_max;
    rs.n_big_cavities = c.nbig;
    rs.n_mid_cand = c.n_mid_cand;
    rs.n_f1_drop = c.n_f1_drop;
    rs.n_f2_drop = c.n_f2_drop;
    M->stats.push_back(rs);
    m.nV += nwin;
    m.nT += fresh;
    m.nS += nwin_mid;
    m.rounds += 1;
    M->serial += 1;
    // this round's lists become the previous ones
    prev_ncc = ncc;
    prev_nmk = nmk;
    prev_fan = c.fan_used;
    std::swap(M->cc.elem, M->prev_cc_elem);
    std::swap(M->cc.key, M->prev_cc_key);
    std::swap(M->cc.p, M->prev_cc_p);
    std::swap(M->mid.elem, M->prev_mid_elem);
    full_scan = false;
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

gdp_status gdp_mesh_refine(gdp_ctx *ctx, gdp_mesh *mesh, double ratio_bound_sq, const gdp_params *params) {
  if (!ctx || !mesh || mesh->ctx != ctx) return GDP_E_ARG;
  gdp_params P;
  if (params) P = *params; else gdp_params_default(&P);
  if (P.block_size == 0) P.block_size = 256;
  if (!(ratio_bound_sq > 0.0) || !std::isfinite(ratio_bound_sq)) return fail(ctx, GDP_E_ARG, "bad ratio bound");
  if (P.prefilter_f1 != 0 && P.prefilter_f1 != 1) return fail(ctx, GDP_E_ARG, "prefilter_f1 must be 0 or 1");
  if (P.cavity_approx_n < 0 || P.cavity_approx_n > kApproxMaxN)
    return fail(ctx, GDP_E_ARG, "cavity_approx_n must be in [0, 16]");
  if (P.cand_cap_K < 0 || P.max_rounds < 0 || (P.priority_mode != 0 && P.priority_mode != 1))
    return fail(ctx, GDP_E_ARG, "bad parameter");
  if (P.block_size < 64 || P.block_size > 1024 || P.block_size % 64) return fail(ctx, GDP_E_ARG, "bad block size");
  if (P.reserve_mode != 0 && P.reserve_mode != 1) return fail(ctx, GDP_E_ARG, "bad reserve mode");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, GDP_E_DEVICE, "hipSetDevice failed");
  return refine_loop(mesh, ratio_bound_sq, &P);
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
  if (!chk(dalloc(&M->d_cnt, 1)) || !chk(hipHostMalloc((void **)&M->h_cnt, sizeof(DevCounters))) ||
      !chk(hipHostMalloc((void **)&M->h_small, 1024 * sizeof(int32_t))) || !chk(dalloc(&M->hist, 256)) ||
      !chk(dalloc(&M->thresh, 1))) {
    free_mesh_arrays(M);
    delete M;
    return fail(ctx, GDP_E_NOMEM, "allocation failed");
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

}  // extern "C"

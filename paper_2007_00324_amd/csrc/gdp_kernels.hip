// gdp_kernels.hip -- gfx950 kernels of one refinement round (Algorithm 1,
// Lines 3-8 of gDP2d, with cavity insertion as in Section 5.2).
//
// Every kernel works on a slot-indexed structure-of-arrays mesh in HBM.  The
// round is deterministic: candidate lists are built with atomics in any
// order, but every decision depends only on the mesh at the start of the
// round, on 64-bit priority keys (unique per element) and on atomicMax,
// which is order independent; vertex ids, triangle slots and subsegment ids
// of the inserted points come from prefix sums over element-indexed bitmaps.
#include "gdp_kernels.h"

namespace gdp {

// ---------------------------------------------------------------------------
// Priorities (Section 4.3: midpoints before circumcenters, then larger
// length / area first; the element id, mixed by a fixed bijection, makes
// every key unique).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t perm32(uint32_t x) {
  // MurmurHash3 32-bit finalizer applied to id + 1 (never 0)
  uint32_t h = x + 1u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__device__ __forceinline__ uint32_t perm32_inv(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7ed1b41du;  // inverse of 0xc2b2ae35 mod 2^32
  h ^= (h >> 13) ^ (h >> 26);
  h *= 0xa5cb9243u;  // inverse of 0x85ebca6b mod 2^32
  h ^= h >> 16;
  return h - 1u;
}

__device__ __forceinline__ uint32_t q31(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  return (uint32_t)((b >> 32) & 0x7fffffffu);
}

__device__ __forceinline__ int comp(const int4 &v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }

struct SplitPt {
  double px, py;
  uint64_t key;
  int bad;
  double d;  // doubled area by the fixed formula (triangles)
};

// Circumcenter / radius-edge test / key of triangle t, in one fixed FP64
// operation order (vertices rotated so the smallest id comes first); a
// needle (non-positive FP64 doubled area, or a circumcenter beyond 2^20)
// is bad, has measure 0 and splits at the midpoint of its longest edge.
__device__ SplitPt tri_split(const DevMesh &m, int t, int4 tri, double B2, double L2, int pm) {
  int v0 = tri.x, v1 = tri.y, v2 = tri.z, ia, ib, ic;
  if (v0 < v1 && v0 < v2) { ia = v0; ib = v1; ic = v2; }
  else if (v1 < v2) { ia = v1; ib = v2; ic = v0; }
  else { ia = v2; ib = v0; ic = v1; }
  double2 A = m.vxy[ia], B = m.vxy[ib], C = m.vxy[ic];
  double ax = A.x, ay = A.y;
  double bx = B.x - ax, by = B.y - ay;
  double cx = C.x - ax, cy = C.y - ay;
  double b2 = bx * bx + by * by;
  double c2 = cx * cx + cy * cy;
  double d = bx * cy - by * cx;
  double ex = C.x - B.x, ey = C.y - B.y;
  double e2 = ex * ex + ey * ey;
  SplitPt r;
  uint64_t q = 0;
  bool needle = true;
  if (d > 0.0) {
    double den = d + d;
    double ux = (cy * b2 - by * c2) / den;
    double uy = (bx * c2 - cx * b2) / den;
    double px = ax + ux, py = ay + uy;
    if (fabs(px) <= 0x1p20 && fabs(py) <= 0x1p20) {
      needle = false;
      r.px = px;
      r.py = py;
      double r2 = ux * ux + uy * uy;
      double lmin2 = b2;
      if (c2 < lmin2) lmin2 = c2;
      if (e2 < lmin2) lmin2 = e2;
      r.bad = r2 > B2 * lmin2 ? 1 : 0;
      if (L2 > 0.0) {
        // edge-length bound (Section 4.1): the longest edge against l^2
        double lmax2 = b2;
        if (c2 > lmax2) lmax2 = c2;
        if (e2 > lmax2) lmax2 = e2;
        if (lmax2 > L2) r.bad = 1;
      }
      q = q31(d);
    }
  }
  if (needle) {
    double2 U = A, W = B;
    double best = b2;
    if (c2 > best) { best = c2; U = A; W = C; }
    if (e2 > best) { best = e2; U = B; W = C; }
    r.px = (U.x + W.x) * 0.5;
    r.py = (U.y + W.y) * 0.5;
    r.bad = 1;
    q = 0;
  }
  if (pm == 1) q = 0;
  // mode 2: a tie-break that does not depend on the slot (the first two ids
  // of the rotation that starts at the smallest id, 22 bits each), above it
  // the measure reduced to 19 bits
  if (pm == 2) r.key = ((q >> 12) << 44) | ((uint64_t)ia << 22) | (uint64_t)ib;
  else r.key = (q << 32) | (uint64_t)perm32((uint32_t)t);
  r.d = d;
  return r;
}

// Splitting point of subsegment k: its midpoint, or with split_mode 1
// (concentric shells) when exactly one endpoint c is an input vertex, the
// point at distance 2^j from c, 2^j the power of two nearest to half the
// length (2^e if len/2 = f 2^e with f > 3/4, else 2^(e-1)), so that
// subsegments meeting at a small input angle are cut on common circles.
__device__ SplitPt seg_split(const DevMesh &m, int k, int pm, int split_mode) {
  int2 s = m.sv[k];
  double2 A = m.vxy[s.x], B = m.vxy[s.y];
  SplitPt r;
  double dx = B.x - A.x, dy = B.y - A.y;
  double len2 = dx * dx + dy * dy;
  const bool ina = split_mode == 1 && m.vkind[s.x] == 0, inb = split_mode == 1 && m.vkind[s.y] == 0;
  if (ina != inb) {
    const double2 C = ina ? A : B, O = ina ? B : A;
    const double len = sqrt(len2);
    int e;
    const double f = frexp(len * 0.5, &e);
    const double d = f > 0.75 ? ldexp(1.0, e) : ldexp(1.0, e - 1);
    const double t = d / len;
    r.px = C.x + (O.x - C.x) * t;
    r.py = C.y + (O.y - C.y) * t;
  } else {
    r.px = (A.x + B.x) * 0.5;
    r.py = (A.y + B.y) * 0.5;
  }
  uint64_t q = pm == 1 ? 0 : (uint64_t)q31(len2);
  r.key = (1ull << 63) | (q << 32) | (uint64_t)perm32((uint32_t)k);
  r.bad = 1;
  return r;
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
// A variable-size allocation by one wave (all 64 lanes take part): one
// atomic per wave instead of one per lane.
__device__ __forceinline__ int wave_alloc(int *counter, int n) {
  int lane = __lane_id();
  int x = n;
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  int total = __shfl(x, 63);
  int base = 0;
  if (lane == 63 && total > 0) base = atomicAdd(counter, total);
  base = __shfl(base, 63);
  return base + x - n;
}

// Encroachment of subsegment ab by p under the round's mode (circle or lens).
__device__ __forceinline__ bool encroached(const Work &w, double2 a, double2 b, double2 p) {
  return encroaches(w.enc_mode, a.x, a.y, b.x, b.y, p.x, p.y, w.tally);
}

// Entry idx of the midpoint list: subsegment k.
__device__ __forceinline__ void put_mid(const Work &w, int idx, int k) {
  w.mid.elem[idx] = k;
  w.mid.state[idx] = 0;
  w.cidx_s[k] = idx;
}

// Flags subsegment k; the first flag of the round appends it to the list.
// (One lane at a time: used where flags are rare; the collection gathers its
// flags and appends them per workgroup, see push_mids.)
__device__ __forceinline__ void flag_mid(const Work &w, int k) {
  if (atomicOr(&w.mflag[k], 1u) == 0u) put_mid(w, atomicAdd(&w.cnt->nmk, 1), k);
}

// Round statistics: a wave-wide sum (every lane of the wave takes part)
// added by one lane to the stat line of the wave.
__device__ __forceinline__ StatLine *stat_line(const Work &w) {
  const unsigned wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  return w.stat + (wave & (kStatStripes - 1));
}
__device__ __forceinline__ void stat_add(const Work &w, int f, uint64_t v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  if (__lane_id() == 0 && v) atomicAdd((unsigned long long *)&stat_line(w)->v[f], (unsigned long long)v);
}
// Four small statistics summed at once: each lane's values must stay below
// 2^10 (the per-thread cavity slices bound them), so a wave's sums fit the
// 16-bit fields of one 64-bit word.
__device__ __forceinline__ void stat_add4(const Work &w, const int f[4], uint32_t a, uint32_t b, uint32_t c,
                                         uint32_t d) {
  uint64_t v = (uint64_t)a | ((uint64_t)b << 16) | ((uint64_t)c << 32) | ((uint64_t)d << 48);
  for (int k = 32; k > 0; k >>= 1) v += __shfl_xor(v, k);
  if (__lane_id() == 0 && v) {
    StatLine *l = stat_line(w);
    for (int i = 0; i < 4; i++) {
      const uint64_t x = (v >> (16 * i)) & 0xffffu;
      if (x) atomicAdd((unsigned long long *)&l->v[f[i]], (unsigned long long)x);
    }
  }
}
// Two statistics summed at once whose wave sums fit 32 bits.
__device__ __forceinline__ void stat_add2(const Work &w, int f0, int f1, uint32_t a, uint32_t b) {
  uint64_t v = (uint64_t)a | ((uint64_t)b << 32);
  for (int k = 32; k > 0; k >>= 1) v += __shfl_xor(v, k);
  if (__lane_id() == 0 && v) {
    StatLine *l = stat_line(w);
    if (v & 0xffffffffu) atomicAdd((unsigned long long *)&l->v[f0], (unsigned long long)(v & 0xffffffffu));
    if (v >> 32) atomicAdd((unsigned long long *)&l->v[f1], (unsigned long long)(v >> 32));
  }
}
__device__ __forceinline__ void stat_max(const Work &w, int f, uint64_t v) {
  for (int d = 32; d > 0; d >>= 1) v = max(v, (uint64_t)__shfl_xor(v, d));
  if (__lane_id() == 0 && v) atomicMax((unsigned long long *)&stat_line(w)->v[f], (unsigned long long)v);
}

__device__ __forceinline__ bool bit_get(const uint32_t *bm, int i) { return (bm[i >> 5] >> (i & 31)) & 1u; }
__device__ __forceinline__ void bit_set(uint32_t *bm, int i) { atomicOr(&bm[i >> 5], 1u << (i & 31)); }

// Rank of bit i among the set bits of bm: the scanned popcounts of the words
// before it (word prefix + tile prefix) and the set bits below it in its word.
__device__ __forceinline__ int bit_rank(const uint32_t *bm, const int32_t *words_prefix, const int32_t *tiles, int i) {
  uint32_t w = bm[i >> 5];
  uint32_t below = (i & 31) ? (w & ((1u << (i & 31)) - 1u)) : 0u;
  return words_prefix[i >> 5] + tiles[(i >> 5) / kScanTileSize] + __popc(below);
}

// Exclusive prefix of the fresh-slot counts at winner r.
__device__ __forceinline__ int fbase_at(const Work &w, int r) { return w.fbase[r] + w.tiles_f[r / kScanTileSize]; }

__device__ __forceinline__ int orient_pts(const Work &w, double2 a, double2 b, double2 c) {
  return orient2d(a.x, a.y, b.x, b.y, c.x, c.y, w.tally);
}

__device__ __forceinline__ int incircle_tri(const DevMesh &m, const Work &w, int4 tri, double2 p) {
  double2 A = m.vxy[tri.x], B = m.vxy[tri.y], C = m.vxy[tri.z];
  return incircle(A.x, A.y, B.x, B.y, C.x, C.y, p.x, p.y, w.tally);
}

__device__ __forceinline__ bool in_sorted(const int32_t *a, int n, int v) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int x = a[mid];
    if (x == v) return true;
    if (x < v) lo = mid + 1; else hi = mid - 1;
  }
  return false;
}

// Work distribution of a phase: item = base + threadIdx.x for base = base0,
// base0 + stride, ...  A grid kernel spreads the items over all workgroups;
// the single-workgroup engine takes them all.  The loops are uniform over a
// workgroup, as the wave-wide operations require.
// blk: every thread of the workgroup runs the loop (grid kernels), so list
// space can be taken once per workgroup; otherwise once per wave (the
// engine, whose waves share one compute unit and see no contention).
struct Lanes {
  int base0, stride, blk;
};
__device__ __forceinline__ Lanes grid_lanes() {
  return {(int)(blockIdx.x * blockDim.x), (int)(gridDim.x * blockDim.x), 1};
}
__device__ __forceinline__ Lanes block_lanes() { return {0, (int)blockDim.x, 0}; }

// n entries per lane from a shared counter: returns this lane's first offset.
// One atomic per workgroup (L.blk) or per wave; the loops that call it are
// uniform over the workgroup.
constexpr int kMaxWaves = 16;
__device__ __forceinline__ int group_alloc(int *counter, int n, const Lanes &L) {
  if (!L.blk) return wave_alloc(counter, n);
  __shared__ int s_part[kMaxWaves];
  __shared__ int s_base;
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  int x = n;
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_part[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) {
      int t = s_part[i];
      s_part[i] = acc;
      acc += t;
    }
    s_base = acc ? atomicAdd(counter, acc) : 0;
  }
  __syncthreads();
  const int r = s_base + s_part[wid] + x - n;
  __syncthreads();
  return r;
}

// The midpoint entries a lane flagged (up to 4), appended together (kept in
// named registers: an indexed array would go to scratch memory).
struct MidFlags {
  int k0 = -1, k1 = -1, k2 = -1, k3 = -1;
  int n = 0;
  __device__ __forceinline__ void push(int k) {
    k3 = n == 3 ? k : k3;
    k2 = n == 2 ? k : k2;
    k1 = n == 1 ? k : k1;
    k0 = n == 0 ? k : k0;
    n++;
  }
};
__device__ __forceinline__ void push_mids(const Work &w, const MidFlags &f, const Lanes &L) {
  const int off = group_alloc(&w.cnt->nmk, f.n, L);
  if (f.n > 0) put_mid(w, off, f.k0);
  if (f.n > 1) put_mid(w, off + 1, f.k1);
  if (f.n > 2) put_mid(w, off + 2, f.k2);
  if (f.n > 3) put_mid(w, off + 3, f.k3);
}
// the first lane of the whole distribution (single writes)
__device__ __forceinline__ bool first_lane(const Lanes &L) { return L.base0 == 0 && threadIdx.x == 0; }

// ---------------------------------------------------------------------------
// R1: collect encroached subsegments and bad triangles (Line 3)
// ---------------------------------------------------------------------------
// Tests one triangle: subsegment sides + encroaching apex, and badness.
__device__ __forceinline__ bool scan_triangle(const DevMesh &m, const Work &w, int i, double B2, int pm,
                                              SplitPt &r, MidFlags &fl) {
  int4 tri = m.tv[i];
  if (tri.w) {
    int4 s = m.ts[i];
    for (int e = 0; e < 3; e++) {
      if (!((tri.w >> e) & 1)) continue;
      int k = comp(s, e);
      int u = comp(tri, e), v = comp(tri, (e + 1) % 3), c = comp(tri, (e + 2) % 3);
      int side = (u == m.sv[k].x) ? 0 : 1;
      w.sadj[2 * k + side] = i * 4 + e;
      double2 U = m.vxy[u], V = m.vxy[v], Cc = m.vxy[c];
      if (encroached(w, U, V, Cc) && atomicOr(&w.mflag[k], 1u) == 0u) fl.push(k);
    }
  }
  r = tri_split(m, i, tri, B2, w.L2, pm);
  return r.bad != 0;
}

__device__ __forceinline__ void append_cc(const Work &w, bool bad, int t, const SplitPt &r, const Lanes &L) {
  int idx = group_alloc(&w.cnt->ncc, bad ? 1 : 0, L);
  if (bad) {
    w.cc.elem[idx] = t;
    w.cc.key[idx] = r.key;
    w.cc.p[idx] = make_double2(r.px, r.py);
    w.cc.state[idx] = 0;
    w.cidx_t[t] = idx;
  }
}

// Full collection over every triangle and subsegment (first round of a call).
__device__ __forceinline__ void scan_part(const DevMesh &m, const Work &w, double B2, int pm, const Lanes &L) {
  const int nT = w.st->nT, nS = w.st->nS, n = max(nT, nS);
  for (int base = L.base0; base < n; base += L.stride) {
    int i = base + threadIdx.x;
    bool bad = false;
    SplitPt r;
    MidFlags fl;
    if (i < nT) bad = scan_triangle(m, w, i, B2, pm, r, fl);
    append_cc(w, bad, i, r, L);
    if (i < nS && m.spend[i] && atomicOr(&w.mflag[i], 1u) == 0u) fl.push(i);
    push_mids(w, fl, L);
  }
}

__global__ void k_scan(DevMesh m, Work w, double B2, int pm) {
  if (w.st->halt) return;
  scan_part(m, w, B2, pm, grid_lanes());
}

// Incremental collection, later rounds.  A triangle that no winner rewrote
// keeps its vertices, so its badness and split point are unchanged: the bad
// triangles of the previous round that were not rewritten are carried over.
// (The carried list and the rewritten slots are collected by one kernel, one
// grid-stride loop each; each loop is uniform over the grid, as the wave-wide
// appends require.)
__device__ __forceinline__ void carry_part(const Work &w, const Lanes &L) {
  const int n_prev = w.st->prev_ncc, prev_serial = w.st->serial - 1;
  for (int base = L.base0; base < n_prev; base += L.stride) {
    int c = base + threadIdx.x;
    bool keep = false;
    int t = 0;
    if (c < n_prev) {
      t = w.prev_cc_elem[c];
      keep = w.tstamp[t] != prev_serial;
    }
    int idx = group_alloc(&w.cnt->ncc, keep ? 1 : 0, L);
    if (keep) {
      w.cc.elem[idx] = t;
      w.cc.key[idx] = w.prev_cc_key[c];
      w.cc.p[idx] = w.prev_cc_p[c];
      w.cc.state[idx] = 0;
      w.cidx_t[t] = idx;
    }
  }
}

// ... and every slot written last round (the fan records) is tested afresh;
// an encroaching apex can only appear on a rewritten triangle.
__device__ __forceinline__ void dirty_part(const DevMesh &m, const Work &w, double B2, int pm, const Lanes &L) {
  const int n_dirty = w.st->prev_fan;
  for (int base = L.base0; base < n_dirty; base += L.stride) {
    int c = base + threadIdx.x;
    bool bad = false;
    SplitPt r;
    MidFlags fl;
    int t = 0;
    if (c < n_dirty) {
      t = w.fan[c].slot;
      bad = scan_triangle(m, w, t, B2, pm, r, fl);
    }
    append_cc(w, bad, t, r, L);
    push_mids(w, fl, L);
  }
}

// ... and last round's flagged subsegments are tested again: pending, or an
// apex still inside the diametric circle (a flagged subsegment the candidate
// cap left out is not pending, and its sides may be unchanged).  The side
// slots are current: rewritten sides were re-scanned just before.
// Returns true if subsegment k is flagged anew.
__device__ __forceinline__ bool pending_one(const DevMesh &m, const Work &w, int k) {
  if (m.spend[k]) return atomicOr(&w.mflag[k], 1u) == 0u;
  for (int side = 0; side < 2; side++) {
    int a = w.sadj[2 * k + side];
    if (a < 0) continue;
    int t = a >> 2, e = a & 3;
    int4 tri = m.tv[t];
    double2 U = m.vxy[comp(tri, e)], V = m.vxy[comp(tri, (e + 1) % 3)], C = m.vxy[comp(tri, (e + 2) % 3)];
    if (encroached(w, U, V, C)) return atomicOr(&w.mflag[k], 1u) == 0u;
  }
  return false;
}

__device__ __forceinline__ void pending_part(const DevMesh &m, const Work &w, const Lanes &L) {
  const int n_prev = w.st->prev_nmk;
  for (int base = L.base0; base < n_prev; base += L.stride) {
    int c = base + threadIdx.x;
    MidFlags fl;
    if (c < n_prev) {
      const int k = w.prev_mid_elem[c];
      if (pending_one(m, w, k)) fl.push(k);
    }
    push_mids(w, fl, L);
  }
}

__global__ void k_collect(DevMesh m, Work w, double B2, int pm) {
  if (w.st->halt) return;
  carry_part(w, grid_lanes());
  dirty_part(m, w, B2, pm, grid_lanes());
}

// Separate launch: it reads side slots that k_collect rewrites.
__global__ void k_pending(DevMesh m, Work w) {
  if (w.st->halt) return;
  pending_part(m, w, grid_lanes());
}

// After the collection: stop if nothing is left (Algorithm 1, the loop ends
// when L is empty) or if the round cap is reached with work left.
// One workgroup.  At the round cap this round's flags are dropped before
// leaving.  Returns the halt code it set (0: the round goes on).
__device__ __forceinline__ int gate_part(const Work &w, int max_rounds) {
  __shared__ int s_h;
  DevState *st = w.st;
  DevCounters *c = w.cnt;
  if (threadIdx.x == 0) {
    s_h = 0;
    if (!st->halt) {
      const int ncc = c->ncc, nmk = c->nmk;
      c->nmk0 = nmk;
      if (ncc == 0 && nmk == 0) s_h = kHaltDone;
      else if (max_rounds > 0 && st->rounds >= max_rounds) s_h = kHaltCap;
      if (s_h) st->halt = s_h;
    }
  }
  __syncthreads();
  const int h = s_h;
  if (h == kHaltCap) {
    const int nmk = c->nmk;
    for (int i = threadIdx.x; i < nmk; i += blockDim.x) w.mflag[w.mid.elem[i]] = 0u;
  }
  return h;
}

__global__ void k_gate(Work w, int max_rounds) { (void)gate_part(w, max_rounds); }

// ---------------------------------------------------------------------------
// R3 (optional): keep the K largest keys.  Keys of both classes are placed in
// one array; a radix select finds the K-th largest (keys are unique).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gather_part(const DevMesh &m, const Work &w, int pm, const Lanes &L) {
  const int ncc = w.cnt->ncc, nmk = w.cnt->nmk;
  if (first_lane(L)) {
    w.sel[0] = 0;  // prefix
    w.sel[1] = 0;  // prefix mask
  }
  for (int base = L.base0; base < ncc + nmk; base += L.stride) {
    int c = base + threadIdx.x;
    if (c >= ncc + nmk) break;
    if (c < ncc) {
      w.keys[c] = w.cc.key[c];
    } else {
      int j = c - ncc;
      SplitPt r = seg_split(m, w.mid.elem[j], pm, w.split_mode);
      w.mid.key[j] = r.key;
      w.mid.p[j] = make_double2(r.px, r.py);
      w.keys[c] = r.key;
    }
  }
}

__global__ void k_gather_keys(DevMesh m, Work w, int pm) {
  if (w.st->halt) return;
  gather_part(m, w, pm, grid_lanes());
}

// Histogram of 8-bit digit `shift` over keys whose higher digits equal the
// prefix chosen so far.
__global__ void k_radix_hist(Work w, int shift) {
  __shared__ int h[256];
  if (w.st->halt) return;
  const int n = w.cnt->ncc + w.cnt->nmk;
  const uint64_t prefix = w.sel[0], pmask = w.sel[1];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    uint64_t k = w.keys[c];
    if ((k & pmask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&w.rhist[i], h[i]);
}

// Picks the digit of the K-th largest key (keys are unique) and clears the
// histogram for the next digit.  With no more than K keys the threshold is 0
// and every key is kept.
__device__ __forceinline__ void radix_pick_part(const Work &w, int shift, int K) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int n = w.cnt->ncc + w.cnt->nmk;
    if (shift == 56) w.sel[2] = (uint64_t)K;
    if (n > K) {
      int64_t remaining = (int64_t)w.sel[2];
      int64_t cum = 0;
      int d = 255;
      for (; d > 0; d--) {
        if (cum + w.rhist[d] >= remaining) break;
        cum += w.rhist[d];
      }
      w.sel[2] = (uint64_t)(remaining - cum);
      w.sel[0] |= (uint64_t)d << shift;
      w.sel[1] |= (uint64_t)0xff << shift;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x) w.rhist[i] = 0;
}

__global__ void k_radix_pick(Work w, int shift, int K) {
  if (w.st->halt) return;
  radix_pick_part(w, shift, K);
}

__device__ __forceinline__ void apply_part(const Work &w, const Lanes &L) {
  const int ncc = w.cnt->ncc, nmk = w.cnt->nmk;
  const uint64_t th = w.sel[0];
  for (int base = L.base0; base < ncc + nmk; base += L.stride) {
    int c = base + threadIdx.x;
    if (c >= ncc + nmk) break;
    if (c < ncc) {
      if (w.cc.key[c] < th) w.cc.state[c] = kStDone | kStSkip;
      else atomicAdd(&w.cnt->n_kept_cc, 1);
    } else {
      int j = c - ncc;
      if (w.mid.key[j] < th) {
        w.mid.state[j] = kStSkip;
        w.mflag[w.mid.elem[j]] = 0u;
      } else {
        atomicAdd(&w.cnt->n_kept_mid, 1);
      }
    }
  }
}

__global__ void k_apply_cap(Work w) {
  if (w.st->halt) return;
  apply_part(w, grid_lanes());
}

// ---------------------------------------------------------------------------
// R4: locate circumcenters by a visibility walk (Line 6); a walk stopped only
// by subsegments turns into the midpoint candidate of the first one.
// ---------------------------------------------------------------------------
// Returns 1 for a coincident point, 2 for a walk blocked by a subsegment.
// The walk length is kept in bits 16-30 of the state of a located point (at
// most 0x7fff) and added to *nsteps.
constexpr int kStepShift = 16;
__device__ __forceinline__ int locate_one(const DevMesh &m, const Work &w, int c, int nS, int &nsteps) {
  if (w.cc.state[c] & kStSkip) return 0;
  int cur = w.cc.elem[c];
  double2 p = w.cc.p[c];
  for (int steps = 1;; steps++) {
    nsteps++;
    if (steps > (1 << 20)) {
      atomicOr(&w.cnt->err, kErrWalk);
      w.cc.state[c] = kStDone;
      return 0;
    }
    // the neighbours are loaded with the vertices (needed unless p is found here)
    int4 tri = m.tv[cur];
    const int4 nb = m.tn[cur];
    double2 A = m.vxy[tri.x], B = m.vxy[tri.y], C = m.vxy[tri.z];
    int s0 = orient_pts(w, A, B, p), s1 = orient_pts(w, B, C, p), s2 = orient_pts(w, C, A, p);
    if (s0 >= 0 && s1 >= 0 && s2 >= 0) {
      int nz = (s0 == 0) + (s1 == 0) + (s2 == 0);
      if (nz >= 2) {
        w.cc.state[c] = kStDone;
        return 1;
      }
      w.cc.loc[c] = cur;
      w.cc.state[c] = kStFound | (min(steps, 0x7fff) << kStepShift);
      return 0;
    }
    int s[3] = {s0, s1, s2};
    int first_neg = -1, next = -1;
    for (int e = 0; e < 3; e++) {
      if (s[e] >= 0) continue;
      if (first_neg < 0) first_neg = e;
      int o = comp(nb, e);
      if (!((tri.w >> e) & 1) && o >= 0) { next = o; break; }
    }
    if (next < 0) {
      int k = comp(m.ts[cur], first_neg);
      if (k < 0 || k >= nS) {  // a hull edge that is not a subsegment
        atomicOr(&w.cnt->err, kErrInput);
        w.cc.state[c] = kStDone;
        return 0;
      }
      flag_mid(w, k);
      w.cc.state[c] = kStDone;
      return 2;
    }
    cur = next;
  }
}

__device__ __forceinline__ void locate_part(const DevMesh &m, const Work &w, const Lanes &L) {
  const int ncc = w.cnt->ncc, nS = w.st->nS;
  int n_coin = 0, n_blk = 0, n_steps = 0;
  for (int base = L.base0; base < ncc; base += L.stride) {
    int c = base + threadIdx.x;
    if (c < ncc) {
      const int r = locate_one(m, w, c, nS, n_steps);
      n_coin += r == 1;
      n_blk += r == 2;
    }
  }
  stat_add(w, kStCoincident, n_coin);
  stat_add(w, kStBlocked, n_blk);
  stat_add(w, kStOrTests, 3 * (uint64_t)n_steps);
}

__global__ void k_locate(DevMesh m, Work w) {
  if (w.st->halt) return;
  locate_part(m, w, grid_lanes());
}

// ---------------------------------------------------------------------------
// Optional semantic prefilters on located circumcenters.
//   F1 (Line 6): one circumcenter per located triangle, the largest key.
//   F2 (Line 7): the first n triangles of the cavity growth order (seed, then
//   breadth first across non-subsegment edges whose far circumcircle strictly
//   holds the point, edges in index order, stopping as soon as n are taken)
//   are marked with atomicMax; a point that does not hold all of them is
//   dropped.  Marks are cleared before the real cavities are grown.
// mode: 0 F1 mark, 1 F1 filter, 2 F1 clear, 3 F2 mark, 4 F2 filter, 5 F2 clear
// ---------------------------------------------------------------------------
constexpr int kApproxMax = 16;
constexpr int kPreBlock = 128;

__device__ __forceinline__ void prefilter_one(const DevMesh &m, const Work &w, int32_t *lds, int ls, int tid, int c, int mode,
                              int n) {
  int st = w.cc.state[c];
  if (!(st & kStFound)) return;
  int loc = w.cc.loc[c];
  uint64_t key = w.cc.key[c];
  if (mode <= 2) {
    if (mode == 0) {
      if (!(st & kStDone)) atomicMax((unsigned long long *)&w.mark[loc], (unsigned long long)key);
    } else if (mode == 1) {
      if (!(st & kStDone) && w.mark[loc] != key) {
        w.cc.state[c] = st | kStDone;
        atomicAdd(&w.cnt->n_f1_drop, 1);
      }
    } else {
      w.mark[loc] = 0ull;
    }
    return;
  }
  if (mode != 5 && (st & kStDone)) return;
  double2 p = w.cc.p[c];
  int len = 0;
  lds[tid] = loc;
  len = 1;
  for (int h = 0; h < len && len < n; h++) {
    int t = lds[h * ls + tid];
    int4 tri = m.tv[t];
    int4 nb = m.tn[t];
    for (int e = 0; e < 3 && len < n; e++) {
      if ((tri.w >> e) & 1) continue;
      int o = comp(nb, e);
      if (o < 0) continue;
      bool in = false;
      for (int q = 0; q < len; q++)
        if (lds[q * ls + tid] == o) { in = true; break; }
      if (in) continue;
      if (incircle_tri(m, w, m.tv[o], p) > 0) lds[(len++) * ls + tid] = o;
    }
  }
  if (mode == 3) {
    for (int j = 0; j < len; j++)
      atomicMax((unsigned long long *)&w.mark[lds[j * ls + tid]], (unsigned long long)key);
  } else if (mode == 4) {
    bool own = true;
    for (int j = 0; j < len && own; j++) own = w.mark[lds[j * ls + tid]] == key;
    if (!own) {
      w.cc.state[c] = st | kStDone;
      atomicAdd(&w.cnt->n_f2_drop, 1);
    }
  } else {
    for (int j = 0; j < len; j++) w.mark[lds[j * ls + tid]] = 0ull;
  }
}

// lds: kApproxMax slices of blockDim.x entries
__device__ __forceinline__ void prefilter_part(const DevMesh &m, const Work &w, int mode, int n, int32_t *lds, const Lanes &L) {
  const int ncc = w.cnt->ncc;
  for (int base = L.base0; base < ncc; base += L.stride) {
    int c = base + threadIdx.x;
    if (c < ncc) prefilter_one(m, w, lds, blockDim.x, threadIdx.x, c, mode, n);
  }
}

__global__ __launch_bounds__(kPreBlock) void k_prefilter(DevMesh m, Work w, int mode, int n) {
  __shared__ int32_t lds[kApproxMax * kPreBlock];
  if (w.st->halt) return;
  prefilter_part(m, w, mode, n, lds, grid_lanes());
}

// ---------------------------------------------------------------------------
// R5 / R6: Bowyer-Watson cavities.  Per-thread growth in an LDS slice; a
// cavity larger than the slice goes to the cooperative kernel below.
// ---------------------------------------------------------------------------
struct CavCheck {
  int nbnd;
  bool fan_bad;
  bool enc;
  int ntest;  // incircle evaluations
};

// per-thread cavity capacity of the grid kernel: 39 slots x 128 threads (plus
// a few bytes) is the most LDS that still lets 8 workgroups (16 waves) share a
// compute unit's 160 KB; larger cavities go to the cooperative kernel
constexpr int kCap = kCavCapDefault;
// per-lane statistics of a per-thread cavity (size, boundary edges, circle
// tests: at most three per slot) stay below 2^10 (see stat_add4)
constexpr int kStat4Cap = 1023 / 3 - 2;
static_assert(kCap <= kStat4Cap, "per-thread cavity statistics fit stat_add4");
constexpr int kCavBlock = kCavBlockSize;

// Grows the cavity of p from the seeds into lds[j * ls + tid] (a slice of
// cap entries).  Returns the size, or -1 if it exceeds cap (the cavity then
// goes to the cooperative path; the set of triangles is the same).
// FILTER: the geometric tests use the FP64 filters alone, and a test they
// cannot decide returns -2 (the cavity then goes to the cooperative path,
// which evaluates exactly); this keeps the exact evaluations, and the
// registers and scratch they need, out of the per-thread kernels.
//
// The boundary checks are made on the way: an edge of a cavity triangle is
// internal iff its neighbour is in the cavity, and that is decided when the
// triangle is taken from the list (a neighbour already listed is internal;
// one that fails the circle test never enters).  For each boundary edge:
// the count, the fan orientation (p strictly left of it), and for
// circumcenters an encroached boundary subsegment (all are flagged; a
// cavity that overflows flags a subset of what the cooperative path flags
// for the same cavity).  The split subsegment of a midpoint (skip_k) is
// not a boundary edge.  A cavity left undecided by a filter (FILTER) has
// flagged a subset too.
template <bool FILTER>
__device__ __forceinline__ int grow_local(const DevMesh &m, const Work &w, int32_t *lds, int ls, int cap, int tid,
                                          const int *seeds, int nseeds, double2 p, int skip_k, bool is_cc,
                                          CavCheck &ck) {
  ck = CavCheck{0, false, false, 0};
  int len = 0;
  for (int s = 0; s < nseeds; s++) {
    bool dup = false;
    for (int q = 0; q < len; q++) dup |= lds[q * ls + tid] == seeds[s];
    if (!dup) lds[(len++) * ls + tid] = seeds[s];
  }
  for (int h = 0; h < len; h++) {
    const int t = lds[h * ls + tid];
    const int4 tri = m.tv[t];
    const int4 nb = m.tn[t];
    // the three neighbours are distinct triangles, so they can be screened
    // against the list together and then tested in edge order
    int o[3];
    bool c[3], in[3];
    for (int e = 0; e < 3; e++) {
      o[e] = comp(nb, e);
      in[e] = false;
    }
    for (int q = 0; q < len; q++) {
      const int x = lds[q * ls + tid];
      in[0] = in[0] || x == o[0];
      in[1] = in[1] || x == o[1];
      in[2] = in[2] || x == o[2];
    }
    // in: internal (a listed neighbour across a non-subsegment edge);
    // c: to be tested by the circle test; the rest (subsegment and hull
    // edges) are boundary
    for (int e = 0; e < 3; e++) {
      const bool sub = (tri.w >> e) & 1;
      in[e] = in[e] && !sub;
      c[e] = !sub && o[e] >= 0 && !in[e];
    }
    if (in[0] && in[1] && in[2]) continue;
    // independent loads: the neighbours' records, this triangle's vertices
    // and subsegments; then only the far vertex of each neighbour
    int4 to[3];
    for (int e = 0; e < 3; e++) to[e] = c[e] ? m.tv[o[e]] : make_int4(0, 0, 0, 0);
    const int4 ts = tri.w ? m.ts[t] : make_int4(-1, -1, -1, 0);
    const double2 P[3] = {m.vxy[tri.x], m.vxy[tri.y], m.vxy[tri.z]};
    double2 F[3];
    int fv[3];
    for (int e = 0; e < 3; e++) {
      fv[e] = -1;
      if (!c[e]) continue;
      const int u = comp(tri, e), v = comp(tri, (e + 1) % 3);
      fv[e] = (to[e].x != u && to[e].x != v) ? to[e].x : ((to[e].y != u && to[e].y != v) ? to[e].y : to[e].z);
      F[e] = m.vxy[fv[e]];
    }
    for (int e = 0; e < 3; e++) {
      if (in[e]) continue;
      const double2 Pu = P[e], Pv = P[(e + 1) % 3];
      if (c[e]) {
        const int u = comp(tri, e);
        // the neighbour's vertices in its own order (the same arguments as
        // a direct evaluation on its record)
        const double2 A = to[e].x == fv[e] ? F[e] : (to[e].x == u ? Pu : Pv);
        const double2 B = to[e].y == fv[e] ? F[e] : (to[e].y == u ? Pu : Pv);
        const double2 C = to[e].z == fv[e] ? F[e] : (to[e].z == u ? Pu : Pv);
        ck.ntest++;
        int in;
        if (FILTER) {
          in = incircle_filter(A.x, A.y, B.x, B.y, C.x, C.y, p.x, p.y);
          if (in == kUndecided) return -2;
        } else {
          in = incircle(A.x, A.y, B.x, B.y, C.x, C.y, p.x, p.y, w.tally);
        }
        if (in > 0) {
          if (len == cap) return -1;
          lds[(len++) * ls + tid] = o[e];
          continue;
        }
      }
      // a boundary edge
      const int sid = ((tri.w >> e) & 1) ? comp(ts, e) : -1;
      if (skip_k >= 0 && sid == skip_k) continue;
      ck.nbnd++;
      if (is_cc && sid >= 0) {
        int enc;
        if (FILTER) {
          enc = encroaches_filter(w.enc_mode, Pu.x, Pu.y, Pv.x, Pv.y, p.x, p.y);
          if (enc == kUndecided) return -2;
        } else {
          enc = encroached(w, Pu, Pv, p) ? 1 : 0;
        }
        if (enc) {
          flag_mid(w, sid);
          ck.enc = true;
        }
      }
      int o;
      if (FILTER) {
        o = orient2d_filter(Pu.x, Pu.y, Pv.x, Pv.y, p.x, p.y);
        if (o == kUndecided) return -2;
      } else {
        o = orient_pts(w, Pu, Pv, p);
      }
      if (o <= 0) ck.fan_bad = true;
    }
  }
  // insertion sort (ascending slots)
  for (int a = 1; a < len; a++) {
    int x = lds[a * ls + tid];
    int b = a - 1;
    while (b >= 0 && lds[b * ls + tid] > x) {
      lds[(b + 1) * ls + tid] = lds[b * ls + tid];
      b--;
    }
    lds[(b + 1) * ls + tid] = x;
  }
  return len;
}

// Outcome of one per-thread cavity: alive (cavity left in the LDS slice),
// dropped (with the counter it feeds) or handed to the cooperative kernel.
struct CavRes {
  int len;        // cavity size when grown (0 otherwise)
  int bnd;        // its boundary edges
  int alive;
  int enc_reject, fan_invalid, unsplittable, mid_cand;
  int ntest;      // incircle evaluations made while growing
};

template <bool FILTER>
__device__ __forceinline__ CavRes cavity_one(const DevMesh &m, const Work &w, int32_t *lds, int ls, int cap, int tid,
                                             int ci, int is_cc) {
  CavRes res{0, 0, 0, 0, 0, 0, 0, 0};
  CandSet S = is_cc ? w.cc : w.mid;
  int st = S.state[ci];
  if (st & (kStDone | kStSkip | kStBig)) return res;
  int seeds[2], nseeds = 0, skip_k = -1, expect = 2;
  double2 p;
  if (is_cc) {
    if (!(st & kStFound)) return res;
    seeds[nseeds++] = S.loc[ci];
    p = S.p[ci];
  } else {
    int k = S.elem[ci];
    res.mid_cand = 1;
    const int a0 = w.sadj[2 * k], a1 = w.sadj[2 * k + 1];  // with the subsegment's record
    SplitPt r = seg_split(m, k, w.pm, w.split_mode);
    S.key[ci] = r.key;
    p = make_double2(r.px, r.py);
    S.p[ci] = p;
    int2 sk = m.sv[k];
    double2 A = m.vxy[sk.x], B = m.vxy[sk.y];
    if ((p.x == A.x && p.y == A.y) || (p.x == B.x && p.y == B.y)) {
      res.unsplittable = 1;
      S.state[ci] = st | kStDone;
      return res;
    }
    if (a0 >= 0) seeds[nseeds++] = a0 >> 2;
    if (a1 >= 0) seeds[nseeds++] = a1 >> 2;
    skip_k = k;
    expect = nseeds == 2 ? 2 : 1;
    S.state[ci] = st | kStFound;
  }
  CavCheck ck;
  int len = grow_local<FILTER>(m, w, lds, ls, cap, tid, seeds, nseeds, p, skip_k, is_cc != 0, ck);
  res.ntest = ck.ntest;
  if (len < 0) {
    S.state[ci] = st | kStBig | kStFound;
    int q = atomicAdd(&w.cnt->nbig, 1);
    if (q < w.big_cap) w.big[q] = (is_cc ? 0 : (int)0x80000000) | ci;
    else atomicOr(&w.cnt->err, kErrCavity);
    return res;
  }
  res.len = len;
  res.bnd = ck.nbnd;
  if (is_cc && ck.enc) {
    res.enc_reject = 1;
    S.state[ci] |= kStDone;
  } else if (ck.fan_bad || ck.nbnd - len != expect) {
    res.fan_invalid = 1;
    S.state[ci] |= kStDone;
  } else {
    res.alive = 1;
  }
  return res;
}

// Per-thread cavities of one class (lds: cap slices of ls entries; the
// threads tid < ls take part).
// The midpoint list is final when this runs for midpoints (they are flagged
// only by the scan, the walk and the circumcenter cavities), so its length
// is read from device memory.  The loop is uniform over the workgroup so
// that pool space and statistics are handled once per wave.
// Candidates [lo, hi) of the class (hi < 0: to the end of the list); tid is
// the thread's index in the group that runs the loop (its LDS slice).
template <bool FILTER = false>
__device__ __forceinline__ void cavity_part(const DevMesh &m, const Work &w, int is_cc, int32_t *lds, int ls, int cap,
                                            const Lanes &L, int lo = 0, int hi = -1, int tid = -1) {
  if (tid < 0) tid = threadIdx.x;
  const int n = hi >= 0 ? hi : (is_cc ? w.cnt->ncc : w.cnt->nmk);
  CandSet S = is_cc ? w.cc : w.mid;
  for (int base = lo + L.base0; base < n; base += L.stride) {
    int ci = base + tid;
    CavRes r{0, 0, 0, 0, 0, 0, 0, 0};
    if (ci < n) r = cavity_one<FILTER>(m, w, lds, ls, cap, tid, ci, is_cc);
    int off = group_alloc(&w.cnt->pool_used, r.alive ? r.len : 0, L);
    bool counted = r.len > 0 && !r.alive;  // dropped cavities count in the statistics now
    if (r.alive) {
      if (off + r.len > w.pool_cap) {
        atomicOr(&w.cnt->err, kErrPool);  // the round is abandoned and run again
      } else {
        // R8 marks are placed as soon as the cavity is known to be valid:
        // validity depends on this cavity alone, and atomicMax is order free.
        uint64_t key = S.key[ci];
        for (int j = 0; j < r.len; j++) {
          int t = lds[j * ls + tid];
          w.pool[off + j] = t;
          atomicMax((unsigned long long *)&w.mark[t], (unsigned long long)key);
        }
        S.off[ci] = off;
        S.len[ci] = r.len;
        S.state[ci] |= kStDone | kStAlive;
        counted = true;
      }
    }
    // (summed per iteration: nothing stays live across the cavity work)
    stat_max(w, kStCavMax, counted ? r.len : 0);
    const int f4a[4] = {kStCavTri, is_cc ? kStCavLen1 : kStCavLen0, is_cc ? kStCavBnd1 : kStCavBnd0, kStInTests};
    const int f4b[4] = {is_cc ? kStMarks1 : kStMarks0, kStEncReject, kStFanInvalid, kStUnsplittable};
    stat_add4(w, f4a, counted ? r.len : 0, r.len, r.bnd, r.ntest);
    stat_add4(w, f4b, (r.alive && counted) ? r.len : 0, r.enc_reject, r.fan_invalid, r.unsplittable);
    stat_add(w, kStMidCand, r.mid_cand);
  }
}

// One kernel symbol per class (circumcenters: IS_CC = 1), so that profiles
// tell them apart, and per slice length CAP (the per-thread capacity; a
// cavity beyond it goes to the cooperative path: perf only).
template <int IS_CC, int CAP>
__global__ __launch_bounds__(kCavBlock, 4) void k_cavity(DevMesh m, Work w) {
  static_assert(CAP <= kStat4Cap, "per-thread cavity statistics fit stat_add4");
  __shared__ int32_t lds[CAP * kCavBlock];
  if (w.st->halt) return;
  cavity_part<true>(m, w, IS_CC, lds, kCavBlock, CAP, grid_lanes());
}
template __global__ void k_cavity<0, kCap>(DevMesh m, Work w);
template __global__ void k_cavity<1, kCap>(DevMesh m, Work w);
template __global__ void k_cavity<0, 24>(DevMesh m, Work w);
template __global__ void k_cavity<1, 24>(DevMesh m, Work w);
template __global__ void k_cavity<0, 12>(DevMesh m, Work w);
template __global__ void k_cavity<1, 12>(DevMesh m, Work w);

// Cooperative growth of one large cavity per workgroup (the tuple-parallel
// ExpandList idea of Section 5.3: the frontier of <point, triangle> tuples
// is processed in parallel, new tuples are reserved with atomics).
constexpr int kBigMax = 4096;
constexpr int kHash = 16384;
constexpr int kBigBlock = 256;

__device__ __forceinline__ int hash_insert(int32_t *hs, int v, int *ovf) {
  uint32_t h = ((uint32_t)v * 2654435761u) & (kHash - 1);
  for (int probe = 0; probe < kHash; probe++) {
    int old = atomicCAS(&hs[h], -1, v);
    if (old == -1) return 1;
    if (old == v) return 0;
    h = (h + 1) & (kHash - 1);
  }
  *ovf = 1;
  return 0;
}

struct BigShared {
  int32_t cav[kBigMax];
  int32_t hs[kHash];
  int s_n, s_head, s_ovf, s_nbnd, s_fanbad, s_enc, s_off, s_r;
};

// Ascending sort of a[0..n) by one workgroup: the bitonic network in its
// all-ascending form (each block of size k first compares mirrored pairs,
// then half-cleaners of strides k/4 .. 1; every compare-exchange puts the
// smaller value at the lower index).  Entries beyond n act as +infinity and
// are never touched, so no padding is stored.
__device__ __forceinline__ void block_sort_asc(int32_t *a, int n) {
  int P = 1;
  while (P < n) P <<= 1;
  const int half = P >> 1;
  for (int k = 2; k <= P; k <<= 1) {
    const int hk = k >> 1;
    __syncthreads();
    for (int idx = threadIdx.x; idx < half; idx += blockDim.x) {
      const int blk = idx / hk, o = idx - blk * hk;
      const int i = blk * k + o, l = blk * k + (k - 1 - o);
      if (l < n) {
        const int x = a[i], y = a[l];
        if (x > y) { a[i] = y; a[l] = x; }
      }
    }
    for (int j = k >> 2; j > 0; j >>= 1) {
      __syncthreads();
      for (int idx = threadIdx.x; idx < half; idx += blockDim.x) {
        const int i = (idx / j) * 2 * j + idx % j, l = i + j;
        if (l < n) {
          const int x = a[i], y = a[l];
          if (x > y) { a[i] = y; a[l] = x; }
        }
      }
    }
  }
  __syncthreads();
}

// The rest of a cooperative cavity once its slots are known (cav[0..len),
// any order; LDS or device memory): sort, boundary checks in parallel over
// the cavity triangles, then drop it or take pool space and place its
// marks.  Uniform over the workgroup; the shared scalars are reset here.
__device__ __forceinline__ void coop_finish(const DevMesh &m, const Work &w, BigShared &sh, CandSet S, int ci,
                                            int is_cc, int skip_k, int expect, double2 p, int32_t *cav, int len) {
  const int tid = threadIdx.x;
  if (tid == 0) { sh.s_nbnd = 0; sh.s_fanbad = 0; sh.s_enc = 0; sh.s_off = -1; }
  block_sort_asc(cav, len);
  for (int j = tid; j < len; j += blockDim.x) {
    int t = cav[j];
    int4 tri = m.tv[t];
    int4 nb = m.tn[t];
    int4 ts = tri.w ? m.ts[t] : make_int4(-1, -1, -1, 0);
    for (int e = 0; e < 3; e++) {
      int sid = ((tri.w >> e) & 1) ? comp(ts, e) : -1;
      if (skip_k >= 0 && sid == skip_k) continue;
      int o = comp(nb, e);
      if (sid < 0 && o >= 0 && in_sorted(cav, len, o)) continue;
      atomicAdd(&sh.s_nbnd, 1);
      double2 U = m.vxy[comp(tri, e)], V = m.vxy[comp(tri, (e + 1) % 3)];
      if (is_cc && sid >= 0 && encroached(w, U, V, p)) {
        flag_mid(w, sid);
        sh.s_enc = 1;
      }
      if (orient_pts(w, U, V, p) <= 0) sh.s_fanbad = 1;
    }
  }
  __syncthreads();
  if (tid == 0) {
    atomicAdd((unsigned long long *)&stat_line(w)->v[kStOrTests], (unsigned long long)sh.s_nbnd);
    bool drop = (is_cc && sh.s_enc) || sh.s_fanbad || sh.s_nbnd - len != expect;
    if (drop) {
      atomicAdd((unsigned long long *)&w.cnt->cav_tri_total, (unsigned long long)len);
      atomicMax(&w.cnt->cav_max, len);
      atomicAdd((is_cc && sh.s_enc) ? &w.cnt->n_enc_reject : &w.cnt->n_fan_invalid, 1);
      S.state[ci] |= kStDone;
    } else {
      int off = atomicAdd(&w.cnt->pool_used, len);
      if (off + len > w.pool_cap) atomicOr(&w.cnt->err, kErrPool);
      else {
        sh.s_off = off;
        atomicAdd((unsigned long long *)&w.cnt->cav_tri_total, (unsigned long long)len);
        atomicMax(&w.cnt->cav_max, len);
      }
    }
  }
  __syncthreads();
  int off = sh.s_off;
  if (off >= 0) {
    uint64_t key = S.key[ci];
    for (int j = tid; j < len; j += blockDim.x) {
      w.pool[off + j] = cav[j];
      atomicMax((unsigned long long *)&w.mark[cav[j]], (unsigned long long)key);
    }
    if (tid == 0) {
      atomicAdd((unsigned long long *)&stat_line(w)->v[is_cc ? kStMarks1 : kStMarks0], (unsigned long long)len);
      S.off[ci] = off;
      S.len[ci] = len;
      S.state[ci] |= kStDone | kStAlive;
    }
  }
  __syncthreads();
}

// Candidate of queue entry b and its growth parameters.
struct CoopCand {
  CandSet S;
  int ci, is_cc, skip_k, expect;
  double2 p;
};
__device__ __forceinline__ CoopCand coop_cand(const Work &w, int b) {
  CoopCand c;
  const int ref = w.big[b];
  c.is_cc = (ref & 0x80000000) ? 0 : 1;
  c.ci = ref & 0x7fffffff;
  c.S = c.is_cc ? w.cc : w.mid;
  c.p = c.S.p[c.ci];
  c.skip_k = c.is_cc ? -1 : c.S.elem[c.ci];
  c.expect = c.is_cc ? 2 : ((w.sadj[2 * c.skip_k] >= 0 && w.sadj[2 * c.skip_k + 1] >= 0) ? 2 : 1);
  return c;
}

// Grows queue entry b (uniform over the workgroup) in LDS: the tuple-
// parallel ExpandList of Section 5.3 (Algorithm 3): the frontier of
// <point, triangle> tuples is expanded in parallel and new tuples are
// reserved with an atomic counter.  A cavity beyond the LDS list (kBigMax
// triangles) continues in device memory (huge_one); when the round was
// started without that path, the round is abandoned and run again with it.
__device__ __forceinline__ void big_one(const DevMesh &m, const Work &w, BigShared &sh, int b) {
  int32_t *cav = sh.cav;
  int32_t *hs = sh.hs;
  int tid = threadIdx.x;
  const int ci0 = w.big[b] & 0x7fffffff;
  const CandSet S0 = (w.big[b] & 0x80000000) ? w.mid : w.cc;
  if (!(S0.state[ci0] & kStBig) || (S0.state[ci0] & (kStDone | kStHuge))) return;
  const CoopCand c = coop_cand(w, b);
  for (int i = tid; i < kHash; i += blockDim.x) hs[i] = -1;
  __syncthreads();
  if (tid == 0) {
    sh.s_n = 0; sh.s_head = 0; sh.s_ovf = 0;
    if (c.is_cc) {
      int t = c.S.loc[c.ci];
      hash_insert(hs, t, &sh.s_ovf);
      cav[sh.s_n++] = t;
    } else {
      int a0 = w.sadj[2 * c.skip_k], a1 = w.sadj[2 * c.skip_k + 1];
      if (a0 >= 0 && hash_insert(hs, a0 >> 2, &sh.s_ovf)) cav[sh.s_n++] = a0 >> 2;
      if (a1 >= 0 && hash_insert(hs, a1 >> 2, &sh.s_ovf)) cav[sh.s_n++] = a1 >> 2;
    }
  }
  __syncthreads();
  for (;;) {
    int lo = sh.s_head, hi = sh.s_n < kBigMax ? sh.s_n : kBigMax;
    int ovf = sh.s_ovf;
    __syncthreads();
    if (lo >= hi || ovf) break;
    if (tid == 0) sh.s_head = hi;
    for (int idx = lo + tid; idx < hi; idx += blockDim.x) {
      int t = cav[idx];
      int4 tri = m.tv[t];
      int4 nb = m.tn[t];
      for (int e = 0; e < 3; e++) {
        if ((tri.w >> e) & 1) continue;
        int o = comp(nb, e);
        if (o < 0) continue;
        if (!hash_insert(hs, o, &sh.s_ovf)) continue;
        atomicAdd((unsigned long long *)&stat_line(w)->v[kStInTests], 1ull);
        if (incircle_tri(m, w, m.tv[o], c.p) > 0) {
          int pos = atomicAdd(&sh.s_n, 1);
          if (pos < kBigMax) cav[pos] = o;
          else sh.s_ovf = 1;
        }
      }
    }
    __syncthreads();
  }
  if (sh.s_ovf) {
    if (tid == 0) {
      if (w.huge_ok) {
        c.S.state[c.ci] |= kStHuge;
        atomicAdd(&w.cnt->nhuge, 1);
      } else {
        atomicOr(&w.cnt->err, kErrHuge);
      }
    }
    __syncthreads();
    return;
  }
  coop_finish(m, w, sh, c.S, c.ci, c.is_cc, c.skip_k, c.expect, c.p, cav, sh.s_n);
}

// A cavity beyond the LDS list, grown by one workgroup in device memory
// with no ceiling (the mesh's triangle count bounds it): the frontier and
// the cavity list live in w.hlist (accepted slots from the bottom, slots
// that failed the circle test from the top; every slot enters at most
// once), visited slots are flagged in w.hvis and cleared again at the end.
// Only one workgroup of a mesh runs this at a time (the flags are shared).
__device__ __noinline__ void huge_one(const DevMesh &m, const Work &w, BigShared &sh, int b) {
  const int tid = threadIdx.x;
  const int ci0 = w.big[b] & 0x7fffffff;
  const CandSet S0 = (w.big[b] & 0x80000000) ? w.mid : w.cc;
  if (!(S0.state[ci0] & kStHuge) || (S0.state[ci0] & kStDone)) return;
  const CoopCand c = coop_cand(w, b);
  int32_t *list = w.hlist;
  const int top = w.hcap - 1;
  if (tid == 0) {
    sh.s_n = 0; sh.s_head = 0; sh.s_r = 0;
    if (c.is_cc) {
      int t = c.S.loc[c.ci];
      w.hvis[t] = 1;
      list[sh.s_n++] = t;
    } else {
      int a0 = w.sadj[2 * c.skip_k], a1 = w.sadj[2 * c.skip_k + 1];
      if (a0 >= 0 && atomicExch(&w.hvis[a0 >> 2], 1) == 0) list[sh.s_n++] = a0 >> 2;
      if (a1 >= 0 && atomicExch(&w.hvis[a1 >> 2], 1) == 0) list[sh.s_n++] = a1 >> 2;
    }
  }
  __syncthreads();
  for (;;) {
    int lo = sh.s_head, hi = sh.s_n;
    __syncthreads();
    if (lo >= hi) break;
    if (tid == 0) sh.s_head = hi;
    for (int idx = lo + tid; idx < hi; idx += blockDim.x) {
      int t = list[idx];
      int4 tri = m.tv[t];
      int4 nb = m.tn[t];
      for (int e = 0; e < 3; e++) {
        if ((tri.w >> e) & 1) continue;
        int o = comp(nb, e);
        if (o < 0) continue;
        if (atomicExch(&w.hvis[o], 1) != 0) continue;
        atomicAdd((unsigned long long *)&stat_line(w)->v[kStInTests], 1ull);
        if (incircle_tri(m, w, m.tv[o], c.p) > 0) list[atomicAdd(&sh.s_n, 1)] = o;
        else list[top - atomicAdd(&sh.s_r, 1)] = o;
      }
    }
    __syncthreads();
  }
  const int len = sh.s_n, nrej = sh.s_r;
  __syncthreads();
  // every visited slot is flagged: clear the flags for the next cavity
  for (int j = tid; j < len; j += blockDim.x) w.hvis[list[j]] = 0;
  for (int j = tid; j < nrej; j += blockDim.x) w.hvis[list[top - j]] = 0;
  coop_finish(m, w, sh, c.S, c.ci, c.is_cc, c.skip_k, c.expect, c.p, list, len);
}

// Large cavities of one class (phase 0: circumcenters, 1: midpoints); the
// workgroups stride over the queue.
__global__ __launch_bounds__(kBigBlock) void k_cavity_big(DevMesh m, Work w, int phase) {
  __shared__ BigShared sh;
  if (w.st->halt) return;
  int nbig = min(w.cnt->nbig, w.big_cap);
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    int ref = w.big[b];
    int is_cc = (ref & 0x80000000) ? 0 : 1;
    if (is_cc != (phase == 0 ? 1 : 0)) continue;
    big_one(m, w, sh, b);
    __syncthreads();
  }
}

// Cavities of one class that outgrew the LDS list, one after the other by
// a single workgroup (launched only on meshes that have needed it).
__global__ __launch_bounds__(kHugeBlock) void k_cavity_huge(DevMesh m, Work w, int phase) {
  __shared__ BigShared sh;
  if (w.st->halt || w.cnt->nhuge == 0) return;
  int nbig = min(w.cnt->nbig, w.big_cap);
  for (int b = 0; b < nbig; b++) {
    int ref = w.big[b];
    int is_cc = (ref & 0x80000000) ? 0 : 1;
    if (is_cc != (phase == 0 ? 1 : 0)) continue;
    huge_one(m, w, sh, b);
  }
}

// ---------------------------------------------------------------------------
// R8: priority marks and ownership
// ---------------------------------------------------------------------------
// Loop bodies that load a few records and then use them are written as
// batches: all loads of a batch are issued before any result is needed
// (the stores in between would otherwise keep the compiler from hoisting
// them), which turns a chain of dependent memory latencies into a few.
constexpr int kIlp = 8;

__device__ __forceinline__ bool cand_at(const Work &w, int c, int ncc, CandSet &S, int &ci, int &is_cc) {
  if (c < ncc) { S = w.cc; ci = c; is_cc = 1; return true; }
  S = w.mid; ci = c - ncc; is_cc = 0; return true;
}

__device__ __forceinline__ void own_one(const Work &w, int c, int ncc, int &lost) {
  CandSet S;
  int ci, is_cc;
  cand_at(w, c, ncc, S, ci, is_cc);
  int st = S.state[ci];
  if (!(st & kStAlive)) return;
  uint64_t key = S.key[ci];
  int off = S.off[ci], len = S.len[ci];
  // independent loads, kIlp slots at a time (the marks are tested after)
  bool own = true;
  for (int j0 = 0; j0 < len && own; j0 += kIlp) {
    int t[kIlp];
    uint64_t mk[kIlp];
#pragma unroll
    for (int i = 0; i < kIlp; i++) t[i] = j0 + i < len ? w.pool[off + j0 + i] : -1;
#pragma unroll
    for (int i = 0; i < kIlp; i++) mk[i] = t[i] >= 0 ? w.mark[t[i]] : key;
#pragma unroll
    for (int i = 0; i < kIlp; i++) own = own && mk[i] == key;
  }
  if (own) {
    S.state[ci] = st | kStW0;
    bit_set(is_cc ? w.w0_t : w.w0_s, S.elem[ci]);
  } else {
    lost = 1;
  }
}

__device__ __forceinline__ void own_part(const Work &w, const Lanes &L) {
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk;
  int n_lost = 0;
  for (int base = L.base0; base < n; base += L.stride) {
    int c = base + threadIdx.x, lost = 0;
    if (c < n) own_one(w, c, ncc, lost);
    n_lost += lost;
  }
  stat_add(w, kStLostMark, n_lost);
}

__global__ void k_own(Work w) {
  if (w.st->halt) return;
  own_part(w, grid_lanes());
}

// R9: Delaunay dependency across a shared non-subsegment cavity edge.
// Returns true if the candidate is dropped.
__device__ __forceinline__ bool dep_one(const DevMesh &m, const Work &w, int c, int ncc, int &ntest) {
  CandSet S;
  int ci, is_cc;
  cand_at(w, c, ncc, S, ci, is_cc);
  int st = S.state[ci];
  if (!(st & kStW0)) return false;
  uint64_t key = S.key[ci];
  double2 p = S.p[ci];
  int off = S.off[ci], len = S.len[ci];
  int skip_k = is_cc ? -1 : S.elem[ci];
  bool drop = false;
  constexpr int B = 2;  // cavity triangles per batch
  for (int j0 = 0; j0 < len && !drop; j0 += B) {
    int tt[B];
    int4 tri_[B], nb_[B], ts_[B];
    uint64_t mo_[B][3];
#pragma unroll
    for (int i = 0; i < B; i++) tt[i] = j0 + i < len ? w.pool[off + j0 + i] : -1;
#pragma unroll
    for (int i = 0; i < B; i++) {
      const bool v = tt[i] >= 0;
      tri_[i] = v ? m.tv[tt[i]] : make_int4(0, 0, 0, 0);
      nb_[i] = v ? m.tn[tt[i]] : make_int4(-1, -1, -1, 0);
      ts_[i] = v ? m.ts[tt[i]] : make_int4(-1, -1, -1, 0);
    }
#pragma unroll
    for (int i = 0; i < B; i++)
#pragma unroll
      for (int e = 0; e < 3; e++) {
        const int o = comp(nb_[i], e);
        const bool sub = ((tri_[i].w >> e) & 1) && comp(ts_[i], e) >= 0;
        mo_[i][e] = (!sub && o >= 0) ? w.mark[o] : 0ull;
      }
#pragma unroll
    for (int i = 0; i < B; i++)
#pragma unroll
    for (int e = 0; e < 3; e++) {
      if (drop || tt[i] < 0) continue;
      const int4 tri = tri_[i];
      // subsegment edges (incl. the split one) and hull edges were given mark 0
      uint64_t mo = mo_[i][e];
      if (mo == key || mo == 0) continue;  // inside this cavity, or unclaimed
      int q_cc = (mo >> 63) ? 0 : 1;
      int qid = (int)perm32_inv((uint32_t)(mo & 0xffffffffu));
      if (!bit_get(q_cc ? w.w0_t : w.w0_s, qid)) continue;
      if (!(key < mo)) continue;  // only the lower key of a dependent pair drops
      double2 q = q_cc ? w.cc.p[w.cidx_t[qid]] : w.mid.p[w.cidx_s[qid]];
      double2 U = m.vxy[comp(tri, e)], V = m.vxy[comp(tri, (e + 1) % 3)];
      ntest++;
      if (incircle(U.x, U.y, V.x, V.y, p.x, p.y, q.x, q.y, w.tally) > 0) drop = true;
    }
  }
  (void)skip_k;
  if (!drop) {
    S.state[ci] = st | kStWin;
    bit_set(is_cc ? w.win_t : w.win_s, S.elem[ci]);
  }
  return drop;
}

__device__ __forceinline__ void dep_part(const DevMesh &m, const Work &w, const Lanes &L) {
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk;
  int n_drop = 0, ntest = 0;
  for (int base = L.base0; base < n; base += L.stride) {
    int c = base + threadIdx.x;
    if (c < n) n_drop += dep_one(m, w, c, ncc, ntest);
  }
  stat_add(w, kStDepDrop, n_drop);
  stat_add(w, kStInTests, ntest);
}

__global__ void k_dep(DevMesh m, Work w) {
  if (w.st->halt) return;
  dep_part(m, w, grid_lanes());
}

// ---------------------------------------------------------------------------
// Prefix sums (block scan + scan of block sums + add)
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;
static_assert(kScanTile == kScanTileSize, "scan tile size shared with the host and the readers");

// Exclusive scan over a workgroup of up to 1024 threads.
__device__ __forceinline__ int block_excl_scan(int v, int *total) {
  __shared__ int warp_sums[16];
  int lane = __lane_id(), wid = threadIdx.x / 64;
  // inclusive wave scan
  int x = v;
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) warp_sums[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < (int)(blockDim.x / 64); i++) {
      int s = warp_sums[i];
      warp_sums[i] = run;
      run += s;
    }
    *total = run;
  }
  __syncthreads();
  int r = x - v + warp_sums[wid];
  __syncthreads();
  return r;
}

// Exclusive scans in two launches: per-tile scans (the workgroups stride
// over the tiles of one or two jobs), then one workgroup per job scans the
// tile totals in place.  A reader adds the tile prefix itself:
// value(i) = out[i] + tiles[i / kScanTile].
__device__ void scan_tile(const ScanJob &j, int n, int tile) {
  __shared__ int s_total;
  int base = tile * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
  for (int i = 0; i < kScanItems; i++) {
    int idx = base + i;
    int x = idx < n ? j.in[idx] : 0;
    if (j.mode == 1) x = __popc((uint32_t)x);
    v[i] = x;
    sum += x;
  }
  int excl = block_excl_scan(sum, &s_total);
  for (int i = 0; i < kScanItems; i++) {
    int idx = base + i;
    if (idx < n) j.out[idx] = excl;
    excl += v[i];
  }
  if (threadIdx.x == 0) j.tiles[tile] = s_total;
  __syncthreads();
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(ScanJob a, ScanJob b, const int32_t *halt) {
  if (*halt) return;
  const int na = *a.n_dev, nb = b.in ? *b.n_dev : 0;
  const int ta = (na + kScanTile - 1) / kScanTile, tb = (nb + kScanTile - 1) / kScanTile;
  for (int tile = blockIdx.x; tile < ta + tb; tile += gridDim.x) {
    if (tile < ta) scan_tile(a, na, tile);
    else scan_tile(b, nb, tile - ta);
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(ScanJob a, ScanJob b, const int32_t *halt) {
  __shared__ int s_total;
  if (*halt) return;
  const ScanJob &j = blockIdx.x == 0 ? a : b;
  if (!j.in) return;
  const int ntiles = (*j.n_dev + kScanTile - 1) / kScanTile;
  int carry = 0;
  for (int start = 0; start < ntiles; start += kScanBlock) {
    int idx = start + threadIdx.x;
    int x = idx < ntiles ? j.tiles[idx] : 0;
    int e = block_excl_scan(x, &s_total);
    if (idx < ntiles) j.tiles[idx] = e + carry;
    carry += s_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *j.total = carry;
}

// ---------------------------------------------------------------------------
// R10: insertion
// ---------------------------------------------------------------------------
// Fresh slots of a winner: two, or one for a midpoint on a hull subsegment.
__device__ __forceinline__ int fresh_of(const Work &w, int is_cc, int e) {
  if (is_cc) return 2;
  return (w.sadj[2 * e] >= 0 && w.sadj[2 * e + 1] >= 0) ? 2 : 1;
}

__device__ __forceinline__ void winner_one(const Work &w, int c, int ncc, int nwin_mid) {
  CandSet S;
  int ci, is_cc;
  cand_at(w, c, ncc, S, ci, is_cc);
  if (!(S.state[ci] & kStWin)) return;
  int e = S.elem[ci];
  int r, fresh;
  if (is_cc) {
    r = nwin_mid + bit_rank(w.win_t, w.rank_t, w.tiles_t, e);
    fresh = 2;
  } else {
    r = bit_rank(w.win_s, w.rank_s, w.tiles_s, e);
    fresh = (w.sadj[2 * e] >= 0 && w.sadj[2 * e + 1] >= 0) ? 2 : 1;
  }
  w.win_ref[r] = (is_cc ? 0 : (int)0x80000000) | ci;
  w.fcount[r] = fresh;
}

// Winner ranks: midpoints by subsegment id, then circumcenters by slot.
// Also sets nwin, and a zero fresh count after the last winner, so that the
// exclusive scan over nwin + 1 entries ends with the total.
__device__ __forceinline__ void winners_part(const Work &w, const Lanes &L) {
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk;
  const int nwin_mid = w.cnt->nwin_mid;
  if (first_lane(L)) {
    int nwin = nwin_mid + w.cnt->nwin_cc;
    w.cnt->nwin = nwin;
    w.cnt->nwin1 = nwin + 1;
    w.fcount[nwin] = 0;
  }
  for (int base = L.base0; base < n; base += L.stride) {
    int c = base + threadIdx.x;
    if (c < n) winner_one(w, c, ncc, nwin_mid);
  }
}

__global__ void k_winners(Work w) {
  if (w.st->halt) return;
  winners_part(w, grid_lanes());
}

__device__ __forceinline__ bool owner_wins(const Work &w, uint64_t mo) {
  if (mo == 0) return false;
  int q_cc = (mo >> 63) ? 0 : 1;
  int qid = (int)perm32_inv((uint32_t)(mo & 0xffffffffu));
  return bit_get(q_cc ? w.win_t : w.win_s, qid);
}

// Fan records of each winner: boundary edges in canonical order (cavity
// slots ascending, edge index 0..2; the split subsegment is skipped).  The
// j-th fan triangle takes the j-th cavity slot, then fresh slots.
__device__ __forceinline__ void record_one(const DevMesh &m, const Work &w, int r, int foff) {
  int ref = w.win_ref[r];
  int is_cc = (ref & 0x80000000) ? 0 : 1;
  int ci = ref & 0x7fffffff;
  CandSet S = is_cc ? w.cc : w.mid;
  uint64_t key = S.key[ci];
  int off = S.off[ci], len = S.len[ci];
  int skip_k = is_cc ? -1 : S.elem[ci];
  int fresh_base = w.st->nT + fbase_at(w, r);
  int b = len + (fbase_at(w, r + 1) - fbase_at(w, r));
  w.fan_off[r] = foff;
  int j = 0;
  constexpr int B = 2;  // cavity triangles per batch
  for (int q0 = 0; q0 < len; q0 += B) {
    int tt[B];
    int4 tri_[B], nb_[B], ts_[B], to_[B][3];
    uint64_t mk_[B][3];
#pragma unroll
    for (int i = 0; i < B; i++) tt[i] = q0 + i < len ? w.pool[off + q0 + i] : -1;
#pragma unroll
    for (int i = 0; i < B; i++) {
      const bool v = tt[i] >= 0;
      tri_[i] = v ? m.tv[tt[i]] : make_int4(0, 0, 0, 0);
      nb_[i] = v ? m.tn[tt[i]] : make_int4(-1, -1, -1, 0);
      ts_[i] = v ? m.ts[tt[i]] : make_int4(-1, -1, -1, 0);
    }
#pragma unroll
    for (int i = 0; i < B; i++)
#pragma unroll
      for (int e = 0; e < 3; e++) {
        const int o = comp(nb_[i], e);
        mk_[i][e] = o >= 0 ? w.mark[o] : 0ull;
        to_[i][e] = o >= 0 ? m.tv[o] : make_int4(0, 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < B; i++)
#pragma unroll
    for (int e = 0; e < 3; e++) {
      if (tt[i] < 0) continue;
      const int t = tt[i];
      const int4 tri = tri_[i], ts = ts_[i];
      int sid = ((tri.w >> e) & 1) ? comp(ts, e) : -1;
      if (skip_k >= 0 && sid == skip_k) continue;
      int o = comp(nb_[i], e);
      if (sid < 0 && o >= 0 && mk_[i][e] == key) continue;
      int slot = j < len ? w.pool[off + j] : fresh_base + (j - len);
      int u = comp(tri, e), v = comp(tri, (e + 1) % 3);
      int jn = -1;
      if (o >= 0) {
        int4 to = to_[i][e];
        if (to.x == v && to.y == u) jn = 0;
        else if (to.y == v && to.z == u) jn = 1;
        else jn = 2;
      }
      if (j >= b) {  // cannot happen for a cavity that passed the boundary count check
        j++;
        continue;
      }
      FanRec f;
      f.slot = slot; f.u = u; f.v = v; f.o = o; f.jn = jn; f.ts = sid;
      w.fan[foff + j] = f;
      w.repl[t * 4 + e] = slot;
      j++;
    }
  }
  if (j != b) {
    atomicOr(&w.cnt->err, kErrCavity);
    if (atomicCAS(&w.cnt->dbg_set, 0, 1) == 0) {
      w.cnt->dbg[0] = is_cc;
      w.cnt->dbg[1] = S.elem[ci];
      w.cnt->dbg[2] = len;
      w.cnt->dbg[3] = b;
      w.cnt->dbg[4] = j;
      w.cnt->dbg[5] = S.state[ci];
    }
  }
}

// The capacity check of the round comes first: every thread evaluates it on
// the same counts; if anything would overflow, the round is abandoned before
// the mesh is written and the host grows the buffers and runs it again.
__device__ __forceinline__ void record_part(const DevMesh &m, const Work &w, const Lanes &L) {
  const DevState *st = w.st;
  DevCounters *c = w.cnt;
  const int nwin = c->nwin;
  const int fresh = fbase_at(w, nwin);
  const int64_t need_fan = (int64_t)c->pool_used + 2 * (int64_t)nwin;
  const bool over = (c->err & (kErrPool | kErrHuge)) || (int64_t)st->nV + nwin > m.capV ||
                    (int64_t)st->nT + fresh > m.capT || (int64_t)st->nS + c->nwin_mid > m.capS ||
                    need_fan > w.fan_cap || nwin + 1 > w.win_cap;
  if (first_lane(L)) {
    c->fresh_total = fresh;
    c->abort = over ? 1 : 0;
  }
  if (over) return;
  for (int base = L.base0; base < nwin; base += L.stride) {
    int r = base + threadIdx.x;
    int b = 0, len = 0, steps = 0, cc = 0;
    if (r < nwin) {
      const int ref = w.win_ref[r];
      cc = (ref & 0x80000000) ? 0 : 1;
      const CandSet S = cc ? w.cc : w.mid;
      len = S.len[ref & 0x7fffffff];
      b = len + (fbase_at(w, r + 1) - fbase_at(w, r));
      if (cc) steps = (S.state[ref & 0x7fffffff] >> kStepShift) & 0x7fff;
    }
    int foff = group_alloc(&w.cnt->fan_used, b, L);
    if (r < nwin) record_one(m, w, r, foff);
    // the winners' share of the round's memory work (winners' cavities are
    // disjoint, so a wave's sums of sizes and fan edges stay below 2^32)
    stat_add2(w, kStWinCav, kStWinBnd, len, b);
    stat_add2(w, kStWinCcCav, kStWinCcBnd, cc ? len : 0, cc ? b : 0);
    stat_add(w, kStWinSteps, steps);
  }
}

__global__ void k_record(DevMesh m, Work w) {
  if (w.st->halt) return;
  record_part(m, w, grid_lanes());
}

__device__ __forceinline__ void write_one(const DevMesh &m, const Work &w, int r, int nV, int nS, int serial) {
  int ref = w.win_ref[r];
  int is_cc = (ref & 0x80000000) ? 0 : 1;
  int ci = ref & 0x7fffffff;
  CandSet S = is_cc ? w.cc : w.mid;
  int len = S.len[ci];
  int b = len + (fbase_at(w, r + 1) - fbase_at(w, r));
  int foff = w.fan_off[r];
  int pid = nV + r;
  double2 p = S.p[ci];
  int k = -1, knew = -1, a = -1, bb = -1;
  if (!is_cc) {
    k = S.elem[ci];
    knew = nS + r;  // midpoint winners take ranks 0..nwin_mid-1
    int2 sk = m.sv[k];
    a = sk.x;
    bb = sk.y;
  }
  // kIlp fan records at a time: the records, then the outside marks, their
  // owners' win bits and replacement slots, each a batch of loads; a fan of
  // at most kIlp records finds its neighbours in registers
  for (int j0 = 0; j0 < b; j0 += kIlp) {
    FanRec F[kIlp];
    uint64_t mo[kIlp];
    bool ow[kIlp];
    int rp[kIlp];
#pragma unroll
    for (int i = 0; i < kIlp; i++) F[i] = j0 + i < b ? w.fan[foff + j0 + i] : FanRec{-1, -2, -2, -1, 0, -1};
#pragma unroll
    for (int i = 0; i < kIlp; i++) mo[i] = F[i].o >= 0 ? w.mark[F[i].o] : 0ull;
#pragma unroll
    for (int i = 0; i < kIlp; i++) ow[i] = F[i].o >= 0 && owner_wins(w, mo[i]);
#pragma unroll
    for (int i = 0; i < kIlp; i++) rp[i] = ow[i] ? w.repl[F[i].o * 4 + F[i].jn] : -1;
#pragma unroll
    for (int i = 0; i < kIlp; i++) {
      if (j0 + i >= b) continue;
      const FanRec f = F[i];
      const int s = f.slot;
      int n0;
      if (f.o < 0) n0 = -1;
      else if (ow[i]) n0 = rp[i];
      else {
        n0 = f.o;
        ((int32_t *)m.tn)[f.o * 4 + f.jn] = s;
      }
      int n1 = -1, n2 = -1;
      if (b <= kIlp) {
#pragma unroll
        for (int g = 0; g < kIlp; g++) {
          if (g >= b) continue;
          if (F[g].u == f.v) n1 = F[g].slot;
          if (F[g].v == f.u) n2 = F[g].slot;
        }
      } else {
        for (int g = 0; g < b; g++) {
          FanRec h = w.fan[foff + g];
          if (h.u == f.v) n1 = h.slot;
          if (h.v == f.u) n2 = h.slot;
        }
      }
      int s1 = -1, s2 = -1;
      if (!is_cc) {
        s1 = f.v == a ? k : (f.v == bb ? knew : -1);
        s2 = f.u == a ? k : (f.u == bb ? knew : -1);
      }
      int mask = (f.ts >= 0 ? 1 : 0) | (s1 >= 0 ? 2 : 0) | (s2 >= 0 ? 4 : 0);
      m.tv[s] = make_int4(f.u, f.v, pid, mask);
      m.tn[s] = make_int4(n0, n1, n2, 0);
      m.ts[s] = make_int4(f.ts, s1, s2, 0);
      w.tstamp[s] = serial;
    }
  }
  m.vxy[pid] = p;
  m.vkind[pid] = is_cc ? 2 : 1;
  if (!is_cc) {
    m.sv[k] = make_int2(a, pid);
    m.sv[knew] = make_int2(pid, bb);
    m.spar[knew] = m.spar[k];
    m.spend[knew] = 0;
    w.sadj[2 * knew] = -1;
    w.sadj[2 * knew + 1] = -1;
    w.mflag[knew] = 0u;
  }
}

__device__ __forceinline__ void write_part(const DevMesh &m, const Work &w, const Lanes &L) {
  if (w.cnt->abort) return;
  const int nwin = w.cnt->nwin, nV = w.st->nV, nS = w.st->nS, serial = w.st->serial;
  for (int base = L.base0; base < nwin; base += L.stride) {
    int r = base + threadIdx.x;
    if (r < nwin) write_one(m, w, r, nV, nS, serial);
  }
}

__global__ void k_write(DevMesh m, Work w) {
  if (w.st->halt) return;
  write_part(m, w, grid_lanes());
}

// R11: clear marks and bitmap bits of every candidate; pending flags.  A
// subsegment is split iff its second endpoint is now a new vertex.  After an
// abandoned round nothing was split and the flags are only released.
__device__ __forceinline__ void finish_one(const DevMesh &m, const Work &w, int c, int ncc, int nV, bool aborted) {
  CandSet S;
  int ci, is_cc;
  cand_at(w, c, ncc, S, ci, is_cc);
  int st = S.state[ci];
  if (st & kStAlive) {
    int off = S.off[ci], len = S.len[ci];
    for (int j0 = 0; j0 < len; j0 += kIlp) {
      int t[kIlp];
#pragma unroll
      for (int i = 0; i < kIlp; i++) t[i] = j0 + i < len ? w.pool[off + j0 + i] : -1;
#pragma unroll
      for (int i = 0; i < kIlp; i++)
        if (t[i] >= 0) w.mark[t[i]] = 0ull;
    }
  }
  int e = S.elem[ci];
  uint32_t bit = 1u << (e & 31);
  if (st & kStW0) atomicAnd(&(is_cc ? w.w0_t : w.w0_s)[e >> 5], ~bit);
  if (st & kStWin) atomicAnd(&(is_cc ? w.win_t : w.win_s)[e >> 5], ~bit);
  if (!is_cc) {
    // pending := (pending or flagged this round) and not split; an entry the
    // cap skipped is not "flagged" unless R4/R5 flagged it again (own entry)
    if (!aborted) {
      bool split = m.sv[e].y >= nV;
      if (!(st & kStSkip)) m.spend[e] = split ? 0 : 1;
      else if (split) m.spend[e] = 0;
    }
    w.mflag[e] = 0u;
  }
}

// End of a round (run by the last workgroup of k_finish to arrive, or by the
// single-workgroup engine): a
// completed round is recorded in the history, the counts advance, this
// round's lists become the previous ones and the counters are cleared for
// the next round.  An error, an abandoned round or a round without winners
// halts instead (the counters stay for the host to read).
// Folds the stat lines into the round counters and clears them (one
// workgroup; ends with a barrier).
__device__ __forceinline__ void round_fold(const Work &w) {
  __shared__ uint64_t s_fold[kStFields];
  DevCounters *c = w.cnt;
  // fold the stat lines into the counters and clear them (read-and-clear
  // atomics: the lines were written by atomics)
  if (threadIdx.x < kStFields) s_fold[threadIdx.x] = 0;
  __syncthreads();
  constexpr int kGroups = (kStFields + 3) / 4;
  for (int idx = threadIdx.x; idx < kGroups * kStatStripes; idx += blockDim.x) {
    // one stripe, four of its fields (independent read-and-clear atomics),
    // combined in LDS
    const int i = idx / kGroups, f0 = (idx % kGroups) * 4;
    for (int f = f0; f < f0 + 4 && f < kStFields; f++) {
      const uint64_t x = atomicExch((unsigned long long *)&w.stat[i].v[f], 0ull);
      if (!x) continue;
      if (f == kStCavMax) atomicMax((unsigned long long *)&s_fold[f], (unsigned long long)x);
      else atomicAdd((unsigned long long *)&s_fold[f], (unsigned long long)x);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c->cav_tri_total += (int64_t)s_fold[kStCavTri];
    c->cav_len[0] += (int64_t)s_fold[kStCavLen0];
    c->cav_len[1] += (int64_t)s_fold[kStCavLen1];
    c->cav_bnd[0] += (int64_t)s_fold[kStCavBnd0];
    c->cav_bnd[1] += (int64_t)s_fold[kStCavBnd1];
    c->n_enc_reject += (int32_t)s_fold[kStEncReject];
    c->n_fan_invalid += (int32_t)s_fold[kStFanInvalid];
    c->n_unsplittable += (int32_t)s_fold[kStUnsplittable];
    c->n_mid_cand += (int32_t)s_fold[kStMidCand];
    c->n_lost_mark += (int32_t)s_fold[kStLostMark];
    c->n_dep_drop += (int32_t)s_fold[kStDepDrop];
    c->n_blocked += (int32_t)s_fold[kStBlocked];
    c->n_coincident += (int32_t)s_fold[kStCoincident];
    c->cav_max = max(c->cav_max, (int32_t)s_fold[kStCavMax]);
    c->n_in_tests += (int64_t)s_fold[kStInTests];
    c->n_or_tests += (int64_t)s_fold[kStOrTests];
    for (int e = 0; e < kExStages; e++) c->n_exact[e] += (int64_t)s_fold[kStExact0 + e];
    c->win_cav += (int64_t)s_fold[kStWinCav];
    c->win_bnd += (int64_t)s_fold[kStWinBnd];
    c->win_steps += (int64_t)s_fold[kStWinSteps];
    c->win_cc_cav += (int64_t)s_fold[kStWinCcCav];
    c->win_cc_bnd += (int64_t)s_fold[kStWinCcBnd];
    c->n_marks[0] += (int64_t)s_fold[kStMarks0];
    c->n_marks[1] += (int64_t)s_fold[kStMarks1];
  }
  __syncthreads();
}

__device__ __forceinline__ void round_end(const Work &w) {
  __shared__ int s_go, s_slot;
  DevState *st = w.st;
  DevCounters *c = w.cnt;
  round_fold(w);
  if (threadIdx.x == 0) {
    s_go = 0;
    s_slot = -1;
    const int err = c->err, nwin = c->nwin;
    if (err & (kErrWalk | kErrInput | kErrCavity)) st->halt = kHaltError;
    else if (c->abort) st->halt = kHaltAbort;
    else if (nwin == 0) st->halt = kHaltStall;
    else {
      s_go = 1;
      const int nh = st->nhist;
      if (nh < w.hist_cap) s_slot = nh;
      st->nhist = nh + 1;
      const int nT = st->nT + c->fresh_total, nS = st->nS + c->nwin_mid;
      st->nV = st->nV + nwin;
      st->nT = nT;
      st->nS = nS;
      st->wT = nT / 32 + 1;
      st->wS = nS / 32 + 1;
      st->rounds = st->rounds + 1;
      st->serial = st->serial + 1;
      st->prev_ncc = c->ncc;
      st->prev_nmk = c->nmk;
      st->prev_fan = c->fan_used;
      st->full = 0;
    }
  }
  __syncthreads();
  if (!s_go) return;
  const int nw = (int)(sizeof(DevCounters) / 4);
  int32_t *src = (int32_t *)c;
  if (s_slot >= 0) {
    int32_t *dst = (int32_t *)&w.hist[s_slot];
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nw; i += blockDim.x) src[i] = 0;
}

__device__ __forceinline__ void finish_part(const DevMesh &m, const Work &w, const Lanes &L) {
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk, nV = w.st->nV;
  // an abandoned round, or one that inserts nothing (the refinement stops
  // there), leaves the pending flags as they were
  bool aborted = w.cnt->abort != 0 || w.cnt->nwin == 0;
  for (int base = L.base0; base < n; base += L.stride) {
    int c = base + threadIdx.x;
    if (c < n) finish_one(m, w, c, ncc, nV, aborted);
  }
}

__global__ void k_finish(DevMesh m, Work w) {
  __shared__ int s_last;
  if (w.st->halt) return;
  finish_part(m, w, grid_lanes());
  // every workgroup has read the counts it needs before it arrives here
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&w.st->done_blocks, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (threadIdx.x == 0) w.st->done_blocks = 0;
  round_end(w);
}

// ---------------------------------------------------------------------------
// Flip-Flop rounds (Section 4.3): Line 6 claims and the end of the round.
// ---------------------------------------------------------------------------
// Edge of the located triangle a circumcenter lies on, + 1, kept in bits 8-9
// of its state (0: strictly inside).
constexpr int kFfEdgeShift = 8;

// A located circumcenter claims its triangle, or both triangles of the
// interior edge it lies on; one on a subsegment encroaches it and flags it.
__global__ void kf_claim_cc(DevMesh m, Work w) {
  if (w.st->halt) return;
  const Lanes L = grid_lanes();
  const int ncc = w.cnt->ncc;
  int n_rej = 0;
  for (int base = L.base0; base < ncc; base += L.stride) {
    const int c = base + threadIdx.x;
    if (c >= ncc) continue;
    const int st = w.cc.state[c];
    if (!(st & kStFound) || (st & kStDone)) continue;
    const int loc = w.cc.loc[c];
    const int4 tri = m.tv[loc];
    const double2 p = w.cc.p[c];
    const double2 A = m.vxy[tri.x], B = m.vxy[tri.y], C = m.vxy[tri.z];
    const int s0 = orient_pts(w, A, B, p), s1 = orient_pts(w, B, C, p), s2 = orient_pts(w, C, A, p);
    const int e = s0 == 0 ? 0 : (s1 == 0 ? 1 : (s2 == 0 ? 2 : -1));
    int c1 = -1;
    if (e >= 0) {
      if ((tri.w >> e) & 1) {
        flag_mid(w, comp(m.ts[loc], e));
        w.cc.state[c] = st | kStDone;
        n_rej++;
        continue;
      }
      c1 = comp(m.tn[loc], e);
    }
    const uint64_t key = w.cc.key[c];
    w.cc.off[c] = loc;
    w.cc.len[c] = c1;
    w.cc.state[c] = (st & ~(3 << kFfEdgeShift)) | ((e + 1) << kFfEdgeShift);
    atomicMax((unsigned long long *)&w.mark[loc], (unsigned long long)key);
    if (c1 >= 0) atomicMax((unsigned long long *)&w.mark[c1], (unsigned long long)key);
  }
  stat_add(w, kStEncReject, n_rej);
}

// A flagged subsegment's split point claims the triangles on its sides
// (4 * slot + edge of each, -1 none); an unsplittable one is dropped.
__global__ void kf_claim_mid(DevMesh m, Work w) {
  if (w.st->halt) return;
  const Lanes L = grid_lanes();
  const int nmk = w.cnt->nmk;
  int n_cand = 0, n_uns = 0;
  for (int base = L.base0; base < nmk; base += L.stride) {
    const int i = base + threadIdx.x;
    if (i >= nmk) continue;
    const int st = w.mid.state[i];
    if (st & kStSkip) continue;
    const int k = w.mid.elem[i];
    n_cand++;
    const SplitPt sp = seg_split(m, k, w.pm, w.split_mode);
    const int2 s = m.sv[k];
    const double2 A = m.vxy[s.x], B = m.vxy[s.y];
    if ((sp.px == A.x && sp.py == A.y) || (sp.px == B.x && sp.py == B.y)) {
      w.mid.state[i] = st | kStDone;
      n_uns++;
      continue;
    }
    const int c0 = w.sadj[2 * k], c1 = w.sadj[2 * k + 1];
    w.mid.key[i] = sp.key;
    w.mid.p[i] = make_double2(sp.px, sp.py);
    w.mid.off[i] = c0;
    w.mid.len[i] = c1;
    w.mid.state[i] = st | kStFound;
    if (c0 >= 0) atomicMax((unsigned long long *)&w.mark[c0 >> 2], (unsigned long long)sp.key);
    if (c1 >= 0) atomicMax((unsigned long long *)&w.mark[c1 >> 2], (unsigned long long)sp.key);
  }
  stat_add(w, kStMidCand, n_cand);
  stat_add(w, kStUnsplittable, n_uns);
}

// Points that hold every claim go to S (midpoint references have bit 30).
__global__ void kf_own(Work w, FfCount *f, uint64_t *skey, int32_t *sref) {
  if (w.st->halt) return;
  const Lanes L = grid_lanes();
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk;
  int n_lost = 0;
  for (int base = L.base0; base < n; base += L.stride) {
    const int c = base + threadIdx.x;
    if (c >= n) continue;
    const bool is_cc = c < ncc;
    const int ci = is_cc ? c : c - ncc;
    const CandSet &S = is_cc ? w.cc : w.mid;
    const int st = S.state[ci];
    if (!(st & kStFound) || (st & (kStDone | kStSkip))) continue;
    const uint64_t key = S.key[ci];
    int c0 = S.off[ci], c1 = S.len[ci];
    if (!is_cc) {
      c0 = c0 >= 0 ? c0 >> 2 : -1;
      c1 = c1 >= 0 ? c1 >> 2 : -1;
    }
    const bool own = (c0 < 0 || w.mark[c0] == key) && (c1 < 0 || w.mark[c1] == key);
    if (!own) { n_lost++; continue; }
    const int idx = FfDevOps::append(&f->np);
    skey[idx] = ~key;
    sref[idx] = is_cc ? ci : (ci | (1 << 30));
    if (!is_cc) FfDevOps::append(&f->nmid);
  }
  stat_add(w, kStLostMark, n_lost);
}

__global__ void kf_clear_marks(Work w) {
  if (w.st->halt) return;
  const Lanes L = grid_lanes();
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk;
  for (int base = L.base0; base < n; base += L.stride) {
    const int c = base + threadIdx.x;
    if (c >= n) continue;
    const bool is_cc = c < ncc;
    const int ci = is_cc ? c : c - ncc;
    const CandSet &S = is_cc ? w.cc : w.mid;
    const int st = S.state[ci];
    if (!(st & kStFound) || (st & kStSkip)) continue;
    if (is_cc && (st & kStDone)) continue;  // dropped before claiming
    int c0 = S.off[ci], c1 = S.len[ci];
    if (!is_cc) {
      if (st & kStDone) continue;
      c0 = c0 >= 0 ? c0 >> 2 : -1;
      c1 = c1 >= 0 ? c1 >> 2 : -1;
    }
    if (c0 >= 0) w.mark[c0] = 0ull;
    if (c1 >= 0) w.mark[c1] = 0ull;
  }
}

// S by rank (the sorted references): point, class, claims, a midpoint's
// subsegment endpoints; every point starts in the mesh and not redundant.
__global__ void kf_gather(DevMesh m, Work w, FfView V, const int32_t *sref) {
  const int np = V.c->np;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < np; r += gridDim.x * blockDim.x) {
    const int ref = sref[r];
    ff_init_point_one<FfDevOps>(V, r);
    if (ref & (1 << 30)) {
      const int i = ref & ((1 << 30) - 1);
      const int k = w.mid.elem[i];
      V.pt[r] = w.mid.p[i];
      V.pinfo[r] = make_int4(1, k, w.mid.off[i], w.mid.len[i]);
      V.pab[r] = m.sv[k];
    } else {
      const int st = w.cc.state[ref];
      V.pt[r] = w.cc.p[ref];
      V.pinfo[r] = make_int4(0, ((st >> kFfEdgeShift) & 3) - 1, w.cc.off[ref], w.cc.len[ref]);
      V.pab[r] = make_int2(-1, -1);
    }
  }
}

// End of a Flip-Flop round (one workgroup): statistics folded in, the counts
// advanced to the compacted mesh, the round recorded, the counters cleared.
// Every element of the round's candidate lists was consumed by the host-side
// sequence, so the next round collects over the whole mesh again.
__global__ void kf_round_end(Work w, const FfCount *f, int32_t nT_new, int32_t nwin, int32_t nwin_mid) {
  __shared__ int s_slot;
  DevState *st = w.st;
  DevCounters *c = w.cnt;
  round_fold(w);
  if (threadIdx.x == 0) {
    c->n_dep_drop += (int32_t)f->n_dep;
    c->n_enc_reject += (int32_t)f->n_enc;
    c->nwin = nwin;
    c->nwin_mid = nwin_mid;
    c->nwin_cc = nwin - nwin_mid;
    c->fresh_total = nT_new - st->nT;
    c->ff_points = f->np;
    c->ff_iters = f->iters;
    c->ff_flips = f->flips;
    c->ff_passes = f->passes;
    c->ff_removals = f->removals;
    c->ff_rm_passes = f->rm_passes;
    const int nh = st->nhist;
    s_slot = nh < w.hist_cap ? nh : -1;
    st->nhist = nh + 1;
    st->nV = st->nV + nwin;
    st->nT = nT_new;
    st->nS = st->nS + nwin_mid;
    st->wT = nT_new / 32 + 1;
    st->wS = st->nS / 32 + 1;
    st->rounds = st->rounds + 1;
    st->serial = st->serial + 1;
    st->prev_ncc = 0;
    st->prev_nmk = 0;
    st->prev_fan = 0;
    st->full = 1;
  }
  __syncthreads();
  const int nw = (int)(sizeof(DevCounters) / 4);
  int32_t *src = (int32_t *)c;
  if (s_slot >= 0) {
    int32_t *dst = (int32_t *)&w.hist[s_slot];
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nw; i += blockDim.x) src[i] = 0;
}

// ---------------------------------------------------------------------------
// Mesh quality (the bad-area measure of Table 1): every triangle is tested
// with the scan's formula; a bad one adds its doubled area / 2.  Each block
// sums its lanes in a fixed tree order; the partials are summed in index
// order by one thread, so the result depends only on the grid shape.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_quality(DevMesh m, double B2, double L2, unsigned long long *n_part,
                                                 double *a_part) {
  __shared__ unsigned long long s_n[256];
  __shared__ double s_a[256];
  unsigned long long n = 0;
  double a = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m.nT; t += gridDim.x * blockDim.x) {
    SplitPt r = tri_split(m, t, m.tv[t], B2, L2, 0);
    if (r.bad) {
      n++;
      a += r.d * 0.5;
    }
  }
  s_n[threadIdx.x] = n;
  s_a[threadIdx.x] = a;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_n[threadIdx.x] += s_n[threadIdx.x + h];
      s_a[threadIdx.x] += s_a[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    n_part[blockIdx.x] = s_n[0];
    a_part[blockIdx.x] = s_a[0];
  }
}

__global__ void k_scatter_copy(const int32_t *src, const CopyEnt *ents, int n) {
  for (int e = blockIdx.x; e < n; e += gridDim.x) {
    const CopyEnt c = ents[e];
    const int32_t *a = src + c.src_off / 4;
    const int64_t words = c.bytes / 4;
    for (int64_t i = threadIdx.x; i < words; i += blockDim.x) c.dst[i] = a[i];
  }
}

__global__ void k_quality_sum(int n_part, const unsigned long long *n_in, const double *a_in,
                              unsigned long long *n_out, double *a_out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  unsigned long long n = 0;
  double a = 0.0;
  for (int i = 0; i < n_part; i++) {
    n += n_in[i];
    a += a_in[i];
  }
  *n_out = n;
  *a_out = a;
}

// ---------------------------------------------------------------------------
// Single-workgroup engine: whole rounds, every phase of Lines 3-9, inside one
// workgroup, with workgroup barriers between the phases instead of kernel
// launches.  Used for rounds too small to fill the chip (the end of a
// refinement, where launch latency dominates) and, one mesh per workgroup,
// for batches of independent meshes.  The phases are the same functions the
// grid kernels run, so the result is identical.
// ---------------------------------------------------------------------------
// Barrier between two phases.  Every wave of the engine runs on one compute
// unit, so the workgroup-scope release / acquire of the barrier is enough to
// make each phase's writes (stores and atomics) visible to the next phase.
__device__ __forceinline__ void phase_sync() { __syncthreads(); }

// Exclusive scan of *j.n_dev entries by one workgroup: complete prefixes in
// j.out, zero tile prefixes (so that readers that add them are unchanged).
__device__ void engine_scan(const ScanJob &j) {
  __shared__ int s_total;
  const int n = *j.n_dev;
  const int chunk = blockDim.x * kScanItems;
  int carry = 0;
  for (int start = 0; start < n; start += chunk) {
    int base = start + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
    for (int i = 0; i < kScanItems; i++) {
      int idx = base + i;
      int x = idx < n ? j.in[idx] : 0;
      if (j.mode == 1) x = __popc((uint32_t)x);
      v[i] = x;
      sum += x;
    }
    int excl = block_excl_scan(sum, &s_total) + carry;
    for (int i = 0; i < kScanItems; i++) {
      int idx = base + i;
      if (idx < n) j.out[idx] = excl;
      excl += v[i];
    }
    carry += s_total;
    __syncthreads();
  }
  for (int t = threadIdx.x; t <= n / kScanTile; t += blockDim.x) j.tiles[t] = 0;
  if (threadIdx.x == 0) *j.total = carry;
}

// Radix select of the K-th largest key by one workgroup (keys are unique);
// the threshold goes to w.sel[0] (0 when no more than K keys).
__device__ void engine_select(const Work &w, int K, int32_t *h) {
  __shared__ uint64_t s_prefix, s_pmask;
  __shared__ int64_t s_rem;
  const int n = w.cnt->ncc + w.cnt->nmk;
  if (threadIdx.x == 0) {
    s_prefix = 0;
    s_pmask = 0;
    s_rem = K;
  }
  __syncthreads();
  if (n > K) {
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
      __syncthreads();
      const uint64_t prefix = s_prefix, pmask = s_pmask;
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        uint64_t k = w.keys[c];
        if ((k & pmask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int64_t cum = 0;
        int d = 255;
        for (; d > 0; d--) {
          if (cum + h[d] >= s_rem) break;
          cum += h[d];
        }
        s_rem -= cum;
        s_prefix |= (uint64_t)d << shift;
        s_pmask |= (uint64_t)0xff << shift;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) w.sel[0] = s_prefix;
}

// Winner ranks by counting (at most kEngRankMax winners): rank = number of
// winners with a smaller (class, element) key, midpoints first, which is the
// order the bitmap ranks give.  Returns false if there are more winners.
constexpr int kEngRankMax = 2048;
__device__ bool engine_rank(const Work &w, int32_t *lds) {
  __shared__ int s_nw, s_nmid;
  int32_t *key = lds, *ref = lds + kEngRankMax;
  if (threadIdx.x == 0) {
    s_nw = 0;
    s_nmid = 0;
  }
  __syncthreads();
  const int ncc = w.cnt->ncc, n = ncc + w.cnt->nmk;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    CandSet S;
    int ci, is_cc;
    cand_at(w, c, ncc, S, ci, is_cc);
    if (!(S.state[ci] & kStWin)) continue;
    int pos = atomicAdd(&s_nw, 1);
    if (!is_cc) atomicAdd(&s_nmid, 1);
    if (pos < kEngRankMax) {
      key[pos] = (int32_t)(((uint32_t)is_cc << 31) | (uint32_t)S.elem[ci]);
      ref[pos] = (is_cc ? 0 : (int)0x80000000) | ci;
    }
  }
  __syncthreads();
  const int nw = s_nw;
  if (nw > kEngRankMax) return false;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    const uint32_t k = (uint32_t)key[i];
    int r = 0;
    for (int j = 0; j < nw; j++) r += (uint32_t)key[j] < k;
    w.win_ref[r] = ref[i];
    w.fcount[r] = fresh_of(w, (k >> 31) != 0, (int)(k & 0x7fffffffu));
  }
  if (threadIdx.x == 0) {
    w.cnt->nwin_mid = s_nmid;
    w.cnt->nwin_cc = nw - s_nmid;
    w.cnt->nwin = nw;
    w.cnt->nwin1 = nw + 1;
    w.fcount[nw] = 0;
  }
  return true;
}

// The single-workgroup engine's large cavities: growth, bitonic sort and
// checks in LDS, as the cooperative kernel does, by the engine's own
// workgroup.  A cavity beyond the LDS list makes the round abandon itself
// (kErrHuge); the host then runs that mesh's rounds on the grid kernels,
// which finish such cavities in device memory.
__device__ __forceinline__ void engine_big_one(const DevMesh &m, const Work &w, BigShared &sh, int b) {
  int32_t *cav = sh.cav;
  int32_t *hs = sh.hs;
  int &s_n = sh.s_n, &s_head = sh.s_head, &s_ovf = sh.s_ovf, &s_nbnd = sh.s_nbnd, &s_fanbad = sh.s_fanbad,
      &s_enc = sh.s_enc, &s_off = sh.s_off;
  int tid = threadIdx.x;
  int ref = w.big[b];
  int is_cc = (ref & 0x80000000) ? 0 : 1;
  int ci = ref & 0x7fffffff;
  CandSet S = is_cc ? w.cc : w.mid;
  if (!(S.state[ci] & kStBig) || (S.state[ci] & kStDone)) return;
  double2 p = S.p[ci];
  int skip_k = is_cc ? -1 : S.elem[ci];
  for (int i = tid; i < kHash; i += blockDim.x) hs[i] = -1;
  __syncthreads();
  int expect = 2;
  if (tid == 0) {
    s_n = 0; s_head = 0; s_ovf = 0; s_nbnd = 0; s_fanbad = 0; s_enc = 0;
    if (is_cc) {
      int t = S.loc[ci];
      hash_insert(hs, t, &s_ovf);
      cav[s_n++] = t;
    } else {
      int a0 = w.sadj[2 * skip_k], a1 = w.sadj[2 * skip_k + 1];
      if (a0 >= 0 && hash_insert(hs, a0 >> 2, &s_ovf)) cav[s_n++] = a0 >> 2;
      if (a1 >= 0 && hash_insert(hs, a1 >> 2, &s_ovf)) cav[s_n++] = a1 >> 2;
    }
  }
  if (!is_cc) expect = (w.sadj[2 * skip_k] >= 0 && w.sadj[2 * skip_k + 1] >= 0) ? 2 : 1;
  __syncthreads();
  for (;;) {
    int lo = s_head, hi = s_n < kBigMax ? s_n : kBigMax;
    int ovf = s_ovf;
    __syncthreads();
    if (lo >= hi || ovf) break;
    if (tid == 0) s_head = hi;
    for (int idx = lo + tid; idx < hi; idx += blockDim.x) {
      int t = cav[idx];
      int4 tri = m.tv[t];
      int4 nb = m.tn[t];
      for (int e = 0; e < 3; e++) {
        if ((tri.w >> e) & 1) continue;
        int o = comp(nb, e);
        if (o < 0) continue;
        if (!hash_insert(hs, o, &s_ovf)) continue;
        if (incircle_tri(m, w, m.tv[o], p) > 0) {
          int pos = atomicAdd(&s_n, 1);
          if (pos < kBigMax) cav[pos] = o;
          else s_ovf = 1;
        }
      }
    }
    __syncthreads();
  }
  if (s_ovf) {
    if (tid == 0) atomicOr(&w.cnt->err, kErrHuge);
    return;
  }
  int len = s_n;
  int P = 1;
  while (P < len) P <<= 1;
  for (int i = len + tid; i < P; i += blockDim.x) cav[i] = 0x7fffffff;
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = tid; i < P; i += blockDim.x) {
        int j = i ^ stride;
        if (j > i) {
          bool up = (i & size) == 0;
          int x = cav[i], y = cav[j];
          if ((x > y) == up) { cav[i] = y; cav[j] = x; }
        }
      }
    }
  __syncthreads();
  // boundary checks, in parallel over cavity triangles
  for (int j = tid; j < len; j += blockDim.x) {
    int t = cav[j];
    int4 tri = m.tv[t];
    int4 nb = m.tn[t];
    int4 ts = tri.w ? m.ts[t] : make_int4(-1, -1, -1, 0);
    for (int e = 0; e < 3; e++) {
      int sid = ((tri.w >> e) & 1) ? comp(ts, e) : -1;
      if (skip_k >= 0 && sid == skip_k) continue;
      int o = comp(nb, e);
      if (sid < 0 && o >= 0 && in_sorted(cav, len, o)) continue;
      atomicAdd(&s_nbnd, 1);
      double2 U = m.vxy[comp(tri, e)], V = m.vxy[comp(tri, (e + 1) % 3)];
      if (is_cc && sid >= 0 && encroached(w, U, V, p)) {
        flag_mid(w, sid);
        s_enc = 1;
      }
      if (orient_pts(w, U, V, p) <= 0) s_fanbad = 1;
    }
  }
  __syncthreads();
  if (tid == 0) {
    s_off = -1;
    bool drop = (is_cc && s_enc) || s_fanbad || s_nbnd - len != expect;
    if (drop) {
      atomicAdd((unsigned long long *)&w.cnt->cav_tri_total, (unsigned long long)len);
      atomicMax(&w.cnt->cav_max, len);
      atomicAdd((is_cc && s_enc) ? &w.cnt->n_enc_reject : &w.cnt->n_fan_invalid, 1);
      S.state[ci] |= kStDone;
    } else {
      int off = atomicAdd(&w.cnt->pool_used, len);
      if (off + len > w.pool_cap) atomicOr(&w.cnt->err, kErrPool);
      else {
        s_off = off;
        atomicAdd((unsigned long long *)&w.cnt->cav_tri_total, (unsigned long long)len);
        atomicMax(&w.cnt->cav_max, len);
      }
    }
  }
  __syncthreads();
  int off = s_off;
  if (off >= 0) {
    uint64_t key = S.key[ci];
    for (int j = tid; j < len; j += blockDim.x) {
      w.pool[off + j] = cav[j];
      atomicMax((unsigned long long *)&w.mark[cav[j]], (unsigned long long)key);
    }
    if (tid == 0) {
      S.off[ci] = off;
      S.len[ci] = len;
      S.state[ci] |= kStDone | kStAlive;
    }
  }
}

// Large cavities of one class, one after the other, by the whole workgroup.
__device__ void engine_big(const DevMesh &m, const Work &w, BigShared &sh, int phase) {
  const int nbig = min(w.cnt->nbig, w.big_cap);
  for (int b = 0; b < nbig; b++) {
    int ref = w.big[b];
    int is_cc = (ref & 0x80000000) ? 0 : 1;
    if (is_cc != (phase == 0 ? 1 : 0)) continue;
    engine_big_one(m, w, sh, b);
    __syncthreads();
  }
}

// The engine's per-thread cavities: half the workgroup, with slices twice as
// long as the grid kernel's (large cavities are common in small meshes with
// clustered points, and the cooperative path runs them one at a time here).
constexpr int kEngCavThreads = kEngBlock / 2;
constexpr int kEngCap = 48;
// midpoint cavities listed before the circumcenter cavities run on the other
// half of the workgroup at the same time, in slices of their own
constexpr int kEngMidCap = 24;
static_assert(kEngCap <= kStat4Cap && kEngMidCap <= kStat4Cap, "engine cavity statistics fit stat_add4");
constexpr int kEngMidLdsWords = kEngMidCap * kEngCavThreads;
constexpr int kEngLdsWords = (kEngCap * kEngCavThreads > (int)(sizeof(BigShared) / 4)) ? kEngCap * kEngCavThreads
                                                                                     : (int)(sizeof(BigShared) / 4);
static_assert(kApproxMax * kEngBlock <= kEngLdsWords, "prefilter slices fit in the engine's LDS");
static_assert(2 * kEngRankMax <= kEngLdsWords, "winner keys fit in the engine's LDS");

// Rounds of one mesh until it halts or round_limit rounds have completed.
__device__ void engine_mesh(const EngDesc &d, int32_t *lds, int round_limit) {
  __shared__ int s_ser, s_full, s_halt, s_mid0;
  const DevMesh &m = d.m;
  DevState *st = d.w[0].st;
  const Lanes L = block_lanes();
  for (int r = 0; r < round_limit; r++) {
    phase_sync();
    if (threadIdx.x == 0) {
      s_halt = st->halt;
      s_ser = st->serial;
      s_full = st->full;
    }
    __syncthreads();
    if (s_halt) break;
    const Work &w = d.w[s_ser & 1];
    // R1 collection
    if (s_full) {
      scan_part(m, w, d.B2, d.pm, L);
    } else {
      carry_part(w, L);
      dirty_part(m, w, d.B2, d.pm, L);
      phase_sync();
      pending_part(m, w, L);
    }
    phase_sync();
    if (gate_part(w, d.max_rounds)) break;
    phase_sync();
    // R3 candidate cap
    if (d.K > 0) {
      gather_part(m, w, d.pm, L);
      phase_sync();
      engine_select(w, d.K, lds);
      phase_sync();
      apply_part(w, L);
      phase_sync();
    }
    // R4 locate, optional prefilters
    locate_part(m, w, L);
    phase_sync();
    if (d.f1)
      for (int mode = 0; mode < 3; mode++) {
        prefilter_part(m, w, mode, 0, lds, L);
        phase_sync();
      }
    if (d.approx_n > 0)
      for (int mode = 3; mode < 6; mode++) {
        prefilter_part(m, w, mode, d.approx_n, lds, L);
        phase_sync();
      }
    // R5/R6 cavities with their marks: the circumcenters on one half of the
    // workgroup while the midpoints listed so far (collection and walks) run
    // on the other; then the midpoints the circumcenter cavities flagged.
    // (Marks are order free and a midpoint cavity depends on no other.)
    BigShared &sh = *reinterpret_cast<BigShared *>(lds);
    const Lanes LC{0, kEngCavThreads, 0};
    if (threadIdx.x == 0) s_mid0 = w.cnt->nmk;
    __syncthreads();
    const int mid0 = s_mid0;
    if (threadIdx.x < kEngCavThreads)
      cavity_part(m, w, 1, lds, kEngCavThreads, kEngCap, LC);
    else
      cavity_part(m, w, 0, lds + kEngLdsWords, kEngCavThreads, kEngMidCap, LC, 0, mid0,
                  (int)threadIdx.x - kEngCavThreads);
    phase_sync();
    engine_big(m, w, sh, 0);
    phase_sync();
    if (threadIdx.x < kEngCavThreads) cavity_part(m, w, 0, lds, kEngCavThreads, kEngCap, LC, mid0);
    phase_sync();
    engine_big(m, w, sh, 1);
    phase_sync();
    // R8 ownership, R9 dependency
    own_part(w, L);
    phase_sync();
    dep_part(m, w, L);
    phase_sync();
    // R10 ranks, fresh slots, capacity check, insertion
    const ScanJob js{(const int32_t *)w.win_s, w.rank_s, &w.st->wS, w.tiles_s, &w.cnt->nwin_mid, 1};
    const ScanJob jt{(const int32_t *)w.win_t, w.rank_t, &w.st->wT, w.tiles_t, &w.cnt->nwin_cc, 1};
    const ScanJob jf{w.fcount, w.fbase, &w.cnt->nwin1, w.tiles_f, &w.cnt->fan_total, 0};
    if (!engine_rank(w, lds)) {  // many winners: bitmap ranks as in the grid kernels
      phase_sync();
      engine_scan(js);
      engine_scan(jt);
      phase_sync();
      winners_part(w, L);
    }
    phase_sync();
    engine_scan(jf);
    phase_sync();
    record_part(m, w, L);
    phase_sync();
    write_part(m, w, L);
    phase_sync();
    finish_part(m, w, L);
    phase_sync();
    round_end(w);
  }
}

// Each workgroup takes meshes from a queue (head counts the taken ones) and
// runs each for at most round_limit rounds.
__global__ __launch_bounds__(kEngBlock) void k_engine(const EngDesc *descs, int n_mesh, int32_t *head,
                                                      int round_limit) {
  __shared__ int32_t lds[kEngLdsWords + kEngMidLdsWords];
  __shared__ int s_i;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_i = atomicAdd(head, 1);
    __syncthreads();
    const int i = s_i;
    if (i >= n_mesh) return;
    engine_mesh(descs[i], lds, round_limit);
  }
}

// ---------------------------------------------------------------------------
// Round-boundary batching: the round's phases for a set of meshes, one
// launch each (gridDim.y = meshes).  The bodies are the single-mesh phases;
// each workgroup copies its mesh's descriptor (mesh arrays and the round's
// workspace, chosen by the mesh's own serial) into registers first.
// ---------------------------------------------------------------------------
#define GANG_MESH                                           \
  const GangDesc &g_ = G[blockIdx.y];                       \
  const int par_ = g_.e.w[0].st->serial & 1;                \
  const DevMesh m = g_.e.m;                                 \
  const Work w = g_.e.w[par_];

__global__ void kg_collect(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt) return;
  if (w.st->full) {
    scan_part(m, w, g_.e.B2, g_.e.pm, grid_lanes());
  } else {
    carry_part(w, grid_lanes());
    dirty_part(m, w, g_.e.B2, g_.e.pm, grid_lanes());
  }
}

__global__ void kg_pending(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt || w.st->full) return;
  pending_part(m, w, grid_lanes());
}

__global__ void kg_gate(const GangDesc *G) {
  GANG_MESH
  (void)m;
  (void)gate_part(w, g_.e.max_rounds);
}

__global__ void kg_gather_keys(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt || g_.e.K <= 0) return;
  gather_part(m, w, g_.e.pm, grid_lanes());
}

__global__ void kg_radix_hist(const GangDesc *G, int shift) {
  __shared__ int h[256];
  GANG_MESH
  (void)m;
  if (w.st->halt || g_.e.K <= 0) return;
  const int n = w.cnt->ncc + w.cnt->nmk;
  const uint64_t prefix = w.sel[0], pmask = w.sel[1];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    uint64_t k = w.keys[c];
    if ((k & pmask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&w.rhist[i], h[i]);
}

__global__ void kg_radix_pick(const GangDesc *G, int shift) {
  GANG_MESH
  (void)m;
  if (w.st->halt || g_.e.K <= 0) return;
  radix_pick_part(w, shift, g_.e.K);
}

__global__ void kg_apply_cap(const GangDesc *G) {
  GANG_MESH
  (void)m;
  if (w.st->halt || g_.e.K <= 0) return;
  apply_part(w, grid_lanes());
}

__global__ void kg_locate(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt) return;
  locate_part(m, w, grid_lanes());
}

__global__ __launch_bounds__(kPreBlock) void kg_prefilter(const GangDesc *G, int mode) {
  __shared__ int32_t lds[kApproxMax * kPreBlock];
  GANG_MESH
  if (w.st->halt) return;
  if (mode < 3 ? !g_.e.f1 : g_.e.approx_n <= 0) return;
  prefilter_part(m, w, mode, mode < 3 ? 0 : g_.e.approx_n, lds, grid_lanes());
}

template <int IS_CC>
__global__ __launch_bounds__(kCavBlock, 4) void kg_cavity(const GangDesc *G) {
  __shared__ int32_t lds[kCap * kCavBlock];
  GANG_MESH
  if (w.st->halt) return;
  cavity_part<true>(m, w, IS_CC, lds, kCavBlock, kCap, grid_lanes());
}
template __global__ void kg_cavity<0>(const GangDesc *G);
template __global__ void kg_cavity<1>(const GangDesc *G);

__global__ __launch_bounds__(kBigBlock) void kg_cavity_big(const GangDesc *G, int phase) {
  __shared__ BigShared sh;
  GANG_MESH
  if (w.st->halt) return;
  int nbig = min(w.cnt->nbig, w.big_cap);
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    int ref = w.big[b];
    int is_cc = (ref & 0x80000000) ? 0 : 1;
    if (is_cc != (phase == 0 ? 1 : 0)) continue;
    big_one(m, w, sh, b);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kHugeBlock) void kg_cavity_huge(const GangDesc *G, int phase) {
  __shared__ BigShared sh;
  GANG_MESH
  if (w.st->halt || w.cnt->nhuge == 0) return;
  int nbig = min(w.cnt->nbig, w.big_cap);
  for (int b = 0; b < nbig; b++) {
    int ref = w.big[b];
    int is_cc = (ref & 0x80000000) ? 0 : 1;
    if (is_cc != (phase == 0 ? 1 : 0)) continue;
    huge_one(m, w, sh, b);
  }
}

__global__ void kg_own(const GangDesc *G) {
  GANG_MESH
  (void)m;
  if (w.st->halt) return;
  own_part(w, grid_lanes());
}

__global__ void kg_dep(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt) return;
  dep_part(m, w, grid_lanes());
}

// which = 0: the two winner bitmaps; 1: the fresh-slot counts.
__global__ __launch_bounds__(kScanBlock) void kg_scan_tiles(const GangDesc *G, int which) {
  const GangDesc &g = G[blockIdx.y];
  if (g.e.w[0].st->halt) return;
  const ScanJob a = which == 0 ? g.js : g.jf;
  const ScanJob b = which == 0 ? g.jt : ScanJob{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
  const int na = *a.n_dev, nb = b.in ? *b.n_dev : 0;
  const int ta = (na + kScanTile - 1) / kScanTile, tb = (nb + kScanTile - 1) / kScanTile;
  for (int tile = blockIdx.x; tile < ta + tb; tile += gridDim.x) {
    if (tile < ta) scan_tile(a, na, tile);
    else scan_tile(b, nb, tile - ta);
  }
}

// Launched with gridDim.x = 2 (both jobs of which = 0; one of which = 1).
__global__ __launch_bounds__(kScanBlock) void kg_scan_sums(const GangDesc *G, int which) {
  __shared__ int s_total;
  const GangDesc &g = G[blockIdx.y];
  if (g.e.w[0].st->halt) return;
  if (which == 1 && blockIdx.x != 0) return;
  const ScanJob j = which == 1 ? g.jf : (blockIdx.x == 0 ? g.js : g.jt);
  const int ntiles = (*j.n_dev + kScanTile - 1) / kScanTile;
  int carry = 0;
  for (int start = 0; start < ntiles; start += kScanBlock) {
    int idx = start + threadIdx.x;
    int x = idx < ntiles ? j.tiles[idx] : 0;
    int e = block_excl_scan(x, &s_total);
    if (idx < ntiles) j.tiles[idx] = e + carry;
    carry += s_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *j.total = carry;
}

__global__ void kg_winners(const GangDesc *G) {
  GANG_MESH
  (void)m;
  if (w.st->halt) return;
  winners_part(w, grid_lanes());
}

__global__ void kg_record(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt) return;
  record_part(m, w, grid_lanes());
}

__global__ void kg_write(const GangDesc *G) {
  GANG_MESH
  if (w.st->halt) return;
  write_part(m, w, grid_lanes());
}

__global__ void kg_finish(const GangDesc *G) {
  __shared__ int s_last;
  GANG_MESH
  if (w.st->halt) return;
  finish_part(m, w, grid_lanes());
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&w.st->done_blocks, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (threadIdx.x == 0) w.st->done_blocks = 0;
  round_end(w);
}

__global__ void kg_status(const GangDesc *G, int rounds, int32_t *out, int stride_words) {
  const GangDesc &g = G[blockIdx.y];
  const Work &w = g.e.w[0];
  int32_t *o = out + (size_t)blockIdx.y * stride_words;
  const int ns = (int)(sizeof(DevState) / 4), nc = (int)(sizeof(DevCounters) / 4);
  const int32_t *st = (const int32_t *)w.st, *cn = (const int32_t *)w.cnt, *hi = (const int32_t *)w.hist;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) o[i] = st[i];
  for (int i = threadIdx.x; i < nc; i += blockDim.x) o[ns + i] = cn[i];
  for (int i = threadIdx.x; i < rounds * nc; i += blockDim.x) o[ns + nc + i] = hi[i];
}
#undef GANG_MESH

// ---------------------------------------------------------------------------
// Measurement: 64-bit atomicMax at random slots of a table in device memory,
// the access pattern of the priority marks (random slot, one read-modify-
// write each).  Slot and value of operation i come from a fixed mix of i.
// ---------------------------------------------------------------------------
__global__ void k_atomic_max_bench(uint64_t *table, uint64_t n_slots, int64_t n_ops, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops; i += stride) {
    uint64_t h = (uint64_t)i * 0x9e3779b97f4a7c15ull + seed;
    h ^= h >> 31;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 29;
    atomicMax((unsigned long long *)&table[h % n_slots], (unsigned long long)(h | 1ull));
  }
}

// ---------------------------------------------------------------------------
// Test entry: the predicates above, one thread per query.
// ---------------------------------------------------------------------------
__global__ void k_predicates(int kind, int n, const double *pts, int32_t *out, uint64_t *tally) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int w = kind == 1 ? 8 : 6;
  const double *q = pts + (size_t)i * w;
  int r = 0;
  if (kind == 0) r = orient2d(q[0], q[1], q[2], q[3], q[4], q[5], tally);
  else if (kind == 1) r = incircle(q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], tally);
  else if (kind == 2) r = indiametral(q[0], q[1], q[2], q[3], q[4], q[5], tally);
  else r = encroaches(1, q[0], q[1], q[2], q[3], q[4], q[5], tally) ? 1 : 0;
  out[i] = r;
}

}  // namespace gdp

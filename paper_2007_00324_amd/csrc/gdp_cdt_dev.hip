// gdp_cdt_dev.hip -- Line 1 of Algorithm 1 on the GPU: the constrained
// Delaunay triangulation of the input PSLG built by kernels, so that a mesh
// can go from its PSLG to the refinement loop without the host builder.
//
// The result is the same triangulation as the host builder's, element for
// element: the CDT is unique once cocircular ties are broken by the symbolic
// perturbation of the lifting map with the smaller vertex id dominant, and
// the canonical form (each triangle rotated so its smallest vertex comes
// first, triangles sorted) fixes the slot order.
//
// Stages, all on one stream:
//   1. Delaunay triangulation of the points and a large enclosing triangle by
//      rounds of parallel Bowyer-Watson insertion.  Each pending point walks
//      to the triangle holding it; each triangle elects one point (largest
//      key); an elected point grows its cavity (triangles whose circle holds
//      it) and stamps its key with atomicMax on the cavity and on the ring of
//      triangles across the cavity boundary; a point whose cavity and ring
//      all still carry its key replaces the cavity by its fan.  Disjoint
//      cavity+ring regions make the insertions of one round independent: a
//      point outside another's region is outside every circle of that
//      other's new fan (the fan triangle on a boundary edge has, on the far
//      side of the edge, a circle inside the circle of the ring triangle).
//   2. Segment recovery by rounds: a segment whose edge is missing walks the
//      triangles it crosses and stamps them and their outer neighbours; a
//      segment that keeps every stamp replaces the crossed triangles by the
//      constrained Delaunay triangulations of the two pseudo-polygons on its
//      sides (recursive choice of the apex whose circle holds no other
//      polygon vertex).  Crossed regions of different winners are disjoint,
//      so the result is the one sequential insertion gives.
//   3. Triangles with an enclosing vertex are dropped; every dropped/kept
//      boundary must be a segment, every vertex used, the kept region a
//      convex disk; the survivors are rotated, sorted by (v0, v1) with a
//      radix sort of this file and renumbered into the refinement's mesh
//      layout.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "gdp_internal.h"

namespace gdp {
namespace {

constexpr int kBlk = 256;        // block of the plain kernels
constexpr int kCavBlk = 128;     // block of the cavity kernels
constexpr int kLdsCap = 32;      // cavity triangles per thread kept in LDS
constexpr int kBigSlots = 64;    // cavities above kLdsCap handled per round
constexpr int kBigCap = 16384;   // triangles of one such cavity (a larger one waits, see mark_cavity)
constexpr int kWalkCap = 1 << 20;   // steps of one walk or rotation

enum CdtErr : int {
  kEOk = 0, kEDup, kEWalk, kECavity, kERepeat, kEOnSeg, kECross, kELeave, kEDir, kEHull, kEUnused,
  kEDisk, kEInternal = 100  // + the site that found an inconsistency
};

const char *cdt_err_text(int e) {
  switch (e) {
    case kEDup: return "duplicate point";
    case kEWalk: return "point location failed";
    case kECavity: return "a Delaunay cavity exceeded the device builder's capacity";
    case kERepeat: return "repeated segment";
    case kEOnSeg: return "a vertex lies in the interior of a segment";
    case kECross: return "segments cross";
    case kELeave: return "segment leaves the domain";
    case kEDir: return "segment direction not found";
    case kEHull: return "a convex hull edge is not covered by a segment";
    case kEUnused: return "a convex hull edge is not covered by a segment";
    case kEDisk: return "the kept region is not a disk";
    default: return "device CDT builder: internal error";
  }
}

std::string cdt_err_string(int e) {
  if (e >= kEInternal) return "device CDT builder: internal error at site " + std::to_string(e - kEInternal);
  return cdt_err_text(e);
}

// Round counters, read back after each round.
struct Ctr {
  int npend;   // entries appended to the next pending list
  int nwin;    // insertions this round
  int nbig;    // big cavity slots taken
  int pool;    // ints of the per-round pool taken
  int err;     // first error code
  int nkeep;   // kept triangles (final stage)
  int nhull;   // boundary edges of the kept region
  int first;   // smallest list index of a pending point (rounds with one forced insertion)
};

struct Bld {
  const double2 *P;  // nv + 3 points: the input, then the enclosing triangle
  int nv;
  int4 *tv, *tn, *ts;  // triangle slots: vertices, neighbours, segment id per edge (-1 none)
  int capT;
  int *ntri;
  uint64_t *pick, *mark;  // per slot: elected key, largest cavity stamp (round << 32 | key)
  uint64_t *ring;         // per slot: largest ring stamp of a point cavity
  int *hint, *state;      // per point: last triangle, -2 / -1 (LDS cavity) / big slot
  int *vt;                // per vertex: an incident triangle
  int *big;               // kBigSlots * kBigCap, or the whole area for the one cavity of a solo round
  int big_all;            // ints of the area (>= capT: room for any cavity)
  int *pool;              // per-round scratch
  int pool_cap;
  Ctr *c;
};

__device__ __forceinline__ void set_err(Ctr *c, int e) { atomicCAS(&c->err, 0, e); }

__device__ __forceinline__ int comp(const int4 &v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }
__device__ __forceinline__ int *comp_ptr(int4 *a, int t, int i) { return reinterpret_cast<int *>(a + t) + i; }

// A fixed bijection of 32-bit ids (MurmurHash3 finalizer of id + 1) makes
// the election keys distinct and spread.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  uint32_t h = x + 1u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Pending points take part in a round's election only while a second mix of
// their id is at most the round's threshold: a random sample of about four
// points per triangle while the mesh is coarse, so the early rounds do not
// walk every point.
__device__ __forceinline__ bool sampled(int p, uint32_t thresh) { return mix32((uint32_t)p ^ 0x5bd1e995u) <= thresh; }

__device__ __forceinline__ int orient_ids(const double2 *P, int a, int b, int c) {
  const double2 A = P[a], B = P[b], C = P[c];
  return orient2d(A.x, A.y, B.x, B.y, C.x, C.y);
}

// incircle with the symbolic perturbation of the lifting map (gdp_exact.h)
// on points given by their ids; equal ids (a chain vertex repeated around a
// slit) keep their argument order.
__device__ int incircle_sos(const double2 *P, int a, int b, int c, int d) {
  const double2 A = P[a], B = P[b], C = P[c], D = P[d];
  return gdp::incircle_sos(A.x, A.y, B.x, B.y, C.x, C.y, D.x, D.y, a, b, c, d);
}

__device__ __forceinline__ int eidx(const int4 &v, int u, int w) {
  if (v.x == u && v.y == w) return 0;
  if (v.y == u && v.z == w) return 1;
  if (v.z == u && v.x == w) return 2;
  return -1;
}

__device__ __forceinline__ int vidx(const int4 &v, int a) { return v.x == a ? 0 : (v.y == a ? 1 : (v.z == a ? 2 : -1)); }

// Variable-size allocation by a whole wave: one atomic per wave.
__device__ __forceinline__ int wave_take(int *counter, int n) {
  const int lane = __lane_id();
  int x = n;
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  const int total = __shfl(x, 63);
  int base = 0;
  if (lane == 63 && total > 0) base = atomicAdd(counter, total);
  base = __shfl(base, 63);
  return base + x - n;
}

struct List {
  int *p;
  int stride;
  __device__ __forceinline__ int &operator[](int i) const { return p[(size_t)i * stride]; }
};

// ---------------------------------------------------------------------------
// Stage 1: Delaunay triangulation by parallel Bowyer-Watson rounds
// ---------------------------------------------------------------------------
__global__ void k_init(Bld b, int *pend) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < b.nv; i += stride) {
    pend[i] = i;
    b.hint[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    b.tv[0] = make_int4(b.nv, b.nv + 1, b.nv + 2, 0);
    b.tn[0] = make_int4(-1, -1, -1, 0);
    b.ts[0] = make_int4(-1, -1, -1, 0);
    *b.ntri = 1;
  }
}

// Walks each pending point to its triangle and elects, per triangle, the
// point with the largest key (waves whose lanes share a triangle combine
// their keys before the atomic).
// relocate = 1: the points outside the sample walk too (their start
// triangles are refreshed each time the mesh has doubled) but do not elect.
__global__ void k_locate(Bld b, const int *pend, int np, uint32_t round, int solo, uint32_t thresh, int relocate) {
  const int lane = __lane_id();
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < np; base += stride) {
    const int i = base + threadIdx.x;
    const int p = i < np ? pend[i] : -1;  // -1: an inserted point left in the list
    bool act = p >= 0;
    int t = 0;
    uint64_t key = 0;
    if (solo && act) atomicMin(&b.c->first, i);
    const bool elect = act && sampled(p, thresh);
    if (!elect && !relocate) act = false;
    if (act) {
      t = b.hint[p];
      int from = -1;
      const double2 q = b.P[p];
      int steps = 0;
      for (;;) {
        const int4 v = b.tv[t];
        const int4 n = b.tn[t];
        int moved = -1;
        for (int e = 0; e < 3; e++) {
          const int o = comp(n, e);
          if (o == from && o >= 0) continue;
          const double2 U = b.P[comp(v, e)], W = b.P[comp(v, (e + 1) % 3)];
          if (orient2d(U.x, U.y, W.x, W.y, q.x, q.y) < 0) { moved = e; break; }
        }
        if (moved < 0) {
          const double2 A = b.P[v.x], B = b.P[v.y], C = b.P[v.z];
          if ((A.x == q.x && A.y == q.y) || (B.x == q.x && B.y == q.y) || (C.x == q.x && C.y == q.y)) {
            set_err(b.c, kEDup);
            act = false;
          }
          break;
        }
        const int o = comp(n, moved);
        if (o < 0 || ++steps > kWalkCap) { set_err(b.c, kEWalk); act = false; break; }
        from = t;
        t = o;
      }
      b.hint[p] = t;
      key = ((uint64_t)round << 32) | mix32((uint32_t)p);
      if (!elect) act = false;
    }
    // combine the keys of lanes that share a triangle while such groups are
    // large (early rounds: few triangles, many points each)
    uint64_t left = __ballot(act);
    for (int it = 0; it < 64 && left; it++) {
      const int leader = __ffsll((unsigned long long)left) - 1;
      const int tl = __shfl(t, leader);
      const bool same = act && t == tl;
      const uint64_t m = __ballot(same);
      if (it > 0 && __popcll(m) < 3) break;
      long long best = same ? (long long)key : 0;
      for (int d = 32; d >= 1; d >>= 1) {
        long long o = __shfl_xor(best, d);
        best = (unsigned long long)o > (unsigned long long)best ? o : best;
      }
      if (lane == leader) atomicMax((unsigned long long *)&b.pick[tl], (unsigned long long)best);
      if (same) act = false;
      left &= ~m;
    }
    if (act) atomicMax((unsigned long long *)&b.pick[t], (unsigned long long)key);
  }
}

// Cavity of point p, breadth first from the triangles already in L[0..n)
// (the caller puts the start triangle there and stamps / checks it).
// mode 0: stamp key on the cavity (mark) and on the ring around it (ring);
// a triangle already stamped with key is already listed.  mode 1: rebuild
// the list from the stamps (pick marks the listed triangles), requiring that
// no larger key holds a cavity triangle in its cavity or ring, nor a ring
// triangle in its cavity.  Rings may overlap: a ring triangle only has one
// neighbour pointer per cavity rewritten.  Returns n when done, -1 when the
// list is full (h and n then allow a resume with a larger list), -2 when a
// larger key holds the region.
__device__ int grow(const Bld &b, int p, List L, int cap, uint64_t key, int mode, int &h, int &n) {
  for (; h < n; h++) {
    const int4 nb = b.tn[L[h]];
    for (int e = 0; e < 3; e++) {
      const int o = comp(nb, e);
      if (o < 0) continue;
      if (mode == 1) {
        const uint64_t m = b.mark[o];
        if (m > key) return -2;
        if (m != key) continue;  // ring
        if (b.ring[o] > key) return -2;
        if (b.pick[o] == key) continue;  // listed
        if (n == cap) return -1;
        b.pick[o] = key;
      } else {
        if (b.mark[o] == key) continue;  // listed
        const int4 v = b.tv[o];
        if (incircle_sos(b.P, v.x, v.y, v.z, p) <= 0) {
          atomicMax((unsigned long long *)&b.ring[o], (unsigned long long)key);
          continue;
        }
        if (n == cap) return -1;
        const uint64_t old = atomicMax((unsigned long long *)&b.mark[o], (unsigned long long)key);
        if (old > key) return -2;
        if (old == key) continue;
      }
      L[n++] = o;
    }
  }
  return n;
}

// Stamps the start triangle and grows the cavity of p (mode 0) in L; on a
// full list continues in a large list of the global pool when one is free.
// Returns the state: -1 (cavity in LDS), a big-list slot, or -2 (none).  A
// cavity beyond a big list waits: the point stays pending, its cavity
// shrinks as its neighbourhood fills in, and a round that inserts nothing
// is followed by a solo round whose one point may use the whole area, which
// holds any cavity (the triangles of a cavity are distinct live slots).
__device__ int mark_cavity(const Bld &b, int p, int t0, uint64_t key, List L, int cap, bool big_only) {
  const uint64_t old = atomicMax((unsigned long long *)&b.mark[t0], (unsigned long long)key);
  if (old > key) return -2;
  int h = 0, n = 1;
  if (big_only) {
    const List G{b.big, 1};
    G[0] = t0;
    const int r = grow(b, p, G, b.big_all, key, 0, h, n);
    if (r == -1) set_err(b.c, kEInternal + 3);
    return r > 0 ? 0 : -2;
  }
  L[0] = t0;
  int r = grow(b, p, L, cap, key, 0, h, n);
  if (r > 0) return -1;
  if (r == -2) return -2;
  const int slot = atomicAdd(&b.c->nbig, 1);
  if (slot >= kBigSlots) return -2;
  const List G{b.big + (size_t)slot * kBigCap, 1};
  for (int k = 0; k < n; k++) G[k] = L[k];
  r = grow(b, p, G, kBigCap, key, 0, h, n);
  return r > 0 ? slot : -2;
}

__global__ __launch_bounds__(kCavBlk) void k_mark(Bld b, const int *pend, int np, uint32_t round, int solo,
                                                  uint32_t thresh) {
  __shared__ int s_list[kLdsCap * kCavBlk];
  const List lds{&s_list[threadIdx.x], kCavBlk};
  const int stride = gridDim.x * blockDim.x;
  const int first = solo ? b.c->first : -1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const int p = pend[i];
    if (p < 0) continue;
    const uint64_t key = ((uint64_t)round << 32) | mix32((uint32_t)p);
    const int t0 = b.hint[p];
    int st = -2;
    if (solo) {
      if (i == first) st = mark_cavity(b, p, t0, key, lds, kLdsCap, true);
    } else if (sampled(p, thresh) && b.pick[t0] == key) {
      st = mark_cavity(b, p, t0, key, lds, kLdsCap, false);
    }
    b.state[p] = st;
  }
}

// compact = 1: the points not inserted go to pend_out; compact = 0: the
// list stays and each inserted point leaves -1 in its entry.
__global__ __launch_bounds__(kCavBlk) void k_insert(Bld b, int *pend, int np, uint32_t round, int *pend_out,
                                                    int compact, int solo) {
  __shared__ int s_list[kLdsCap * kCavBlk];
  const List lds{&s_list[threadIdx.x], kCavBlk};
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < np; base += stride) {
    const int i = base + threadIdx.x;
    int p = i < np ? pend[i] : -1;
    const bool act = p >= 0;
    int n = -2;
    List L = lds;
    if (act) {
      const int st = b.state[p];
      if (st != -2) {
        const uint64_t key = ((uint64_t)round << 32) | mix32((uint32_t)p);
        int cap = kLdsCap;
        if (st >= 0) { L = List{b.big + (size_t)st * kBigCap, 1}; cap = solo ? b.big_all : kBigCap; }
        const int t0 = b.hint[p];
        if (b.mark[t0] == key && b.ring[t0] <= key) {
          b.pick[t0] = key;
          L[0] = t0;
          int h = 0, m = 1;
          n = grow(b, p, L, cap, key, 1, h, m);
        }
      }
    }
    const bool win = n > 0;
    const int fresh = wave_take(b.ntri, win ? 2 : 0);
    const int bo = wave_take(&b.c->pool, win ? 4 * (n + 2) : 0);
    if (compact) {
      const int po = wave_take(&b.c->npend, act && !win ? 1 : 0);
      if (act && !win) pend_out[po] = p;
    }
    if (!win) continue;
    if (!compact) pend[i] = -1;
    if (fresh + 2 > b.capT || bo + 4 * (n + 2) > b.pool_cap) { set_err(b.c, kEInternal + 1); continue; }
    int *B = b.pool + bo;
    const uint64_t key = ((uint64_t)round << 32) | mix32((uint32_t)p);
    // the cavity boundary as a cycle: from a boundary edge (u, w), rotate
    // around w inside the cavity to the next boundary edge
    int ft = -1, fe = -1;
    for (int h = 0; h < n && ft < 0; h++) {
      const int4 nbv = b.tn[L[h]];
      for (int e = 0; e < 3; e++) {
        const int o = comp(nbv, e);
        if (o < 0 || b.mark[o] != key) { ft = L[h]; fe = e; break; }
      }
    }
    bool linked = ft >= 0;
    int nb = 0, ct = ft, ce = fe;
    while (linked) {
      if (nb >= n + 2) { linked = false; break; }
      const int4 v = b.tv[ct];
      const int o = comp(b.tn[ct], ce);
      const int u = comp(v, ce), w = comp(v, (ce + 1) % 3);
      const int oe = o >= 0 ? eidx(b.tv[o], w, u) : -1;
      if (o >= 0 && oe < 0) { linked = false; break; }
      B[4 * nb] = u;
      B[4 * nb + 1] = w;
      B[4 * nb + 2] = o;
      B[4 * nb + 3] = oe;
      nb++;
      int t2 = ct, e2 = (ce + 1) % 3;
      for (int guard = 0;; guard++) {
        const int n2 = comp(b.tn[t2], e2);
        if (n2 < 0 || b.mark[n2] != key) break;
        const int k = vidx(b.tv[n2], w);
        if (k < 0 || guard > n) { linked = false; break; }
        t2 = n2;
        e2 = k;
      }
      ct = t2;
      ce = e2;
      if (ct == ft && ce == fe) break;
    }
    linked = linked && nb == n + 2;
    if (!linked) { set_err(b.c, kEInternal + 2); continue; }
    atomicAdd(&b.c->nwin, 1);
    for (int j = 0; j < nb; j++) {
      const int u = B[4 * j], w = B[4 * j + 1], o = B[4 * j + 2], oe = B[4 * j + 3];
      const int jn = j + 1 == nb ? 0 : j + 1, jp = j == 0 ? nb - 1 : j - 1;
      const int s = j < n ? L[j] : fresh + (j - n);
      const int sn = jn < n ? L[jn] : fresh + (jn - n);
      const int sp = jp < n ? L[jp] : fresh + (jp - n);
      b.tv[s] = make_int4(u, w, p, 0);
      b.tn[s] = make_int4(o, sn, sp, 0);
      b.ts[s] = make_int4(-1, -1, -1, 0);
      if (o >= 0) *comp_ptr(b.tn, o, oe) = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Stage 2: segment recovery
// ---------------------------------------------------------------------------
__global__ void k_vt(Bld b, int nt) {
  const int stride = gridDim.x * blockDim.x;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
    const int4 v = b.tv[t];
    b.vt[v.x] = t;
    b.vt[v.y] = t;
    b.vt[v.z] = t;
  }
}

// Around vertex a: the edge a-b (returns 1 with t, i of edge a->b or b->a),
// else the triangle whose wedge at a holds the direction to b (returns 0,
// t = that triangle), else an error code < 0.
__device__ int around(const Bld &b, int a, int bb, int &tout, int &iout) {
  const int start = b.vt[a];
  int cur = start, found = -1, onseg = 0;
  const double2 A = b.P[a], Bp = b.P[bb];
  for (int guard = 0; guard < kWalkCap; guard++) {
    const int4 v = b.tv[cur];
    const int k = vidx(v, a);
    if (k < 0) return -(kEInternal + 3);
    const int u = comp(v, (k + 1) % 3), w = comp(v, (k + 2) % 3);
    if (u == bb) { tout = cur; iout = k; return 1; }
    if (w == bb) { tout = cur; iout = (k + 2) % 3; return 1; }
    if (found < 0) {
      const double2 U = b.P[u], W = b.P[w];
      const int ou = orient2d(A.x, A.y, U.x, U.y, Bp.x, Bp.y);
      const int ow = orient2d(A.x, A.y, W.x, W.y, Bp.x, Bp.y);
      if (ou == 0 && (U.x - A.x) * (Bp.x - A.x) + (U.y - A.y) * (Bp.y - A.y) > 0) onseg = 1;
      if (ou > 0 && ow < 0) found = cur;
    }
    const int nx = comp(b.tn[cur], (k + 2) % 3);
    if (nx < 0) return -(kEInternal + 4);
    if (nx == start) break;
    cur = nx;
  }
  if (found < 0) return onseg ? -kEOnSeg : -kEDir;
  tout = found;
  return 0;
}

// Outputs of one walk along segment a->b from the triangle at a.
struct WalkOut {
  int *crossed;        // k
  int *lc, *lo, *lcn;  // left chain L_1..L_m; out tri / segment id of edge L_{i+1}->L_i (m + 1)
  int *rc, *ro, *rcn;  // right chain R_1..R_n; out of edge R_i->R_{i+1} (n + 1)
};

// Walks the triangles crossed by a->b.  mode 0: stamp the crossed triangles
// and their outer neighbours; mode 1: require the stamp before reading a
// triangle; mode 2: as mode 1 and fill w.  Returns the number of crossed
// triangles, or -2 for a foreign stamp, or -(error code + 16).
__device__ int seg_walk(const Bld &b, int a, int bb, int t0, uint64_t key, int mode, const WalkOut &w,
                        int &m_out, int &n_out) {
  auto stamp = [&](int t) -> bool {
    if (t < 0) return true;
    if (mode == 0) { atomicMax((unsigned long long *)&b.mark[t], (unsigned long long)key); return true; }
    return b.mark[t] == key;
  };
  if (!stamp(t0)) return -2;
  int4 v = b.tv[t0];
  int4 nb = b.tn[t0];
  int4 sg = b.ts[t0];
  const int k0 = vidx(v, a);
  if (k0 < 0) return -(kEInternal + 5 + 16);
  int R = comp(v, (k0 + 1) % 3), L = comp(v, (k0 + 2) % 3);
  int m = 0, n = 0, kc = 0;
  {
    const int ol = comp(nb, (k0 + 2) % 3), orr = comp(nb, k0);
    if (!stamp(ol) || !stamp(orr)) return -2;
    if (mode == 2) {
      w.lo[0] = ol; w.lcn[0] = comp(sg, (k0 + 2) % 3);
      w.ro[0] = orr; w.rcn[0] = comp(sg, k0);
      w.lc[0] = L; w.rc[0] = R;
      w.crossed[0] = t0;
    }
    m = 1; n = 1; kc = 1;
  }
  int cur = t0;
  const double2 A = b.P[a], Bp = b.P[bb];
  for (int guard = 0;; guard++) {
    if (guard > kWalkCap) return -(kEInternal + 6 + 16);
    const int e = eidx(v, R, L);
    if (e < 0) return -(kEInternal + 7 + 16);
    if (comp(sg, e) >= 0) return -(kECross + 16);
    const int nx = comp(nb, e);
    if (nx < 0) return -(kELeave + 16);
    if (!stamp(nx)) return -2;
    v = b.tv[nx];
    nb = b.tn[nx];
    sg = b.ts[nx];
    const int j = eidx(v, L, R);
    if (j < 0) return -(kEInternal + 8 + 16);
    const int wv = comp(v, (j + 2) % 3);
    if (mode == 2) w.crossed[kc] = nx;
    kc++;
    if (wv == bb) {
      const int orr = comp(nb, (j + 1) % 3), ol = comp(nb, (j + 2) % 3);
      if (!stamp(orr) || !stamp(ol)) return -2;
      if (mode == 2) {
        w.ro[n] = orr; w.rcn[n] = comp(sg, (j + 1) % 3);
        w.lo[m] = ol; w.lcn[m] = comp(sg, (j + 2) % 3);
      }
      break;
    }
    const double2 W = b.P[wv];
    const int o = orient2d(A.x, A.y, Bp.x, Bp.y, W.x, W.y);
    if (o == 0) return -(kEOnSeg + 16);
    if (o > 0) {
      const int ol = comp(nb, (j + 2) % 3);
      if (!stamp(ol)) return -2;
      if (mode == 2) { w.lo[m] = ol; w.lcn[m] = comp(sg, (j + 2) % 3); w.lc[m] = wv; }
      m++;
      L = wv;
    } else {
      const int orr = comp(nb, (j + 1) % 3);
      if (!stamp(orr)) return -2;
      if (mode == 2) { w.ro[n] = orr; w.rcn[n] = comp(sg, (j + 1) % 3); w.rc[n] = wv; }
      n++;
      R = wv;
    }
    cur = nx;
  }
  (void)cur;
  m_out = m;
  n_out = n;
  return kc;
}

__global__ void k_seg_mark(Bld b, const int2 *seg, const int *list, int nl, uint32_t round, int *sstart) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += stride) {
    const int s = list[i];
    const int2 ab = seg[s];
    int t = -1, e = -1;
    const int r = around(b, ab.x, ab.y, t, e);
    if (r < 0) { set_err(b.c, -r); sstart[s] = -1; continue; }
    if (r == 1) {
      // the edge is there: constrain both sides
      const int o = comp(b.tn[t], e);
      const int prev = atomicCAS(comp_ptr(b.ts, t, e), -1, s);
      if (prev != -1 && prev != s) set_err(b.c, kERepeat);
      if (o >= 0) {
        const int4 vt = b.tv[t];
        const int oe = eidx(b.tv[o], comp(vt, (e + 1) % 3), comp(vt, e));
        if (oe < 0) { set_err(b.c, kEInternal + 9); sstart[s] = -1; continue; }
        const int p2 = atomicCAS(comp_ptr(b.ts, o, oe), -1, s);
        if (p2 != -1 && p2 != s) set_err(b.c, kERepeat);
      }
      sstart[s] = -1;
      continue;
    }
    const uint64_t key = ((uint64_t)round << 32) | mix32((uint32_t)s);
    int m, n;
    const int kc = seg_walk(b, ab.x, ab.y, t, key, 0, WalkOut{}, m, n);
    if (kc < -2) { set_err(b.c, -kc - 16); sstart[s] = -1; continue; }
    sstart[s] = t;
  }
}

// Constrained Delaunay triangulation of the pseudo-polygon with base p->q
// and chain c[0..m) (from the p side to the q side, left of p->q); out[i] is
// the outer triangle / segment id across the polygon edge E[i+1]->E[i] of
// E = (p, c_0, .., c_{m-1}, q).  New triangles take the slots slot[*next..].
// Returns the slot of the triangle on the base.
__device__ int tri_poly(const Bld &b, int p, int q, const int *c, int m, const int *out, const int *outcn,
                        const int *slot, int &next, int *stk) {
  auto E = [&](int i) { return i == 0 ? p : (i == m + 1 ? q : c[i - 1]); };
  auto link_out = [&](int s, int ei, int x, int y, int oi) {
    // edge ei of s runs x->y; the outer triangle sees it as y->x
    const int o = out[oi];  // -2: a slit edge, linked inside the region afterwards
    *comp_ptr(b.tn, s, ei) = o;
    *comp_ptr(b.ts, s, ei) = outcn[oi];
    if (o >= 0) {
      const int oe = eidx(b.tv[o], y, x);
      if (oe >= 0) *comp_ptr(b.tn, o, oe) = s;
      else set_err(b.c, kEInternal + 10);
    }
  };
  int sp = 0, root = -1;
  stk[0] = 0; stk[1] = m; stk[2] = -1; stk[3] = 0;
  sp = 1;
  while (sp > 0) {
    sp--;
    const int lo = stk[4 * sp], hi = stk[4 * sp + 1], ps = stk[4 * sp + 2], pe = stk[4 * sp + 3];
    const int u = E(lo), w = E(hi + 1);
    int best = lo;
    for (int k = lo + 1; k < hi; k++)
      if (incircle_sos(b.P, u, w, c[best], c[k]) > 0) best = k;
    const int cb = c[best];
    const int s = slot[next++];
    b.tv[s] = make_int4(u, w, cb, 0);
    b.tn[s] = make_int4(ps, -1, -1, 0);
    b.ts[s] = make_int4(-1, -1, -1, 0);
    if (ps >= 0) *comp_ptr(b.tn, ps, pe) = s;
    else root = s;
    b.vt[u] = s; b.vt[w] = s; b.vt[cb] = s;
    // edge 1: w -> cb; the sub-polygon (best + 1, hi) or the polygon edge E[hi+1] -> E[hi]
    if (best + 1 < hi) { stk[4 * sp] = best + 1; stk[4 * sp + 1] = hi; stk[4 * sp + 2] = s; stk[4 * sp + 3] = 1; sp++; }
    else link_out(s, 1, w, cb, hi);
    // edge 2: cb -> u; the sub-polygon (lo, best) or the polygon edge E[lo+1] -> E[lo]
    if (best > lo) { stk[4 * sp] = lo; stk[4 * sp + 1] = best; stk[4 * sp + 2] = s; stk[4 * sp + 3] = 2; sp++; }
    else link_out(s, 2, cb, u, lo);
  }
  return root;
}

__global__ void k_seg_insert(Bld b, const int2 *seg, const int *list, int nl, uint32_t round, const int *sstart,
                             int *list_out) {
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < nl; base += stride) {
    const int i = base + threadIdx.x;
    bool act = i < nl;
    int s = -1, kc = -2, m = 0, n = 0, t0 = -1;
    int2 ab = make_int2(0, 0);
    uint64_t key = 0;
    if (act) {
      s = list[i];
      t0 = sstart[s];
      if (t0 < 0) act = false;  // constrained in place (or failed)
    }
    if (act) {
      ab = seg[s];
      key = ((uint64_t)round << 32) | mix32((uint32_t)s);
      kc = seg_walk(b, ab.x, ab.y, t0, key, 1, WalkOut{}, m, n);
      if (kc < -2) { set_err(b.c, -kc - 16); act = false; }
    }
    const bool win = act && kc > 0;
    const int need = win ? kc + 3 * (m + 1) + 3 * (n + 1) + 4 * (kc + 2) + (m + n + 2) : 0;
    const int po = wave_take(&b.c->pool, need);
    const int lo = wave_take(&b.c->npend, act && !win ? 1 : 0);
    if (act && !win) list_out[lo] = s;
    if (!win) continue;
    if (po + need > b.pool_cap) { set_err(b.c, kEInternal + 11); continue; }
    int *q = b.pool + po;
    WalkOut w;
    w.crossed = q; q += kc;
    w.lc = q; q += m + 1;
    w.lo = q; q += m + 1;
    w.lcn = q; q += m + 1;
    w.rc = q; q += n + 1;
    w.ro = q; q += n + 1;
    w.rcn = q; q += n + 1;
    int *stk = q; q += 4 * (kc + 2);
    int *rev = q;  // right chain reversed, then its outs reversed
    int m2, n2;
    if (seg_walk(b, ab.x, ab.y, t0, key, 2, w, m2, n2) != kc || m2 != m || n2 != n) { set_err(b.c, kEInternal + 12); continue; }
    // Where the crossed region wraps around a vertex, an edge of a chain has
    // crossed triangles on both sides (a slit): it stays an edge of the new
    // triangulation, linked between the two new triangles that carry it.
    int nslit = 0;
    for (int k = 0; k <= m + n + 1; k++) {
      int *op = k <= m ? &w.lo[k] : &w.ro[k - m - 1];
      if (*op < 0) continue;
      for (int x = 0; x < kc; x++)
        if (w.crossed[x] == *op) { *op = -2; nslit++; break; }
    }
    atomicAdd(&b.c->nwin, 1);
    int next = 0;
    const int rl = tri_poly(b, ab.x, ab.y, w.lc, m, w.lo, w.lcn, w.crossed, next, stk);
    // right side: base b->a, chain R_n..R_1, out[i] = edge R_{n-i} -> R_{n+1-i}
    for (int k = 0; k < n; k++) rev[k] = w.rc[n - 1 - k];
    for (int k = 0; k <= n / 2; k++) {
      const int x = n - k;
      int t1 = w.ro[k]; w.ro[k] = w.ro[x]; w.ro[x] = t1;
      int t2 = w.rcn[k]; w.rcn[k] = w.rcn[x]; w.rcn[x] = t2;
    }
    const int rr = tri_poly(b, ab.y, ab.x, rev, n, w.ro, w.rcn, w.crossed, next, stk);
    if (next != kc) { set_err(b.c, kEInternal + 13); continue; }
    *comp_ptr(b.tn, rl, 0) = rr;
    *comp_ptr(b.tn, rr, 0) = rl;
    *comp_ptr(b.ts, rl, 0) = s;
    *comp_ptr(b.ts, rr, 0) = s;
    for (int x = 0; x < kc && nslit > 0; x++) {
      const int t = w.crossed[x];
      const int4 tv = b.tv[t];
      for (int e = 0; e < 3; e++) {
        if (*comp_ptr(b.tn, t, e) != -2) continue;
        const int u = comp(tv, e), v = comp(tv, (e + 1) % 3);
        int found = -1;
        for (int y = 0; y < kc && found < 0; y++) {
          const int ye = eidx(b.tv[w.crossed[y]], v, u);
          if (ye >= 0) { found = y; *comp_ptr(b.tn, w.crossed[y], ye) = t; }
        }
        if (found < 0) { set_err(b.c, kEInternal + 15); continue; }
        *comp_ptr(b.tn, t, e) = w.crossed[found];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stage 3: outside removal, checks, canonical order
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_out(const Bld &b, int t) {
  if (t < 0) return true;
  const int4 v = b.tv[t];
  return v.x >= b.nv || v.y >= b.nv || v.z >= b.nv;
}

__global__ void k_keep(Bld b, int nt, int *used, uint64_t *keys, int *vals) {
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < nt; base += stride) {
    const int t = base + threadIdx.x;
    bool keep = false;
    int hull = 0;
    uint64_t key = 0;
    if (t < nt && !is_out(b, t)) {
      keep = true;
      const int4 v = b.tv[t], n = b.tn[t], sg = b.ts[t];
      used[v.x] = 1; used[v.y] = 1; used[v.z] = 1;
      for (int e = 0; e < 3; e++) {
        if (!is_out(b, comp(n, e))) continue;
        hull++;
        if (comp(sg, e) < 0) { set_err(b.c, kEHull); continue; }
        // the boundary must turn left at its end vertex
        const int u = comp(v, e), x = comp(v, (e + 1) % 3);
        int cur = t, ce = (e + 1) % 3;
        for (int guard = 0; guard < kWalkCap; guard++) {
          const int o = comp(b.tn[cur], ce);
          if (is_out(b, o)) break;
          cur = o;
          ce = vidx(b.tv[o], x);
          if (ce < 0) { set_err(b.c, kEInternal + 14); ce = 0; break; }
        }
        const int y = comp(b.tv[cur], (ce + 1) % 3);
        if (orient_ids(b.P, u, x, y) < 0) set_err(b.c, kEDisk);
      }
      const int r = (v.y < v.x && v.y < v.z) ? 1 : ((v.z < v.x && v.z < v.y) ? 2 : 0);
      key = ((uint64_t)(uint32_t)comp(v, r) << 32) | (uint32_t)comp(v, (r + 1) % 3);
    }
    const int slot = wave_take(&b.c->nkeep, keep ? 1 : 0);
    const int hsum = wave_take(&b.c->nhull, hull);
    (void)hsum;
    if (keep) { keys[slot] = key; vals[slot] = t; }
  }
}

__global__ void k_used(Bld b, const int *used) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < b.nv; i += stride)
    if (!used[i]) set_err(b.c, kEUnused);
}

__global__ void k_newid(int nk, const int *vals, int *newid) {
  const int stride = gridDim.x * blockDim.x;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += stride) newid[vals[k]] = k;
}

__global__ void k_emit(Bld b, int nk, const int *vals, const int *newid, int4 *otv, int4 *otn, int4 *ots) {
  const int stride = gridDim.x * blockDim.x;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += stride) {
    const int t = vals[k];
    const int4 v = b.tv[t], n = b.tn[t], sg = b.ts[t];
    const int r = (v.y < v.x && v.y < v.z) ? 1 : ((v.z < v.x && v.z < v.y) ? 2 : 0);
    int vv[3], nn[3], ss[3];
    for (int i = 0; i < 3; i++) {
      const int src = (r + i) % 3;
      vv[i] = comp(v, src);
      const int o = comp(n, src);
      nn[i] = is_out(b, o) ? -1 : newid[o];
      ss[i] = comp(sg, src);
    }
    const int mask = (ss[0] >= 0 ? 1 : 0) | (ss[1] >= 0 ? 2 : 0) | (ss[2] >= 0 ? 4 : 0);
    otv[k] = make_int4(vv[0], vv[1], vv[2], mask);
    otn[k] = make_int4(nn[0], nn[1], nn[2], 0);
    ots[k] = make_int4(ss[0], ss[1], ss[2], 0);
  }
}

// ---------------------------------------------------------------------------
// Canonical order: least-significant-digit radix sort of (key, value) pairs
// by 8-bit digits, one stable counting pass per digit that varies:
//   1. tile histograms (a tile is kSortThreads x kSortItems keys), written
//      digit-major, so that
//   2. one exclusive scan gives every (digit, tile) its output offset;
//   3. each tile scatters its keys in their input order: items are taken
//      kSortThreads at a time; inside a wave, lanes with the same digit find
//      each other by eight ballots (one per digit bit) and rank themselves by
//      the lanes below; the waves' digit counts, taken in wave order, and the
//      running count of the tile's earlier items complete the rank.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / 64;

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint64_t *keys, int n, int shift, int ntiles,
                                                            int *hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; j++) {
    const int i = base + j * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1);
  }
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of hist[0..m) in place by one workgroup of kSortScanThreads:
// each thread sums a contiguous chunk, the chunk sums are scanned in LDS, then
// each thread rewrites its chunk.
constexpr int kSortScanThreads = 1024;
__global__ __launch_bounds__(kSortScanThreads) void k_sort_scan(int *hist, int m) {
  __shared__ int part[kSortScanThreads];
  const int chunk = (m + kSortScanThreads - 1) / kSortScanThreads;
  const int lo = threadIdx.x * chunk, hi = min(m, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; i++) s += hist[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < kSortScanThreads; i++) {
      const int x = part[i];
      part[i] = run;
      run += x;
    }
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int i = lo; i < hi; i++) {
    const int x = hist[i];
    hist[i] = run;
    run += x;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t *keys, const int *vals,
                                                               uint64_t *keys_out, int *vals_out, int n, int shift,
                                                               int ntiles, const int *offs) {
  __shared__ int run[256];       // items of the tile ranked so far, per digit
  __shared__ int wcnt[kSortWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  run[threadIdx.x] = offs[threadIdx.x * ntiles + blockIdx.x];
  for (int w = 0; w < kSortWaves; w++) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int j = 0; j < kSortItems; j++) {
    const int i = base + j * kSortThreads + threadIdx.x;
    const bool act = i < n;
    const uint64_t k = act ? keys[i] : 0ull;
    const int v = act ? vals[i] : 0;
    const int d = (int)((k >> shift) & 0xff);
    uint64_t peers = __ballot(act);
    for (int bit = 0; bit < 8; bit++) {
      const uint64_t m = __ballot((d >> bit) & 1);
      peers &= ((d >> bit) & 1) ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (act && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (act) {
      int pos = run[d] + rank;
      for (int w = 0; w < wave; w++) pos += wcnt[w][d];
      keys_out[pos] = k;
      vals_out[pos] = v;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < kSortWaves; w++) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

// Sorts n pairs by key bits [0, 32 + vbits) and [32, 32 + vbits) (a key is
// (a << 32) | b with a, b < 2^vbits); the result ends in (k1, v1).  hist
// holds 256 * ceil(n / kSortTile) ints.
hipError_t radix_sort_pairs(hipStream_t stream, uint64_t *k0, int *v0, uint64_t *k1, int *v1, int n, int vbits,
                            int *hist) {
  if (n <= 0) return hipSuccess;
  const int ntiles = (n + kSortTile - 1) / kSortTile;
  int shifts[16], ns = 0;
  for (int half = 0; half < 2; half++)
    for (int b = 0; b < vbits; b += 8) shifts[ns++] = 32 * half + b;
  uint64_t *kin = k0, *kout = k1;
  int *vin = v0, *vout = v1;
  for (int p = 0; p < ns; p++) {
    k_sort_hist<<<ntiles, kSortThreads, 0, stream>>>(kin, n, shifts[p], ntiles, hist);
    k_sort_scan<<<1, kSortScanThreads, 0, stream>>>(hist, 256 * ntiles);
    k_sort_scatter<<<ntiles, kSortThreads, 0, stream>>>(kin, vin, kout, vout, n, shifts[p], ntiles, hist);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  // after an odd number of passes the result is in (k1, v1); else copy it there
  if (kin != k1) {
    hipError_t e = hipMemcpyAsync(k1, kin, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(v1, vin, sizeof(int) * n, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

__global__ void k_iota(int n, int *a) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = i;
}

int grid_for(int n, int blk) { return std::max(1, std::min((n + blk - 1) / blk, 4096)); }

}  // namespace

// Sorts n (64-bit key, int) pairs by the whole key (8 digit passes); the
// result ends in (k1, v1).  hist holds 256 * ceil(n / 2048) ints.
static_assert(kSortPairsTile == kSortTile, "the sort's tile as declared in gdp_internal.h");
hipError_t sort_pairs_u64(hipStream_t stream, uint64_t *k0, int *v0, uint64_t *k1, int *v1, int n, int *hist) {
  return radix_sort_pairs(stream, k0, v0, k1, v1, n, 32, hist);
}

// Builds the CDT of the PSLG whose vertices (nv, the first nv entries of
// d_xy, which has room for nv + 3) and segments (d_seg) are on the device;
// writes the canonical triangles to otv / otn / ots (capacity cap_out) and
// their count to *n_tri.  Coordinates and segment endpoints are checked by
// the caller.  Returns GDP_OK, GDP_E_INPUT (invalid PSLG, err set),
// GDP_E_NOMEM or GDP_E_DEVICE.
void dev_cdt_work_free(DevCdtWork &ws) {
  if (ws.mem) (void)hipFree(ws.mem);
  if (ws.hctr) (void)hipHostFree(ws.hctr);
  ws = DevCdtWork();
}

int dev_cdt_build(hipStream_t stream, int32_t nv, double2 *d_xy, int32_t ns, const int2 *d_seg, int4 *otv,
                  int4 *otn, int4 *ots, int32_t cap_out, int32_t *n_tri, DevCdtStats *stats, std::string &err,
                  DevCdtWork *ws) {
  if (nv < 3) { err = "bad arguments"; return GDP_E_ARG; }
  // enclosing triangle, as the host builder places it
  std::vector<double2> hxy(nv);
  if (hipMemcpyAsync(hxy.data(), d_xy, sizeof(double2) * nv, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) { err = "copy failed"; return GDP_E_DEVICE; }
  double mx = 1.0;
  for (int i = 0; i < nv; i++) mx = std::max(mx, std::max(std::fabs(hxy[i].x), std::fabs(hxy[i].y)));
  const double Lb = std::exp2(std::ceil(std::log2(mx)) + 1.0);
  const double2 enc[3] = {make_double2(-4 * Lb, -4 * Lb), make_double2(8 * Lb, -4 * Lb), make_double2(-4 * Lb, 8 * Lb)};
  const int capT = 2 * nv + 8;
  const int pool_cap = std::max(16 * capT + 4096, 8 * (kBigCap + 8));
  void *mem = nullptr;
  // layout
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
  const size_t o_tv = take(sizeof(int4) * capT), o_tn = take(sizeof(int4) * capT), o_ts = take(sizeof(int4) * capT);
  const size_t o_pick = take(8 * (size_t)capT), o_mark = take(8 * (size_t)capT), o_ring = take(8 * (size_t)capT);
  const size_t o_hint = take(4 * (size_t)nv), o_state = take(4 * (size_t)std::max(nv, ns));
  const int big_all = std::max(kBigSlots * kBigCap, capT);
  const size_t o_vt = take(4 * (size_t)(nv + 3)), o_big = take(4 * (size_t)big_all);
  const size_t o_pool = take(4 * (size_t)pool_cap);
  const size_t o_p0 = take(4 * (size_t)std::max(nv, ns)), o_p1 = take(4 * (size_t)std::max(nv, ns));
  const size_t o_ctr = take(sizeof(Ctr)), o_ntri = take(4), o_used = take(4 * (size_t)nv);
  const size_t o_keys = take(8 * (size_t)capT), o_keys2 = take(8 * (size_t)capT);
  const size_t o_vals = take(4 * (size_t)capT), o_vals2 = take(4 * (size_t)capT), o_newid = take(4 * (size_t)capT);
  const size_t o_sort = take(4 * 256 * (size_t)((capT + kSortTile - 1) / kSortTile));
  Ctr *hctr = nullptr;
  if (ws) {
    // every earlier build on the workspace has finished (each one ends with
    // a stream synchronisation), so its scratch can be replaced
    if (ws->bytes < off) {
      if (ws->mem) (void)hipFree(ws->mem);
      ws->mem = nullptr;
      ws->bytes = 0;
      if (hipMalloc(&ws->mem, off) != hipSuccess) { ws->mem = nullptr; err = "device allocation failed"; return GDP_E_NOMEM; }
      ws->bytes = off;
    }
    if (!ws->hctr && hipHostMalloc(&ws->hctr, sizeof(Ctr)) != hipSuccess) { ws->hctr = nullptr; err = "host allocation failed"; return GDP_E_NOMEM; }
    mem = ws->mem;
    hctr = (Ctr *)ws->hctr;
  } else {
    if (hipMalloc(&mem, off) != hipSuccess) { err = "device allocation failed"; return GDP_E_NOMEM; }
    if (hipHostMalloc((void **)&hctr, sizeof(Ctr)) != hipSuccess) { (void)hipFree(mem); err = "host allocation failed"; return GDP_E_NOMEM; }
  }
  char *base = (char *)mem;
  auto done = [&](int rc) {
    (void)hipStreamSynchronize(stream);
    if (!ws) {
      (void)hipFree(mem);
      (void)hipHostFree(hctr);
    }
    return rc;
  };
  Bld b;
  b.P = d_xy;
  b.nv = nv;
  b.tv = (int4 *)(base + o_tv); b.tn = (int4 *)(base + o_tn); b.ts = (int4 *)(base + o_ts);
  b.capT = capT;
  b.ntri = (int *)(base + o_ntri);
  b.pick = (uint64_t *)(base + o_pick); b.mark = (uint64_t *)(base + o_mark); b.ring = (uint64_t *)(base + o_ring);
  b.hint = (int *)(base + o_hint); b.state = (int *)(base + o_state);
  b.vt = (int *)(base + o_vt); b.big = (int *)(base + o_big);
  b.big_all = big_all;
  b.pool = (int *)(base + o_pool); b.pool_cap = pool_cap;
  b.c = (Ctr *)(base + o_ctr);
  int *pl[2] = {(int *)(base + o_p0), (int *)(base + o_p1)};
  if (hipMemcpyAsync(d_xy + nv, enc, sizeof(enc), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemsetAsync(b.pick, 0, 8 * (size_t)capT, stream) != hipSuccess ||
      hipMemsetAsync(b.mark, 0, 8 * (size_t)capT, stream) != hipSuccess ||
      hipMemsetAsync(b.ring, 0, 8 * (size_t)capT, stream) != hipSuccess ||
      hipMemsetAsync(b.c, 0, sizeof(Ctr), stream) != hipSuccess)
    { err = "device call failed"; return done(GDP_E_DEVICE); }
  k_init<<<grid_for(nv, kBlk), kBlk, 0, stream>>>(b, pl[0]);
  auto round_trip = [&]() -> bool {
    if (hipMemcpyAsync(hctr, b.c, sizeof(Ctr), hipMemcpyDeviceToHost, stream) != hipSuccess) return false;
    return hipStreamSynchronize(stream) == hipSuccess;
  };
  uint32_t round = 0;
  // np: points still to insert; nl: entries of the pending list (inserted
  // points stay in it as -1 until more than an eighth of it is stale)
  int np = nv, nl = nv, cur = 0, solo = 0, dt_rounds = 0, seg_rounds = 0;
  int64_t t_reloc = 1;  // triangles at the last refresh of every start triangle
  while (np > 0) {
    round++;
    dt_rounds++;
    const int compact = (nl - np) * 8 >= nl;
    const int64_t ntri = 1 + 2 * (int64_t)(nv - np);
    const double frac = solo ? 1.0 : 4.0 * (double)ntri / (double)np;
    const uint32_t thresh = frac >= 1.0 ? 0xffffffffu : (uint32_t)(frac * 4294967296.0);
    int relocate = 0;
    if (thresh != 0xffffffffu && ntri >= 2 * t_reloc) { relocate = 1; t_reloc = ntri; }
    if (hipMemsetAsync(b.c, 0, 4 * sizeof(int), stream) != hipSuccess ||
        hipMemsetAsync(&b.c->first, 0x7f, sizeof(int), stream) != hipSuccess) { err = "device call failed"; return done(GDP_E_DEVICE); }
    k_locate<<<grid_for(nl, kBlk), kBlk, 0, stream>>>(b, pl[cur], nl, round, solo, thresh, relocate);
    k_mark<<<grid_for(nl, kCavBlk), kCavBlk, 0, stream>>>(b, pl[cur], nl, round, solo, thresh);
    k_insert<<<grid_for(nl, kCavBlk), kCavBlk, 0, stream>>>(b, pl[cur], nl, round, pl[cur ^ 1], compact, solo);
    if (!round_trip()) { err = "device call failed"; return done(GDP_E_DEVICE); }
    if (hctr->err) { err = std::string("points (round " + std::to_string(dt_rounds) + "): ") + cdt_err_string(hctr->err); return done(hctr->err == kECavity ? GDP_E_CAVITY : (hctr->err >= kEInternal ? GDP_E_DEVICE : GDP_E_INPUT)); }
    if (compact && hctr->npend != np - hctr->nwin) { err = "device CDT builder: lost points"; return done(GDP_E_DEVICE); }
    if (solo && hctr->nwin == 0) { err = "device CDT builder: no insertion progress"; return done(GDP_E_DEVICE); }
    solo = hctr->nwin == 0;
    np -= hctr->nwin;
    if (compact) {
      nl = np;
      cur ^= 1;
    }
  }
  int nt = 0;
  if (hipMemcpyAsync(&nt, b.ntri, 4, hipMemcpyDeviceToHost, stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
    { err = "device call failed"; return done(GDP_E_DEVICE); }
  if (nt != 2 * nv + 1) { err = "device CDT builder: triangle count"; return done(GDP_E_DEVICE); }
  // segments
  k_vt<<<grid_for(nt, kBlk), kBlk, 0, stream>>>(b, nt);
  int *sstart = b.state;
  nl = ns;
  cur = 0;
  if (ns > 0) k_iota<<<grid_for(ns, kBlk), kBlk, 0, stream>>>(ns, pl[0]);
  while (nl > 0) {
    round++;
    seg_rounds++;
    if (hipMemsetAsync(b.c, 0, 4 * sizeof(int), stream) != hipSuccess) { err = "device call failed"; return done(GDP_E_DEVICE); }
    k_seg_mark<<<grid_for(nl, kBlk), kBlk, 0, stream>>>(b, d_seg, pl[cur], nl, round, sstart);
    k_seg_insert<<<grid_for(nl, kBlk), kBlk, 0, stream>>>(b, d_seg, pl[cur], nl, round, sstart, pl[cur ^ 1]);
    if (!round_trip()) { err = "device call failed"; return done(GDP_E_DEVICE); }
    if (hctr->err) { err = std::string("segments (round " + std::to_string(seg_rounds) + "): ") + cdt_err_string(hctr->err); return done(hctr->err >= kEInternal ? GDP_E_DEVICE : GDP_E_INPUT); }
    if (hctr->npend > 0 && hctr->nwin == 0 && hctr->npend == nl) { err = "device CDT builder: no segment progress"; return done(GDP_E_DEVICE); }
    nl = hctr->npend;
    cur ^= 1;
  }
  // outside removal and canonical order
  int *used = (int *)(base + o_used);
  uint64_t *keys = (uint64_t *)(base + o_keys), *keys2 = (uint64_t *)(base + o_keys2);
  int *vals = (int *)(base + o_vals), *vals2 = (int *)(base + o_vals2), *newid = (int *)(base + o_newid);
  if (hipMemsetAsync(used, 0, 4 * (size_t)nv, stream) != hipSuccess || hipMemsetAsync(b.c, 0, sizeof(Ctr), stream) != hipSuccess)
    { err = "device call failed"; return done(GDP_E_DEVICE); }
  k_keep<<<grid_for(nt, kBlk), kBlk, 0, stream>>>(b, nt, used, keys, vals);
  k_used<<<grid_for(nv, kBlk), kBlk, 0, stream>>>(b, used);
  if (!round_trip()) { err = "device call failed"; return done(GDP_E_DEVICE); }
  if (hctr->err) { err = std::string("final: ") + cdt_err_string(hctr->err); return done(hctr->err >= kEInternal ? GDP_E_DEVICE : GDP_E_INPUT); }
  const int nk = hctr->nkeep;
  if ((int64_t)nk != 2 * (int64_t)nv - hctr->nhull - 2) { err = "the kept region is not a disk"; return done(GDP_E_INPUT); }
  if (nk > cap_out) { err = "output capacity"; return done(GDP_E_NOMEM); }
  int vbits = 1;
  while (vbits < 31 && (1 << vbits) < nv + 3) vbits++;
  if (radix_sort_pairs(stream, keys, vals, keys2, vals2, nk, vbits, (int *)(base + o_sort)) != hipSuccess)
    { err = "sort failed"; return done(GDP_E_DEVICE); }
  k_newid<<<grid_for(nk, kBlk), kBlk, 0, stream>>>(nk, vals2, newid);
  k_emit<<<grid_for(nk, kBlk), kBlk, 0, stream>>>(b, nk, vals2, newid, otv, otn, ots);
  if (hipStreamSynchronize(stream) != hipSuccess || hipGetLastError() != hipSuccess)
    { err = "device call failed"; return done(GDP_E_DEVICE); }
  *n_tri = nk;
  if (stats) { stats->dt_rounds = dt_rounds; stats->seg_rounds = seg_rounds; }
  return done(GDP_OK);
}

}  // namespace gdp

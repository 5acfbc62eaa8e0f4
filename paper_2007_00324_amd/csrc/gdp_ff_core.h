// gdp_ff_core.h -- Line 8 of Algorithm 1 by Flip-Flop insertion (Section 4.3):
// the per-element steps of the kernels in gdp_ff.hip.
//
// The points S that survive Line 6 (each triangle split by at most one point,
// the one of highest priority) are all added by splitting the triangles they
// claimed: 1-3 for a point inside a triangle, 2-4 for a point on an interior
// edge (a midpoint, or a circumcenter on an edge), 1-2 for a midpoint of a
// hull subsegment.  Edges that are not locally Delaunay under the symbolic
// perturbation of the lifting map are then flipped (2-2) in parallel passes
// until the triangulation is the CDT of the old vertices and S.  A point of S
// joined by an edge to a point of S of higher priority, or a circumcenter
// inside the diametric circle (lens) of a subsegment opposite it, is
// redundant (Sections 4.2, 4.3): redundant points are taken out, each by
// flips that lower its degree followed by a flop (3-1; 2-1 or 4-2 beside a
// subsegment), done by one thread as the ear clipping of the point's link,
// then Lawson flips again.  This repeats until no point is redundant.
//
// The CDT is unique under the perturbation, so the order of flips and
// removals does not change the result; slots are assigned freely and the
// round ends by moving live triangles into the holes.  Points of S carry
// provisional vertex ids nV + rank (rank = position in decreasing key order,
// so a smaller id means a larger key); the ids are compacted at the end.
//
// Every step is a function of (view, element index) templated on the atomic
// operations, so the kernels (device atomics) and a sequential host run
// (plain operations, used to test the steps on the CPU) execute the same code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gdp_exact.h"

namespace gdp {

// Device counters of one Flip-Flop round.
struct FfCount {
  int32_t np, nmid;       // points of S (midpoints first in rank order)
  int32_t n_alloc;        // next fresh triangle slot
  int32_t n_list[2];      // lengths of the two worklists (one read, one built per pass)
  int32_t n_cnd[2];       // flip candidates of a pass (by the parity of the pass)
  int32_t n_touched;      // slots written this round (each once)
  int32_t n_red;          // redundant points found by the last detection
  int32_t n_left;         // redundant points a removal pass left for the next one
  int32_t n_dead;         // slots freed by removals
  int32_t pool_used, pool_short;
  int32_t n_hole, n_mover;
  int32_t err;            // first inconsistency found (site number), 0 none
  int32_t flags;          // subsegments newly flagged by encroaching circumcenters
  int32_t nwin, nwin_mid; // points of S kept, of which midpoints (after the last pass)
  int64_t flips, removals, n_dep, n_enc, iters, passes, rm_passes;
};

// Everything the steps read and write.
struct FfView {
  // mesh
  double2 *vxy;
  int32_t *vkind;
  int4 *tv, *tn, *ts;
  int2 *sv;
  int32_t *spar, *spend;
  uint32_t *mflag;
  int32_t nV, nT, nS;     // counts when the round started
  int32_t enc_mode;
  // points of S by rank
  double2 *pt;
  int4 *pinfo;            // x: 1 midpoint / 0 circumcenter; y: subsegment k (midpoint) or
                          //    edge index (circumcenter on an edge) or -1; z, w: claimed
                          //    triangles (midpoints: 4 * slot + edge of each side, -1 none)
  int2 *pab;              // a midpoint's subsegment endpoints (a, b) as the round started
  int4 *pslots;           // slots written by the point's split
  int32_t *alive, *red, *vtri, *newid;
  int32_t *newid_tiles;   // final rank of r = newid[r] + newid_tiles[r / kFfScanTile] (a tiled scan)
  // per slot
  int4 *grp;              // slots that replaced a triangle split this round
  int32_t *sstamp, *wstamp, *tstamp, *moved;
  uint64_t *claim;
  // lists
  int32_t *list_in, *list_out, *touched, *dead, *hole, *mover;
  int4 *fc0, *fc1;        // flip candidates: (t, e, o, j), the four outer slots
  uint64_t *fprio;
  int32_t cand_cap;
  // counters of the running pass (entries of FfCount): input and output list
  // lengths, this pass's candidates and the next pass's
  int32_t *n_in, *n_out, *n_cand, *n_cand_next;
  // per vertex / subsegment
  uint64_t *vmark;
  int32_t *sflag;         // [nS + nmid] flagged by an encroaching circumcenter (provisional ids)
  int32_t *mid_rank;      // [nS] 1 + rank of the subsegment's midpoint in S, 0 none
  int32_t *mid_elem, *mid_state;  // the round's midpoint candidate list
  int32_t nmk;
  int32_t *pool;
  int64_t pool_cap;
  FfCount *c;
};

// Candidate state bit of the refinement round (a cap-skipped entry).
constexpr int kFfStSkip = 64;
// Tile of the scan that ranks the kept points (the refinement's scan tile).
constexpr int kFfScanTile = 2048;
constexpr int kFfWalkCap = 1 << 20;

// Atomic operations of the kernels.  Additions to a shared counter are
// combined per wave first (one atomic for the active lanes of the wave, each
// lane getting its own offset): a pass appends thousands of entries to the
// same few counters, and atomics on one address are serialised.
struct FfDevOps {
  // returns the counter's value before this lane's share (lanes ordered by id)
  __device__ static int add(int32_t *p, int v) {
    const uint64_t mask = __ballot(1);
    const int lane = __lane_id();
    int prefix = 0, total = 0;
    for (uint64_t m = mask; m; m &= m - 1) {
      const int b = __ffsll((unsigned long long)m) - 1;
      const int vb = __shfl(v, b);
      prefix += b < lane ? vb : 0;
      total += vb;
    }
    int base = 0;
    if (lane == __ffsll((unsigned long long)mask) - 1) base = atomicAdd(p, total);
    return __builtin_amdgcn_readfirstlane(base) + prefix;
  }
  // add(p, 1)
  __device__ static int append(int32_t *p) {
    const uint64_t mask = __ballot(1);
    const int rank = __popcll(mask & ((1ull << __lane_id()) - 1));
    int base = 0;
    if (rank == 0) base = atomicAdd(p, __popcll(mask));
    return __builtin_amdgcn_readfirstlane(base) + rank;
  }
  __device__ static void add64(int64_t *p, int64_t v) {
    const uint64_t mask = __ballot(1);
    const int lane = __lane_id();
    long long total = 0;
    for (uint64_t m = mask; m; m &= m - 1) total += __shfl((long long)v, __ffsll((unsigned long long)m) - 1);
    if (lane == __ffsll((unsigned long long)mask) - 1 && total)
      atomicAdd((unsigned long long *)p, (unsigned long long)total);
  }
  __device__ static int exch(int32_t *p, int v) { return atomicExch(p, v); }
  __device__ static int or32(int32_t *p, int v) { return atomicOr(p, v); }
  __device__ static void max64(uint64_t *p, uint64_t v) {
    atomicMax((unsigned long long *)p, (unsigned long long)v);
  }
  __device__ static void err(int32_t *p, int site) { atomicCAS(p, 0, site); }
};

// ... and of a sequential run on the host.
struct FfHostOps {
  static int add(int32_t *p, int v) { const int o = *p; *p += v; return o; }
  static int append(int32_t *p) { return (*p)++; }
  static void add64(int64_t *p, int64_t v) { *p += v; }
  static int exch(int32_t *p, int v) { const int o = *p; *p = v; return o; }
  static int or32(int32_t *p, int v) { const int o = *p; *p |= v; return o; }
  static void max64(uint64_t *p, uint64_t v) { if (v > *p) *p = v; }
  static void err(int32_t *p, int site) { if (*p == 0) *p = site; }
};

GDP_HD int ffc(const int4 &v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }
GDP_HD int ff_eidx(const int4 &t, int u, int w) {
  if (t.x == u && t.y == w) return 0;
  if (t.y == u && t.z == w) return 1;
  if (t.z == u && t.x == w) return 2;
  return -1;
}
GDP_HD int ff_vidx(const int4 &t, int a) { return t.x == a ? 0 : (t.y == a ? 1 : (t.z == a ? 2 : -1)); }
GDP_HD int ff_sid(const int4 &tv, const int4 &ts, int e) { return ((tv.w >> e) & 1) ? ffc(ts, e) : -1; }
GDP_HD void ff_set(const FfView &V, int4 *arr, int slot, int e, int val) {
  ((int32_t *)arr)[(size_t)slot * 4 + e] = val;
}

// Writes a triangle (a, b, c) with the neighbour and subsegment of edges
// (a,b), (b,c), (c,a), rotated so that its smallest vertex comes first.
GDP_HD void ff_store(const FfView &V, int slot, int a, int b, int c, int na, int nb, int nc, int sa, int sb,
                     int sc) {
  int v0 = a, v1 = b, v2 = c, n0 = na, n1 = nb, n2 = nc, s0 = sa, s1 = sb, s2 = sc;
  if (b < a && b < c) {
    v0 = b; v1 = c; v2 = a; n0 = nb; n1 = nc; n2 = na; s0 = sb; s1 = sc; s2 = sa;
  } else if (c < a && c < b) {
    v0 = c; v1 = a; v2 = b; n0 = nc; n1 = na; n2 = nb; s0 = sc; s1 = sa; s2 = sb;
  }
  const int mask = (s0 >= 0 ? 1 : 0) | (s1 >= 0 ? 2 : 0) | (s2 >= 0 ? 4 : 0);
  V.tv[slot] = make_int4(v0, v1, v2, mask);
  V.tn[slot] = make_int4(n0, n1, n2, 0);
  V.ts[slot] = make_int4(s0, s1, s2, 0);
}

template <class O>
GDP_HD void ff_push(int32_t *list, int32_t *cnt, int32_t *stamps, int stamp, int slot) {
  if (O::exch(&stamps[slot], stamp) != stamp) list[O::append(cnt)] = slot;
}

// Both lists a written slot goes to: the flip worklist and the touched list.
template <class O>
GDP_HD void ff_wrote(const FfView &V, int slot, int wstamp, int tstamp) {
  ff_push<O>(V.list_out, V.n_out, V.wstamp, wstamp, slot);
  ff_push<O>(V.touched, &V.c->n_touched, V.tstamp, tstamp, slot);
}

// Every point of S starts in the mesh and not redundant.
template <class O>
GDP_HD void ff_init_point_one(const FfView &V, int r) {
  V.alive[r] = 1;
  V.red[r] = 0;
}

// ---------------------------------------------------------------------------
// Insertion by splits (every claimed triangle is split by one point)
// ---------------------------------------------------------------------------
// 2-4 split of edge e0 = (u, v) of t0 (t1 holds (v, u) at e1, or -1 on the
// hull) at p; s_up / s_pv: subsegment ids of the halves (u,p) and (p,v).
template <class O>
GDP_HD void ff_split_edge(const FfView &V, int r, int p, int t0, int e0, int t1, int e1, int s_up, int s_pv,
                          int split_stamp, int wst, int tst) {
  const int4 a0 = V.tv[t0], n0 = V.tn[t0], z0 = V.ts[t0];
  const int u = ffc(a0, e0), v = ffc(a0, (e0 + 1) % 3), w = ffc(a0, (e0 + 2) % 3);
  const int n_vw = ffc(n0, (e0 + 1) % 3), n_wu = ffc(n0, (e0 + 2) % 3);
  const int s_vw = ff_sid(a0, z0, (e0 + 1) % 3), s_wu = ff_sid(a0, z0, (e0 + 2) % 3);
  const int nnew = t1 >= 0 ? 2 : 1;
  const int base = O::add(&V.c->n_alloc, nnew);
  const int A = t0, B = base, C = t1, D = t1 >= 0 ? base + 1 : -1;
  if (t1 >= 0) {
    const int4 a1 = V.tv[t1], n1 = V.tn[t1], z1 = V.ts[t1];
    const int x = ffc(a1, (e1 + 2) % 3);
    const int n_ux = ffc(n1, (e1 + 1) % 3), n_xv = ffc(n1, (e1 + 2) % 3);
    const int s_ux = ff_sid(a1, z1, (e1 + 1) % 3), s_xv = ff_sid(a1, z1, (e1 + 2) % 3);
    ff_store(V, C, v, p, x, B, D, n_xv, s_pv, -1, s_xv);
    ff_store(V, D, p, u, x, A, n_ux, C, s_up, s_ux, -1);
    V.grp[t1] = make_int4(C, D, -1, -1);
    V.sstamp[t1] = split_stamp;
  }
  ff_store(V, A, u, p, w, D, B, n_wu, s_up, -1, s_wu);
  ff_store(V, B, p, v, w, C, n_vw, A, s_pv, s_vw, -1);
  V.grp[t0] = make_int4(A, B, -1, -1);
  V.sstamp[t0] = split_stamp;
  V.pslots[r] = make_int4(A, B, C, D);
  ff_wrote<O>(V, A, wst, tst);
  ff_wrote<O>(V, B, wst, tst);
  if (C >= 0) { ff_wrote<O>(V, C, wst, tst); ff_wrote<O>(V, D, wst, tst); }
}

template <class O>
GDP_HD void ff_split_one(const FfView &V, int r, int split_stamp, int wst, int tst) {
  const int4 info = V.pinfo[r];
  const int p = V.nV + r;
  V.vxy[p] = V.pt[r];
  V.vkind[p] = info.x ? 1 : 2;
  if (info.x) {
    // midpoint of subsegment k = (a, b): first half (a, p) keeps k, the
    // second (p, b) takes the provisional id nS + r
    const int k = info.y, ks = V.nS + r;
    const int2 ab = V.pab[r];
    int c0 = info.z, c1 = info.w;
    if (c0 < 0) { c0 = c1; c1 = -1; }
    const int t0 = c0 >> 2, e0 = c0 & 3;
    const int u = ffc(V.tv[t0], e0);
    const int s_up = u == ab.x ? k : ks, s_pv = u == ab.x ? ks : k;
    V.mid_rank[k] = r + 1;
    V.vtri[r] = t0;
    ff_split_edge<O>(V, r, p, t0, e0, c1 >= 0 ? (c1 >> 2) : -1, c1 >= 0 ? (c1 & 3) : -1, s_up, s_pv, split_stamp,
                     wst, tst);
    return;
  }
  const int t0 = info.z;
  V.vtri[r] = t0;
  if (info.y >= 0) {
    // circumcenter on the interior edge info.y of t0 (not a subsegment)
    const int e0 = info.y;
    const int4 a0 = V.tv[t0];
    const int t1 = ffc(V.tn[t0], e0);
    if (t1 < 0) { O::err(&V.c->err, 20); return; }
    const int e1 = ff_eidx(V.tv[t1], ffc(a0, (e0 + 1) % 3), ffc(a0, e0));
    if (e1 < 0) { O::err(&V.c->err, 1); return; }
    ff_split_edge<O>(V, r, p, t0, e0, t1, e1, -1, -1, split_stamp, wst, tst);
    return;
  }
  // 1-3 split of t0 = (a, b, c)
  const int4 a0 = V.tv[t0], n0 = V.tn[t0], z0 = V.ts[t0];
  const int a = a0.x, b = a0.y, c = a0.z;
  const int base = O::add(&V.c->n_alloc, 2);
  const int A = t0, B = base, C = base + 1;
  ff_store(V, A, a, b, p, n0.x, B, C, ff_sid(a0, z0, 0), -1, -1);
  ff_store(V, B, b, c, p, n0.y, C, A, ff_sid(a0, z0, 1), -1, -1);
  ff_store(V, C, c, a, p, n0.z, A, B, ff_sid(a0, z0, 2), -1, -1);
  V.grp[t0] = make_int4(A, B, C, -1);
  V.sstamp[t0] = split_stamp;
  V.pslots[r] = make_int4(A, B, C, -1);
  ff_wrote<O>(V, A, wst, tst);
  ff_wrote<O>(V, B, wst, tst);
  ff_wrote<O>(V, C, wst, tst);
}

// After all splits: an outer edge of a new triangle still names the old
// neighbour.  If that neighbour was split too, the edge is in one of its
// replacements; otherwise the neighbour's back pointer is set here (one
// writer per edge).
template <class O>
GDP_HD void ff_split_fix_one(const FfView &V, int r, int split_stamp) {
  const int4 sl = V.pslots[r];
  for (int q = 0; q < 4; q++) {
    const int s = ffc(sl, q < 3 ? q : 0) ;
    const int slot = q == 3 ? sl.w : s;
    if (slot < 0) continue;
    const int4 t = V.tv[slot], nb = V.tn[slot];
    for (int e = 0; e < 3; e++) {
      const int o = ffc(nb, e);
      if (o < 0 || o == sl.x || o == sl.y || o == sl.z || o == sl.w) continue;
      const int x = ffc(t, e), y = ffc(t, (e + 1) % 3);
      if (V.sstamp[o] == split_stamp) {
        const int4 g = V.grp[o];
        int found = -1;
        for (int h = 0; h < 3 && found < 0; h++) {
          const int cand = ffc(g, h);
          if (cand >= 0 && ff_eidx(V.tv[cand], y, x) >= 0) found = cand;
        }
        if (found < 0) { O::err(&V.c->err, 2); continue; }
        ff_set(V, V.tn, slot, e, found);
      } else {
        const int j = ff_eidx(V.tv[o], y, x);
        if (j < 0) { O::err(&V.c->err, 3); continue; }
        ff_set(V, V.tn, o, j, slot);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Lawson flips.  A pass checks the edges of the triangles on its worklist; a
// non-locally-Delaunay, non-subsegment edge (t, e | o, j) claims t, o and the
// four triangles around them with one 64-bit atomicMax of (pass, edge); a
// flip whose six claims all hold is applied, so it is the only writer of the
// six triangles in that pass.
// ---------------------------------------------------------------------------
template <class O>
GDP_HD void ff_flip_check_one(const FfView &V, int i, int in_stamp, uint64_t pass) {
  const int t = V.list_in[i];
  const int4 a = V.tv[t];
  if (a.x < 0) return;  // freed by a removal
  const int4 na = V.tn[t];
  for (int e = 0; e < 3; e++) {
    if ((a.w >> e) & 1) continue;
    const int o = ffc(na, e);
    if (o < 0) continue;
    if (o < t && V.wstamp[o] == in_stamp) continue;  // the lower slot on the list checks the edge
    const int u = ffc(a, e), v = ffc(a, (e + 1) % 3), w = ffc(a, (e + 2) % 3);
    const int4 b = V.tv[o];
    const int j = ff_eidx(b, v, u);
    if (j < 0) { O::err(&V.c->err, 4); continue; }
    const int d = ffc(b, (j + 2) % 3);
    const double2 U = V.vxy[u], W = V.vxy[v], C = V.vxy[w], D = V.vxy[d];
    if (incircle_sos(U.x, U.y, W.x, W.y, C.x, C.y, D.x, D.y, u, v, w, d) <= 0) continue;
    const int4 nb = V.tn[o];
    const int n_vw = ffc(na, (e + 1) % 3), n_wu = ffc(na, (e + 2) % 3);
    const int n_ud = ffc(nb, (j + 1) % 3), n_dv = ffc(nb, (j + 2) % 3);
    const uint64_t prio = (pass << 40) | (uint64_t)(t < o ? 4 * (int64_t)t + e : 4 * (int64_t)o + j);
    const int idx = O::append(V.n_cand);
    if (idx >= V.cand_cap) continue;  // no room and no claims: ff_flip_requeue_one
    O::max64(&V.claim[t], prio);
    O::max64(&V.claim[o], prio);
    if (n_vw >= 0) O::max64(&V.claim[n_vw], prio);
    if (n_wu >= 0) O::max64(&V.claim[n_wu], prio);
    if (n_ud >= 0) O::max64(&V.claim[n_ud], prio);
    if (n_dv >= 0) O::max64(&V.claim[n_dv], prio);
    V.fc0[idx] = make_int4(t, e, o, j);
    V.fc1[idx] = make_int4(n_vw, n_wu, n_ud, n_dv);
    V.fprio[idx] = prio;
  }
}

// Duties of one thread of a pass's check launch: the output list starts
// empty (nothing writes it during the check), and a pass is counted; of its
// apply launch: the next pass's candidate count starts at zero.
template <class O>
GDP_HD void ff_check_begin(const FfView &V) {
  *V.n_out = 0;
  if (*V.n_in > 0) V.c->passes++;
}
template <class O>
GDP_HD void ff_apply_begin(const FfView &V) { *V.n_cand_next = 0; }

// After a pass whose candidates overflowed their list (more candidates than
// room, and those without room placed no claims): every triangle of the
// input list is checked again in the next pass.
template <class O>
GDP_HD void ff_flip_requeue_one(const FfView &V, int i, int wst) {
  const int t = V.list_in[i];
  if (V.tv[t].x >= 0) ff_push<O>(V.list_out, V.n_out, V.wstamp, wst, t);
}

template <class O>
GDP_HD void ff_flip_apply_one(const FfView &V, int i, int wst, int tst) {
  if (i >= V.cand_cap) return;
  const int4 f = V.fc0[i], g = V.fc1[i];
  const uint64_t prio = V.fprio[i];
  const int t = f.x, e = f.y, o = f.z, j = f.w;
  bool win = V.claim[t] == prio && V.claim[o] == prio;
  for (int q = 0; q < 4 && win; q++) {
    const int s = ffc(g, q < 3 ? q : 0);
    const int x = q == 3 ? g.w : s;
    if (x >= 0 && V.claim[x] != prio) win = false;
  }
  if (!win) {
    ff_push<O>(V.list_out, V.n_out, V.wstamp, wst, t);  // the edge is checked again
    return;
  }
  // t = (u, v, w) with edge e = (u, v); o = (v, u, d) with edge j = (v, u).
  // The flip replaces (u, v) by (w, d): (u, d, w) in t, (d, v, w) in o.
  const int4 a = V.tv[t], za = V.ts[t], b = V.tv[o], zb = V.ts[o];
  const int u = ffc(a, e), v = ffc(a, (e + 1) % 3), w = ffc(a, (e + 2) % 3), d = ffc(b, (j + 2) % 3);
  const int s_vw = ff_sid(a, za, (e + 1) % 3), s_wu = ff_sid(a, za, (e + 2) % 3);
  const int s_ud = ff_sid(b, zb, (j + 1) % 3), s_dv = ff_sid(b, zb, (j + 2) % 3);
  const int n_vw = g.x, n_wu = g.y, n_ud = g.z, n_dv = g.w;
  ff_store(V, t, u, d, w, n_ud, o, n_wu, s_ud, -1, s_wu);
  ff_store(V, o, d, v, w, n_dv, n_vw, t, s_dv, s_vw, -1);
  if (n_ud >= 0) {
    const int q = ff_eidx(V.tv[n_ud], d, u);
    if (q < 0) O::err(&V.c->err, 5);
    else ff_set(V, V.tn, n_ud, q, t);
  }
  if (n_vw >= 0) {
    const int q = ff_eidx(V.tv[n_vw], w, v);
    if (q < 0) O::err(&V.c->err, 6);
    else ff_set(V, V.tn, n_vw, q, o);
  }
  O::add64(&V.c->flips, 1);
  ff_wrote<O>(V, t, wst, tst);
  ff_wrote<O>(V, o, wst, tst);
}

// ---------------------------------------------------------------------------
// Redundant points
// ---------------------------------------------------------------------------
// A triangle holding each live point of S (any one; written from the
// touched list, which holds every triangle with a new vertex).
template <class O>
GDP_HD void ff_vtri_one(const FfView &V, int i, int np) {
  const int s = V.touched[i];
  const int4 t = V.tv[s];
  if (t.x < 0) return;
  for (int q = 0; q < 3; q++) {
    const int x = ffc(t, q);
    if (x >= V.nV && x < V.nV + np) V.vtri[x - V.nV] = s;
  }
}

// The star of vertex p in counter-clockwise order: calls f(slot, index of p)
// for each triangle, starting at the hull side for a vertex on the hull.
// Returns the number of triangles (0 on an inconsistency).
template <class F>
GDP_HD int ff_star(const FfView &V, int p, int t0, bool &open, F &&f) {
  int start = t0;
  open = false;
  for (int steps = 0;; steps++) {
    if (steps > kFfWalkCap) return 0;
    const int4 t = V.tv[start];
    const int i = ff_vidx(t, p);
    if (i < 0) return 0;
    const int prev = ffc(V.tn[start], i);  // across (p, next vertex): clockwise
    if (prev < 0) { open = true; break; }
    if (prev == t0) { start = t0; break; }
    start = prev;
  }
  int n = 0, t = start;
  for (;;) {
    const int4 tri = V.tv[t];
    const int i = ff_vidx(tri, p);
    if (i < 0 || n > kFfWalkCap) return 0;
    f(t, i);
    n++;
    const int nxt = ffc(V.tn[t], (i + 2) % 3);  // across (previous vertex, p): counter-clockwise
    if (nxt < 0 || nxt == start) break;
    t = nxt;
  }
  return n;
}

template <class O>
GDP_HD void ff_detect_one(const FfView &V, int r) {
  if (!V.alive[r]) return;
  const int p = V.nV + r;
  const bool is_cc = V.pinfo[r].x == 0;
  const double2 P = V.vxy[p];
  bool dep = false, enc = false;
  bool open;
  const int n = ff_star(V, p, V.vtri[r], open, [&](int t, int i) {
    const int4 tri = V.tv[t];
    const int u = ffc(tri, (i + 1) % 3), w = ffc(tri, (i + 2) % 3);
    if ((u >= V.nV && u < p) || (w >= V.nV && w < p)) dep = true;
    if (is_cc && ((tri.w >> ((i + 1) % 3)) & 1)) {
      const double2 A = V.vxy[u], B = V.vxy[w];
      if (encroaches(V.enc_mode, A.x, A.y, B.x, B.y, P.x, P.y)) {
        enc = true;
        const int sid = ffc(V.ts[t], (i + 1) % 3);
        if (O::or32(&V.sflag[sid], 1) == 0) O::append(&V.c->flags);
      }
    }
  });
  if (n == 0) { O::err(&V.c->err, 7); return; }
  if (enc || dep) {
    V.red[r] = enc ? 2 : 1;
    O::append(&V.c->n_red);
    if (enc) O::add64(&V.c->n_enc, 1);
    else O::add64(&V.c->n_dep, 1);
  }
}

// Removal passes: a redundant point stamps itself and its neighbours with
// (pass, rank); it is removed in the pass only if every stamp is its own, so
// no two removals of a pass are within two edges of each other and their
// stars, and the triangles around them, are disjoint.
template <class O>
GDP_HD void ff_rm_mark_one(const FfView &V, int r, uint64_t pbase) {
  if (!V.alive[r] || !V.red[r]) return;
  const int p = V.nV + r;
  const uint64_t prio = pbase | (uint64_t)(r + 1);
  O::max64(&V.vmark[p], prio);
  bool open;
  const int n = ff_star(V, p, V.vtri[r], open, [&](int t, int i) {
    const int4 tri = V.tv[t];
    O::max64(&V.vmark[ffc(tri, (i + 1) % 3)], prio);
    O::max64(&V.vmark[ffc(tri, (i + 2) % 3)], prio);
  });
  if (n == 0) O::err(&V.c->err, 8);
}

// Ear clipping of one polygon (m vertices, counter-clockwise) held in the
// pool: pv vertex ids, info[q] the outer neighbour of edge (pv[q], pv[q+1])
// (>= 0 a slot, -1 none, -2 matched later), sd[q] its subsegment id.  Emits
// triangles into ev (3 ids each) and en / es (neighbour code and subsegment
// per edge).  Returns the number emitted, -1 if no ear was found.
//
// The polygon is the link of the removed point P, so it is star-shaped from
// P (P inside it, or on its closing edge): a convex corner b between a and c
// with P strictly on the other side of the chord a-c is an ear (the triangle
// lies in the wedge a-P-c, which holds no other link vertex) -- that is a
// flip of the edge P-b.  Only when no such corner is left (P on every
// remaining chord) is a corner tested against all remaining vertices.
GDP_HD int ff_clip(const FfView &V, double2 P, int m, int *pv, int *info, int *sd, int *nx, int *pr, int *ev,
                   int *en, int *es, int ne) {
  for (int q = 0; q < m; q++) { nx[q] = (q + 1) % m; pr[q] = (q + m - 1) % m; }
  int left = m, cur = 0, tries = 0;
  bool general = false;  // the slow ear test, once the fast one found nothing in a full turn
  while (left > 3) {
    const int a = pr[cur], b = cur, c = nx[cur];
    const double2 A = V.vxy[pv[a]], B = V.vxy[pv[b]], C = V.vxy[pv[c]];
    bool ear = orient2d(A.x, A.y, B.x, B.y, C.x, C.y) > 0;
    if (ear && !general) {
      ear = orient2d(A.x, A.y, C.x, C.y, P.x, P.y) > 0;
    } else if (ear) {
      for (int q = nx[c]; ear && q != a; q = nx[q]) {
        const double2 Q = V.vxy[pv[q]];
        if (orient2d(A.x, A.y, B.x, B.y, Q.x, Q.y) >= 0 && orient2d(B.x, B.y, C.x, C.y, Q.x, Q.y) >= 0 &&
            orient2d(C.x, C.y, A.x, A.y, Q.x, Q.y) >= 0)
          ear = false;
      }
    }
    if (!ear) {
      cur = nx[cur];
      if (++tries > left) {
        if (general) return -1;
        general = true;
        tries = 0;
      }
      continue;
    }
    // triangle (a, b, c): edges (a,b), (b,c) from the polygon; (c,a) new
    ev[3 * ne] = pv[a]; ev[3 * ne + 1] = pv[b]; ev[3 * ne + 2] = pv[c];
    en[3 * ne] = info[a]; en[3 * ne + 1] = info[b]; en[3 * ne + 2] = -2;
    es[3 * ne] = sd[a]; es[3 * ne + 1] = sd[b]; es[3 * ne + 2] = -1;
    ne++;
    info[a] = -2;  // the polygon's new edge (a, c): matched later
    sd[a] = -1;
    nx[a] = c;
    pr[c] = a;
    left--;
    cur = a;
    tries = 0;
    general = false;
  }
  const int a = pr[cur], b = cur, c = nx[cur];
  ev[3 * ne] = pv[a]; ev[3 * ne + 1] = pv[b]; ev[3 * ne + 2] = pv[c];
  en[3 * ne] = info[a]; en[3 * ne + 1] = info[b]; en[3 * ne + 2] = info[c];
  es[3 * ne] = sd[a]; es[3 * ne + 1] = sd[b]; es[3 * ne + 2] = sd[c];
  return ne + 1;
}

template <class O>
GDP_HD void ff_rm_decide_one(const FfView &V, int r, uint64_t pbase) {
  if (!V.alive[r] || !V.red[r]) return;
  const int p = V.nV + r;
  const uint64_t prio = pbase | (uint64_t)(r + 1);
  bool own = V.vmark[p] == prio, open;
  const int k = ff_star(V, p, V.vtri[r], open, [&](int t, int i) {
    const int4 tri = V.tv[t];
    if (V.vmark[ffc(tri, (i + 1) % 3)] != prio || V.vmark[ffc(tri, (i + 2) % 3)] != prio) own = false;
  });
  if (k == 0) { O::err(&V.c->err, 9); return; }
  if (own) V.red[r] |= 4;
  else O::append(&V.c->n_left);
}

template <class O>
GDP_HD void ff_rm_apply_one(const FfView &V, int r, int wst, int tst) {
  if (!V.alive[r] || !(V.red[r] & 4)) return;
  const int p = V.nV + r;
  bool open;
  const int k = ff_star(V, p, V.vtri[r], open, [&](int, int) {});
  if (k == 0) { O::err(&V.c->err, 19); return; }
  // pool layout, k + 2 entries each: ring, star, outer neighbour, outer
  // subsegment; then the clipping arrays and up to k emitted triangles
  const int64_t L = k + 2;
  const int64_t need = 11 * L + 9 * L;
  const int64_t base = O::add(&V.c->pool_used, (int)need);
  if (base + need > V.pool_cap) {
    O::or32(&V.c->pool_short, 1);
    O::append(&V.c->n_left);
    V.red[r] &= 3;  // tried again in the next pass
    return;
  }
  int *ring = V.pool + base, *star = ring + L, *onb = star + L, *osd = onb + L;
  int *pv = osd + L, *info = pv + L, *sd = info + L, *nx = sd + L, *pr = nx + L, *tmp = pr + L, *tmp2 = tmp + L;
  int *ev = tmp2 + L, *en = ev + 3 * L, *es = en + 3 * L;
  int j = 0, last_w = -1;
  ff_star(V, p, V.vtri[r], open, [&](int t, int i) {
    const int4 tri = V.tv[t];
    ring[j] = ffc(tri, (i + 1) % 3);
    last_w = ffc(tri, (i + 2) % 3);
    star[j] = t;
    onb[j] = ffc(V.tn[t], (i + 1) % 3);
    osd[j] = ff_sid(tri, V.ts[t], (i + 1) % 3);
    j++;
  });
  int nring = k;
  if (open) ring[nring++] = last_w;
  const int4 info4 = V.pinfo[r];
  int ne = 0;
  // A rounded midpoint lies off its segment by rounding, so one side of its
  // link can be the single edge (a, b) (a sliver triangle (p, a, b)): that
  // side has nothing to fill, and the triangle X across (a, b) takes the
  // restored subsegment.
  int sl_x = -1, sl_u = -1, sl_v = -1;
  if (info4.x == 0) {
    // circumcenter: one closed polygon, the link
    for (int q = 0; q < k; q++) { pv[q] = ring[q]; info[q] = onb[q]; sd[q] = osd[q]; }
    ne = ff_clip(V, V.vxy[p], k, pv, info, sd, nx, pr, ev, en, es, 0);
  } else {
    const int2 ab = V.pab[r];
    const int kseg = info4.y;
    if (open) {
      // hull subsegment: the chain ring[0..k] closed by the restored subsegment
      if (k == 1) {
        sl_x = onb[0]; sl_u = ring[0]; sl_v = ring[1];
      } else {
        for (int q = 0; q < k; q++) { pv[q] = ring[q]; info[q] = onb[q]; sd[q] = osd[q]; }
        pv[k] = ring[k]; info[k] = -1; sd[k] = kseg;
        ne = ff_clip(V, V.vxy[p], k + 1, pv, info, sd, nx, pr, ev, en, es, 0);
      }
    } else {
      int ia = -1, ib = -1;
      for (int q = 0; q < k; q++) {
        if (ring[q] == ab.x) ia = q;
        if (ring[q] == ab.y) ib = q;
      }
      if (ia < 0 || ib < 0) { O::err(&V.c->err, 10); return; }
      // two polygons: ring[ia..ib] and ring[ib..ia], each closed by (b, a) / (a, b)
      for (int side = 0; side < 2 && ne >= 0; side++) {
        const int from = side == 0 ? ia : ib, to = side == 0 ? ib : ia;
        if ((from + 1) % k == to) {
          if (sl_x >= 0) { O::err(&V.c->err, 11); return; }
          sl_x = onb[from]; sl_u = ring[from]; sl_v = ring[to];
          continue;
        }
        int m = 0;
        for (int q = from; q != to; q = (q + 1) % k) { pv[m] = ring[q]; info[m] = onb[q]; sd[m] = osd[q]; m++; }
        pv[m] = ring[to]; info[m] = -2; sd[m] = kseg; m++;
        ne = ff_clip(V, V.vxy[p], m, pv, info, sd, nx, pr, ev, en, es, ne);
      }
    }
  }
  if (ne < 0 || ne > k) { O::err(&V.c->err, 12); return; }
  // slots: the first ne star slots; the rest are freed
  for (int q = 0; q < ne; q++) tmp[q] = star[q];
  // neighbours: outer slots as found, the others are the emitted triangle
  // holding the reversed edge, or the sliver's outer triangle
  int sl_partner = -1;
  for (int q = 0; q < ne; q++) {
    int nn[3];
    for (int h = 0; h < 3; h++) {
      const int x = ev[3 * q + h], y = ev[3 * q + (h + 1) % 3];
      int code = en[3 * q + h];
      if (code == -2) {
        code = -1;
        for (int g = 0; g < ne && code < 0; g++) {
          if (g == q) continue;
          for (int hh = 0; hh < 3; hh++)
            if (ev[3 * g + hh] == y && ev[3 * g + (hh + 1) % 3] == x) code = tmp[g];
        }
        if (code < 0 && sl_x >= 0 && x == sl_u && y == sl_v) {
          code = sl_x;
          sl_partner = tmp[q];
        }
        if (code < 0) O::err(&V.c->err, 13);
      }
      nn[h] = code;
    }
    ff_store(V, tmp[q], ev[3 * q], ev[3 * q + 1], ev[3 * q + 2], nn[0], nn[1], nn[2], es[3 * q], es[3 * q + 1],
             es[3 * q + 2]);
    for (int h = 0; h < 3; h++) {
      const int x = ev[3 * q + h], y = ev[3 * q + (h + 1) % 3];
      if (en[3 * q + h] >= 0) {
        const int o = en[3 * q + h];
        const int jj = ff_eidx(V.tv[o], y, x);
        if (jj < 0) O::err(&V.c->err, 14);
        else ff_set(V, V.tn, o, jj, tmp[q]);
      }
      if (x >= V.nV && x != p && x < V.nV + V.c->np) V.vtri[x - V.nV] = tmp[q];
    }
    ff_wrote<O>(V, tmp[q], wst, tst);
  }
  if (sl_u >= 0) {
    // X holds (v, u): it becomes the subsegment, facing the other side's
    // triangle (none on the hull)
    if (sl_x < 0) { O::err(&V.c->err, 18); return; }
    const int4 tx = V.tv[sl_x];
    const int jx = ff_eidx(tx, sl_v, sl_u);
    if (jx < 0 || (!open && sl_partner < 0)) { O::err(&V.c->err, 18); return; }
    ff_set(V, V.tn, sl_x, jx, open ? -1 : sl_partner);
    ff_set(V, V.ts, sl_x, jx, info4.y);
    V.tv[sl_x] = make_int4(tx.x, tx.y, tx.z, tx.w | (1 << jx));
    ff_wrote<O>(V, sl_x, wst, tst);
  }
  for (int q = ne; q < k; q++) {
    V.tv[star[q]] = make_int4(-1, -1, -1, 0);
    V.tn[star[q]] = make_int4(-1, -1, -1, 0);
    V.dead[O::append(&V.c->n_dead)] = star[q];
  }
  V.alive[r] = 0;
  V.red[r] = 0;
  O::add64(&V.c->removals, 1);
}

// ---------------------------------------------------------------------------
// End of the round
// ---------------------------------------------------------------------------
GDP_HD int ff_newid(const FfView &V, int r) { return V.newid[r] + V.newid_tiles[r / kFfScanTile]; }

// Final ids: newid[r] = rank of r among the live points (an exclusive scan).
template <class O>
GDP_HD void ff_final_point_one(const FfView &V, int r) {
  if (!V.alive[r]) return;
  const int4 info = V.pinfo[r];
  const int id = V.nV + ff_newid(V, r);
  V.vxy[id] = V.pt[r];
  V.vkind[id] = info.x ? 1 : 2;
  if (info.x) {
    const int k = info.y, knew = V.nS + ff_newid(V, r);  // midpoints come first in rank order
    const int2 ab = V.pab[r];
    V.sv[k] = make_int2(ab.x, id);
    V.sv[knew] = make_int2(id, ab.y);
    V.spar[knew] = V.spar[k];
    V.spend[knew] = V.sflag[V.nS + r] ? 1 : 0;
  }
}

// Vertex and subsegment ids of every live triangle written this round.  The
// renumbering keeps the order of the ids, so the rotation stays canonical.
template <class O>
GDP_HD void ff_final_tri_one(const FfView &V, int i) {
  const int s = V.touched[i];
  int4 t = V.tv[s];
  if (t.x < 0) return;
  int4 z = V.ts[s];
  int v[3] = {t.x, t.y, t.z}, sid[3] = {z.x, z.y, z.z};
  for (int q = 0; q < 3; q++) {
    if (v[q] >= V.nV) {
      const int r = v[q] - V.nV;
      if (!V.alive[r]) O::err(&V.c->err, 15);
      v[q] = V.nV + ff_newid(V, r);
    }
    if (((t.w >> q) & 1) && sid[q] >= V.nS) {
      const int r = sid[q] - V.nS;
      if (!V.alive[r]) O::err(&V.c->err, 16);
      sid[q] = V.nS + ff_newid(V, r);
    }
  }
  V.tv[s] = make_int4(v[0], v[1], v[2], t.w);
  V.ts[s] = make_int4(sid[0], sid[1], sid[2], z.w);
}

// Pending flags of the round's midpoint candidates: pending := (pending or
// flagged this round) and not split (an entry the candidate cap skipped is
// not flagged).
template <class O>
GDP_HD void ff_final_mid_one(const FfView &V, int i) {
  const int k = V.mid_elem[i];
  const int st = V.mid_state[i];
  const int rr = V.mid_rank[k];
  const bool split = rr > 0 && V.alive[rr - 1];
  if (!(st & kFfStSkip)) V.spend[k] = split ? 0 : 1;
  else if (split) V.spend[k] = 0;
  V.mflag[k] = 0u;
}

// ... and the flags raised by encroaching circumcenters: on the piece they
// name, or on the whole subsegment when its split was undone.  Clears the
// per-subsegment state of the round.
template <class O>
GDP_HD void ff_final_flag_one(const FfView &V, int k, int nmid) {
  if (k < V.nS) {
    if (V.sflag[k]) V.spend[k] = 1;
    const int rr = V.mid_rank[k];
    if (rr > 0 && !V.alive[rr - 1] && V.sflag[V.nS + rr - 1]) V.spend[k] = 1;
    V.mid_rank[k] = 0;
    V.sflag[k] = 0;
  } else if (k < V.nS + nmid) {
    // read by ff_final_point_one and by the line above before this runs
  }
}
template <class O>
GDP_HD void ff_final_flag_clear_one(const FfView &V, int r) { V.sflag[V.nS + r] = 0; }

// Compaction: live triangles above the final count move into the holes
// below it.  Holes are the freed slots below the count (from the list of
// freed slots); movers are the live slots from the count up.
template <class O>
GDP_HD void ff_compact_hole_one(const FfView &V, int i, int n_live) {
  const int s = V.dead[i];
  if (s < n_live) V.hole[O::append(&V.c->n_hole)] = s;
}
template <class O>
GDP_HD void ff_compact_mover_one(const FfView &V, int s) {
  if (V.tv[s].x >= 0) V.mover[O::append(&V.c->n_mover)] = s;
}
template <class O>
GDP_HD void ff_compact_move_one(const FfView &V, int i) {
  const int h = V.hole[i], s = V.mover[i];
  V.tv[h] = V.tv[s];
  V.tn[h] = V.tn[s];
  V.ts[h] = V.ts[s];
  V.moved[s] = h;
}
template <class O>
GDP_HD void ff_compact_fix_one(const FfView &V, int i, int n_live) {
  const int h = V.hole[i];
  const int4 t = V.tv[h], nb = V.tn[h];
  for (int e = 0; e < 3; e++) {
    const int n = ffc(nb, e);
    if (n < 0) continue;
    const int n2 = n >= n_live ? V.moved[n] : n;
    if (n2 != n) ff_set(V, V.tn, h, e, n2);
    const int x = ffc(t, e), y = ffc(t, (e + 1) % 3);
    const int j = ff_eidx(V.tv[n2], y, x);
    if (j < 0) { O::err(&V.c->err, 17); continue; }
    ff_set(V, V.tn, n2, j, h);
  }
}

// Canonical rotation (smallest vertex first) of an existing triangle.
template <class O>
GDP_HD void ff_rotate_one(const FfView &V, int s) {
  const int4 t = V.tv[s], n = V.tn[s], z = V.ts[s];
  if (t.x < t.y && t.x < t.z) return;
  ff_store(V, s, t.x, t.y, t.z, n.x, n.y, n.z, ff_sid(t, z, 0), ff_sid(t, z, 1), ff_sid(t, z, 2));
}

}  // namespace gdp

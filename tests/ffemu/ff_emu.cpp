// ff_emu.cpp -- a sequential host run of the Flip-Flop steps of
// gdp_ff_core.h (TEST INFRASTRUCTURE: it checks the steps on the CPU
// against the oracle before they run as kernels; the product library does
// not contain it).
//
// Each "launch" runs the step for element 0, 1, ... in turn with plain
// operations in place of atomics: a legal schedule of the kernels.
#include <algorithm>
#include <cstring>
#include <vector>

#include "gdp_ff_core.h"

using namespace gdp;

namespace {
struct Bufs {
  std::vector<double2> vxy, pt;
  std::vector<int32_t> vkind, spar, spend, alive, red, vtri, newid, sstamp, wstamp, tstamp, moved;
  std::vector<int32_t> l0, l1, touched, dead, hole, mover, sflag, mid_rank, mid_elem, mid_state, pool, ntiles;
  std::vector<uint32_t> mflag;
  std::vector<int4> tv, tn, ts, pinfo, pslots, grp, fc0, fc1;
  std::vector<int2> sv, pab;
  std::vector<uint64_t> claim, fprio, vmark;
};
// Every live triangle strictly counter-clockwise, neighbours mutual, the
// subsegment bits equal on both sides of an edge.  Returns 0 or a code.
int validate(const Bufs &B, int n_alloc) {
  for (int s = 0; s < n_alloc; s++) {
    const int4 t = B.tv[s];
    if (t.x < 0) continue;
    const double2 A = B.vxy[t.x], Bp = B.vxy[t.y], Cp = B.vxy[t.z];
    if (orient2d(A.x, A.y, Bp.x, Bp.y, Cp.x, Cp.y) <= 0) return 1;
    for (int e = 0; e < 3; e++) {
      const int o = ffc(B.tn[s], e);
      if (o < 0) continue;
      const int4 u = B.tv[o];
      if (u.x < 0) return 2;
      const int j = ff_eidx(u, ffc(t, (e + 1) % 3), ffc(t, e));
      if (j < 0) return 3;
      if (ffc(B.tn[o], j) != s) return 4;
      if (((t.w >> e) & 1) != ((u.w >> j) & 1)) return 5;
    }
  }
  return 0;
}
// Element order of one emulated launch: 0, 1, ... or, with a seed, a
// pseudo-random permutation (another legal schedule of the same kernel).
struct Order {
  uint64_t seed;
  std::vector<int> idx;
  const std::vector<int> &of(int n) {
    idx.resize(n);
    for (int i = 0; i < n; i++) idx[i] = i;
    if (seed) {
      for (int i = n - 1; i > 0; i--) {
        seed = seed * 6364136223846793005ull + 1442695040888963407ull;
        const int j = (int)((seed >> 33) % (uint64_t)(i + 1));
        std::swap(idx[i], idx[j]);
      }
    }
    return idx;
  }
};
}  // namespace

extern "C" int ffemu_round(int nV, int nT, int nS, int enc_mode, double *xy, int *vkind, int capV, int *tv, int *tn,
                           int *ts, int capT, int *sv, int *spar, int *spend, int capS, int np, int nmid,
                           const double *pxy, const int *pinfo, const int *pab, int nmk, const int *mid_elem,
                           const int *mid_state, int64_t *out, int cand_cap, uint64_t order_seed) {
  Order ord{order_seed, {}};
  using O = FfHostOps;
  Bufs B;
  B.vxy.resize(capV);
  for (int i = 0; i < nV; i++) B.vxy[i] = make_double2(xy[2 * i], xy[2 * i + 1]);
  B.vkind.assign(vkind, vkind + capV);
  B.tv.resize(capT); B.tn.resize(capT); B.ts.resize(capT);
  for (int i = 0; i < nT; i++) {
    B.tv[i] = make_int4(tv[4 * i], tv[4 * i + 1], tv[4 * i + 2], tv[4 * i + 3]);
    B.tn[i] = make_int4(tn[4 * i], tn[4 * i + 1], tn[4 * i + 2], tn[4 * i + 3]);
    B.ts[i] = make_int4(ts[4 * i], ts[4 * i + 1], ts[4 * i + 2], ts[4 * i + 3]);
  }
  B.sv.resize(capS);
  for (int i = 0; i < nS; i++) B.sv[i] = make_int2(sv[2 * i], sv[2 * i + 1]);
  B.spar.assign(spar, spar + capS);
  B.spend.assign(spend, spend + capS);
  B.mflag.assign(capS, 0u);
  B.pt.resize(np + 1); B.pinfo.resize(np + 1); B.pab.resize(np + 1); B.pslots.resize(np + 1);
  for (int r = 0; r < np; r++) {
    B.pt[r] = make_double2(pxy[2 * r], pxy[2 * r + 1]);
    B.pinfo[r] = make_int4(pinfo[4 * r], pinfo[4 * r + 1], pinfo[4 * r + 2], pinfo[4 * r + 3]);
    B.pab[r] = make_int2(pab[2 * r], pab[2 * r + 1]);
  }
  B.alive.assign(np + 1, 7); B.red.assign(np + 1, 7); B.vtri.assign(np + 1, -1); B.newid.assign(np + 1, 0);
  B.sstamp.assign(capT, 0); B.wstamp.assign(capT, 0); B.tstamp.assign(capT, 0); B.moved.assign(capT, -1);
  B.grp.resize(capT); B.claim.assign(capT, 0);
  B.l0.resize(capT); B.l1.resize(capT); B.touched.resize(capT); B.dead.resize(capT); B.hole.resize(capT);
  B.mover.resize(capT);
  B.ntiles.assign(np / kFfScanTile + 2, 0);  // the host run ranks in one tile
  B.fc0.resize(3 * (size_t)capT); B.fc1.resize(3 * (size_t)capT); B.fprio.resize(3 * (size_t)capT);
  B.vmark.assign(capV, 0);
  B.sflag.assign(capS + np + 1, 0);
  B.mid_rank.assign(capS, 0);
  B.mid_elem.assign(mid_elem, mid_elem + nmk);
  B.mid_state.assign(mid_state, mid_state + nmk);
  B.pool.resize(40 * (size_t)capT + 1024);
  FfCount C;
  memset(&C, 0, sizeof C);
  C.np = np; C.nmid = nmid; C.n_alloc = nT;
  FfView V;
  memset(&V, 0, sizeof V);
  V.vxy = B.vxy.data(); V.vkind = B.vkind.data(); V.tv = B.tv.data(); V.tn = B.tn.data(); V.ts = B.ts.data();
  V.sv = B.sv.data(); V.spar = B.spar.data(); V.spend = B.spend.data(); V.mflag = B.mflag.data();
  V.nV = nV; V.nT = nT; V.nS = nS; V.enc_mode = enc_mode;
  V.pt = B.pt.data(); V.pinfo = B.pinfo.data(); V.pab = B.pab.data(); V.pslots = B.pslots.data();
  V.alive = B.alive.data(); V.red = B.red.data(); V.vtri = B.vtri.data(); V.newid = B.newid.data();
  V.grp = B.grp.data(); V.sstamp = B.sstamp.data(); V.wstamp = B.wstamp.data(); V.tstamp = B.tstamp.data();
  V.moved = B.moved.data(); V.claim = B.claim.data();
  V.touched = B.touched.data(); V.dead = B.dead.data(); V.hole = B.hole.data(); V.mover = B.mover.data();
  V.newid_tiles = B.ntiles.data();
  V.fc0 = B.fc0.data(); V.fc1 = B.fc1.data(); V.fprio = B.fprio.data(); V.cand_cap = cand_cap > 0 ? cand_cap : 3 * capT;
  V.vmark = B.vmark.data(); V.sflag = B.sflag.data(); V.mid_rank = B.mid_rank.data();
  V.mid_elem = B.mid_elem.data(); V.mid_state = B.mid_state.data(); V.nmk = nmk;
  V.pool = B.pool.data(); V.pool_cap = (int64_t)B.pool.size();
  V.c = &C;
  int32_t *lists[2] = {B.l0.data(), B.l1.data()};
  int cur = 0, stamp = 0;
  uint64_t pass = 0;
  auto target = [&](int out) {  // writers of the next worklist
    V.list_out = lists[out];
    V.n_out = &C.n_list[out];
    C.n_list[out] = 0;
  };
  const int tst = ++stamp;
  // splits write the first worklist
  int wst = ++stamp;
  target(0);
  for (int r : ord.of(np)) ff_init_point_one<O>(V, r);
  for (int r : ord.of(np)) ff_split_one<O>(V, r, 1, wst, tst);
  for (int r : ord.of(np)) ff_split_fix_one<O>(V, r, 1);
  int bad = validate(B, C.n_alloc);
  if (bad) { out[11] = 1000 + bad; return 200; }
  cur = 0;
  int in_stamp = wst;
  auto lawson = [&]() {
    C.n_cnd[0] = C.n_cnd[1] = 0;
    for (;;) {
      if (C.n_list[cur] == 0 || C.err) return;
      wst = ++stamp;
      pass++;
      V.list_in = lists[cur];
      V.list_out = lists[cur ^ 1];
      V.n_in = &C.n_list[cur];
      V.n_out = &C.n_list[cur ^ 1];
      V.n_cand = &C.n_cnd[pass & 1];
      V.n_cand_next = &C.n_cnd[(pass + 1) & 1];
      ff_check_begin<O>(V);
      const int n_in = *V.n_in;
      for (int i : ord.of(n_in)) ff_flip_check_one<O>(V, i, in_stamp, pass);
      const int nc = *V.n_cand;
      ff_apply_begin<O>(V);
      for (int i : ord.of(std::min(nc, V.cand_cap))) ff_flip_apply_one<O>(V, i, wst, tst);
      if (nc > V.cand_cap)
        for (int i = 0; i < n_in; i++) ff_flip_requeue_one<O>(V, i, wst);
      in_stamp = wst;
      cur ^= 1;
      const int bad2 = validate(B, C.n_alloc);
      if (bad2) { out[11] = 2000 + bad2 + 10 * (int)C.passes; C.err = 201; return; }
    }
  };
  lawson();
  for (int it = 0; it < 1000 && !C.err; it++) {
    C.iters++;
    for (int i : ord.of(C.n_touched)) ff_vtri_one<O>(V, i, np);
    C.n_red = 0;
    for (int r : ord.of(np)) ff_detect_one<O>(V, r);
    if (C.n_red == 0 || C.err) break;
    // removals write the next worklist
    wst = ++stamp;
    target(cur);
    for (int guard = 0;; guard++) {
      if (guard > 100000) { C.err = 99; break; }
      pass++;
      const uint64_t pbase = pass << 32;
      C.n_left = 0;
      C.pool_used = 0;
      for (int r : ord.of(np)) ff_rm_mark_one<O>(V, r, pbase);
      for (int r : ord.of(np)) ff_rm_decide_one<O>(V, r, pbase);
      for (int r : ord.of(np)) ff_rm_apply_one<O>(V, r, wst, tst);
      const int bad3 = validate(B, C.n_alloc);
      if (bad3) { out[11] = 3000 + bad3; C.err = 202; break; }
      if (C.n_left == 0 || C.err) break;
    }
    in_stamp = wst;
    lawson();
  }
  // final ids
  int nwin = 0, nmid_win = 0;
  for (int r = 0; r < np; r++) {
    B.newid[r] = nwin;
    nwin += B.alive[r];
    if (r < nmid) nmid_win += B.alive[r];
  }
  for (int r = 0; r < np; r++) ff_final_point_one<O>(V, r);
  for (int i = 0; i < C.n_touched; i++) ff_final_tri_one<O>(V, i);
  for (int i = 0; i < nmk; i++) ff_final_mid_one<O>(V, i);
  for (int k = 0; k < nS; k++) ff_final_flag_one<O>(V, k, nmid);
  for (int r = 0; r < nmid; r++) ff_final_flag_clear_one<O>(V, r);
  const int n_live = C.n_alloc - C.n_dead;
  for (int i : ord.of(C.n_dead)) ff_compact_hole_one<O>(V, i, n_live);
  for (int j : ord.of(C.n_alloc - n_live)) ff_compact_mover_one<O>(V, n_live + j);
  if (C.n_hole != C.n_mover) C.err = C.err ? C.err : 98;
  for (int i = 0; i < C.n_hole; i++) ff_compact_move_one<O>(V, i);
  for (int i = 0; i < C.n_hole; i++) ff_compact_fix_one<O>(V, i, n_live);
  // results
  const int nV2 = nV + nwin, nS2 = nS + nmid_win;
  if (nV2 > capV || n_live > capT || nS2 > capS) return 97;
  for (int i = 0; i < nV2; i++) { xy[2 * i] = B.vxy[i].x; xy[2 * i + 1] = B.vxy[i].y; vkind[i] = B.vkind[i]; }
  for (int i = 0; i < n_live; i++) {
    const int4 a = B.tv[i], b = B.tn[i], c = B.ts[i];
    tv[4 * i] = a.x; tv[4 * i + 1] = a.y; tv[4 * i + 2] = a.z; tv[4 * i + 3] = a.w;
    tn[4 * i] = b.x; tn[4 * i + 1] = b.y; tn[4 * i + 2] = b.z; tn[4 * i + 3] = b.w;
    ts[4 * i] = c.x; ts[4 * i + 1] = c.y; ts[4 * i + 2] = c.z; ts[4 * i + 3] = c.w;
  }
  for (int i = 0; i < nS2; i++) { sv[2 * i] = B.sv[i].x; sv[2 * i + 1] = B.sv[i].y; spar[i] = B.spar[i]; spend[i] = B.spend[i]; }
  out[0] = nV2; out[1] = n_live; out[2] = nS2; out[3] = C.iters; out[4] = C.flips; out[5] = C.removals;
  out[6] = C.n_dep; out[7] = C.n_enc; out[8] = C.flags; out[9] = C.err; out[10] = C.passes;
  return C.err;
}

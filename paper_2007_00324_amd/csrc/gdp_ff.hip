// gdp_ff.hip -- the Flip-Flop insertion of Line 8 (Section 4.3) as kernels:
// grid-stride loops over the elements, each element one step of
// gdp_ff_core.h with device atomics.  The host sequence that drives them
// (one round: splits, flip passes, detection, removal passes, final ids,
// compaction) is ff_loop / ff_line8 in gdp_api.hip.
#include "gdp_kernels.h"

namespace gdp {

using DO = FfDevOps;
static_assert(kFfScanTile == kScanTileSize, "the ranks are scanned with the refinement's tile");

#define FF_LOOP(i, n) \
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

__global__ void kf_split(FfView V, int split_stamp, int wst, int tst) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_split_one<DO>(V, r, split_stamp, wst, tst);
}

__global__ void kf_split_fix(FfView V, int split_stamp) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_split_fix_one<DO>(V, r, split_stamp);
}

// Control words moved by one thread: op 0 empties worklist count `arg` and
// both candidate counts, op 1 starts a removal pass, op 2 a detection, op 4
// the compaction lists.
__global__ void kf_ctl(FfCount *c, int op, int arg) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  switch (op) {
    case 0:
      c->n_list[arg] = 0;
      c->n_cnd[0] = 0;
      c->n_cnd[1] = 0;
      break;
    case 1:
      c->n_left = 0;
      c->pool_used = 0;
      c->pool_short = 0;
      c->rm_passes++;
      break;
    case 2:
      c->n_red = 0;
      c->iters++;
      break;
    default:
      c->n_hole = 0;
      c->n_mover = 0;
      break;
  }
}

// A flip pass is these two launches: the list lengths and candidate counts
// are entries of FfCount chosen by the host (two lists and two candidate
// counts alternate), so no launch is needed between passes.
__global__ void kf_flip_check(FfView V, int in_stamp, uint64_t pass) {
  const int n = *V.n_in;
  if (blockIdx.x == 0 && threadIdx.x == 0) ff_check_begin<DO>(V);
  FF_LOOP(i, n) ff_flip_check_one<DO>(V, i, in_stamp, pass);
}

__global__ void kf_flip_apply(FfView V, int wst, int tst) {
  const int nc = *V.n_cand;
  if (blockIdx.x == 0 && threadIdx.x == 0) ff_apply_begin<DO>(V);
  FF_LOOP(i, min(nc, V.cand_cap)) ff_flip_apply_one<DO>(V, i, wst, tst);
  if (nc > V.cand_cap) {
    const int n_in = *V.n_in;
    FF_LOOP(i, n_in) ff_flip_requeue_one<DO>(V, i, wst);
  }
}

__global__ void kf_vtri(FfView V) {
  const int n = V.c->n_touched, np = V.c->np;
  FF_LOOP(i, n) ff_vtri_one<DO>(V, i, np);
}

__global__ void kf_detect(FfView V) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_detect_one<DO>(V, r);
}

__global__ void kf_rm_mark(FfView V, uint64_t pbase) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_rm_mark_one<DO>(V, r, pbase);
}

__global__ void kf_rm_decide(FfView V, uint64_t pbase) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_rm_decide_one<DO>(V, r, pbase);
}

__global__ void kf_rm_apply(FfView V, int wst, int tst) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_rm_apply_one<DO>(V, r, wst, tst);
}

// The number of kept midpoints (the midpoints are ranks 0..nmid-1), once
// the ranks are scanned (one thread).
__global__ void kf_nwin_mid(FfView V) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int np = V.c->np, nmid = V.c->nmid;
  V.c->nwin_mid = nmid < np ? ff_newid(V, nmid) : V.c->nwin;
}

__global__ void kf_final_point(FfView V) {
  const int np = V.c->np;
  FF_LOOP(r, np) ff_final_point_one<DO>(V, r);
}

__global__ void kf_final_tri(FfView V) {
  const int n = V.c->n_touched;
  FF_LOOP(i, n) ff_final_tri_one<DO>(V, i);
}

__global__ void kf_final_mid(FfView V) {
  FF_LOOP(i, V.nmk) ff_final_mid_one<DO>(V, i);
}

__global__ void kf_final_flag(FfView V) {
  const int nmid = V.c->nmid;
  FF_LOOP(k, V.nS) ff_final_flag_one<DO>(V, k, nmid);
}

__global__ void kf_final_flag_clear(FfView V) {
  const int nmid = V.c->nmid;
  FF_LOOP(r, nmid) ff_final_flag_clear_one<DO>(V, r);
}

__global__ void kf_compact_list(FfView V, int n_alloc, int n_live) {
  const int nd = V.c->n_dead;
  FF_LOOP(i, nd) ff_compact_hole_one<DO>(V, i, n_live);
  FF_LOOP(j, n_alloc - n_live) ff_compact_mover_one<DO>(V, n_live + j);
}

__global__ void kf_compact_move(FfView V) {
  const int n = min(V.c->n_hole, V.c->n_mover);
  FF_LOOP(i, n) ff_compact_move_one<DO>(V, i);
}

__global__ void kf_compact_fix(FfView V, int n_live) {
  const int n = min(V.c->n_hole, V.c->n_mover);
  FF_LOOP(i, n) ff_compact_fix_one<DO>(V, i, n_live);
}

__global__ void kf_rotate(FfView V, int n) {
  FF_LOOP(s, n) ff_rotate_one<DO>(V, s);
}

__global__ void kf_all_slots(FfView V, int n, int wst) {
  FF_LOOP(s, n) {
    V.wstamp[s] = wst;
    V.list_out[s] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *V.n_out = n;
}

#undef FF_LOOP

}  // namespace gdp

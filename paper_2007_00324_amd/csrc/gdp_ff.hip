// gdp_ff.hip -- the Flip-Flop insertion of Line 8 (Section 4.3) as kernels:
// grid-stride loops over the elements, each element one step of
// gdp_ff_core.h with device atomics.  The host sequence that drives them
// (one round: splits, flip passes, detection, removal passes, final ids,
// compaction) is ff_loop / ff_line8 in gdp_api.hip.
#include "gdp_kernels.h"

namespace gdp {

using DO = FfDevOps;

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

// The control words of a pass are moved by one thread before the pass:
// op 0 starts a flip pass (the last output list becomes the input), op 1 a
// removal pass, op 2 a detection, op 3 empties the output list, op 4 the
// compaction lists.
__global__ void kf_ctl(FfCount *c, int op) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  switch (op) {
    case 0:
      c->n_in = c->n_out;
      c->n_out = 0;
      c->n_cand = 0;
      c->cand_over = 0;
      if (c->n_in > 0) c->passes++;
      break;
    case 1:
      c->n_left = 0;
      c->pool_used = 0;
      c->pool_short = 0;
      break;
    case 2:
      c->n_red = 0;
      c->iters++;
      break;
    case 3:
      c->n_out = 0;
      break;
    default:
      c->n_hole = 0;
      c->n_mover = 0;
      break;
  }
}

__global__ void kf_flip_check(FfView V, int in_stamp, uint64_t pass) {
  const int n = V.c->n_in;
  FF_LOOP(i, n) ff_flip_check_one<DO>(V, i, in_stamp, pass);
}

__global__ void kf_flip_apply(FfView V, int wst, int tst) {
  const int n = min(V.c->n_cand, V.cand_cap);
  FF_LOOP(i, n) ff_flip_apply_one<DO>(V, i, wst, tst);
  if (V.c->cand_over) {
    const int n_in = V.c->n_in;
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

// One workgroup: newid = exclusive prefix of alive over the ranks; the
// totals (kept points, kept midpoints) go to the counters.  Each thread
// sums a contiguous chunk, the chunk sums are scanned in LDS, then each
// thread writes its chunk.
constexpr int kFfScanThreads = 1024;
__global__ __launch_bounds__(kFfScanThreads) void kf_newid(FfView V) {
  __shared__ int part[kFfScanThreads];
  __shared__ int s_total;
  const int np = V.c->np, nmid = V.c->nmid;
  const int chunk = (np + kFfScanThreads - 1) / kFfScanThreads;
  const int lo = threadIdx.x * chunk, hi = min(np, lo + chunk);
  int s = 0;
  for (int r = lo; r < hi; r++) s += V.alive[r];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < kFfScanThreads; i++) {
      const int x = part[i];
      part[i] = run;
      run += x;
    }
    s_total = run;
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int r = lo; r < hi; r++) {
    V.newid[r] = run;
    if (r == nmid) V.c->nwin_mid = run;
    run += V.alive[r];
  }
  if (threadIdx.x == 0) {
    V.c->nwin = s_total;
    if (nmid >= np) V.c->nwin_mid = s_total;
  }
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
  FF_LOOP(s, n_alloc) ff_compact_list_one<DO>(V, s, n_live);
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
  if (blockIdx.x == 0 && threadIdx.x == 0) V.c->n_out = n;
}

#undef FF_LOOP

}  // namespace gdp

/*
 * gdp2d.h -- C ABI of the gfx950 (MI355X) 2D constrained Delaunay refinement
 * library.
 *
 * What it computes (Chen, Tan, Ong, "On Designing GPU Algorithms with
 * Applications to Mesh Refinement", Section 4, Algorithm 1 gDP2d):
 *   input  : a planar straight-line graph (PSLG) -- vertices P and
 *            non-crossing segments E -- and a quality bound;
 *   output : a constrained Delaunay triangulation of the convex hull of P in
 *            which every segment is a union of subsegments, no triangle has a
 *            radius-edge ratio above B (the ratio of Section 5.1, used here in
 *            2D) and no subsegment is encroached in Ruppert's sense
 *            (Section 4.2), plus the Steiner vertices that were added.
 * Line 1 (the initial CDT) runs on the host; Lines 2-9 run as a sequence of
 * deterministic rounds of HIP kernels on one GPU, where each round collects
 * encroached subsegments and bad triangles, computes midpoints and
 * circumcenters, locates them by walking, grows Bowyer-Watson cavities,
 * resolves overlapping cavities with 64-bit priority marks (atomicMax) and a
 * Delaunay-dependency test, and inserts the winners.
 *
 * Conventions for every call:
 *   - every function returns gdp_status (GDP_OK == 0; errors are negative);
 *     no exception or signal crosses the boundary;
 *   - after an error, gdp_last_error(ctx) describes it; output handles are
 *     set to NULL;
 *   - host arrays passed in are read during the call only (copied); the
 *     caller keeps ownership;
 *   - a gdp_mesh is owned by the library and lives in device memory until
 *     gdp_mesh_free;
 *   - one context is used by one host thread at a time (calls on the same
 *     context do not run concurrently);
 *   - vertex ids: input vertices keep their ids 0..n-1; Steiner vertices
 *     follow in insertion order; triangle vertices are counter-clockwise;
 *     edge i of triangle t joins vertex i and vertex (i+1) mod 3.
 */
#ifndef GDP2D_H
#define GDP2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GDP_OK = 0,
  GDP_E_ARG = -1,     /* invalid argument (NULL pointer, bad size, bad parameter) */
  GDP_E_INPUT = -2,   /* invalid PSLG: non-finite / out-of-range coordinate, duplicate
                         point, bad or repeated segment, crossing segments, a vertex in
                         a segment's interior, a hull edge that is not a segment */
  GDP_E_NOMEM = -3,   /* host or device allocation failed */
  GDP_E_DEVICE = -4,  /* a HIP call failed */
  GDP_E_NOTERM = -5,  /* max_rounds reached with work left; the mesh stays valid */
  GDP_E_STALL = -6,   /* a round had candidates but inserted nothing */
  GDP_E_BUSY = -7,    /* reserved */
  GDP_E_WALK = -8,    /* a point-location walk exceeded its step cap */
  GDP_E_CAVITY = -9   /* a cavity failed an internal consistency check (its fan did not
                         match its boundary; not expected for valid input) */
} gdp_status;

typedef struct gdp_ctx gdp_ctx;
typedef struct gdp_mesh gdp_mesh;

/* A PSLG: xy holds 2*n_vertices doubles (x0, y0, x1, y1, ...); seg holds
   2*n_segments vertex ids.  Every nonzero coordinate must have magnitude in
   [2^-100, 2^20].  The convex hull boundary must be covered by segments. */
typedef struct {
  int32_t n_vertices;
  const double *xy;
  int32_t n_segments;
  const int32_t *seg;
} gdp_pslg;

/* Refinement parameters.  The first group changes the mesh (semantic); the
   second only changes speed (every value gives a bit-identical mesh). */
typedef struct {
  /* semantic */
  int32_t cand_cap_K;       /* 0 = unlimited; else keep the K largest priorities per
                               round (Rule 2 filter as a candidate limit) */
  int32_t priority_mode;    /* 0: class|q(measure)|perm32(id); 1: class|perm32(id);
                               2: as 0 for subsegments; a triangle's tie-break is
                               its first two vertex ids from the smallest (22 bits
                               each, over q(measure) cut to 19 bits), so no key
                               depends on the slot a triangle occupies (needs
                               fewer than 2^22 vertices; Flip-Flop insertion
                               only, see insert_mode) */
  int32_t max_rounds;       /* 0 = no cap; else stop with GDP_E_NOTERM */
  int32_t prefilter_f1;     /* 1: keep one circumcenter per located triangle, the
                               largest key (Line 6 filter, Section 4.3) */
  int32_t cavity_approx_n;  /* 0 = off; 1..16: drop a circumcenter that does not hold
                               the largest key on the first n triangles of its
                               cavity growth order (Line 7 filter, Section 4.3) */
  /* perf only */
  int32_t block_size;       /* threads per workgroup for the per-element kernels
                               (64..1024, multiple of 64; 0 = default 256) */
  int32_t profile_kernels;  /* 1 = time every kernel launch with HIP events (adds
                               overhead; read with gdp_mesh_kernel_profile) */
  int32_t reserve_mode;     /* 0 = grow buffers before each group of rounds from the
                               last counts; 1 = grow only after a round was
                               abandoned for lack of room (then it is run again) */
  int32_t rounds_per_sync;  /* rounds queued on the stream between two host
                               synchronisations (1..64; 0 = automatic: one while
                               rounds are large, more as they shrink) */
  int32_t tail_engine_max;  /* rounds whose previous round had at most this many
                               candidates run whole inside one workgroup (0 =
                               default 1024; negative = never) */
  /* semantic (quality criteria of Section 4.1) */
  int32_t encroach_mode;    /* 0: a subsegment is encroached by a vertex or splitting
                               point strictly inside its diametric circle (Ruppert);
                               1: strictly inside its diametric lens, the points that
                               see it under more than 120 degrees (Chew) */
  int32_t split_mode;       /* 0: subsegments split at their midpoint; 1: concentric
                               shells: a subsegment with exactly one input-vertex
                               endpoint c is split at distance 2^j from c, 2^j the
                               power of two nearest to half its length */
  double max_edge_len_sq;   /* 0 = off; else l^2 for the edge-length bound l: a
                               triangle with an edge longer than l is bad too */
  /* perf only (batched form) */
  int32_t batch_engine_max_v; /* gdp_refine_batch: meshes with more input vertices
                               run in shared rounds (each phase one launch for all
                               of them, over the whole chip), the others one
                               workgroup each in the single-workgroup engine;
                               0 = every mesh in the engine */
  /* perf only */
  int32_t cavity_thread_cap;  /* per-thread cavity slots of the grid path (0 = 39;
                               12, 24 or 39): larger cavities go to the cooperative
                               path (Rule 3) */
  /* semantic */
  int32_t insert_mode;      /* Line 8 insertion.  0: Bowyer-Watson cavities with
                               priority marks and the dependency test (Section 5.2);
                               1: Flip-Flop (Section 4.3): every point kept by Line 6
                               (one point per split triangle, its largest key) is
                               added by splits, edges are flipped to the CDT, and
                               points joined to a point of larger key, or
                               circumcenters encroaching a subsegment opposite them
                               (flagged pending), are removed by flips and a flop,
                               until none is left.  Needs priority_mode 2 (triangles
                               end in slots of the flips' choosing); each triangle
                               is kept rotated so its smallest vertex comes first;
                               gdp_mesh_refine only (not the batched or serving
                               forms).  A refine call in this mode starts by
                               flipping the mesh to the CDT under the symbolic
                               perturbation of the lifting map. */
  /* perf only (batched form) */
  int32_t batch_line1_device_min_v; /* gdp_refine_batch: inputs with at least this
                               many vertices get their initial CDT (Line 1) from
                               the device builder of gdp_mesh_create_device (the
                               same CDT), on library threads with streams of their
                               own, while host threads build the others; 0 = every
                               input on the host */
} gdp_params;

/* Per-kernel totals of the last profiled gdp_mesh_refine. */
typedef struct {
  char name[24];
  int64_t launches;
  double total_ms;     /* sum of event-timed launch durations */
  int64_t items;       /* work items over all launches (triangles, candidates, ...) */
  int64_t alg_bytes;   /* algorithmic HBM bytes (k_scan and k_cavity_cc; 0 otherwise) */
} gdp_kernel_prof;

typedef struct {
  int32_t n_vertices, n_triangles, n_subsegments;
  int32_t n_input_vertices, n_input_segments;
  int32_t rounds;
  /* rounds of the device CDT builder that made the mesh (point insertion,
     segment recovery); 0 for meshes built on the host or uploaded */
  int32_t cdt_point_rounds, cdt_segment_rounds;
  /* FP64 filter fallbacks of the last gdp_mesh_refine: predicate calls whose
     floating-point filter could not decide the sign and that were evaluated
     exactly (orient2d, diametral test, incircle; the per-stage split is in
     gdp_round_stats) */
  int64_t fallbacks;
} gdp_mesh_info;

/* Per-round counters (device-side counts copied back after every round). */
typedef struct {
  int64_t n_enc, n_bad, n_kept_mid, n_kept_cc;
  int64_t n_blocked, n_coincident, n_enc_reject, n_mid_cand, n_unsplittable;
  int64_t n_fan_invalid, n_lost_mark, n_dep_drop, n_ins_mid, n_ins_cc;
  int64_t cav_tri_total, cav_max, n_big_cavities;
  int64_t n_f1_drop, n_f2_drop;
  /* predicate calls: incircle tests of cavity growth and of the dependency
     test; orient2d tests of the walk (three per step) and of the fan check */
  int64_t n_incircle_tests, n_orient_tests;
  /* of those, evaluated exactly after the FP64 filter failed, per stage:
     orient2d, diametral dot product, incircle on exact coordinate
     differences, incircle on raw coordinates */
  int64_t n_exact_orient, n_exact_dot, n_exact_incircle_b, n_exact_incircle_c;
  /* the inserted points (all classes): sum of cavity sizes |C|, of fan
     (boundary) edges b, and of the walk steps of the circumcenters; then |C|
     and b of the circumcenters alone.  With these the memory work of a
     sequential insertion of the same points can be priced. */
  int64_t win_cav_tri, win_fan_edges, win_walk_steps, win_cc_cav_tri, win_cc_fan_edges;
  /* cooperative cavities that outgrew the workgroup's local list and were
     finished in device memory */
  int64_t n_huge_cavities;
  /* priority marks placed (64-bit atomicMax, one per cavity triangle of a
     valid cavity): midpoint cavities, circumcenter cavities */
  int64_t n_marks_mid, n_marks_cc;
  /* Flip-Flop rounds (insert_mode 1): points added in Line 8, CDTs examined
     for redundant points, 2-2 flips, flip passes, points removed, removal
     passes */
  int64_t n_ff_points, n_ff_iters, n_flips, n_flip_passes, n_removals, n_removal_passes;
} gdp_round_stats;

/* Fills *p with the defaults (all zero, block_size 256). */
void gdp_params_default(gdp_params *p);

/* Creates a context on HIP device `device`, issuing work on `hip_stream`
   (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL means
   the default stream).  The stream must outlive the context. */
gdp_status gdp_ctx_create(int device, void *hip_stream, gdp_ctx **out);
void gdp_ctx_destroy(gdp_ctx *ctx);
const char *gdp_last_error(const gdp_ctx *ctx);
const char *gdp_status_str(gdp_status s);

/* Line 1 of Algorithm 1 on the host: builds the canonical constrained
   Delaunay triangulation of *pslg (cocircular ties broken by a symbolic
   perturbation in which a smaller vertex id dominates; triangles rotated so
   the smallest id comes first and sorted lexicographically) and uploads it
   to the device.  Subsegment k of the result is input segment k. */
gdp_status gdp_mesh_create(gdp_ctx *ctx, const gdp_pslg *pslg, gdp_mesh **out);

/* Line 1 of Algorithm 1 on the device (Section 4.3 names the initial CDT as
   the first step; Section 7.1 builds it on the CPU): the same canonical CDT
   as gdp_mesh_create, element for element, built by kernels on the context
   stream from the host arrays of *pslg (copied to the device; the caller
   keeps ownership).  Points are inserted by rounds of parallel
   Bowyer-Watson insertion, missing segments recovered by rounds of
   pseudo-polygon retriangulation.  Blocks until done.  Errors:
   GDP_E_ARG (NULL, fewer than 3 vertices), GDP_E_INPUT (invalid PSLG: the
   host builder's checks; its message may differ), GDP_E_NOMEM,
   GDP_E_DEVICE.  Cavities of any size are handled (one larger than a
   round's per-point lists waits for a round of its own).  On error
   *out = NULL. */
gdp_status gdp_mesh_create_device(gdp_ctx *ctx, const gdp_pslg *pslg, gdp_mesh **out);

/* Same CDT, host only (no device needed).  Writes the counts to *n_tri and,
   when the pointers are non-NULL and cap_tri >= *n_tri, tri/nbr/seg
   (3 * n_tri int32 each: vertices, neighbour across edge i or -1, segment id
   on edge i or -1).  Call once with cap_tri = 0 to size the buffers. */
gdp_status gdp_cdt_host(const gdp_pslg *pslg, int32_t *n_tri, int32_t cap_tri, int32_t *tri,
                        int32_t *nbr, int32_t *seg, char *err, int32_t err_len);

/* Uploads a mesh given as arrays (e.g. a state saved at a round boundary):
   xy[2V], vkind[V], tri/nbr/sub_on_edge[3T], sub_v[2S], sub_parent[S],
   sub_pending[S] (0/1), plus the counts and the round number.  Shapes and
   index ranges are checked; geometry is not. */
gdp_status gdp_mesh_upload(gdp_ctx *ctx, int32_t n_v, int32_t n_input_v, const double *xy,
                           const int32_t *vkind, int32_t n_t, const int32_t *tri,
                           const int32_t *nbr, const int32_t *sub_on_edge, int32_t n_s,
                           int32_t n_input_s, const int32_t *sub_v, const int32_t *sub_parent,
                           const uint8_t *sub_pending, int32_t rounds, gdp_mesh **out);

/* Lines 2-9 of Algorithm 1 on the GPU, in place, until no encroached
   subsegment or bad triangle remains.  ratio_bound_sq is B^2 passed exactly
   (B = sqrt(2) -> 2.0): a triangle is bad when its FP64 circumradius^2
   exceeds ratio_bound_sq times its shortest edge^2.  Blocks until done. */
gdp_status gdp_mesh_refine(gdp_ctx *ctx, gdp_mesh *mesh, double ratio_bound_sq,
                           const gdp_params *params);

/* gdp_mesh_create followed by gdp_mesh_refine. */
gdp_status gdp_refine(gdp_ctx *ctx, const gdp_pslg *pslg, double ratio_bound_sq,
                      const gdp_params *params, gdp_mesh **out);

gdp_status gdp_mesh_info_get(const gdp_mesh *mesh, gdp_mesh_info *info);

/* The quality of a mesh under the criteria of Section 4.1 (the same FP64
   test as the refinement's scan, with bound ratio_bound_sq and, if
   max_edge_len_sq > 0, the edge-length bound): *n_bad gets the number of bad
   triangles and *bad_area the area they cover (the bad-area measure of
   Table 1: half the FP64 doubled area of each, summed on the device in a
   fixed order per launch shape).  Bad triangles remain near input angles
   below 60 degrees.  Computed by kernels on the context stream; blocks until
   done.  GDP_E_ARG for a bad bound or null output. */
gdp_status gdp_mesh_quality(gdp_ctx *ctx, const gdp_mesh *mesh, double ratio_bound_sq, double max_edge_len_sq,
                            int64_t *n_bad, double *bad_area);

/* Zero-copy view of a mesh in device memory (Section 4.1: the output is the
   refined CDT with its Steiner vertices and subsegments).  Every pointer is a
   device address on the mesh's context device; the arrays belong to the
   library and stay valid until the mesh is freed or passed to a call that
   modifies it (gdp_mesh_refine, gdp_mesh_assign), which may move them.  A
   caller may wrap them (e.g. as torch tensors) without taking ownership.
   Layout, counts as in gdp_mesh_info:
     xy          : 2V doubles, x then y of each vertex;
     vkind       : V int32 (0 input, 1 midpoint, 2 circumcenter);
     tri         : 4T int32, (v0, v1, v2, m) per triangle, counter-clockwise,
                   bit i of m set when edge i (v_i, v_{i+1 mod 3}) is a subsegment;
     nbr         : 4T int32, (n0, n1, n2, 0): the triangle across edge i or -1;
     sub_on_edge : 4T int32, (s0, s1, s2, 0): the subsegment on edge i or -1;
     sub_v       : 2S int32 endpoints; sub_parent: S int32 input segment;
     sub_pending : S int32 (0/1).
   GDP_E_ARG for a NULL argument. */
typedef struct {
  int32_t n_vertices, n_triangles, n_subsegments;
  int32_t tri_stride; /* int32 per triangle record: 4 */
  const double *xy;
  const int32_t *vkind;
  const int32_t *tri;
  const int32_t *nbr;
  const int32_t *sub_on_edge;
  const int32_t *sub_v;
  const int32_t *sub_parent;
  const int32_t *sub_pending;
} gdp_device_views;
gdp_status gdp_mesh_device_views(const gdp_mesh *mesh, gdp_device_views *out);

/* The refinement's geometric predicates (Section 4.1 and Section 4.2:
   circumcircle and diametral-circle tests; Section 7: exact arithmetic),
   evaluated for testing on n queries of one kind, in the same code the
   kernels run:
     kind 0: orient2d(a, b, c)           pts: 6 doubles per query (ax ay bx by cx cy),
             signs[i] = 1 counter-clockwise, -1 clockwise, 0 collinear;
     kind 1: incircle(a, b, c, d)         8 doubles; 1 if d is strictly inside the
             circle through a, b, c (counter-clockwise), -1 outside, 0 on it;
     kind 2: indiametral(a, b, c)         6 doubles; 1 if c is strictly inside the
             circle with diameter ab, -1 outside, 0 on it;
     kind 3: lens encroachment of ab by c 6 doubles; 1 if c is strictly inside the
             diametric lens of ab (the points seeing ab under more than 120
             degrees), else 0.
   ctx non-NULL: one thread per query on the context's device and stream
   (blocks until done; host arrays are copied); ctx NULL: on the host.
   stage_counts (optional, 4 entries) receives the exact evaluations made,
   per stage: orient2d, diametral dot product, incircle on exact differences,
   incircle on raw coordinates.  Coordinates must satisfy the range of
   gdp_pslg.  GDP_E_ARG for a bad kind, n < 0 or NULL arrays with n > 0. */
gdp_status gdp_predicates_eval(gdp_ctx *ctx, int32_t kind, int32_t n, const double *pts, int32_t *signs,
                               int64_t *stage_counts);

/* Measurement of the conflict step's memory pattern (Section 5.2: each
   cavity triangle takes the largest priority of the cavities that hold it,
   here a 64-bit atomicMax): n_ops atomicMax operations on random slots of a
   table of n_slots 64-bit words in device memory, one thread per operation
   in a grid-stride loop.  *ms gets the device time of the timed launch (a
   first launch warms the table).  Blocks until done.  GDP_E_ARG for
   non-positive sizes, GDP_E_NOMEM when the table does not fit. */
gdp_status gdp_bench_atomic_max(gdp_ctx *ctx, int64_t n_slots, int64_t n_ops, double *ms);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops that forbid allocation): gdp_mesh_quality without
   any allocation and without blocking.  The two results go to caller device
   memory (*d_n_bad, *d_bad_area) on the context stream, equal to
   gdp_mesh_quality's; the per-workgroup partial sums live in a static
   device array of the library (16 KB per device, resolved when a context is
   created on the device).  Calls that overlap on one device share that
   array and race: serialise them (e.g. one stream).  GDP_E_ARG for a bad
   bound, NULL pointers, or partials beyond the array (not reachable with
   the fixed grid of at most 512 workgroups); GDP_E_DEVICE if the array's
   address could not be resolved or a launch failed. */
gdp_status gdp_mesh_quality_noalloc(gdp_ctx *ctx, const gdp_mesh *mesh, double ratio_bound_sq,
                                    double max_edge_len_sq, unsigned long long *d_n_bad, double *d_bad_area);

/* Copies the mesh to caller buffers sized from gdp_mesh_info_get (any pointer
   may be NULL to skip that array): xy[2V], vkind[V] (0 input, 1 midpoint,
   2 circumcenter), tri/nbr/sub_on_edge[3T], sub_v[2S], sub_parent[S] (input
   segment of each subsegment), sub_pending[S]. */
gdp_status gdp_mesh_download(gdp_ctx *ctx, const gdp_mesh *mesh, double *xy, int32_t *vkind,
                             int32_t *tri, int32_t *nbr, int32_t *sub_on_edge, int32_t *sub_v,
                             int32_t *sub_parent, uint8_t *sub_pending);

/* Copies up to cap per-round records of the last gdp_mesh_refine; *n gets
   the number of rounds recorded. */
gdp_status gdp_mesh_round_stats(const gdp_mesh *mesh, gdp_round_stats *stats, int32_t cap,
                                int32_t *n);

/* Device-resident refinement timing of the last gdp_mesh_refine:
   *ms = wall time between HIP events recorded before the first and after the
   last round on the context stream. */
gdp_status gdp_mesh_last_refine_ms(const gdp_mesh *mesh, double *ms);

/* Kernel timing table of the last refine run with profile_kernels = 1:
   writes up to cap records, *n gets the number of kernel kinds. */
gdp_status gdp_mesh_kernel_profile(const gdp_mesh *mesh, gdp_kernel_prof *out, int32_t cap, int32_t *n);

/* Batched form: refines count independent PSLGs (pslgs[i] with bound
   ratio_bound_sq[i], the same params for all).  Line 1 runs on the host for
   every input (in parallel), then every mesh is refined by Lines 2-9 in one
   persistent launch in which each workgroup takes meshes from a queue,
   largest first, and runs every round of a mesh by itself.  Each mesh is
   bit-identical to gdp_refine on the same input.  outs[i] receives the mesh
   (free with gdp_mesh_free; the meshes of a batch share one device
   allocation, released with the last of them) or NULL if status[i]
   (optional, count entries) is an error; status[i] = GDP_E_NOTERM keeps the
   mesh.  A mesh that outgrows its estimated room is refined again on its
   own.  *elapsed_ms (optional) receives the device time of the launch.
   Returns GDP_OK unless the call itself failed. */
gdp_status gdp_refine_batch(gdp_ctx *ctx, const gdp_pslg *pslgs, const double *ratio_bound_sq,
                            const gdp_params *params, int32_t count, gdp_mesh **outs, gdp_status *status,
                            double *elapsed_ms);

/* ---- Serving form ----------------------------------------------------------
   A server refines meshing jobs as they arrive, with continuous batching:
   arrived jobs are admitted while there is a free slot and room in the
   server's device memory (each job's region is sized from its initial CDT),
   admitted jobs are refined at once, side by side on the device, and
   finished jobs leave, freeing their slot and region for the next arrival.
   By default (mode 0) the rounds are shared (Rule 4 of Section 2: groups of
   work merged into one launch): one library thread runs the rounds of every
   active job together, one kernel launch per phase of the round for all of
   them, and jobs join and leave between groups of two rounds.  In mode 1
   each admitted job runs its rounds on a slot of its own (one stream and one
   library thread per slot).  With gdp_server_engine_jobs, small jobs are
   instead refined together, one workgroup each, in launches of the
   single-workgroup engine.  Each result is bit-identical to gdp_refine on
   the same input.  A job that outgrows its region is refined
   again on its own.  Latency is measured from arrival.  Line 1 (the initial
   CDT, Section 4.3) runs by default in the caller's thread at prepare, before
   arrival; with gdp_server_line1 it runs in the server after arrival (and so
   counts in the latency), on host threads or, for large jobs, by the device
   builder of gdp_mesh_create_device. */
typedef struct gdp_server gdp_server;

typedef struct {
  double submit_ms;  /* arrival, ms since the server was created */
  double line1_ms;   /* end of Line 1 in the server (0 when it ran at prepare) */
  double admit_ms;   /* admission into a slot */
  double done_ms;    /* completion */
} gdp_job_times;

/* hbm_budget: bytes of device memory for job regions; max_slots: jobs active
   at once (in the shared rounds, or on their own streams in mode 1). */
gdp_status gdp_server_create(gdp_ctx *ctx, size_t hbm_budget, int32_t max_slots, gdp_server **out);
/* mode 0: shared rounds (default); 1: a stream and a thread per slot.
   Applies to jobs admitted afterwards.  rounds_per_group (perf only): shared
   rounds run between two reads of the jobs' states, 1..8, 0 = default 2
   (jobs join and leave only between groups).  GDP_E_ARG for other values. */
gdp_status gdp_server_mode(gdp_server *srv, int32_t mode, int32_t rounds_per_group);
/* Jobs with at most max_input_vertices input vertices go to the batched
   launches (0: every job takes a slot).  Applies to jobs admitted afterwards.
   GDP_E_ARG for a negative value. */
gdp_status gdp_server_engine_jobs(gdp_server *srv, int32_t max_input_vertices);
/* Line 1 inside the server (Section 4.3 Line 1, the initial CDT): from now on
   gdp_server_prepare only copies the job's input (checking its coordinates
   and segment endpoints), and Line 1 runs after arrival: on one of
   host_threads (1..64) library threads, or, for a job with at least
   device_min_vertices input vertices (0: never), on the device by the kernels
   of gdp_mesh_create_device (the same CDT), on a library thread and stream of
   its own that takes the job's region first and builds the CDT inside it
   (such jobs then run in the shared rounds whatever the mode).  A Line-1
   failure ends the job with its status (GDP_E_INPUT for an invalid PSLG).
   Must be called before the first job is prepared: GDP_E_BUSY otherwise;
   GDP_E_ARG for values out of range. */
gdp_status gdp_server_line1(gdp_server *srv, int32_t host_threads, int32_t device_min_vertices);
/* Line 1 for a job (host) without letting it arrive, unless gdp_server_line1
   moved it into the server; *job identifies it. */
gdp_status gdp_server_prepare(gdp_server *srv, const gdp_pslg *pslg, double ratio_bound_sq,
                              const gdp_params *params, uint64_t *job);
/* The prepared job arrives: it is queued for admission (first come, first served). */
gdp_status gdp_server_arrive(gdp_server *srv, uint64_t job);
/* gdp_server_prepare followed by gdp_server_arrive. */
gdp_status gdp_server_submit(gdp_server *srv, const gdp_pslg *pslg, double ratio_bound_sq,
                             const gdp_params *params, uint64_t *job);
/* GDP_E_BUSY while the job is not finished (*out = NULL).  Once finished the
   job's status is returned, *out receives its mesh (the caller owns it and
   frees it with gdp_mesh_free; NULL on error) and the job id is released.
   *times (optional) is filled either way. */
gdp_status gdp_server_poll(gdp_server *srv, uint64_t job, gdp_mesh **out, gdp_job_times *times);
/* gdp_server_poll that blocks until the job has finished (a prepared job
   must still arrive; GDP_E_BUSY if the server is being destroyed first). */
gdp_status gdp_server_wait(gdp_server *srv, uint64_t job, gdp_mesh **out, gdp_job_times *times);
/* Finishes every job that has arrived, frees the jobs nobody took, stops the
   worker.  Meshes already handed out stay valid. */
void gdp_server_destroy(gdp_server *srv);

/* Copies the state of src (vertices, triangles, subsegments, counters) into
   dst on the device, growing dst only if it is too small; both meshes must
   belong to ctx.  Used to restart refinement from a resident initial CDT. */
gdp_status gdp_mesh_assign(gdp_ctx *ctx, gdp_mesh *dst, const gdp_mesh *src);

/* New device mesh with the same state and capacities as src. */
gdp_status gdp_mesh_clone(gdp_ctx *ctx, const gdp_mesh *src, gdp_mesh **out);

void gdp_mesh_free(gdp_mesh *mesh);

#ifdef __cplusplus
}
#endif
#endif

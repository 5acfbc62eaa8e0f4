/*
 * orc.h -- CPU oracle for round-synchronous 2D constrained Delaunay refinement.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference that the GPU path is compared against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never links, includes or calls anything here.
 *
 * What it computes (Chen, Tan, Ong, "On Designing GPU Algorithms with
 * Applications to Mesh Refinement"):
 *   - Line 1 of Algorithm 1 (gDP2d): the constrained Delaunay triangulation of
 *     the input PSLG (Section 4, definitions of PSLG / subsegment / CDT).
 *     Cocircular ties are broken by a symbolic perturbation of the lifting
 *     map, so the CDT is unique and canonical.
 *   - Lines 2-9 of Algorithm 1 as a deterministic round: collect encroached
 *     subsegments and bad triangles, compute midpoints / circumcenters,
 *     prioritize and locate by walking (midpoint replacement when a subsegment
 *     blocks the walk), grow Bowyer-Watson cavities, resolve overlaps by
 *     priority marks and the Delaunay-dependency test of Section 5 (gQM3d
 *     insertion), and insert the winners.
 * Every arithmetic step is plain: exact signs come from multi-precision
 * integers, the floating-point formulas are evaluated in one fixed order
 * (build with -ffp-contract=off).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_ARG = -1,
  ORC_E_INPUT = -2,
  ORC_E_NOMEM = -3,
  ORC_E_NOTERM = -5, /* round cap reached with work left; mesh is valid */
  ORC_E_STALL = -6,  /* a round had candidates but inserted nothing */
  ORC_E_WALK = -8    /* a locate walk exceeded its step cap */
};

/* Vertex kinds. */
enum { ORC_VK_INPUT = 0, ORC_VK_MIDPOINT = 1, ORC_VK_CIRCUMCENTER = 2 };

typedef struct orc_mesh {
  int32_t nV, nT, nS;          /* live counts */
  int32_t n_input_v, n_input_s;
  int32_t capV, capT, capS;
  int32_t rounds;              /* rounds executed so far */
  double *x, *y;               /* [capV] */
  int32_t *vkind;              /* [capV] */
  int32_t *tv, *tn, *ts;       /* [3*capT]: vertices (CCW), neighbour across edge i,
                                  subsegment id on edge i (-1 none); edge i = (tv[i], tv[i+1]) */
  int32_t *sv;                 /* [2*capS]: subsegment endpoints (sv0, sv1) */
  int32_t *sparent;            /* [capS]: input segment id */
  uint8_t *spend;              /* [capS]: pending-split flag carried to the next round */
} orc_mesh;

typedef struct orc_params {
  int32_t cand_cap_K;     /* 0 = unlimited; else keep the K largest keys per round */
  int32_t priority_mode;  /* 0: class|q(measure)|perm32(id); 1: class|perm32(id);
                             2: as 0 for subsegments, and for triangles
                             q(measure) reduced to 19 bits | first two vertex
                             ids of the triangle (smallest first), 22 bits
                             each: a key that does not depend on the slot */
  int32_t max_rounds;     /* stop after this many rounds (ORC_E_NOTERM if work left) */
  int32_t prefilter_f1;   /* 1: keep one circumcenter per located triangle (max key) */
  int32_t cavity_approx_n;/* n > 0: drop circumcenters that lose a mark on the first
                             n triangles of their cavity growth order */
  int32_t encroach_mode;  /* 0: diametric circle (Ruppert); 1: diametric lens (Chew) */
  int32_t split_mode;     /* 0: subsegment midpoints; 1: concentric shells around input
                             vertices (see orc_midpoint) */
  double max_edge_len_sq; /* 0 = off; else a triangle with an edge longer than l
                             (squared length > l^2) is bad as well */
  int32_t insert_mode;    /* 0: cavities, marks and the dependency test (Section 5.2);
                             1: Flip-Flop (Section 4.3 Line 8, see orc_ff.c);
                             needs priority_mode 2 */
} orc_params;

typedef struct orc_round_stats {
  int64_t n_enc, n_bad, n_kept_mid, n_kept_cc;
  int64_t n_blocked, n_coincident, n_enc_reject, n_mid_cand, n_unsplittable;
  int64_t n_fan_invalid, n_lost_mark, n_dep_drop, n_ins_mid, n_ins_cc;
  int64_t cav_tri_total, cav_max, walk_steps;
  int64_t n_f1_drop, n_f2_drop;
  int64_t n_ff_points, n_ff_iters; /* Flip-Flop: points added in Line 8, CDTs examined */
} orc_round_stats;

/* Builds the canonical CDT of the PSLG.  xy: 2*nv doubles; seg: 2*ns vertex ids.
   On error returns ORC_E_INPUT / ORC_E_ARG and writes a message to err. */
int orc_cdt_build(int32_t nv, const double *xy, int32_t ns, const int32_t *seg,
                  orc_mesh **out, char *err, int32_t errlen);

/* Runs refinement rounds in place.  stats (optional) receives one record per
   executed round, up to stats_cap records; *n_stats gets the count. */
int orc_refine(orc_mesh *m, double ratio_bound_sq, const orc_params *p,
               orc_round_stats *stats, int32_t stats_cap, int32_t *n_stats,
               char *err, int32_t errlen);

orc_mesh *orc_mesh_clone(const orc_mesh *m);
/* A mesh from caller arrays (copied; no check): xy[2nv], vkind[nv],
   tv/tn/ts[3nt], sv[2ns], sparent[ns], spend[ns].  NULL on failure. */
orc_mesh *orc_mesh_from_arrays(int32_t nv, int32_t n_input_v, const double *xy, const int32_t *vkind,
                               int32_t nt, const int32_t *tv, const int32_t *tn, const int32_t *ts,
                               int32_t ns, int32_t n_input_s, const int32_t *sv, const int32_t *sparent,
                               const uint8_t *spend);

/* Classic sequential Ruppert refinement of a CDT in place (one insertion at
   a time from a priority queue, insertion by Lawson flips; the sequential
   point-count reference, Ruppert mode, midpoint splits).  max_insertions > 0
   caps the Steiner points (ORC_E_NOTERM when reached).  The mesh keeps the
   orc_mesh conventions (CCW triangles, neighbours, subsegment ids) but not
   the round oracle's slot order. */
int orc_ruppert(orc_mesh *m, double ratio_bound_sq, int64_t max_insertions, int64_t *n_unsplittable,
                char *err, int32_t errlen);
void orc_mesh_free(orc_mesh *m);

/* Exact predicates on FP64 points (p = {x, y}); return -1, 0 or +1. */
int orc_orient2d(const double *a, const double *b, const double *c);
int orc_incircle(const double *a, const double *b, const double *c, const double *d);
int orc_indiametral(const double *a, const double *b, const double *c);
/* Does p encroach subsegment ab?  mode 0: strictly inside the diametric
   circle (exact).  mode 1: strictly inside the diametric lens, the region
   from which ab is seen under more than 120 degrees (exact circle test,
   then a fixed-order FP64 test of the angle). */
int orc_encroaches(int32_t mode, const double *a, const double *b, const double *p);
/* incircle with the symbolic-perturbation tie-break (vertex ids ia..id). */
int orc_incircle_sos(const double *a, const double *b, const double *c, const double *d,
                     int32_t ia, int32_t ib, int32_t ic, int32_t id);
/* Counts of exact (multi-precision) evaluations since load. */
void orc_exact_counts(int64_t *orient, int64_t *incircle, int64_t *indiam);

/* Fixed-order FP64 formulas (refinement Line 5 / Line 6). */
uint32_t orc_perm32(uint32_t x);
void orc_circumcenter(const orc_mesh *m, int32_t t, double ratio_bound_sq, double max_edge_len_sq,
                      double *px, double *py, int32_t *bad, uint64_t *key,
                      int32_t priority_mode);
void orc_midpoint(const orc_mesh *m, int32_t k, double *mx, double *my, uint64_t *key,
                  int32_t priority_mode, int32_t split_mode);

/* Checkers.  Each returns the number of violations found. */
int64_t orc_check_topology(const orc_mesh *m, char *err, int32_t errlen);
int64_t orc_check_local_delaunay(const orc_mesh *m);
int64_t orc_check_quality(const orc_mesh *m, double ratio_bound_sq, double max_edge_len_sq);
int64_t orc_check_encroached(const orc_mesh *m, int32_t encroach_mode);
/* Bad triangles of a mesh under the criteria and the area they cover (the
   bad-area measure of Table 1): each bad triangle adds half its fixed-order
   FP64 doubled area, summed in slot order. */
void orc_mesh_quality(const orc_mesh *m, double ratio_bound_sq, double max_edge_len_sq, int64_t *n_bad,
                      double *bad_area);
int64_t orc_check_cdt_bruteforce(const orc_mesh *m);
int64_t orc_check_subsegments(const orc_mesh *m, const double *in_xy, const int32_t *in_seg,
                              char *err, int32_t errlen);
double orc_area_sum(const orc_mesh *m);
int32_t orc_hull_vertex_count(const orc_mesh *m);

#ifdef __cplusplus
}
#endif
#endif

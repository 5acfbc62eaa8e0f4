/*
 * orc_ruppert.c -- a classic sequential Ruppert refinement (oracle side).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Purpose: an independent point count for the round-synchronous oracle.  The
 * paper compares the number of points its parallel refinement outputs with
 * a sequential refiner's on the same input (Table 1: gDP2d against Triangle,
 * 0.96-1.10 times as many output points); this file is the sequential side
 * of that comparison.  It shares only the exact predicates and the CDT input
 * with the round oracle: its own priority queue, its own point location, its
 * own insertion (Lawson flips after a 1-3 or 2-4 split instead of
 * Bowyer-Watson cavities) and its own circumcenter formula.
 *
 * The method (Ruppert's algorithm as Section 4.2 states its rules):
 *   - one element at a time from a max-priority queue; subsegments come
 *     before triangles, longer subsegments / larger triangles first
 *     (the priorities of Section 4.3);
 *   - an encroached subsegment (a vertex strictly inside its diametric
 *     circle; the apex test on the two adjacent triangles) is split at its
 *     midpoint;
 *   - a bad triangle (circumradius^2 > B^2 * shortest edge^2) is split at its
 *     circumcenter, unless the circumcenter would encroach a subsegment
 *     (one on the boundary of its conflict region), or lies beyond a
 *     subsegment seen from the triangle: then those subsegments are split
 *     instead and the triangle waits in the queue;
 *   - after an insertion the triangles around the new vertex and the
 *     subsegments opposite it are tested and queued.
 * Ties in the predicates follow strict inequalities (a point on a circle is
 * outside it), as in the round oracle.
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NXT(i) (((i) + 1) % 3)
#define PRV(i) (((i) + 2) % 3)

typedef struct {
  int cls;          /* 1 subsegment, 0 triangle */
  double measure;   /* length^2 of the subsegment, doubled area of the triangle */
  int32_t id;       /* subsegment id or triangle slot */
  int32_t a, b, c;  /* the element's vertices when queued (stale check) */
  int forced;       /* subsegment: split even if no vertex encroaches it now */
  int retries;      /* triangle: times its circumcenter was rejected */
} qent;

typedef struct {
  orc_mesh *m;
  int32_t *vtri;    /* a triangle incident to each vertex */
  int32_t capVT;
  qent *heap;
  int64_t nh, caph;
  int32_t *stack, nstack, capstack;
  int32_t *touched, ntouched, captouched;
  int32_t *cav, ncav, capcav;
  int32_t *mark;    /* per-triangle epoch stamp for the conflict flood */
  int32_t capmark, epoch;
  double B2;
  int64_t n_unsplittable, n_coincident, n_given_up;
} rstate;

static int grow_i32(int32_t **a, int32_t *cap, int64_t need) {
  if (need <= *cap) return 0;
  int64_t c = *cap ? *cap : 256;
  while (c < need) c *= 2;
  int32_t *p = realloc(*a, sizeof(int32_t) * (size_t)c);
  if (!p) return -1;
  *a = p;
  *cap = (int32_t)c;
  return 0;
}

static int mesh_room(rstate *S, int32_t needV, int32_t needT, int32_t needS) {
  orc_mesh *m = S->m;
  if (needV > m->capV) {
    int32_t c = m->capV * 2 + 16;
    while (c < needV) c *= 2;
    double *x = realloc(m->x, sizeof(double) * (size_t)c);
    if (!x) return -1;
    m->x = x;
    double *y = realloc(m->y, sizeof(double) * (size_t)c);
    if (!y) return -1;
    m->y = y;
    int32_t *k = realloc(m->vkind, sizeof(int32_t) * (size_t)c);
    if (!k) return -1;
    m->vkind = k;
    m->capV = c;
  }
  if (needV > S->capVT) {
    int32_t c = S->capVT * 2 + 16;
    while (c < needV) c *= 2;
    int32_t *p = realloc(S->vtri, sizeof(int32_t) * (size_t)c);
    if (!p) return -1;
    S->vtri = p;
    S->capVT = c;
  }
  if (needT > m->capT) {
    int32_t c = m->capT * 2 + 16;
    while (c < needT) c *= 2;
    int32_t *p;
    if (!(p = realloc(m->tv, sizeof(int32_t) * 3 * (size_t)c))) return -1;
    m->tv = p;
    if (!(p = realloc(m->tn, sizeof(int32_t) * 3 * (size_t)c))) return -1;
    m->tn = p;
    if (!(p = realloc(m->ts, sizeof(int32_t) * 3 * (size_t)c))) return -1;
    m->ts = p;
    m->capT = c;
  }
  if (needT > S->capmark) {
    int32_t old = S->capmark;
    if (grow_i32(&S->mark, &S->capmark, needT)) return -1;
    for (int32_t t = old; t < S->capmark; t++) S->mark[t] = 0;
  }
  if (needS > m->capS) {
    int32_t c = m->capS * 2 + 16;
    while (c < needS) c *= 2;
    int32_t *p;
    if (!(p = realloc(m->sv, sizeof(int32_t) * 2 * (size_t)c))) return -1;
    m->sv = p;
    if (!(p = realloc(m->sparent, sizeof(int32_t) * (size_t)c))) return -1;
    m->sparent = p;
    uint8_t *q = realloc(m->spend, (size_t)c);
    if (!q) return -1;
    m->spend = q;
    m->capS = c;
  }
  return 0;
}

/* ---- priority queue: subsegments first, then larger measure, then smaller id ---- */
static int qless(const qent *x, const qent *y) {
  if (x->cls != y->cls) return x->cls < y->cls;
  if (x->measure != y->measure) return x->measure < y->measure;
  return x->id > y->id;
}

static int qpush(rstate *S, const qent *e) {
  if (S->nh + 1 > S->caph) {
    int64_t c = S->caph ? S->caph * 2 : 1024;
    qent *h = realloc(S->heap, sizeof(qent) * (size_t)c);
    if (!h) return -1;
    S->heap = h;
    S->caph = c;
  }
  int64_t i = S->nh++;
  S->heap[i] = *e;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!qless(&S->heap[p], &S->heap[i])) break;
    qent t = S->heap[p];
    S->heap[p] = S->heap[i];
    S->heap[i] = t;
    i = p;
  }
  return 0;
}

static qent qpop(rstate *S) {
  qent top = S->heap[0];
  S->heap[0] = S->heap[--S->nh];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, g = i;
    if (l < S->nh && qless(&S->heap[g], &S->heap[l])) g = l;
    if (r < S->nh && qless(&S->heap[g], &S->heap[r])) g = r;
    if (g == i) break;
    qent t = S->heap[g];
    S->heap[g] = S->heap[i];
    S->heap[i] = t;
    i = g;
  }
  return top;
}

static inline void P(const orc_mesh *m, int32_t v, double *p) { p[0] = m->x[v]; p[1] = m->y[v]; }

/* Circumcenter relative to the triangle's first vertex, by the textbook
   formula with the determinant D = 2 * ((b-a) x (c-a)); also the circumradius
   squared and the shortest edge squared. */
static void tri_geom(const orc_mesh *m, int32_t t, double *ox, double *oy, double *r2, double *l2,
                     double *area2) {
  const int32_t *v = &m->tv[3 * t];
  double ax = m->x[v[0]], ay = m->y[v[0]];
  double bx = m->x[v[1]] - ax, by = m->y[v[1]] - ay;
  double cx = m->x[v[2]] - ax, cy = m->y[v[2]] - ay;
  double D = 2.0 * (bx * cy - by * cx);
  double bb = bx * bx + by * by, cc = cx * cx + cy * cy;
  double ux = (cy * bb - by * cc) / D, uy = (bx * cc - cx * bb) / D;
  double dx = cx - bx, dy = cy - by, dd = dx * dx + dy * dy;
  double l = bb < cc ? bb : cc;
  if (dd < l) l = dd;
  *ox = ax + ux;
  *oy = ay + uy;
  *r2 = ux * ux + uy * uy;
  *l2 = l;
  *area2 = D * 0.5;
}

/* Triangles whose FP64 area is not positive have no usable circumcenter and
   are left alone (none arise on the inputs this is run on). */
static int queue_tri_retry(rstate *S, int32_t t, int retries) {
  double ox, oy, r2, l2, a2;
  tri_geom(S->m, t, &ox, &oy, &r2, &l2, &a2);
  if (!(a2 > 0.0) || !(r2 > S->B2 * l2)) return 0;
  qent e = {0, a2, t, S->m->tv[3 * t], S->m->tv[3 * t + 1], S->m->tv[3 * t + 2], 0, retries};
  return qpush(S, &e);
}

static int queue_tri(rstate *S, int32_t t) { return queue_tri_retry(S, t, 0); }

static int queue_seg(rstate *S, int32_t k, int forced) {
  const orc_mesh *m = S->m;
  int32_t a = m->sv[2 * k], b = m->sv[2 * k + 1];
  double dx = m->x[b] - m->x[a], dy = m->y[b] - m->y[a];
  qent e = {1, dx * dx + dy * dy, k, a, b, -1, forced, 0};
  return qpush(S, &e);
}

/* The triangle holding the directed edge (a, b): rotate around a. */
static int find_edge(rstate *S, int32_t a, int32_t b, int32_t *tout, int *iout) {
  const orc_mesh *m = S->m;
  int32_t t0 = S->vtri[a];
  for (int dir = 0; dir < 2; dir++) {
    int32_t t = t0;
    for (int64_t guard = 0; t >= 0 && guard < (int64_t)m->nT + 4; guard++) {
      int i = -1;
      for (int q = 0; q < 3; q++)
        if (m->tv[3 * t + q] == a) i = q;
      if (i < 0) return -1;
      if (m->tv[3 * t + NXT(i)] == b) { *tout = t; *iout = i; return 0; }
      /* counter-clockwise around a crosses edge PRV(i) = (c, a); clockwise crosses edge i */
      t = dir == 0 ? m->tn[3 * t + PRV(i)] : m->tn[3 * t + i];
      if (t == t0) break;
    }
  }
  return -1;
}

/* Writes triangle t = (u, v, w) with neighbours / subsegments per edge and
   records it as touched. */
static int put_tri(rstate *S, int32_t t, int32_t u, int32_t v, int32_t w, const int32_t *nb,
                   const int32_t *sg) {
  orc_mesh *m = S->m;
  m->tv[3 * t] = u; m->tv[3 * t + 1] = v; m->tv[3 * t + 2] = w;
  for (int i = 0; i < 3; i++) { m->tn[3 * t + i] = nb[i]; m->ts[3 * t + i] = sg[i]; }
  S->vtri[u] = t; S->vtri[v] = t; S->vtri[w] = t;
  if (grow_i32(&S->touched, &S->captouched, (int64_t)S->ntouched + 1)) return -1;
  S->touched[S->ntouched++] = t;
  return 0;
}

/* Points the neighbour across directed edge (u, v) of triangle n (stored as
   (v, u) in n) back at t. */
static void relink(orc_mesh *m, int32_t n, int32_t u, int32_t v, int32_t t) {
  if (n < 0) return;
  for (int q = 0; q < 3; q++)
    if (m->tv[3 * n + q] == v && m->tv[3 * n + NXT(q)] == u) { m->tn[3 * n + q] = t; return; }
}

static int push_stack(rstate *S, int32_t t) {
  if (grow_i32(&S->stack, &S->capstack, (int64_t)S->nstack + 1)) return -1;
  S->stack[S->nstack++] = t;
  return 0;
}

/* Lawson flips around the new vertex p: every stacked triangle is (p, x, y);
   its edge (x, y) is flipped when it is not a subsegment and the far apex
   lies strictly inside the circle through p, x, y. */
static int legalize(rstate *S, int32_t p) {
  orc_mesh *m = S->m;
  while (S->nstack > 0) {
    int32_t t = S->stack[--S->nstack];
    if (m->tv[3 * t] != p) continue;
    if (m->ts[3 * t + 1] >= 0) continue;
    int32_t n = m->tn[3 * t + 1];
    if (n < 0) continue;
    int32_t x = m->tv[3 * t + 1], y = m->tv[3 * t + 2];
    int j = -1;
    for (int q = 0; q < 3; q++)
      if (m->tv[3 * n + q] == y && m->tv[3 * n + NXT(q)] == x) j = q;
    if (j < 0) return -1;
    int32_t z = m->tv[3 * n + PRV(j)];
    double pp[2], px[2], py[2], pz[2];
    P(m, p, pp); P(m, x, px); P(m, y, py); P(m, z, pz);
    if (orc_incircle(pp, px, py, pz) <= 0) continue;
    /* t = (p, x, y), n = (y, x, z) -> t = (p, x, z), n = (p, z, y) */
    int32_t t_px = m->tn[3 * t], t_yp = m->tn[3 * t + 2];
    int32_t s_px = m->ts[3 * t], s_yp = m->ts[3 * t + 2];
    int32_t n_xz = m->tn[3 * n + NXT(j)], n_zy = m->tn[3 * n + PRV(j)];
    int32_t s_xz = m->ts[3 * n + NXT(j)], s_zy = m->ts[3 * n + PRV(j)];
    int32_t nb1[3] = {t_px, n_xz, n}, sg1[3] = {s_px, s_xz, -1};
    int32_t nb2[3] = {t, n_zy, t_yp}, sg2[3] = {-1, s_zy, s_yp};
    if (put_tri(S, t, p, x, z, nb1, sg1) || put_tri(S, n, p, z, y, nb2, sg2)) return -1;
    relink(m, n_xz, x, z, t);
    relink(m, t_yp, y, p, n);
    if (push_stack(S, t) || push_stack(S, n)) return -1;
  }
  return 0;
}

static int32_t new_vertex(rstate *S, double x, double y, int kind) {
  orc_mesh *m = S->m;
  if (mesh_room(S, m->nV + 1, m->nT + 4, m->nS + 1)) return -1;
  int32_t v = m->nV++;
  m->x[v] = x; m->y[v] = y; m->vkind[v] = kind;
  return v;
}

/* Inserts p strictly inside triangle t (1-3 split). */
static int insert_in_tri(rstate *S, int32_t t, int32_t p) {
  orc_mesh *m = S->m;
  int32_t a = m->tv[3 * t], b = m->tv[3 * t + 1], c = m->tv[3 * t + 2];
  int32_t nab = m->tn[3 * t], nbc = m->tn[3 * t + 1], nca = m->tn[3 * t + 2];
  int32_t sab = m->ts[3 * t], sbc = m->ts[3 * t + 1], sca = m->ts[3 * t + 2];
  int32_t t1 = m->nT++, t2 = m->nT++;
  int32_t nb0[3] = {t2, nab, t1}, sg0[3] = {-1, sab, -1};
  int32_t nb1[3] = {t, nbc, t2}, sg1[3] = {-1, sbc, -1};
  int32_t nb2[3] = {t1, nca, t}, sg2[3] = {-1, sca, -1};
  if (put_tri(S, t, p, a, b, nb0, sg0) || put_tri(S, t1, p, b, c, nb1, sg1) ||
      put_tri(S, t2, p, c, a, nb2, sg2))
    return -1;
  relink(m, nbc, b, c, t1);
  relink(m, nca, c, a, t2);
  if (push_stack(S, t) || push_stack(S, t1) || push_stack(S, t2)) return -1;
  return legalize(S, p);
}

/* Inserts p on edge i of triangle t (2-4 split, 1-2 on the hull).  When the
   edge carries subsegment k, k keeps its first endpoint and a new subsegment
   takes the second. */
static int insert_on_edge(rstate *S, int32_t t, int i, int32_t p) {
  orc_mesh *m = S->m;
  int32_t a = m->tv[3 * t + i], b = m->tv[3 * t + NXT(i)], c = m->tv[3 * t + PRV(i)];
  int32_t k = m->ts[3 * t + i], n = m->tn[3 * t + i];
  int32_t s_a = -1, s_b = -1; /* subsegment ids on (a, p) and (p, b) */
  if (k >= 0) {
    int32_t kn = m->nS++;
    int32_t s0 = m->sv[2 * k], s1 = m->sv[2 * k + 1];
    m->sv[2 * k] = s0; m->sv[2 * k + 1] = p;
    m->sv[2 * kn] = p; m->sv[2 * kn + 1] = s1;
    m->sparent[kn] = m->sparent[k];
    m->spend[kn] = 0;
    m->spend[k] = 0;
    s_a = (a == s0) ? k : kn;
    s_b = (b == s1) ? kn : k;
  }
  int32_t nbc = m->tn[3 * t + NXT(i)], nca = m->tn[3 * t + PRV(i)];
  int32_t sbc = m->ts[3 * t + NXT(i)], sca = m->ts[3 * t + PRV(i)];
  int32_t t1 = m->nT++;
  int32_t n1 = -1, d = -1, j = -1, nad = -1, ndb = -1, sad = -1, sdb = -1;
  if (n >= 0) {
    for (int q = 0; q < 3; q++)
      if (m->tv[3 * n + q] == b && m->tv[3 * n + NXT(q)] == a) j = q;
    if (j < 0) return -1;
    d = m->tv[3 * n + PRV(j)];
    ndb = m->tn[3 * n + PRV(j)];
    nad = m->tn[3 * n + NXT(j)];
    sdb = m->ts[3 * n + PRV(j)];
    sad = m->ts[3 * n + NXT(j)];
    n1 = m->nT++;
  }
  /* t = (p, c, a), t1 = (p, b, c) above the edge; n = (p, a, d), n1 = (p, d, b) below */
  int32_t nbt[3] = {t1, nca, n >= 0 ? n : -1}, sgt[3] = {-1, sca, s_a};
  int32_t nbt1[3] = {n >= 0 ? n1 : -1, nbc, t}, sgt1[3] = {s_b, sbc, -1};
  if (put_tri(S, t, p, c, a, nbt, sgt) || put_tri(S, t1, p, b, c, nbt1, sgt1)) return -1;
  relink(m, nbc, b, c, t1);
  if (push_stack(S, t) || push_stack(S, t1)) return -1;
  if (n >= 0) {
    int32_t nbn[3] = {t, nad, n1}, sgn[3] = {s_a, sad, -1};
    int32_t nbn1[3] = {n, ndb, t1}, sgn1[3] = {-1, sdb, s_b};
    if (put_tri(S, n, p, a, d, nbn, sgn) || put_tri(S, n1, p, d, b, nbn1, sgn1)) return -1;
    relink(m, ndb, d, b, n1);
    if (push_stack(S, n) || push_stack(S, n1)) return -1;
  }
  return legalize(S, p);
}

/* Is subsegment k (edge i of triangle t) encroached by the apex of t? */
static int apex_encroaches(const orc_mesh *m, int32_t t, int i) {
  double a[2], b[2], c[2];
  P(m, m->tv[3 * t + i], a);
  P(m, m->tv[3 * t + NXT(i)], b);
  P(m, m->tv[3 * t + PRV(i)], c);
  return orc_encroaches(0, a, b, c) > 0;
}

/* Queues what an insertion may have created: bad triangles among the
   touched ones, and encroached subsegments on their edges. */
static int after_insert(rstate *S) {
  orc_mesh *m = S->m;
  for (int32_t q = 0; q < S->ntouched; q++) {
    int32_t t = S->touched[q];
    int dup = 0;
    for (int32_t r = 0; r < q && !dup; r++) dup = S->touched[r] == t;
    if (dup) continue;
    if (queue_tri(S, t)) return -1;
    for (int i = 0; i < 3; i++) {
      int32_t k = m->ts[3 * t + i];
      if (k >= 0 && apex_encroaches(m, t, i) && queue_seg(S, k, 0)) return -1;
    }
  }
  S->ntouched = 0;
  return 0;
}

/* Splits subsegment k at its midpoint.  Returns 1 if it was unsplittable. */
static int split_seg(rstate *S, int32_t k) {
  orc_mesh *m = S->m;
  int32_t a = m->sv[2 * k], b = m->sv[2 * k + 1];
  double mx = (m->x[a] + m->x[b]) * 0.5, my = (m->y[a] + m->y[b]) * 0.5;
  if ((mx == m->x[a] && my == m->y[a]) || (mx == m->x[b] && my == m->y[b])) {
    S->n_unsplittable++;
    return 1;
  }
  int32_t t;
  int i;
  if (find_edge(S, a, b, &t, &i) && find_edge(S, b, a, &t, &i)) return -1;
  int32_t p = new_vertex(S, mx, my, ORC_VK_MIDPOINT);
  if (p < 0) return -1;
  S->ntouched = 0;
  if (insert_on_edge(S, t, i, p)) return -1;
  return after_insert(S);
}

/* Is subsegment k still encroached (apex test on both sides)? */
static int seg_encroached(rstate *S, int32_t k) {
  const orc_mesh *m = S->m;
  int32_t a = m->sv[2 * k], b = m->sv[2 * k + 1], t;
  int i;
  if (!find_edge(S, a, b, &t, &i) && apex_encroaches(m, t, i)) return 1;
  if (!find_edge(S, b, a, &t, &i) && apex_encroaches(m, t, i)) return 1;
  return 0;
}

/* Tries to split bad triangle t at its circumcenter.  Returns 0 after an
   insertion or a deferral (subsegments queued), <0 on error. */
static int split_tri(rstate *S, int32_t t, int retries) {
  orc_mesh *m = S->m;
  double ox, oy, r2, l2, a2;
  tri_geom(m, t, &ox, &oy, &r2, &l2, &a2);
  double p[2] = {ox, oy};
  if (!(a2 > 0.0) || !isfinite(ox) || !isfinite(oy)) return 0;
  /* visibility walk from t */
  int32_t cur = t;
  int on_edge = -1;
  for (int64_t steps = 0;; steps++) {
    if (steps > (1 << 22)) return -1;
    int s[3];
    for (int i = 0; i < 3; i++) {
      double u[2], v[2];
      P(m, m->tv[3 * cur + i], u);
      P(m, m->tv[3 * cur + NXT(i)], v);
      s[i] = orc_orient2d(u, v, p);
    }
    if (s[0] >= 0 && s[1] >= 0 && s[2] >= 0) {
      int nz = (s[0] == 0) + (s[1] == 0) + (s[2] == 0);
      if (nz >= 2) { S->n_coincident++; return 0; }
      for (int i = 0; i < 3; i++)
        if (s[i] == 0) on_edge = i;
      break;
    }
    int moved = 0, first = -1;
    for (int i = 0; i < 3 && !moved; i++) {
      if (s[i] >= 0) continue;
      if (first < 0) first = i;
      if (m->ts[3 * cur + i] < 0 && m->tn[3 * cur + i] >= 0) { cur = m->tn[3 * cur + i]; moved = 1; }
    }
    if (!moved) {
      /* the circumcenter lies beyond a subsegment: split that one instead */
      int32_t k = m->ts[3 * cur + first];
      if (k < 0) return -1;
      if (queue_seg(S, k, 1) || queue_tri_retry(S, t, retries + 1)) return -1;
      return 0;
    }
  }
  /* conflict region: flood across non-subsegment edges whose far circle
     strictly holds p; subsegments on its boundary are tested for encroachment */
  S->epoch++;
  S->ncav = 0;
  if (grow_i32(&S->cav, &S->capcav, 1)) return -1;
  S->cav[S->ncav++] = cur;
  S->mark[cur] = S->epoch;
  int enc = 0;
  for (int32_t h = 0; h < S->ncav; h++) {
    int32_t c = S->cav[h];
    for (int i = 0; i < 3; i++) {
      int32_t k = m->ts[3 * c + i];
      if (k >= 0) {
        double u[2], v[2];
        P(m, m->tv[3 * c + i], u);
        P(m, m->tv[3 * c + NXT(i)], v);
        if (orc_encroaches(0, u, v, p) > 0) {
          enc = 1;
          if (queue_seg(S, k, 1)) return -1;
        }
        continue;
      }
      int32_t n = m->tn[3 * c + i];
      if (n < 0 || S->mark[n] == S->epoch) continue;
      double u[2], v[2], w[2];
      P(m, m->tv[3 * n], u);
      P(m, m->tv[3 * n + 1], v);
      P(m, m->tv[3 * n + 2], w);
      if (orc_incircle(u, v, w, p) > 0) {
        S->mark[n] = S->epoch;
        if (grow_i32(&S->cav, &S->capcav, (int64_t)S->ncav + 1)) return -1;
        S->cav[S->ncav++] = n;
      }
    }
  }
  if (enc) {
    /* the subsegments go first; the triangle waits (and is given up after
       many rejections, which only unsplittable subsegments could cause) */
    if (retries >= 64) { S->n_given_up++; return 0; }
    return queue_tri_retry(S, t, retries + 1);
  }
  int32_t pv = new_vertex(S, ox, oy, ORC_VK_CIRCUMCENTER);
  if (pv < 0) return -1;
  S->ntouched = 0;
  if (on_edge >= 0) {
    if (insert_on_edge(S, cur, on_edge, pv)) return -1;
  } else if (insert_in_tri(S, cur, pv)) {
    return -1;
  }
  return after_insert(S);
}

int orc_ruppert(orc_mesh *m, double ratio_bound_sq, int64_t max_insertions, int64_t *n_unsplittable,
                char *err, int32_t errlen) {
  if (err && errlen > 0) err[0] = 0;
  if (!m || !(ratio_bound_sq > 0.0) || !isfinite(ratio_bound_sq)) {
    if (err && errlen > 0) snprintf(err, (size_t)errlen, "bad arguments");
    return ORC_E_ARG;
  }
  rstate S;
  memset(&S, 0, sizeof S);
  S.m = m;
  S.B2 = ratio_bound_sq;
  int rc = ORC_OK;
  if (mesh_room(&S, m->nV + 1, m->nT + 4, m->nS + 1)) { rc = ORC_E_NOMEM; goto done; }
  for (int32_t t = 0; t < m->nT; t++)
    for (int i = 0; i < 3; i++) S.vtri[m->tv[3 * t + i]] = t;
  for (int32_t t = 0; t < m->nT; t++) {
    if (queue_tri(&S, t)) { rc = ORC_E_NOMEM; goto done; }
    for (int i = 0; i < 3; i++) {
      int32_t k = m->ts[3 * t + i];
      if (k >= 0 && (m->spend[k] || apex_encroaches(m, t, i)) && queue_seg(&S, k, m->spend[k])) {
        rc = ORC_E_NOMEM;
        goto done;
      }
    }
  }
  int32_t nv0 = m->nV;
  while (S.nh > 0) {
    if (max_insertions > 0 && m->nV - nv0 >= max_insertions) { rc = ORC_E_NOTERM; break; }
    qent e = qpop(&S);
    int r = 0;
    if (e.cls == 1) {
      if (m->sv[2 * e.id] != e.a || m->sv[2 * e.id + 1] != e.b) continue; /* already split */
      if (!e.forced && !seg_encroached(&S, e.id)) continue;
      r = split_seg(&S, e.id);
      if (r == 1) r = 0;
    } else {
      const int32_t *v = &m->tv[3 * e.id];
      if (e.id >= m->nT || v[0] != e.a || v[1] != e.b || v[2] != e.c) continue; /* rewritten */
      r = split_tri(&S, e.id, e.retries);
    }
    if (r < 0) {
      rc = ORC_E_NOMEM;
      if (err && errlen > 0) snprintf(err, (size_t)errlen, "sequential refinement failed");
      break;
    }
  }
done:
  if (n_unsplittable) *n_unsplittable = S.n_unsplittable;
  free(S.vtri); free(S.heap); free(S.stack); free(S.touched); free(S.cav); free(S.mark);
  return rc;
}

/*
 * orc_cdt.c -- Line 1 of Algorithm 1 (gDP2d): the constrained Delaunay
 * triangulation of the input PSLG, built the plain way (oracle).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Definitions follow Section 4 (PSLG, subsegment, CDT).  Steps:
 *   1. validate the input (finite, no duplicate points, segment ids in range,
 *      no zero-length or repeated segments);
 *   2. strictly convex hull (monotone chain), fan-triangulated;
 *   3. every other point inserted one at a time (split the containing triangle
 *      or edge), each followed by Lawson flips, which keeps the triangulation
 *      Delaunay for the perturbed incircle test (orc_incircle_sos);
 *   4. every segment recovered by flipping the edges that cross it until the
 *      segment is an edge (a crossing edge whose quadrilateral is convex is
 *      always available), failing on a crossed segment or on a vertex in the
 *      segment's interior;
 *   5. a global Lawson pass over non-constrained edges;
 *   6. every hull edge must be a segment;
 *   7. canonical form: each triangle rotated so its smallest vertex id comes
 *      first, triangles sorted lexicographically.
 * Under the perturbation the CDT is unique, so the canonical arrays are a
 * function of the input alone.
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t nv;
  const double *xy;
  int32_t nt, capt;
  int32_t *tv, *tn, *tc; /* tc: segment id on edge or -1 */
  int32_t *vt;           /* vertex -> an incident triangle */
  char *err;
  int32_t errlen;
} cdt;

#define P(c, v) (&(c)->xy[2 * (v)])
#define NXT(i) (((i) + 1) % 3)
#define PRV(i) (((i) + 2) % 3)

static void seterr(cdt *c, const char *msg) {
  if (c->err && c->errlen > 0) {
    strncpy(c->err, msg, (size_t)c->errlen - 1);
    c->err[c->errlen - 1] = 0;
  }
}

static int grow_tris(cdt *c, int32_t need) {
  if (need <= c->capt) return 0;
  int32_t cap = c->capt ? c->capt : 64;
  while (cap < need) cap *= 2;
  int32_t *a = realloc(c->tv, sizeof(int32_t) * 3 * (size_t)cap);
  if (!a) return -1;
  c->tv = a;
  a = realloc(c->tn, sizeof(int32_t) * 3 * (size_t)cap);
  if (!a) return -1;
  c->tn = a;
  a = realloc(c->tc, sizeof(int32_t) * 3 * (size_t)cap);
  if (!a) return -1;
  c->tc = a;
  c->capt = cap;
  return 0;
}

static int32_t new_tri(cdt *c, int32_t a, int32_t b, int32_t d) {
  if (grow_tris(c, c->nt + 1)) return -1;
  int32_t t = c->nt++;
  c->tv[3 * t] = a; c->tv[3 * t + 1] = b; c->tv[3 * t + 2] = d;
  for (int i = 0; i < 3; i++) { c->tn[3 * t + i] = -1; c->tc[3 * t + i] = -1; }
  c->vt[a] = t; c->vt[b] = t; c->vt[d] = t;
  return t;
}

static int edge_index(const cdt *c, int32_t t, int32_t u, int32_t v) {
  for (int i = 0; i < 3; i++)
    if (c->tv[3 * t + i] == u && c->tv[3 * t + NXT(i)] == v) return i;
  return -1;
}

static int vert_index(const cdt *c, int32_t t, int32_t u) {
  for (int i = 0; i < 3; i++)
    if (c->tv[3 * t + i] == u) return i;
  return -1;
}

/* Point the neighbour across edge (u,v) of triangle n (if any) back at t. */
static void relink(cdt *c, int32_t n, int32_t u, int32_t v, int32_t t) {
  if (n < 0) return;
  int j = edge_index(c, n, v, u);
  c->tn[3 * n + j] = t;
}

/* Triangle that holds the directed edge (u,v), or -1: rotate around u. */
static int32_t find_edge(const cdt *c, int32_t u, int32_t v) {
  int32_t start = c->vt[u];
  int32_t t = start;
  /* counter-clockwise sweep */
  for (int guard = 0; guard < (1 << 24); guard++) {
    int i = vert_index(c, t, u);
    if (c->tv[3 * t + NXT(i)] == v) return t;
    int32_t n = c->tn[3 * t + PRV(i)]; /* across (prev, u) */
    if (n < 0) break;
    t = n;
    if (t == start) return -1;
  }
  /* clockwise sweep from the start */
  t = start;
  for (int guard = 0; guard < (1 << 24); guard++) {
    int i = vert_index(c, t, u);
    if (c->tv[3 * t + NXT(i)] == v) return t;
    int32_t n = c->tn[3 * t + i]; /* across (u, next) */
    if (n < 0) return -1;
    t = n;
    if (t == start) return -1;
  }
  return -1;
}

/* Flip edge i of triangle t.  t = (u,v,w) with edge i = (u,v); n = (v,u,x).
   Afterwards t = (w,u,x) and n = (x,v,w). */
static void flip(cdt *c, int32_t t, int i) {
  int32_t u = c->tv[3 * t + i], v = c->tv[3 * t + NXT(i)], w = c->tv[3 * t + PRV(i)];
  int32_t n = c->tn[3 * t + i];
  int j = edge_index(c, n, v, u);
  int32_t x = c->tv[3 * n + PRV(j)];
  int32_t A = c->tn[3 * t + NXT(i)], Ac = c->tc[3 * t + NXT(i)]; /* (v,w) */
  int32_t B = c->tn[3 * t + PRV(i)], Bc = c->tc[3 * t + PRV(i)]; /* (w,u) */
  int32_t C = c->tn[3 * n + NXT(j)], Cc = c->tc[3 * n + NXT(j)]; /* (u,x) */
  int32_t D = c->tn[3 * n + PRV(j)], Dc = c->tc[3 * n + PRV(j)]; /* (x,v) */
  c->tv[3 * t] = w; c->tv[3 * t + 1] = u; c->tv[3 * t + 2] = x;
  c->tn[3 * t] = B; c->tc[3 * t] = Bc;
  c->tn[3 * t + 1] = C; c->tc[3 * t + 1] = Cc;
  c->tn[3 * t + 2] = n; c->tc[3 * t + 2] = -1;
  c->tv[3 * n] = x; c->tv[3 * n + 1] = v; c->tv[3 * n + 2] = w;
  c->tn[3 * n] = D; c->tc[3 * n] = Dc;
  c->tn[3 * n + 1] = A; c->tc[3 * n + 1] = Ac;
  c->tn[3 * n + 2] = t; c->tc[3 * n + 2] = -1;
  relink(c, C, u, x, t);
  relink(c, A, v, w, n);
  c->vt[u] = t; c->vt[w] = t; c->vt[x] = n; c->vt[v] = n;
}

/* Is edge i of t locally Delaunay under the perturbed incircle test? */
static int locally_delaunay(const cdt *c, int32_t t, int i) {
  int32_t n = c->tn[3 * t + i];
  if (n < 0 || c->tc[3 * t + i] >= 0) return 1;
  int32_t a = c->tv[3 * t], b = c->tv[3 * t + 1], d = c->tv[3 * t + 2];
  int j = edge_index(c, n, c->tv[3 * t + NXT(i)], c->tv[3 * t + i]);
  int32_t x = c->tv[3 * n + PRV(j)];
  return orc_incircle_sos(P(c, a), P(c, b), P(c, d), P(c, x), a, b, d, x) <= 0;
}

typedef struct { int32_t *a; int64_t n, cap; } istack;
static int ipush(istack *s, int32_t u, int32_t v) {
  if (s->n + 2 > s->cap) {
    int64_t cap = s->cap ? s->cap * 2 : 256;
    int32_t *a = realloc(s->a, sizeof(int32_t) * (size_t)cap);
    if (!a) return -1;
    s->a = a; s->cap = cap;
  }
  s->a[s->n++] = u; s->a[s->n++] = v;
  return 0;
}

/* Lawson flips driven by a stack of (u,v) edges. */
static int lawson(cdt *c, istack *st) {
  while (st->n > 0) {
    int32_t v = st->a[--st->n], u = st->a[--st->n];
    int32_t t = find_edge(c, u, v);
    if (t < 0) continue;
    int i = edge_index(c, t, u, v);
    if (locally_delaunay(c, t, i)) continue;
    int32_t w = c->tv[3 * t + PRV(i)];
    int32_t n = c->tn[3 * t + i];
    int j = edge_index(c, n, v, u);
    int32_t x = c->tv[3 * n + PRV(j)];
    flip(c, t, i);
    if (ipush(st, u, x) || ipush(st, x, v) || ipush(st, v, w) || ipush(st, w, u)) return -1;
  }
  return 0;
}

/* Visibility walk to the triangle containing vertex p. Returns t; *zero gets
   the index of the single edge containing p (-1 if p is interior). */
static int32_t locate(cdt *c, int32_t start, int32_t p, int *zero, int *nz) {
  int32_t t = start;
  for (int64_t step = 0; step < ((int64_t)1 << 32); step++) {
    int s[3];
    int moved = 0;
    for (int i = 0; i < 3; i++)
      s[i] = orc_orient2d(P(c, c->tv[3 * t + i]), P(c, c->tv[3 * t + NXT(i)]), P(c, p));
    for (int i = 0; i < 3; i++) {
      if (s[i] < 0) {
        int32_t n = c->tn[3 * t + i];
        if (n < 0) return -1;
        t = n;
        moved = 1;
        break;
      }
    }
    if (!moved) {
      *nz = 0;
      *zero = -1;
      for (int i = 0; i < 3; i++)
        if (s[i] == 0) { (*nz)++; *zero = i; }
      return t;
    }
  }
  return -1;
}

static int insert_point(cdt *c, int32_t p, int32_t *last, istack *st) {
  int zero, nz;
  int32_t t = locate(c, *last, p, &zero, &nz);
  if (t < 0) { seterr(c, "point location left the hull"); return ORC_E_INPUT; }
  if (nz >= 2) { seterr(c, "duplicate point"); return ORC_E_INPUT; }
  if (nz == 0) {
    int32_t a = c->tv[3 * t], b = c->tv[3 * t + 1], d = c->tv[3 * t + 2];
    int32_t na = c->tn[3 * t], nb = c->tn[3 * t + 1], nd = c->tn[3 * t + 2];
    /* t -> (a,b,p); t1 = (b,d,p); t2 = (d,a,p) */
    int32_t t1 = new_tri(c, b, d, p);
    int32_t t2 = new_tri(c, d, a, p);
    if (t1 < 0 || t2 < 0) return ORC_E_NOMEM;
    c->tv[3 * t + 2] = p;
    c->tn[3 * t] = na; c->tn[3 * t + 1] = t1; c->tn[3 * t + 2] = t2;
    c->tn[3 * t1] = nb; c->tn[3 * t1 + 1] = t2; c->tn[3 * t1 + 2] = t;
    c->tn[3 * t2] = nd; c->tn[3 * t2 + 1] = t; c->tn[3 * t2 + 2] = t1;
    relink(c, nb, b, d, t1);
    relink(c, nd, d, a, t2);
    c->vt[a] = t; c->vt[b] = t; c->vt[d] = t1; c->vt[p] = t;
    if (ipush(st, a, b) || ipush(st, b, d) || ipush(st, d, a)) return ORC_E_NOMEM;
  } else {
    /* p on edge `zero` = (u,v) of t = (u,v,w); the other side n = (v,u,x) */
    int i = zero;
    int32_t u = c->tv[3 * t + i], v = c->tv[3 * t + NXT(i)], w = c->tv[3 * t + PRV(i)];
    int32_t n = c->tn[3 * t + i];
    int32_t tA = c->tn[3 * t + NXT(i)]; /* (v,w) */
    int32_t tB = c->tn[3 * t + PRV(i)]; /* (w,u) */
    /* t -> (u,p,w) ; t1 = (p,v,w) */
    int32_t t1 = new_tri(c, p, v, w);
    if (t1 < 0) return ORC_E_NOMEM;
    c->tv[3 * t] = u; c->tv[3 * t + 1] = p; c->tv[3 * t + 2] = w;
    c->tn[3 * t + 1] = t1; c->tn[3 * t + 2] = tB;
    c->tn[3 * t1 + 1] = tA; c->tn[3 * t1 + 2] = t;
    relink(c, tA, v, w, t1);
    c->vt[u] = t; c->vt[w] = t; c->vt[p] = t; c->vt[v] = t1;
    if (n >= 0) {
      int j = edge_index(c, n, v, u);
      int32_t x = c->tv[3 * n + PRV(j)];
      int32_t nC = c->tn[3 * n + NXT(j)]; /* (u,x) */
      int32_t nD = c->tn[3 * n + PRV(j)]; /* (x,v) */
      /* n -> (v,p,x) ; n1 = (p,u,x) */
      int32_t n1 = new_tri(c, p, u, x);
      if (n1 < 0) return ORC_E_NOMEM;
      c->tv[3 * n] = v; c->tv[3 * n + 1] = p; c->tv[3 * n + 2] = x;
      c->tn[3 * n] = t1; c->tn[3 * n + 1] = n1; c->tn[3 * n + 2] = nD;
      c->tn[3 * n1] = t; c->tn[3 * n1 + 1] = nC; c->tn[3 * n1 + 2] = n;
      relink(c, nC, u, x, n1);
      c->tn[3 * t] = n1;   /* (u,p) <-> (p,u) */
      c->tn[3 * t1] = n;   /* (p,v) <-> (v,p) */
      c->vt[x] = n; c->vt[v] = n;
      if (ipush(st, u, x) || ipush(st, x, v)) return ORC_E_NOMEM;
    } else {
      c->tn[3 * t] = -1;
      c->tn[3 * t1] = -1;
    }
    if (ipush(st, v, w) || ipush(st, w, u)) return ORC_E_NOMEM;
  }
  *last = c->vt[p];
  int r = lawson(c, st);
  if (r) return ORC_E_NOMEM;
  *last = c->vt[p];
  return ORC_OK;
}

/* Hilbert index of (x, y) on a 2^16 grid (bit-interleaving rotation form). */
static uint64_t hilbert16(uint32_t x, uint32_t y) {
  uint64_t d = 0;
  for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
    uint32_t rx = (x & s) > 0, ry = (y & s) > 0;
    d += (uint64_t)s * s * ((3 * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) { x = s - 1 - x; y = s - 1 - y; }
      uint32_t t = x; x = y; y = t;
    }
  }
  return d;
}

typedef struct { uint64_t key; int32_t v; } vkey;
static int cmp_vkey(const void *a, const void *b) {
  const vkey *x = a, *y = b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v);
}

static const double *g_sort_xy;
static int cmp_xy(const void *a, const void *b) {
  int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
  const double *p = g_sort_xy + 2 * i, *q = g_sort_xy + 2 * j;
  if (p[0] != q[0]) return p[0] < q[0] ? -1 : 1;
  if (p[1] != q[1]) return p[1] < q[1] ? -1 : 1;
  return i < j ? -1 : (i > j);
}

typedef struct { int32_t a, b, s; } segkey;
static int cmp_seg(const void *x, const void *y) {
  const segkey *p = x, *q = y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return 0;
}

/* Recover segment s = (a,b) as an edge by flips. */
static int recover_segment(cdt *c, int32_t a, int32_t b, int32_t s) {
  int32_t t0 = find_edge(c, a, b);
  int32_t t1 = find_edge(c, b, a);
  if (t0 < 0 && t1 < 0) {
    /* find the triangle around a whose open wedge contains direction a->b */
    int32_t start = c->vt[a], t = start, found = -1;
    /* sweep all triangles around a, both directions */
    int dir_done = 0;
    for (int pass = 0; pass < 2 && found < 0; pass++) {
      t = start;
      for (int guard = 0; guard < (1 << 24); guard++) {
        int i = vert_index(c, t, a);
        int32_t u = c->tv[3 * t + NXT(i)], v = c->tv[3 * t + PRV(i)];
        int ou = orc_orient2d(P(c, a), P(c, u), P(c, b));
        int ov = orc_orient2d(P(c, a), P(c, v), P(c, b));
        double dxu = c->xy[2 * u] - c->xy[2 * a], dyu = c->xy[2 * u + 1] - c->xy[2 * a + 1];
        double dxb = c->xy[2 * b] - c->xy[2 * a], dyb = c->xy[2 * b + 1] - c->xy[2 * a + 1];
        if (ou == 0 && dxu * dxb + dyu * dyb > 0) {
          seterr(c, "a vertex lies in the interior of a segment");
          return ORC_E_INPUT;
        }
        if (ou > 0 && ov < 0) { found = t; break; }
        int32_t n = pass == 0 ? c->tn[3 * t + PRV(i)] : c->tn[3 * t + i];
        if (n < 0 || n == start) break;
        t = n;
      }
      dir_done++;
    }
    (void)dir_done;
    if (found < 0) { seterr(c, "segment direction not found around its endpoint"); return ORC_E_INPUT; }
    /* walk along a->b collecting crossed edges as (left, right) pairs */
    istack q = {0};
    int i = vert_index(c, found, a);
    int32_t R = c->tv[3 * found + NXT(i)], L = c->tv[3 * found + PRV(i)];
    /* orient(a,b,R) < 0 (right), orient(a,b,L) > 0 (left) */
    t = found;
    for (int64_t guard = 0;; guard++) {
      if (guard > ((int64_t)1 << 30)) { free(q.a); seterr(c, "segment walk did not end"); return ORC_E_INPUT; }
      int e = edge_index(c, t, R, L);
      if (c->tc[3 * t + e] >= 0) { free(q.a); seterr(c, "segments cross"); return ORC_E_INPUT; }
      if (ipush(&q, R, L)) { free(q.a); return ORC_E_NOMEM; }
      int32_t n = c->tn[3 * t + e];
      if (n < 0) { free(q.a); seterr(c, "segment leaves the hull"); return ORC_E_INPUT; }
      int j = edge_index(c, n, L, R);
      int32_t w = c->tv[3 * n + PRV(j)];
      if (w == b) break;
      int o = orc_orient2d(P(c, a), P(c, b), P(c, w));
      if (o == 0) { free(q.a); seterr(c, "a vertex lies in the interior of a segment"); return ORC_E_INPUT; }
      if (o > 0) L = w; else R = w;
      t = n;
    }
    /* flip crossing edges until none is left (queue order) */
    int64_t head = 0;
    int64_t stuck = 0;
    while (head < q.n) {
      int32_t u = q.a[head], v = q.a[head + 1];
      head += 2;
      int32_t tt = find_edge(c, u, v);
      if (tt < 0) continue;
      int e = edge_index(c, tt, u, v);
      int32_t w = c->tv[3 * tt + PRV(e)];
      int32_t n = c->tn[3 * tt + e];
      int j = edge_index(c, n, v, u);
      int32_t x = c->tv[3 * n + PRV(j)];
      int o1 = orc_orient2d(P(c, w), P(c, x), P(c, u));
      int o2 = orc_orient2d(P(c, w), P(c, x), P(c, v));
      if (o1 * o2 < 0) {
        flip(c, tt, e);
        stuck = 0;
        if (!(w == a || w == b || x == a || x == b)) {
          int ow = orc_orient2d(P(c, a), P(c, b), P(c, w));
          int ox = orc_orient2d(P(c, a), P(c, b), P(c, x));
          if (ow * ox < 0) {
            int32_t l = ow > 0 ? w : x, r = ow > 0 ? x : w;
            if (ipush(&q, r, l)) { free(q.a); return ORC_E_NOMEM; }
          }
        }
      } else {
        if (ipush(&q, u, v)) { free(q.a); return ORC_E_NOMEM; }
        if (++stuck > (q.n - head) + 4) { free(q.a); seterr(c, "segment recovery stalled"); return ORC_E_INPUT; }
      }
      /* compact the queue occasionally */
      if (head > 4096 && head * 2 > q.n) {
        memmove(q.a, q.a + head, sizeof(int32_t) * (size_t)(q.n - head));
        q.n -= head;
        head = 0;
      }
    }
    free(q.a);
    t0 = find_edge(c, a, b);
    t1 = find_edge(c, b, a);
    if (t0 < 0 && t1 < 0) { seterr(c, "segment not recovered"); return ORC_E_INPUT; }
  }
  if (t0 >= 0) c->tc[3 * t0 + edge_index(c, t0, a, b)] = s;
  if (t1 >= 0) c->tc[3 * t1 + edge_index(c, t1, b, a)] = s;
  return ORC_OK;
}

typedef struct { int32_t v[3]; int32_t old; } ctri;
static int cmp_ctri(const void *x, const void *y) {
  const ctri *p = x, *q = y;
  for (int i = 0; i < 3; i++)
    if (p->v[i] != q->v[i]) return p->v[i] < q->v[i] ? -1 : 1;
  return 0;
}

static orc_mesh *mesh_alloc(int32_t capV, int32_t capT, int32_t capS) {
  orc_mesh *m = calloc(1, sizeof(orc_mesh));
  if (!m) return NULL;
  m->capV = capV; m->capT = capT; m->capS = capS;
  m->x = malloc(sizeof(double) * (size_t)capV);
  m->y = malloc(sizeof(double) * (size_t)capV);
  m->vkind = malloc(sizeof(int32_t) * (size_t)capV);
  m->tv = malloc(sizeof(int32_t) * 3 * (size_t)capT);
  m->tn = malloc(sizeof(int32_t) * 3 * (size_t)capT);
  m->ts = malloc(sizeof(int32_t) * 3 * (size_t)capT);
  m->sv = malloc(sizeof(int32_t) * 2 * (size_t)capS);
  m->sparent = malloc(sizeof(int32_t) * (size_t)capS);
  m->spend = malloc((size_t)capS);
  if (!m->x || !m->y || !m->vkind || !m->tv || !m->tn || !m->ts || !m->sv || !m->sparent || !m->spend) {
    orc_mesh_free(m);
    return NULL;
  }
  return m;
}

void orc_mesh_free(orc_mesh *m) {
  if (!m) return;
  free(m->x); free(m->y); free(m->vkind);
  free(m->tv); free(m->tn); free(m->ts);
  free(m->sv); free(m->sparent); free(m->spend);
  free(m);
}

orc_mesh *orc_mesh_from_arrays(int32_t nv, int32_t n_input_v, const double *xy, const int32_t *vkind,
                               int32_t nt, const int32_t *tv, const int32_t *tn, const int32_t *ts,
                               int32_t ns, int32_t n_input_s, const int32_t *sv, const int32_t *sparent,
                               const uint8_t *spend) {
  if (nv < 0 || nt < 0 || ns < 0) return NULL;
  orc_mesh *m = mesh_alloc(nv + 16, nt + 16, ns + 16);
  if (!m) return NULL;
  m->nV = nv; m->nT = nt; m->nS = ns; m->n_input_v = n_input_v; m->n_input_s = n_input_s;
  for (int32_t i = 0; i < nv; i++) { m->x[i] = xy[2 * i]; m->y[i] = xy[2 * i + 1]; m->vkind[i] = vkind[i]; }
  memcpy(m->tv, tv, sizeof(int32_t) * 3 * (size_t)nt);
  memcpy(m->tn, tn, sizeof(int32_t) * 3 * (size_t)nt);
  memcpy(m->ts, ts, sizeof(int32_t) * 3 * (size_t)nt);
  memcpy(m->sv, sv, sizeof(int32_t) * 2 * (size_t)ns);
  memcpy(m->sparent, sparent, sizeof(int32_t) * (size_t)ns);
  memcpy(m->spend, spend, (size_t)ns);
  return m;
}

orc_mesh *orc_mesh_clone(const orc_mesh *s) {
  orc_mesh *m = mesh_alloc(s->capV, s->capT, s->capS);
  if (!m) return NULL;
  m->nV = s->nV; m->nT = s->nT; m->nS = s->nS;
  m->n_input_v = s->n_input_v; m->n_input_s = s->n_input_s; m->rounds = s->rounds;
  memcpy(m->x, s->x, sizeof(double) * (size_t)s->nV);
  memcpy(m->y, s->y, sizeof(double) * (size_t)s->nV);
  memcpy(m->vkind, s->vkind, sizeof(int32_t) * (size_t)s->nV);
  memcpy(m->tv, s->tv, sizeof(int32_t) * 3 * (size_t)s->nT);
  memcpy(m->tn, s->tn, sizeof(int32_t) * 3 * (size_t)s->nT);
  memcpy(m->ts, s->ts, sizeof(int32_t) * 3 * (size_t)s->nT);
  memcpy(m->sv, s->sv, sizeof(int32_t) * 2 * (size_t)s->nS);
  memcpy(m->sparent, s->sparent, sizeof(int32_t) * (size_t)s->nS);
  memcpy(m->spend, s->spend, (size_t)s->nS);
  return m;
}

int orc_cdt_build(int32_t nv, const double *xy, int32_t ns, const int32_t *seg,
                  orc_mesh **out, char *err, int32_t errlen) {
  *out = NULL;
  if (err && errlen > 0) err[0] = 0;
  cdt C = {0};
  C.err = err; C.errlen = errlen;
  if (nv < 3 || !xy || ns < 0 || (ns > 0 && !seg)) { seterr(&C, "bad arguments"); return ORC_E_ARG; }
  for (int64_t i = 0; i < 2 * (int64_t)nv; i++) {
    double a = fabs(xy[i]);
    if (!isfinite(xy[i]) || a > 0x1p20 || (a != 0.0 && a < 0x1p-100)) {
      seterr(&C, "coordinate not finite, or nonzero with magnitude outside [2^-100, 2^20]");
      return ORC_E_INPUT;
    }
  }
  int rc = ORC_OK;
  int32_t *ord = malloc(sizeof(int32_t) * (size_t)nv);
  C.vt = malloc(sizeof(int32_t) * (size_t)nv);
  uint8_t *onhull = calloc((size_t)nv, 1);
  int32_t *hull = malloc(sizeof(int32_t) * 2 * ((size_t)nv + 1));
  istack st = {0};
  if (!ord || !C.vt || !onhull || !hull) { rc = ORC_E_NOMEM; goto done; }
  C.nv = nv; C.xy = xy;
  for (int32_t i = 0; i < nv; i++) { ord[i] = i; C.vt[i] = -1; }
  g_sort_xy = xy;
  qsort(ord, (size_t)nv, sizeof(int32_t), cmp_xy);
  for (int32_t i = 1; i < nv; i++) {
    const double *p = xy + 2 * ord[i], *q = xy + 2 * ord[i - 1];
    if (p[0] == q[0] && p[1] == q[1]) { seterr(&C, "duplicate point"); rc = ORC_E_INPUT; goto done; }
  }
  /* segment validation */
  if (ns > 0) {
    segkey *sk = malloc(sizeof(segkey) * (size_t)ns);
    if (!sk) { rc = ORC_E_NOMEM; goto done; }
    for (int32_t s = 0; s < ns; s++) {
      int32_t a = seg[2 * s], b = seg[2 * s + 1];
      if (a < 0 || b < 0 || a >= nv || b >= nv || a == b) {
        free(sk); seterr(&C, "segment endpoint out of range or zero length"); rc = ORC_E_INPUT; goto done;
      }
      sk[s].a = a < b ? a : b; sk[s].b = a < b ? b : a; sk[s].s = s;
    }
    qsort(sk, (size_t)ns, sizeof(segkey), cmp_seg);
    for (int32_t s = 1; s < ns; s++)
      if (sk[s].a == sk[s - 1].a && sk[s].b == sk[s - 1].b) {
        free(sk); seterr(&C, "repeated segment"); rc = ORC_E_INPUT; goto done;
      }
    free(sk);
  }
  /* strictly convex hull, monotone chain over the (x, y)-sorted order */
  int32_t h = 0;
  for (int32_t k = 0; k < nv; k++) {
    int32_t p = ord[k];
    while (h >= 2 && orc_orient2d(xy + 2 * hull[h - 2], xy + 2 * hull[h - 1], xy + 2 * p) <= 0) h--;
    hull[h++] = p;
  }
  int32_t lower = h + 1;
  for (int32_t k = nv - 2; k >= 0; k--) {
    int32_t p = ord[k];
    while (h >= lower && orc_orient2d(xy + 2 * hull[h - 2], xy + 2 * hull[h - 1], xy + 2 * p) <= 0) h--;
    hull[h++] = p;
  }
  h--; /* last point repeats the first */
  if (h < 3) { seterr(&C, "all points are collinear"); rc = ORC_E_INPUT; goto done; }
  for (int32_t i = 0; i < h; i++) onhull[hull[i]] = 1;
  /* fan from hull[0] */
  for (int32_t i = 1; i + 1 < h; i++) {
    int32_t t = new_tri(&C, hull[0], hull[i], hull[i + 1]);
    if (t < 0) { rc = ORC_E_NOMEM; goto done; }
    if (i > 1) { C.tn[3 * t] = t - 1; C.tn[3 * (t - 1) + 2] = t; } /* share (h0, h_i) */
  }
  /* make the fan Delaunay */
  for (int32_t t = 0; t < C.nt; t++)
    for (int i = 0; i < 3; i++)
      if (C.tn[3 * t + i] > t)
        if (ipush(&st, C.tv[3 * t + i], C.tv[3 * t + NXT(i)])) { rc = ORC_E_NOMEM; goto done; }
  if (lawson(&C, &st)) { rc = ORC_E_NOMEM; goto done; }
  /* insert the rest in Hilbert order */
  {
    double lox = xy[0], hix = xy[0], loy = xy[1], hiy = xy[1];
    for (int32_t i = 0; i < nv; i++) {
      if (xy[2 * i] < lox) lox = xy[2 * i];
      if (xy[2 * i] > hix) hix = xy[2 * i];
      if (xy[2 * i + 1] < loy) loy = xy[2 * i + 1];
      if (xy[2 * i + 1] > hiy) hiy = xy[2 * i + 1];
    }
    double sx = hix > lox ? 65535.0 / (hix - lox) : 0, sy = hiy > loy ? 65535.0 / (hiy - loy) : 0;
    vkey *vk = malloc(sizeof(vkey) * (size_t)nv);
    if (!vk) { rc = ORC_E_NOMEM; goto done; }
    int32_t m = 0;
    for (int32_t i = 0; i < nv; i++) {
      if (onhull[i]) continue;
      uint32_t gx = (uint32_t)((xy[2 * i] - lox) * sx), gy = (uint32_t)((xy[2 * i + 1] - loy) * sy);
      if (gx > 65535) gx = 65535;
      if (gy > 65535) gy = 65535;
      vk[m].key = hilbert16(gx, gy);
      vk[m].v = i;
      m++;
    }
    qsort(vk, (size_t)m, sizeof(vkey), cmp_vkey);
    int32_t last = 0;
    for (int32_t k = 0; k < m; k++) {
      rc = insert_point(&C, vk[k].v, &last, &st);
      if (rc) { free(vk); goto done; }
    }
    free(vk);
  }
  /* segments */
  for (int32_t s = 0; s < ns; s++) {
    rc = recover_segment(&C, seg[2 * s], seg[2 * s + 1], s);
    if (rc) goto done;
  }
  /* global Lawson over non-constrained interior edges */
  for (int32_t t = 0; t < C.nt; t++)
    for (int i = 0; i < 3; i++)
      if (C.tn[3 * t + i] > t && C.tc[3 * t + i] < 0)
        if (ipush(&st, C.tv[3 * t + i], C.tv[3 * t + NXT(i)])) { rc = ORC_E_NOMEM; goto done; }
  if (lawson(&C, &st)) { rc = ORC_E_NOMEM; goto done; }
  /* hull edges must be segments */
  for (int32_t t = 0; t < C.nt; t++)
    for (int i = 0; i < 3; i++)
      if (C.tn[3 * t + i] < 0 && C.tc[3 * t + i] < 0) {
        seterr(&C, "a convex hull edge is not covered by a segment");
        rc = ORC_E_INPUT;
        goto done;
      }
  /* canonical form */
  {
    int32_t nt = C.nt;
    ctri *ct = malloc(sizeof(ctri) * (size_t)nt);
    int32_t *newid = malloc(sizeof(int32_t) * (size_t)nt);
    int32_t *rot = malloc(sizeof(int32_t) * (size_t)nt);
    if (!ct || !newid || !rot) { free(ct); free(newid); free(rot); rc = ORC_E_NOMEM; goto done; }
    for (int32_t t = 0; t < nt; t++) {
      int r = 0;
      for (int i = 1; i < 3; i++)
        if (C.tv[3 * t + i] < C.tv[3 * t + r]) r = i;
      rot[t] = r;
      for (int i = 0; i < 3; i++) ct[t].v[i] = C.tv[3 * t + (r + i) % 3];
      ct[t].old = t;
    }
    qsort(ct, (size_t)nt, sizeof(ctri), cmp_ctri);
    for (int32_t k = 0; k < nt; k++) newid[ct[k].old] = k;
    orc_mesh *M = mesh_alloc(nv + 16, nt + 16, ns + 16);
    if (!M) { free(ct); free(newid); free(rot); rc = ORC_E_NOMEM; goto done; }
    M->nV = nv; M->nT = nt; M->nS = ns; M->n_input_v = nv; M->n_input_s = ns;
    for (int32_t i = 0; i < nv; i++) { M->x[i] = xy[2 * i]; M->y[i] = xy[2 * i + 1]; M->vkind[i] = ORC_VK_INPUT; }
    for (int32_t k = 0; k < nt; k++) {
      int32_t t = ct[k].old, r = rot[t];
      for (int i = 0; i < 3; i++) {
        int src = (r + i) % 3;
        M->tv[3 * k + i] = C.tv[3 * t + src];
        int32_t n = C.tn[3 * t + src];
        M->tn[3 * k + i] = n < 0 ? -1 : newid[n];
        M->ts[3 * k + i] = C.tc[3 * t + src];
      }
    }
    for (int32_t s = 0; s < ns; s++) {
      M->sv[2 * s] = seg[2 * s]; M->sv[2 * s + 1] = seg[2 * s + 1];
      M->sparent[s] = s; M->spend[s] = 0;
    }
    free(ct); free(newid); free(rot);
    *out = M;
  }
done:
  free(ord); free(C.vt); free(onhull); free(hull); free(st.a);
  free(C.tv); free(C.tn); free(C.tc);
  return rc;
}

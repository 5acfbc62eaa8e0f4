/*
 * orc_ff.c -- Line 8 of Algorithm 1 (gDP2d) by Flip-Flop insertion
 * (Section 4.3), written from what the insertion produces (oracle).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Section 4.3 inserts the splitting points that survive Lines 6-7 with flips
 * (2-2) and flops (3-1): all points are added, and then points that are
 * redundant are taken out again, until the triangulation is a CDT in which no
 * point is redundant.  A point is redundant when it is connected by an edge
 * to a splitting point of higher priority (the two are Delaunay dependent),
 * or when it is a circumcenter that encroaches a subsegment, whose midpoint
 * is then inserted instead (the termination rules of Section 4.2).
 *
 * The CDT of a point set and a set of subsegments is unique under the
 * symbolic perturbation of the lifting map (smaller vertex id dominant), so
 * every flip and flop order that reaches a CDT reaches the same one.  The
 * oracle therefore takes the definition, not the flips:
 *
 *   Line 6  every splitting point claims the triangles it splits: the
 *           triangle that holds a circumcenter in its interior, both
 *           triangles of the edge a circumcenter lies on, the one or two
 *           triangles of a midpoint's subsegment.  Each triangle is split by
 *           at most one point, the one of highest priority: a point goes on
 *           only if it holds every triangle it claims.  A circumcenter on a
 *           subsegment encroaches it: it is dropped and the subsegment is
 *           flagged for its midpoint in this round.
 *   Line 8  S = the points that went on, ordered by priority (largest key
 *           first; that is also the order of their vertex ids).  Repeat:
 *             T = CDT(old vertices + S), each subsegment whose midpoint is in
 *                 S split there;
 *             a point p of S is redundant if an edge of T joins it to a
 *                 point of S of larger key, or if p is a circumcenter, the
 *                 edge opposite p in a triangle of T is a subsegment, and p
 *                 encroaches that subsegment (which is flagged);
 *             stop if no point is redundant; else remove every redundant
 *                 point from S.
 *           The last T is the new mesh.
 *
 * The triangle keys of this insertion must not depend on where a triangle is
 * stored (a flip process leaves triangles in slots of its own choosing), so it
 * runs with priority mode 2: a triangle's key tie-break is the pair of its
 * first two vertex ids (smallest id first), and the mesh is kept in the
 * canonical form of orc_cdt_build (each triangle rotated so that its smallest
 * vertex id comes first), which fixes the walk of Line 6 as well.
 */
#include "orc.h"
#include "orc_ff.h"

#include <stdlib.h>
#include <string.h>

#define NXT(i) (((i) + 1) % 3)
#define PRV(i) (((i) + 2) % 3)

typedef struct {
  uint64_t key;
  double x, y;
  int32_t cls;   /* 1 midpoint, 0 circumcenter */
  int32_t id;    /* subsegment k, or the bad triangle's slot */
  int32_t c0, c1; /* claimed triangles (c1 = -1: one) */
  int32_t edge;   /* circumcenter on edge `edge` of c0 (-1: inside) */
} ffpt;

/* The points S of the last Flip-Flop round, in key order, with what Line 6
   decided for them (kept for tests that drive other implementations of
   Line 8 from the same S). */
static struct {
  int64_t n, cap;
  double *xy;
  int32_t *cls, *id, *c0, *c1, *edge;
  uint64_t *key;
  int64_t nflag, capflag;
  int32_t *flagged; /* subsegments flagged for their midpoint when Line 8 starts */
} g_last;

static void record_last(const ffpt *pts, int64_t np, const int32_t *edge_of) {
  if (np > g_last.cap) {
    int64_t cap = np + 64;
    double *xy = realloc(g_last.xy, sizeof(double) * 2 * (size_t)cap);
    if (xy) g_last.xy = xy;
    int32_t *a = realloc(g_last.cls, sizeof(int32_t) * (size_t)cap);
    if (a) g_last.cls = a;
    int32_t *b = realloc(g_last.id, sizeof(int32_t) * (size_t)cap);
    if (b) g_last.id = b;
    int32_t *c = realloc(g_last.c0, sizeof(int32_t) * (size_t)cap);
    if (c) g_last.c0 = c;
    int32_t *d = realloc(g_last.c1, sizeof(int32_t) * (size_t)cap);
    if (d) g_last.c1 = d;
    int32_t *e = realloc(g_last.edge, sizeof(int32_t) * (size_t)cap);
    if (e) g_last.edge = e;
    uint64_t *k = realloc(g_last.key, sizeof(uint64_t) * (size_t)cap);
    if (k) g_last.key = k;
    if (!xy || !a || !b || !c || !d || !e || !k) { g_last.n = 0; return; }
    g_last.cap = cap;
  }
  for (int64_t i = 0; i < np; i++) {
    g_last.xy[2 * i] = pts[i].x; g_last.xy[2 * i + 1] = pts[i].y;
    g_last.cls[i] = pts[i].cls; g_last.id[i] = pts[i].id;
    g_last.c0[i] = pts[i].c0; g_last.c1[i] = pts[i].c1;
    g_last.edge[i] = edge_of[i];
    g_last.key[i] = pts[i].key;
  }
  g_last.n = np;
}

static void record_flagged(const uint8_t *mflag, int32_t nS) {
  int64_t n = 0;
  for (int32_t k = 0; k < nS; k++) n += mflag[k] != 0;
  if (n > g_last.capflag) {
    int32_t *a = realloc(g_last.flagged, sizeof(int32_t) * (size_t)(n + 64));
    if (!a) { g_last.nflag = 0; return; }
    g_last.flagged = a;
    g_last.capflag = n + 64;
  }
  n = 0;
  for (int32_t k = 0; k < nS; k++)
    if (mflag[k]) g_last.flagged[n++] = k;
  g_last.nflag = n;
}

int64_t orc_ff_last_flagged(int64_t cap, int32_t *ks) {
  int64_t n = g_last.nflag < cap ? g_last.nflag : cap;
  for (int64_t i = 0; i < n; i++) ks[i] = g_last.flagged[i];
  return g_last.nflag;
}

int64_t orc_ff_last_points(int64_t cap, double *xy, int32_t *cls, int32_t *id, int32_t *c0, int32_t *c1,
                           int32_t *edge, uint64_t *key) {
  int64_t n = g_last.n < cap ? g_last.n : cap;
  for (int64_t i = 0; i < n; i++) {
    xy[2 * i] = g_last.xy[2 * i]; xy[2 * i + 1] = g_last.xy[2 * i + 1];
    cls[i] = g_last.cls[i]; id[i] = g_last.id[i]; c0[i] = g_last.c0[i]; c1[i] = g_last.c1[i];
    edge[i] = g_last.edge[i]; key[i] = g_last.key[i];
  }
  return g_last.n;
}

static void ff_err(char *err, int32_t errlen, const char *msg) {
  if (err && errlen > 0) {
    strncpy(err, msg, (size_t)errlen - 1);
    err[errlen - 1] = 0;
  }
}

static int cmp_key_desc(const void *a, const void *b) {
  uint64_t x = ((const ffpt *)a)->key, y = ((const ffpt *)b)->key;
  return x > y ? -1 : (x < y);
}

/* Replaces m's triangles by those of T (same vertex ids, subsegment ids on
   edges = indices of T's segment list = m's subsegment ids). */
static int take_triangles(orc_mesh *m, const orc_mesh *T) {
  if (T->nT > m->capT) {
    int32_t cap = T->nT + T->nT / 2 + 16;
    int32_t *a = realloc(m->tv, sizeof(int32_t) * 3 * (size_t)cap);
    if (!a) return -1;
    m->tv = a;
    a = realloc(m->tn, sizeof(int32_t) * 3 * (size_t)cap);
    if (!a) return -1;
    m->tn = a;
    a = realloc(m->ts, sizeof(int32_t) * 3 * (size_t)cap);
    if (!a) return -1;
    m->ts = a;
    m->capT = cap;
  }
  memcpy(m->tv, T->tv, sizeof(int32_t) * 3 * (size_t)T->nT);
  memcpy(m->tn, T->tn, sizeof(int32_t) * 3 * (size_t)T->nT);
  memcpy(m->ts, T->ts, sizeof(int32_t) * 3 * (size_t)T->nT);
  m->nT = T->nT;
  return 0;
}

int orc_ff_canonical(orc_mesh *m, char *err, int32_t errlen) {
  double *xy = malloc(sizeof(double) * 2 * (size_t)m->nV);
  if (!xy) return ORC_E_NOMEM;
  for (int32_t v = 0; v < m->nV; v++) { xy[2 * v] = m->x[v]; xy[2 * v + 1] = m->y[v]; }
  orc_mesh *T = NULL;
  int rc = orc_cdt_build(m->nV, xy, m->nS, m->sv, &T, err, errlen);
  free(xy);
  if (rc) return rc;
  rc = take_triangles(m, T) ? ORC_E_NOMEM : ORC_OK;
  orc_mesh_free(T);
  return rc;
}

int orc_ff_round(orc_mesh *m, const orc_params *prm, const int32_t *tloc, const double *tpx, const double *tpy,
                 const uint64_t *tkey, uint8_t *mflag, const int32_t *sadj, orc_round_stats *st,
                 char *err, int32_t errlen) {
  const int32_t nV = m->nV, nT = m->nT, nS = m->nS;
  int rc = ORC_OK;
  ffpt *pts = NULL;
  int64_t np = 0;
  uint64_t *mark = calloc((size_t)nT + 1, sizeof(uint64_t));
  uint8_t *enc_flag = NULL; /* [nS + new halves] flagged by an encroaching circumcenter */
  uint8_t *alive = NULL, *redundant = NULL, *encr = NULL;
  int32_t *vid = NULL, *mid_of = NULL, *seg = NULL, *knew = NULL;
  double *xy = NULL;
  int64_t nfl = 0, capfl = 0;
  int32_t *fl_k = NULL;   /* flagged subsegments as (subsegment, half: 0 whole or first, 1 second) */
  uint8_t *fl_h = NULL;
  orc_mesh *T = NULL;
  pts = malloc(sizeof(ffpt) * ((size_t)nT + nS + 1));
  mid_of = malloc(sizeof(int32_t) * ((size_t)nS + 1));
  if (!mark || !pts || !mid_of) { rc = ORC_E_NOMEM; goto out; }

  /* ---- Line 6: claims.  Circumcenters first: one on a subsegment flags it. */
  for (int32_t t = 0; t < nT; t++) {
    int32_t loc = tloc[t];
    if (loc < 0) continue;
    double p[2] = {tpx[t], tpy[t]};
    int s[3];
    for (int i = 0; i < 3; i++) {
      double a[2] = {m->x[m->tv[3 * loc + i]], m->y[m->tv[3 * loc + i]]};
      double b[2] = {m->x[m->tv[3 * loc + NXT(i)]], m->y[m->tv[3 * loc + NXT(i)]]};
      s[i] = orc_orient2d(a, b, p);
    }
    int e = s[0] == 0 ? 0 : (s[1] == 0 ? 1 : (s[2] == 0 ? 2 : -1));
    ffpt *q = &pts[np];
    q->key = tkey[t]; q->x = p[0]; q->y = p[1]; q->cls = 0; q->id = t; q->c0 = loc; q->c1 = -1; q->edge = e;
    if (e >= 0) {
      int32_t k = m->ts[3 * loc + e];
      if (k >= 0) {
        mflag[k] = 1;
        if (st) st->n_enc_reject++;
        continue;
      }
      q->c1 = m->tn[3 * loc + e];
    }
    np++;
  }
  for (int32_t k = 0; k < nS; k++) {
    if (!mflag[k]) continue;
    if (st) st->n_mid_cand++;
    double mx, my;
    uint64_t key;
    orc_midpoint(m, k, &mx, &my, &key, prm->priority_mode, prm->split_mode);
    int32_t a = m->sv[2 * k], b = m->sv[2 * k + 1];
    if ((mx == m->x[a] && my == m->y[a]) || (mx == m->x[b] && my == m->y[b])) {
      if (st) st->n_unsplittable++;
      continue;
    }
    ffpt *q = &pts[np++];
    q->key = key; q->x = mx; q->y = my; q->cls = 1; q->id = k; q->edge = -1;
    q->c0 = sadj[2 * k] >= 0 ? sadj[2 * k] / 3 : -1;
    q->c1 = sadj[2 * k + 1] >= 0 ? sadj[2 * k + 1] / 3 : -1;
    if (q->c0 < 0) { q->c0 = q->c1; q->c1 = -1; }
    if (q->c0 < 0) { ff_err(err, errlen, "subsegment without an adjacent triangle"); rc = ORC_E_INPUT; goto out; }
  }
  for (int64_t i = 0; i < np; i++) {
    if (pts[i].key > mark[pts[i].c0]) mark[pts[i].c0] = pts[i].key;
    if (pts[i].c1 >= 0 && pts[i].key > mark[pts[i].c1]) mark[pts[i].c1] = pts[i].key;
  }
  {
    int64_t w = 0;
    for (int64_t i = 0; i < np; i++) {
      int own = mark[pts[i].c0] == pts[i].key && (pts[i].c1 < 0 || mark[pts[i].c1] == pts[i].key);
      if (own) pts[w++] = pts[i];
      else if (st) st->n_lost_mark++;
    }
    np = w;
  }
  qsort(pts, (size_t)np, sizeof(ffpt), cmp_key_desc);
  if (st) st->n_ff_points = np;
  {
    int32_t *edge_of = malloc(sizeof(int32_t) * ((size_t)np + 1));
    if (edge_of) {
      for (int64_t i = 0; i < np; i++) edge_of[i] = pts[i].edge;
      record_last(pts, np, edge_of);
      free(edge_of);
    }
    record_flagged(mflag, nS);
  }

  /* ---- Line 8: the CDT of the old vertices and S, until no point of S is
     redundant ---- */
  alive = malloc((size_t)np + 1);
  redundant = malloc((size_t)np + 1);
  encr = malloc((size_t)np + 1);
  vid = malloc(sizeof(int32_t) * ((size_t)np + 1));
  xy = malloc(sizeof(double) * 2 * ((size_t)nV + np + 1));
  seg = malloc(sizeof(int32_t) * 2 * ((size_t)nS + np + 1));
  int32_t *owner = malloc(sizeof(int32_t) * ((size_t)nV + np + 1)); /* vertex id -> index in pts */
  if (!alive || !redundant || !encr || !vid || !xy || !seg || !owner) { free(owner); rc = ORC_E_NOMEM; goto out; }
  for (int64_t i = 0; i < np; i++) alive[i] = 1;
  for (int32_t v = 0; v < nV; v++) { xy[2 * v] = m->x[v]; xy[2 * v + 1] = m->y[v]; }
  int64_t iters = 0;
  for (;;) {
    iters++;
    /* vertex ids and the segment list of this S */
    int32_t nv = nV, nsg = nS;
    for (int32_t k = 0; k < nS; k++) mid_of[k] = -1;
    for (int64_t i = 0; i < np; i++) {
      if (!alive[i]) continue;
      vid[i] = nv;
      owner[nv] = (int32_t)i;
      xy[2 * nv] = pts[i].x;
      xy[2 * nv + 1] = pts[i].y;
      nv++;
      if (pts[i].cls) mid_of[pts[i].id] = (int32_t)i;
    }
    for (int32_t k = 0; k < nS; k++) {
      seg[2 * k] = m->sv[2 * k];
      seg[2 * k + 1] = mid_of[k] >= 0 ? vid[mid_of[k]] : m->sv[2 * k + 1];
    }
    for (int64_t i = 0; i < np; i++)
      if (alive[i] && pts[i].cls) {
        seg[2 * nsg] = vid[i];
        seg[2 * nsg + 1] = m->sv[2 * pts[i].id + 1];
        nsg++;
      }
    if (T) { orc_mesh_free(T); T = NULL; }
    rc = orc_cdt_build(nv, xy, nsg, seg, &T, err, errlen);
    if (rc) { free(owner); goto out; }
    /* redundancy */
    for (int64_t i = 0; i < np; i++) { redundant[i] = 0; encr[i] = 0; }
    for (int32_t t = 0; t < T->nT; t++)
      for (int i = 0; i < 3; i++) {
        int32_t v = T->tv[3 * t + i];
        if (v < nV) continue;
        int32_t pi = owner[v];
        int32_t u = T->tv[3 * t + NXT(i)], w = T->tv[3 * t + PRV(i)];
        if ((u >= nV && pts[owner[u]].key > pts[pi].key) || (w >= nV && pts[owner[w]].key > pts[pi].key))
          redundant[pi] = 1;
        int32_t sk = T->ts[3 * t + NXT(i)]; /* edge (u, w), opposite v */
        if (!pts[pi].cls && sk >= 0) {
          double a[2] = {xy[2 * u], xy[2 * u + 1]}, b[2] = {xy[2 * w], xy[2 * w + 1]};
          double p[2] = {pts[pi].x, pts[pi].y};
          if (orc_encroaches(prm->encroach_mode, a, b, p)) {
            redundant[pi] = 1;
            encr[pi] = 1;
            /* remember the flagged subsegment: index < nS is k itself (its
               first half when split); index >= nS is the second half of the
               split subsegment of the sk-nS-th alive midpoint */
            if (nfl + 1 > capfl) {
              capfl = capfl ? 2 * capfl : 256;
              int32_t *a1 = realloc(fl_k, sizeof(int32_t) * (size_t)capfl);
              uint8_t *a2 = a1 ? realloc(fl_h, (size_t)capfl) : NULL;
              if (a1) fl_k = a1;
              if (!a1 || !a2) { free(owner); rc = ORC_E_NOMEM; goto out; }
              fl_h = a2;
            }
            if (sk < nS) { fl_k[nfl] = sk; fl_h[nfl] = 0; }
            else {
              int32_t r = sk - nS, k = -1;
              for (int64_t j = 0; j < np && k < 0; j++)
                if (alive[j] && pts[j].cls && r-- == 0) k = pts[j].id;
              fl_k[nfl] = k; fl_h[nfl] = 1;
            }
            nfl++;
          }
        }
      }
    int64_t nred = 0;
    for (int64_t i = 0; i < np; i++)
      if (alive[i] && redundant[i]) {
        nred++;
        alive[i] = 0;
        if (st) { if (encr[i]) st->n_enc_reject++; else st->n_dep_drop++; }
      }
    if (nred == 0) break;
  }
  free(owner);
  if (st) st->n_ff_iters = iters;

  /* ---- install T ---- */
  int64_t nwin = 0, nmid = 0;
  for (int64_t i = 0; i < np; i++)
    if (alive[i]) { nwin++; nmid += pts[i].cls; }
  {
    /* capacity: vertices and subsegments */
    int32_t needV = nV + (int32_t)nwin, needS = nS + (int32_t)nmid;
    if (needV > m->capV) {
      int32_t cap = needV + needV / 2 + 16;
      double *x = realloc(m->x, sizeof(double) * (size_t)cap);
      if (!x) { rc = ORC_E_NOMEM; goto out; }
      m->x = x;
      double *y = realloc(m->y, sizeof(double) * (size_t)cap);
      if (!y) { rc = ORC_E_NOMEM; goto out; }
      m->y = y;
      int32_t *kd = realloc(m->vkind, sizeof(int32_t) * (size_t)cap);
      if (!kd) { rc = ORC_E_NOMEM; goto out; }
      m->vkind = kd;
      m->capV = cap;
    }
    if (needS > m->capS) {
      int32_t cap = needS + needS / 2 + 16;
      int32_t *a = realloc(m->sv, sizeof(int32_t) * 2 * (size_t)cap);
      if (!a) { rc = ORC_E_NOMEM; goto out; }
      m->sv = a;
      a = realloc(m->sparent, sizeof(int32_t) * (size_t)cap);
      if (!a) { rc = ORC_E_NOMEM; goto out; }
      m->sparent = a;
      uint8_t *b = realloc(m->spend, (size_t)cap);
      if (!b) { rc = ORC_E_NOMEM; goto out; }
      m->spend = b;
      m->capS = cap;
    }
  }
  knew = malloc(sizeof(int32_t) * ((size_t)nS + 1));
  enc_flag = calloc((size_t)nS + (size_t)nmid + 1, 1);
  if (!knew || !enc_flag) { rc = ORC_E_NOMEM; goto out; }
  for (int32_t k = 0; k < nS; k++) knew[k] = -1;
  {
    int32_t v = nV, s = nS;
    for (int64_t i = 0; i < np; i++) {
      if (!alive[i]) continue;
      m->x[v] = pts[i].x;
      m->y[v] = pts[i].y;
      m->vkind[v] = pts[i].cls ? ORC_VK_MIDPOINT : ORC_VK_CIRCUMCENTER;
      if (pts[i].cls) {
        int32_t k = pts[i].id;
        knew[k] = s;
        m->sv[2 * s] = v;
        m->sv[2 * s + 1] = m->sv[2 * k + 1];
        m->sparent[s] = m->sparent[k];
        m->spend[s] = 0;
        m->sv[2 * k + 1] = v;
        s++;
        if (st) st->n_ins_mid++;
      } else if (st) {
        st->n_ins_cc++;
      }
      v++;
    }
  }
  if (take_triangles(m, T)) { rc = ORC_E_NOMEM; goto out; }
  /* flags raised by encroaching circumcenters, on the final subsegment ids */
  for (int64_t j = 0; j < nfl; j++) {
    int32_t k = fl_k[j];
    if (k < 0) continue;
    enc_flag[fl_h[j] && knew[k] >= 0 ? knew[k] : k] = 1;
  }
  /* ---- R11: pending flags.  A subsegment that was pending or flagged and
     was not split stays pending; a flag raised in Line 8 holds on the piece
     it names (a flag on the second half of a split that was undone lands on
     the whole subsegment). ---- */
  for (int32_t k = 0; k < nS; k++) {
    int split = knew[k] >= 0;
    m->spend[k] = (((m->spend[k] || mflag[k]) && !split) || enc_flag[k]) ? 1 : 0;
  }
  for (int32_t k = nS; k < nS + (int32_t)nmid; k++) m->spend[k] = enc_flag[k];
  m->nV = nV + (int32_t)nwin;
  m->nS = nS + (int32_t)nmid;
  if (nwin == 0) {
    int any = 0;
    for (int64_t j = 0; j < nfl; j++) any |= fl_k[j] >= 0;
    if (!any) {
      ff_err(err, errlen, "round had candidates but inserted nothing");
      rc = ORC_E_STALL;
      goto out;
    }
  }
out:
  free(mark); free(enc_flag); free(pts); free(alive); free(redundant); free(encr); free(vid);
  free(mid_of); free(seg); free(knew); free(xy); free(fl_k); free(fl_h);
  if (T) orc_mesh_free(T);
  return rc;
}

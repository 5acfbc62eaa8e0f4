/*
 * orc_refine.c -- Lines 2-9 of Algorithm 1 (gDP2d) as a deterministic,
 * round-synchronous refinement, executed sequentially (oracle).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * One round, in the order of Algorithm 1:
 *   R1 (Line 3)  collect encroached subsegments (pending flag, or an adjacent
 *                apex strictly inside the diametric circle, Ruppert mode, or
 *                inside the diametric lens, Chew mode; Section 4.1/4.2
 *                definition of encroachment) and bad triangles
 *                (circumradius^2 > B^2 * shortest edge^2, the radius-edge
 *                form of the angle bound, or, when a length bound l is set,
 *                an edge longer than l; Section 4.1).  Stop when there are
 *                none.
 *   R2 (Line 5)  splitting points: midpoints of subsegments, circumcenters of
 *                triangles; priorities per Section 4.3 (midpoints first, then
 *                larger length / area first), made unique by a fixed
 *                bijective hash of the element id.
 *   R3 (Rule 2)  optional cap: keep only the K highest priorities.
 *   R4 (Line 6)  locate each circumcenter by a visibility walk from its
 *                triangle; a walk stopped only by subsegments turns into the
 *                midpoint candidate of the first blocking subsegment.
 *   R5 (Line 7/8) circumcenter cavities (Bowyer-Watson growth across
 *                non-subsegment edges whose far triangle's circumcircle holds
 *                the point strictly); a circumcenter that encroaches a
 *                subsegment on its cavity boundary is dropped and that
 *                subsegment is split instead (Section 4.2 termination rule).
 *   R6           midpoint cavities, grown from both sides of the subsegment.
 *   R8           priority marks: every triangle keeps the largest key of the
 *                cavities that contain it; a point survives only if it holds
 *                every triangle of its cavity (Section 5.2 marking rule, taken
 *                after all marks are placed so the result does not depend on
 *                timing).
 *   R9           Delaunay dependency (Section 5.2): for surviving p, q whose
 *                cavities share a non-subsegment edge (u,v), if q lies strictly
 *                inside the circle (u,v,p) the lower priority is dropped.
 *   R10          insert: vertex ids, triangle slots and subsegment ids are
 *                assigned in a fixed order; every new triangle is (u, v, p)
 *                over a cavity boundary edge (u, v).
 *   R11          pending flags and the round counter.
 */
#include "orc.h"
#include "orc_ff.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NXT(i) (((i) + 1) % 3)
#define PRV(i) (((i) + 2) % 3)

typedef struct {
  int cls;          /* 1 = subsegment midpoint, 0 = circumcenter */
  int32_t id;       /* subsegment k or triangle slot t */
  double px, py;
  uint64_t key;
  int64_t cav_off;  /* into the cavity pool (sorted slots) */
  int32_t ncav;
  int alive, w0, win;
} cand;

typedef struct { int32_t *a; int64_t n, cap; } ivec;
static int ivec_push(ivec *v, int32_t x) {
  if (v->n + 1 > v->cap) {
    int64_t cap = v->cap ? v->cap * 2 : 1024;
    int32_t *a = realloc(v->a, sizeof(int32_t) * (size_t)cap);
    if (!a) return -1;
    v->a = a; v->cap = cap;
  }
  v->a[v->n++] = x;
  return 0;
}

static void set_err(char *err, int32_t errlen, const char *msg) {
  if (err && errlen > 0) {
    strncpy(err, msg, (size_t)errlen - 1);
    err[errlen - 1] = 0;
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return x < y ? -1 : (x > y);
}

static int cmp_u64_desc(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x > y ? -1 : (x < y);
}

static int ensure_cap(orc_mesh *m, int32_t needV, int32_t needT, int32_t needS) {
  if (needV > m->capV) {
    int32_t cap = m->capV;
    while (cap < needV) cap = cap + cap / 2 + 16;
    double *x = realloc(m->x, sizeof(double) * (size_t)cap);
    if (!x) return -1;
    m->x = x;
    double *y = realloc(m->y, sizeof(double) * (size_t)cap);
    if (!y) return -1;
    m->y = y;
    int32_t *k = realloc(m->vkind, sizeof(int32_t) * (size_t)cap);
    if (!k) return -1;
    m->vkind = k;
    m->capV = cap;
  }
  if (needT > m->capT) {
    int32_t cap = m->capT;
    while (cap < needT) cap = cap + cap / 2 + 16;
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
  if (needS > m->capS) {
    int32_t cap = m->capS;
    while (cap < needS) cap = cap + cap / 2 + 16;
    int32_t *a = realloc(m->sv, sizeof(int32_t) * 2 * (size_t)cap);
    if (!a) return -1;
    m->sv = a;
    a = realloc(m->sparent, sizeof(int32_t) * (size_t)cap);
    if (!a) return -1;
    m->sparent = a;
    uint8_t *b = realloc(m->spend, (size_t)cap);
    if (!b) return -1;
    m->spend = b;
    m->capS = cap;
  }
  return 0;
}

static inline void vxy(const orc_mesh *m, int32_t v, double *p) { p[0] = m->x[v]; p[1] = m->y[v]; }

/* Is slot t in the sorted cavity list? */
static int in_cav(const int32_t *cav, int32_t n, int32_t t) {
  int32_t lo = 0, hi = n - 1;
  while (lo <= hi) {
    int32_t mid = (lo + hi) / 2;
    if (cav[mid] == t) return 1;
    if (cav[mid] < t) lo = mid + 1; else hi = mid - 1;
  }
  return 0;
}

/* Constrained Bowyer-Watson growth from the seeds: cross a non-subsegment
   edge iff the far triangle's circumcircle strictly contains p.  Appends the
   cavity (sorted ascending) to the pool. */
static int grow_cavity(const orc_mesh *m, const int32_t *seeds, int nseeds, const double *p,
                       int32_t *stamp, int32_t epoch, ivec *pool, int64_t *off, int32_t *ncav) {
  int64_t base = pool->n;
  for (int s = 0; s < nseeds; s++) {
    if (stamp[seeds[s]] == epoch) continue;
    stamp[seeds[s]] = epoch;
    if (ivec_push(pool, seeds[s])) return -1;
  }
  for (int64_t h = base; h < pool->n; h++) {
    int32_t t = pool->a[h];
    for (int i = 0; i < 3; i++) {
      if (m->ts[3 * t + i] >= 0) continue;
      int32_t n = m->tn[3 * t + i];
      if (n < 0 || stamp[n] == epoch) continue;
      double a[2], b[2], c[2];
      vxy(m, m->tv[3 * n], a);
      vxy(m, m->tv[3 * n + 1], b);
      vxy(m, m->tv[3 * n + 2], c);
      if (orc_incircle(a, b, c, p) > 0) {
        stamp[n] = epoch;
        if (ivec_push(pool, n)) return -1;
      }
    }
  }
  *off = base;
  *ncav = (int32_t)(pool->n - base);
  qsort(pool->a + base, (size_t)*ncav, sizeof(int32_t), cmp_i32);
  return 0;
}

/* Boundary edges of a cavity in canonical order: cavity slots ascending,
   edge index 0..2; the subsegment being split (skip_k) is not a boundary. */
typedef struct { int32_t t, i, u, v, n, ts; } bedge;

static int cavity_boundary(const orc_mesh *m, const int32_t *cav, int32_t ncav, int32_t skip_k,
                           bedge **out, int32_t *nb, int32_t *capb) {
  *nb = 0;
  for (int32_t c = 0; c < ncav; c++) {
    int32_t t = cav[c];
    for (int i = 0; i < 3; i++) {
      int32_t s = m->ts[3 * t + i];
      if (skip_k >= 0 && s == skip_k) continue;
      int32_t n = m->tn[3 * t + i];
      if (s < 0 && n >= 0 && in_cav(cav, ncav, n)) continue;
      if (*nb + 1 > *capb) {
        int32_t cap = *capb ? *capb * 2 : 64;
        bedge *a = realloc(*out, sizeof(bedge) * (size_t)cap);
        if (!a) return -1;
        *out = a;
        *capb = cap;
      }
      bedge *e = &(*out)[(*nb)++];
      e->t = t; e->i = i;
      e->u = m->tv[3 * t + i];
      e->v = m->tv[3 * t + NXT(i)];
      e->n = n;
      e->ts = s;
    }
  }
  return 0;
}

/* Every fan triangle (u, v, p) must be strictly CCW and the cavity must be a
   disk with all vertices on its boundary: #boundary - #cavity = expect. */
static int fan_ok(const orc_mesh *m, const bedge *b, int32_t nb, int32_t ncav, const double *p,
                  int expect) {
  if (nb - ncav != expect) return 0;
  for (int32_t j = 0; j < nb; j++) {
    double a[2], c[2];
    vxy(m, b[j].u, a);
    vxy(m, b[j].v, c);
    if (orc_orient2d(a, c, p) <= 0) return 0;
  }
  return 1;
}

typedef struct {
  int32_t slot, u, v, n, jn, ts;
} fanrec;

static const cand *g_cands;
static int cmp_win_idx(const void *a, const void *b) {
  const cand *p = &g_cands[*(const int32_t *)a], *q = &g_cands[*(const int32_t *)b];
  if (p->cls != q->cls) return p->cls > q->cls ? -1 : 1; /* midpoints first */
  return p->id < q->id ? -1 : (p->id > q->id);
}

static int edge_index(const orc_mesh *m, int32_t t, int32_t u, int32_t v) {
  for (int i = 0; i < 3; i++)
    if (m->tv[3 * t + i] == u && m->tv[3 * t + NXT(i)] == v) return i;
  return -1;
}

/* The first n triangles of the cavity growth order (seed, then breadth
   first across non-subsegment edges whose far triangle's circumcircle
   strictly holds p, edges in index order); stops as soon as n are taken. */
static int32_t approx_cavity(const orc_mesh *m, int32_t seed, const double *p, int32_t n,
                             int32_t *stamp, int32_t epoch, int32_t *out) {
  int32_t len = 0;
  out[len++] = seed;
  stamp[seed] = epoch;
  for (int32_t h = 0; h < len && len < n; h++) {
    int32_t t = out[h];
    for (int i = 0; i < 3 && len < n; i++) {
      if (m->ts[3 * t + i] >= 0) continue;
      int32_t o = m->tn[3 * t + i];
      if (o < 0 || stamp[o] == epoch) continue;
      double a[2], b[2], c[2];
      vxy(m, m->tv[3 * o], a);
      vxy(m, m->tv[3 * o + 1], b);
      vxy(m, m->tv[3 * o + 2], c);
      if (orc_incircle(a, b, c, p) > 0) {
        stamp[o] = epoch;
        out[len++] = o;
      }
    }
  }
  return len;
}

/* One round.  Returns 1 if the mesh had nothing to refine, 0 after a round,
   <0 on error. */
static int one_round(orc_mesh *m, double B2, const orc_params *prm, orc_round_stats *st,
                     int only_check, char *err, int32_t errlen) {
  const int32_t nT = m->nT, nS = m->nS, nV = m->nV;
  int rc = 0;
  int pm = prm->priority_mode;
  uint8_t *enc = calloc((size_t)nS + 1, 1);
  uint8_t *mflag = calloc((size_t)nS + 1, 1);
  int32_t *sadj = malloc(sizeof(int32_t) * 2 * ((size_t)nS + 1));
  uint8_t *bad = calloc((size_t)nT + 1, 1);
  double *tpx = malloc(sizeof(double) * ((size_t)nT + 1));
  double *tpy = malloc(sizeof(double) * ((size_t)nT + 1));
  uint64_t *tkey = malloc(sizeof(uint64_t) * ((size_t)nT + 1));
  uint64_t *mark = calloc((size_t)nT + 1, sizeof(uint64_t));
  int32_t *markc = malloc(sizeof(int32_t) * ((size_t)nT + 1));
  int32_t *stamp = malloc(sizeof(int32_t) * ((size_t)nT + 1));
  cand *cands = NULL;
  int64_t ncand = 0, capcand = 0;
  ivec pool = {0};
  bedge *bb = NULL;
  int32_t nb = 0, capb = 0;
  fanrec *fr = NULL;
  int32_t *repl = NULL;
  uint8_t *inW = NULL;
  int32_t *wl = NULL;
  int64_t *foff = NULL;
  uint64_t *keys = NULL;
  int32_t *tloc = NULL;
  if (!enc || !mflag || !sadj || !bad || !tpx || !tpy || !tkey || !mark || !markc || !stamp) {
    rc = ORC_E_NOMEM;
    goto out;
  }
  for (int32_t t = 0; t < nT; t++) stamp[t] = -1;
  for (int64_t k = 0; k < 2 * (int64_t)nS; k++) sadj[k] = -1;
  if (pm == 2 && nV >= (1 << 22)) {
    set_err(err, errlen, "priority mode 2 keys hold vertex ids below 2^22");
    rc = ORC_E_INPUT;
    goto out;
  }

  /* ---- R1: collect ---- */
  for (int32_t k = 0; k < nS; k++) enc[k] = m->spend[k] ? 1 : 0;
  for (int32_t t = 0; t < nT; t++) {
    for (int i = 0; i < 3; i++) {
      int32_t k = m->ts[3 * t + i];
      if (k < 0) continue;
      int32_t u = m->tv[3 * t + i], v = m->tv[3 * t + NXT(i)], c = m->tv[3 * t + PRV(i)];
      int side = (u == m->sv[2 * k] && v == m->sv[2 * k + 1]) ? 0 : 1;
      sadj[2 * k + side] = 3 * t + i;
      double a[2], b[2], cc[2];
      vxy(m, u, a);
      vxy(m, v, b);
      vxy(m, c, cc);
      if (orc_encroaches(prm->encroach_mode, a, b, cc)) enc[k] = 1;
    }
  }
  int64_t n_enc = 0, n_bad = 0;
  for (int32_t k = 0; k < nS; k++) n_enc += enc[k];
  for (int32_t t = 0; t < nT; t++) {
    int32_t b;
    orc_circumcenter(m, t, B2, prm->max_edge_len_sq, &tpx[t], &tpy[t], &b, &tkey[t], pm);
    bad[t] = (uint8_t)b;
    n_bad += b;
  }
  if (st) { memset(st, 0, sizeof *st); st->n_enc = n_enc; st->n_bad = n_bad; }
  if (n_enc == 0 && n_bad == 0) { rc = 1; goto out; }
  if (only_check) { rc = 2; goto out; }

  /* ---- R2/R3: priorities and the optional cap ---- */
  uint64_t thresh = 0;
  if (prm->cand_cap_K > 0 && n_enc + n_bad > prm->cand_cap_K) {
    keys = malloc(sizeof(uint64_t) * (size_t)(n_enc + n_bad));
    if (!keys) { rc = ORC_E_NOMEM; goto out; }
    int64_t nk = 0;
    for (int32_t k = 0; k < nS; k++)
      if (enc[k]) {
        double mx, my;
        uint64_t key;
        orc_midpoint(m, k, &mx, &my, &key, pm, prm->split_mode);
        keys[nk++] = key;
      }
    for (int32_t t = 0; t < nT; t++)
      if (bad[t]) keys[nk++] = tkey[t];
    qsort(keys, (size_t)nk, sizeof(uint64_t), cmp_u64_desc);
    thresh = keys[prm->cand_cap_K - 1];
  }
  for (int32_t k = 0; k < nS; k++)
    if (enc[k]) {
      double mx, my;
      uint64_t key;
      orc_midpoint(m, k, &mx, &my, &key, pm, prm->split_mode);
      if (key >= thresh) { mflag[k] = 1; if (st) st->n_kept_mid++; }
    }

  /* ---- R4: locate circumcenters ---- */
  tloc = malloc(sizeof(int32_t) * ((size_t)nT + 1));
  if (!tloc) { rc = ORC_E_NOMEM; goto out; }
  for (int32_t t = 0; t < nT; t++) {
    tloc[t] = -1;
    if (!bad[t] || tkey[t] < thresh) continue;
    if (st) st->n_kept_cc++;
    double p[2] = {tpx[t], tpy[t]};
    int32_t cur = t;
    int64_t steps = 0;
    int outcome = 0; /* 1 found, 2 coincident, 3 blocked */
    int32_t blocked_k = -1;
    for (;;) {
      if (++steps > (1 << 20)) { set_err(err, errlen, "locate walk exceeded its step cap"); rc = ORC_E_WALK; goto out; }
      int s[3];
      for (int i = 0; i < 3; i++) {
        double a[2], b[2];
        vxy(m, m->tv[3 * cur + i], a);
        vxy(m, m->tv[3 * cur + NXT(i)], b);
        s[i] = orc_orient2d(a, b, p);
      }
      if (s[0] >= 0 && s[1] >= 0 && s[2] >= 0) {
        int nz = (s[0] == 0) + (s[1] == 0) + (s[2] == 0);
        outcome = nz >= 2 ? 2 : 1;
        break;
      }
      int moved = 0, first_neg = -1;
      for (int i = 0; i < 3; i++) {
        if (s[i] >= 0) continue;
        if (first_neg < 0) first_neg = i;
        if (m->ts[3 * cur + i] < 0 && m->tn[3 * cur + i] >= 0) {
          cur = m->tn[3 * cur + i];
          moved = 1;
          break;
        }
      }
      if (!moved) {
        outcome = 3;
        blocked_k = m->ts[3 * cur + first_neg];
        break;
      }
    }
    if (st) st->walk_steps += steps;
    if (outcome == 2) { if (st) st->n_coincident++; continue; }
    if (outcome == 3) {
      if (blocked_k < 0) { set_err(err, errlen, "walk blocked by a hull edge without a segment"); rc = ORC_E_INPUT; goto out; }
      mflag[blocked_k] = 1;
      if (st) st->n_blocked++;
      continue;
    }
    tloc[t] = cur;
  }

  /* ---- F1 (Line 6, optional): one circumcenter per located triangle, the
     highest priority one ---- */
  if (prm->prefilter_f1) {
    for (int32_t t = 0; t < nT; t++)
      if (tloc[t] >= 0 && tkey[t] > mark[tloc[t]]) mark[tloc[t]] = tkey[t];
    for (int32_t t = 0; t < nT; t++)
      if (tloc[t] >= 0 && mark[tloc[t]] != tkey[t]) {
        tloc[t] = -1;
        if (st) st->n_f1_drop++;
      }
    for (int32_t t = 0; t < nT; t++) mark[t] = 0;
  }

  /* ---- F2 (Line 7, optional): approximate cavities of n triangles, first
     n of the growth order; a circumcenter that does not hold the largest key
     on all of them is dropped ---- */
  if (prm->cavity_approx_n > 0) {
    int32_t n = prm->cavity_approx_n;
    int32_t *ap = malloc(sizeof(int32_t) * (size_t)n);
    if (!ap) { rc = ORC_E_NOMEM; goto out; }
    int32_t epoch = 0x40000000;
    for (int pass = 0; pass < 2; pass++) {
      for (int32_t t = 0; t < nT; t++) {
        if (tloc[t] < 0) continue;
        double p[2] = {tpx[t], tpy[t]};
        int32_t len = approx_cavity(m, tloc[t], p, n, stamp, epoch++, ap);
        int own = 1;
        for (int32_t j = 0; j < len; j++) {
          if (pass == 0) { if (tkey[t] > mark[ap[j]]) mark[ap[j]] = tkey[t]; }
          else if (mark[ap[j]] != tkey[t]) own = 0;
        }
        if (pass == 1 && !own) {
          tloc[t] = -2; /* dropped; marks of pass 0 stay until cleared below */
          if (st) st->n_f2_drop++;
        }
      }
    }
    free(ap);
    for (int32_t t = 0; t < nT; t++) {
      mark[t] = 0;
      stamp[t] = -1;
    }
    for (int32_t t = 0; t < nT; t++)
      if (tloc[t] == -2) tloc[t] = -1;
  }

  /* ---- Line 8 by Flip-Flop (orc_ff.c) in place of R5-R10 ---- */
  if (prm->insert_mode == 1) {
    rc = orc_ff_round(m, prm, tloc, tpx, tpy, tkey, mflag, sadj, st, err, errlen);
    if (rc == 0) m->rounds++;
    goto out;
  }

  /* ---- R5: circumcenter cavities ---- */
  for (int32_t t = 0; t < nT; t++) {
    if (tloc[t] < 0) continue;
    double p[2] = {tpx[t], tpy[t]};
    int32_t cur = tloc[t];
    if (ncand + 1 > capcand) {
      capcand = capcand ? capcand * 2 : 1024;
      cand *a = realloc(cands, sizeof(cand) * (size_t)capcand);
      if (!a) { rc = ORC_E_NOMEM; goto out; }
      cands = a;
    }
    cand *cd = &cands[ncand];
    memset(cd, 0, sizeof *cd);
    cd->cls = 0; cd->id = t; cd->px = p[0]; cd->py = p[1]; cd->key = tkey[t];
    if (grow_cavity(m, &cur, 1, p, stamp, (int32_t)(ncand), &pool, &cd->cav_off, &cd->ncav)) { rc = ORC_E_NOMEM; goto out; }
    if (cavity_boundary(m, pool.a + cd->cav_off, cd->ncav, -1, &bb, &nb, &capb)) { rc = ORC_E_NOMEM; goto out; }
    int encroaches = 0;
    for (int32_t j = 0; j < nb; j++) {
      if (bb[j].ts < 0) continue;
      double a[2], b[2];
      vxy(m, bb[j].u, a);
      vxy(m, bb[j].v, b);
      if (orc_encroaches(prm->encroach_mode, a, b, p)) { mflag[bb[j].ts] = 1; encroaches = 1; }
    }
    if (st) {
      st->cav_tri_total += cd->ncav;
      if (cd->ncav > st->cav_max) st->cav_max = cd->ncav;
    }
    if (encroaches) { if (st) st->n_enc_reject++; ncand++; continue; }
    if (!fan_ok(m, bb, nb, cd->ncav, p, 2)) { if (st) st->n_fan_invalid++; ncand++; continue; }
    cd->alive = 1;
    ncand++;
  }

  /* ---- R6: midpoint cavities ---- */
  for (int32_t k = 0; k < nS; k++) {
    if (!mflag[k]) continue;
    if (st) st->n_mid_cand++;
    double mx, my;
    uint64_t key;
    orc_midpoint(m, k, &mx, &my, &key, pm, prm->split_mode);
    int32_t a = m->sv[2 * k], b = m->sv[2 * k + 1];
    if ((mx == m->x[a] && my == m->y[a]) || (mx == m->x[b] && my == m->y[b])) {
      if (st) st->n_unsplittable++;
      continue;
    }
    int32_t seeds[2];
    int ns = 0;
    for (int side = 0; side < 2; side++)
      if (sadj[2 * k + side] >= 0) seeds[ns++] = sadj[2 * k + side] / 3;
    if (ns == 0) { set_err(err, errlen, "subsegment without an adjacent triangle"); rc = ORC_E_INPUT; goto out; }
    if (ncand + 1 > capcand) {
      capcand = capcand ? capcand * 2 : 1024;
      cand *aa = realloc(cands, sizeof(cand) * (size_t)capcand);
      if (!aa) { rc = ORC_E_NOMEM; goto out; }
      cands = aa;
    }
    cand *cd = &cands[ncand];
    memset(cd, 0, sizeof *cd);
    cd->cls = 1; cd->id = k; cd->px = mx; cd->py = my; cd->key = key;
    double p[2] = {mx, my};
    if (grow_cavity(m, seeds, ns, p, stamp, (int32_t)ncand, &pool, &cd->cav_off, &cd->ncav)) { rc = ORC_E_NOMEM; goto out; }
    if (cavity_boundary(m, pool.a + cd->cav_off, cd->ncav, k, &bb, &nb, &capb)) { rc = ORC_E_NOMEM; goto out; }
    if (st) {
      st->cav_tri_total += cd->ncav;
      if (cd->ncav > st->cav_max) st->cav_max = cd->ncav;
    }
    if (!fan_ok(m, bb, nb, cd->ncav, p, ns == 2 ? 2 : 1)) { if (st) st->n_fan_invalid++; ncand++; continue; }
    cd->alive = 1;
    ncand++;
  }

  /* ---- R8: marks and ownership ---- */
  for (int64_t c = 0; c < ncand; c++) {
    if (!cands[c].alive) continue;
    const int32_t *cav = pool.a + cands[c].cav_off;
    for (int32_t j = 0; j < cands[c].ncav; j++) {
      int32_t t = cav[j];
      if (cands[c].key > mark[t]) { mark[t] = cands[c].key; markc[t] = (int32_t)c; }
    }
  }
  for (int64_t c = 0; c < ncand; c++) {
    if (!cands[c].alive) continue;
    const int32_t *cav = pool.a + cands[c].cav_off;
    int own = 1;
    for (int32_t j = 0; j < cands[c].ncav; j++)
      if (mark[cav[j]] != cands[c].key) { own = 0; break; }
    cands[c].w0 = own;
    if (!own && st) st->n_lost_mark++;
  }

  /* ---- R9: Delaunay dependency between neighbouring winners ---- */
  for (int64_t c = 0; c < ncand; c++) {
    if (!cands[c].w0) continue;
    const int32_t *cav = pool.a + cands[c].cav_off;
    if (cavity_boundary(m, cav, cands[c].ncav, cands[c].cls ? cands[c].id : -1, &bb, &nb, &capb)) { rc = ORC_E_NOMEM; goto out; }
    int drop = 0;
    double p[2] = {cands[c].px, cands[c].py};
    for (int32_t j = 0; j < nb && !drop; j++) {
      if (bb[j].ts >= 0 || bb[j].n < 0) continue;
      int32_t o = bb[j].n;
      if (mark[o] == 0) continue;
      const cand *q = &cands[markc[o]];
      if (markc[o] == c || !q->w0) continue;
      double u[2], v[2], qp[2] = {q->px, q->py};
      vxy(m, bb[j].u, u);
      vxy(m, bb[j].v, v);
      if (orc_incircle(u, v, p, qp) > 0 && cands[c].key < q->key) drop = 1;
    }
    cands[c].win = !drop;
    if (drop && st) st->n_dep_drop++;
  }

  /* ---- R10: insertion ---- */
  int64_t nwin = 0;
  for (int64_t c = 0; c < ncand; c++) nwin += cands[c].win;
  if (nwin == 0) {
    set_err(err, errlen, "round had candidates but inserted nothing");
    rc = ORC_E_STALL;
    goto out;
  }
  wl = malloc(sizeof(int32_t) * (size_t)nwin);
  foff = malloc(sizeof(int64_t) * ((size_t)nwin + 1));
  repl = malloc(sizeof(int32_t) * 3 * ((size_t)nT + 1));
  inW = calloc((size_t)nT + 1, 1);
  if (!wl || !foff || !repl || !inW) { rc = ORC_E_NOMEM; goto out; }
  {
    int64_t w = 0;
    for (int64_t c = 0; c < ncand; c++)
      if (cands[c].win) wl[w++] = (int32_t)c;
  }
  g_cands = cands;
  qsort(wl, (size_t)nwin, sizeof(int32_t), cmp_win_idx);
  for (int64_t k = 0; k < 3 * (int64_t)nT; k++) repl[k] = -1;
  /* record phase: boundary of each winner, slot for each fan triangle */
  int64_t total_fan = 0;
  for (int64_t w = 0; w < nwin; w++) {
    const cand *cd = &cands[wl[w]];
    total_fan += cd->ncav + (cd->cls && sadj[2 * cd->id] >= 0 && sadj[2 * cd->id + 1] >= 0 ? 2 : (cd->cls ? 1 : 2));
  }
  fr = malloc(sizeof(fanrec) * (size_t)(total_fan + 1));
  if (!fr) { rc = ORC_E_NOMEM; goto out; }
  int32_t fresh_next = nT;
  int64_t nmid_win = 0;
  int64_t fpos = 0;
  for (int64_t w = 0; w < nwin; w++) {
    const cand *cd = &cands[wl[w]];
    const int32_t *cav = pool.a + cd->cav_off;
    if (cavity_boundary(m, cav, cd->ncav, cd->cls ? cd->id : -1, &bb, &nb, &capb)) { rc = ORC_E_NOMEM; goto out; }
    foff[w] = fpos;
    for (int32_t j = 0; j < nb; j++) {
      fanrec *f = &fr[fpos + j];
      f->slot = j < cd->ncav ? cav[j] : fresh_next + (j - cd->ncav);
      f->u = bb[j].u; f->v = bb[j].v; f->n = bb[j].n; f->ts = bb[j].ts;
      f->jn = f->n >= 0 ? edge_index(m, f->n, f->v, f->u) : -1;
      repl[3 * bb[j].t + bb[j].i] = f->slot;
    }
    fresh_next += nb - cd->ncav;
    fpos += nb;
    for (int32_t j = 0; j < cd->ncav; j++) inW[cav[j]] = 1;
    if (cd->cls) nmid_win++;
  }
  foff[nwin] = fpos;
  if (ensure_cap(m, nV + (int32_t)nwin, fresh_next, nS + (int32_t)nmid_win)) { rc = ORC_E_NOMEM; goto out; }
  /* write phase */
  {
    int32_t mid_rank = 0;
    for (int64_t w = 0; w < nwin; w++) {
      const cand *cd = &cands[wl[w]];
      int32_t pid = nV + (int32_t)w;
      int32_t k = cd->cls ? cd->id : -1, knew = -1, a = -1, b = -1;
      if (cd->cls) {
        knew = nS + mid_rank++;
        a = m->sv[2 * k];
        b = m->sv[2 * k + 1];
      }
      m->x[pid] = cd->px;
      m->y[pid] = cd->py;
      m->vkind[pid] = cd->cls ? ORC_VK_MIDPOINT : ORC_VK_CIRCUMCENTER;
      int64_t f0 = foff[w], f1 = foff[w + 1];
      for (int64_t j = f0; j < f1; j++) {
        const fanrec *f = &fr[j];
        int32_t s = f->slot;
        m->tv[3 * s] = f->u; m->tv[3 * s + 1] = f->v; m->tv[3 * s + 2] = pid;
        /* edge 0: the old boundary edge */
        if (f->n < 0) m->tn[3 * s] = -1;
        else if (inW[f->n]) m->tn[3 * s] = repl[3 * f->n + f->jn];
        else { m->tn[3 * s] = f->n; m->tn[3 * f->n + f->jn] = s; }
        m->ts[3 * s] = f->ts;
        /* edge 1 (v, p) and edge 2 (p, u): neighbours inside the fan */
        int32_t n1 = -1, n2 = -1;
        for (int64_t g = f0; g < f1; g++) {
          if (fr[g].u == f->v) n1 = fr[g].slot;
          if (fr[g].v == f->u) n2 = fr[g].slot;
        }
        m->tn[3 * s + 1] = n1;
        m->tn[3 * s + 2] = n2;
        m->ts[3 * s + 1] = cd->cls ? (f->v == a ? k : (f->v == b ? knew : -1)) : -1;
        m->ts[3 * s + 2] = cd->cls ? (f->u == a ? k : (f->u == b ? knew : -1)) : -1;
      }
      if (cd->cls) {
        m->sv[2 * knew] = pid;
        m->sv[2 * knew + 1] = b;
        m->sparent[knew] = m->sparent[k];
        m->spend[knew] = 0;
        m->sv[2 * k + 1] = pid;
        if (st) st->n_ins_mid++;
      } else if (st) {
        st->n_ins_cc++;
      }
    }
  }
  /* ---- R11: pending flags, counters ----
     A subsegment that was pending or flagged this round and was not split
     stays pending; a split subsegment now ends at a new vertex. */
  for (int32_t k = 0; k < nS; k++) {
    int split = m->sv[2 * k + 1] >= nV;
    m->spend[k] = ((m->spend[k] || mflag[k]) && !split) ? 1 : 0;
  }
  for (int32_t k = nS; k < nS + (int32_t)nmid_win; k++) m->spend[k] = 0;
  m->nV = nV + (int32_t)nwin;
  m->nT = fresh_next;
  m->nS = nS + (int32_t)nmid_win;
  m->rounds++;
  rc = 0;
out:
  free(enc); free(mflag); free(sadj); free(bad); free(tpx); free(tpy); free(tkey);
  free(mark); free(markc); free(stamp); free(cands); free(pool.a); free(bb); free(fr);
  free(repl); free(inW); free(wl); free(foff); free(keys); free(tloc);
  return rc;
}

int orc_refine(orc_mesh *m, double B2, const orc_params *p, orc_round_stats *stats,
               int32_t stats_cap, int32_t *n_stats, char *err, int32_t errlen) {
  if (err && errlen > 0) err[0] = 0;
  if (n_stats) *n_stats = 0;
  if (!m || !p || !(B2 > 0.0) || !isfinite(B2)) { set_err(err, errlen, "bad arguments"); return ORC_E_ARG; }
  if ((p->prefilter_f1 != 0 && p->prefilter_f1 != 1) || p->cavity_approx_n < 0 || p->cand_cap_K < 0 ||
      p->priority_mode < 0 || p->priority_mode > 2 || (p->encroach_mode != 0 && p->encroach_mode != 1) ||
      (p->insert_mode != 0 && p->insert_mode != 1) || (p->insert_mode == 1 && p->priority_mode != 2) ||
      (p->split_mode != 0 && p->split_mode != 1) ||
      !(p->max_edge_len_sq >= 0.0) || !isfinite(p->max_edge_len_sq)) {
    set_err(err, errlen, "unsupported parameter");
    return ORC_E_ARG;
  }
  int32_t max_rounds = p->max_rounds > 0 ? p->max_rounds : (1 << 20);
  int32_t ns = 0;
  if (p->insert_mode == 1) {
    /* Flip-Flop rounds keep the canonical CDT (see orc_ff.c) */
    int r = orc_ff_canonical(m, err, errlen);
    if (r) return r;
  }
  for (;;) {
    orc_round_stats rs;
    int only_check = m->rounds >= max_rounds;
    int r = one_round(m, B2, p, &rs, only_check, err, errlen);
    if (r == 1) return ORC_OK;
    if (r == 2) { set_err(err, errlen, "round cap reached"); return ORC_E_NOTERM; }
    if (r < 0) return r;
    if (stats && ns < stats_cap) stats[ns] = rs;
    ns++;
    if (n_stats) *n_stats = ns < stats_cap ? ns : stats_cap;
  }
}

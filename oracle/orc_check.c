/*
 * orc_check.c -- post-condition checkers for refined meshes (oracle side).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The checks restate what the paper fixes for the output (Section 4:
 * triangulation of the convex hull that contains every input vertex and
 * segment; constrained Delaunay: no vertex visible from a triangle lies
 * strictly inside its circumcircle; quality: no triangle with radius-edge
 * ratio above B; Ruppert mode: no subsegment encroached by a visible vertex).
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NXT(i) (((i) + 1) % 3)
#define PRV(i) (((i) + 2) % 3)

static void wr(char *err, int32_t errlen, const char *msg, long long a, long long b) {
  if (err && errlen > 0 && err[0] == 0) snprintf(err, (size_t)errlen, "%s (%lld, %lld)", msg, a, b);
}

static inline void vxy(const orc_mesh *m, int32_t v, double *p) { p[0] = m->x[v]; p[1] = m->y[v]; }

int64_t orc_check_topology(const orc_mesh *m, char *err, int32_t errlen) {
  int64_t bad = 0;
  if (err && errlen > 0) err[0] = 0;
  uint8_t *used = calloc((size_t)m->nV + 1, 1);
  for (int32_t t = 0; t < m->nT; t++) {
    double a[2], b[2], c[2];
    for (int i = 0; i < 3; i++) {
      int32_t v = m->tv[3 * t + i];
      if (v < 0 || v >= m->nV) { bad++; wr(err, errlen, "vertex id out of range", t, v); continue; }
      used[v] = 1;
    }
    vxy(m, m->tv[3 * t], a);
    vxy(m, m->tv[3 * t + 1], b);
    vxy(m, m->tv[3 * t + 2], c);
    if (orc_orient2d(a, b, c) <= 0) { bad++; wr(err, errlen, "triangle not CCW", t, 0); }
    for (int i = 0; i < 3; i++) {
      int32_t n = m->tn[3 * t + i], s = m->ts[3 * t + i];
      int32_t u = m->tv[3 * t + i], v = m->tv[3 * t + NXT(i)];
      if (n < 0) {
        if (s < 0) { bad++; wr(err, errlen, "hull edge without subsegment", t, i); }
        continue;
      }
      if (n >= m->nT) { bad++; wr(err, errlen, "neighbour out of range", t, i); continue; }
      int j = -1;
      for (int q = 0; q < 3; q++)
        if (m->tv[3 * n + q] == v && m->tv[3 * n + NXT(q)] == u) j = q;
      if (j < 0 || m->tn[3 * n + j] != t) { bad++; wr(err, errlen, "neighbour not symmetric", t, i); continue; }
      if (m->ts[3 * n + j] != s) { bad++; wr(err, errlen, "subsegment mark not symmetric", t, i); }
    }
    for (int i = 0; i < 3; i++) {
      int32_t s = m->ts[3 * t + i];
      if (s < 0) continue;
      if (s >= m->nS) { bad++; wr(err, errlen, "subsegment id out of range", t, s); continue; }
      int32_t u = m->tv[3 * t + i], v = m->tv[3 * t + NXT(i)];
      int32_t a0 = m->sv[2 * s], b0 = m->sv[2 * s + 1];
      if (!((u == a0 && v == b0) || (u == b0 && v == a0))) { bad++; wr(err, errlen, "subsegment endpoints differ", t, s); }
    }
  }
  for (int32_t v = 0; v < m->nV; v++)
    if (!used[v]) { bad++; wr(err, errlen, "vertex in no triangle", v, 0); }
  free(used);
  /* Euler for a disk: T = 2V - h - 2 */
  int32_t h = orc_hull_vertex_count(m);
  if ((int64_t)m->nT != 2 * (int64_t)m->nV - h - 2) { bad++; wr(err, errlen, "Euler relation fails", m->nT, h); }
  return bad;
}

int32_t orc_hull_vertex_count(const orc_mesh *m) {
  int32_t h = 0;
  for (int32_t t = 0; t < m->nT; t++)
    for (int i = 0; i < 3; i++)
      if (m->tn[3 * t + i] < 0) h++;
  return h; /* hull is a single cycle: edges == vertices */
}

int64_t orc_check_local_delaunay(const orc_mesh *m) {
  int64_t bad = 0;
  for (int32_t t = 0; t < m->nT; t++) {
    double a[2], b[2], c[2], d[2];
    vxy(m, m->tv[3 * t], a);
    vxy(m, m->tv[3 * t + 1], b);
    vxy(m, m->tv[3 * t + 2], c);
    for (int i = 0; i < 3; i++) {
      int32_t n = m->tn[3 * t + i];
      if (n < 0 || m->ts[3 * t + i] >= 0) continue;
      int32_t u = m->tv[3 * t + i], v = m->tv[3 * t + NXT(i)], x = -1;
      for (int q = 0; q < 3; q++)
        if (m->tv[3 * n + q] == v && m->tv[3 * n + NXT(q)] == u) x = m->tv[3 * n + PRV(q)];
      if (x < 0) { bad++; continue; }
      vxy(m, x, d);
      if (orc_incircle(a, b, c, d) > 0) bad++;
    }
  }
  return bad;
}

int64_t orc_check_quality(const orc_mesh *m, double B2, double L2) {
  int64_t bad = 0;
  for (int32_t t = 0; t < m->nT; t++) {
    double px, py;
    int32_t b;
    uint64_t key;
    orc_circumcenter(m, t, B2, L2, &px, &py, &b, &key, 0);
    bad += b;
  }
  return bad;
}

void orc_mesh_quality(const orc_mesh *m, double B2, double L2, int64_t *n_bad, double *bad_area) {
  int64_t n = 0;
  double area = 0.0;
  for (int32_t t = 0; t < m->nT; t++) {
    double px, py;
    int32_t b;
    uint64_t key;
    orc_circumcenter(m, t, B2, L2, &px, &py, &b, &key, 0);
    if (!b) continue;
    /* doubled area with the circumcenter formula's operand order: vertices
       rotated so that the smallest id comes first */
    int32_t v0 = m->tv[3 * t], v1 = m->tv[3 * t + 1], v2 = m->tv[3 * t + 2], ia, ib, ic;
    if (v0 < v1 && v0 < v2) { ia = v0; ib = v1; ic = v2; }
    else if (v1 < v2) { ia = v1; ib = v2; ic = v0; }
    else { ia = v2; ib = v0; ic = v1; }
    double bx = m->x[ib] - m->x[ia], by = m->y[ib] - m->y[ia];
    double cx = m->x[ic] - m->x[ia], cy = m->y[ic] - m->y[ia];
    double d = bx * cy - by * cx;
    n++;
    area += d * 0.5;
  }
  *n_bad = n;
  *bad_area = area;
}

int64_t orc_check_encroached(const orc_mesh *m, int32_t mode) {
  int64_t bad = 0;
  for (int32_t t = 0; t < m->nT; t++)
    for (int i = 0; i < 3; i++) {
      if (m->ts[3 * t + i] < 0) continue;
      double a[2], b[2], c[2];
      vxy(m, m->tv[3 * t + i], a);
      vxy(m, m->tv[3 * t + NXT(i)], b);
      vxy(m, m->tv[3 * t + PRV(i)], c);
      if (orc_encroaches(mode, a, b, c)) bad++;
    }
  return bad;
}

/* Does segment pq properly cross subsegment ab (interiors meet at one point)? */
static int proper_cross(const double *p, const double *q, const double *a, const double *b) {
  int o1 = orc_orient2d(p, q, a), o2 = orc_orient2d(p, q, b);
  int o3 = orc_orient2d(a, b, p), o4 = orc_orient2d(a, b, q);
  return o1 * o2 < 0 && o3 * o4 < 0;
}

/* Brute force, for tiny meshes: a vertex strictly inside a triangle's
   circumcircle is a violation when the segments from it to all three
   triangle vertices cross no subsegment. */
int64_t orc_check_cdt_bruteforce(const orc_mesh *m) {
  int64_t bad = 0;
  for (int32_t t = 0; t < m->nT; t++) {
    int32_t tv[3] = {m->tv[3 * t], m->tv[3 * t + 1], m->tv[3 * t + 2]};
    double a[2], b[2], c[2];
    vxy(m, tv[0], a);
    vxy(m, tv[1], b);
    vxy(m, tv[2], c);
    for (int32_t v = 0; v < m->nV; v++) {
      if (v == tv[0] || v == tv[1] || v == tv[2]) continue;
      double p[2];
      vxy(m, v, p);
      if (orc_incircle(a, b, c, p) <= 0) continue;
      int visible = 1;
      for (int j = 0; j < 3 && visible; j++) {
        double q[2];
        vxy(m, tv[j], q);
        for (int32_t s = 0; s < m->nS; s++) {
          double sa[2], sb[2];
          vxy(m, m->sv[2 * s], sa);
          vxy(m, m->sv[2 * s + 1], sb);
          if (proper_cross(p, q, sa, sb)) { visible = 0; break; }
        }
      }
      if (visible) bad++;
    }
  }
  return bad;
}

/* Every input segment is the union of a simple chain of subsegments from its
   first to its second endpoint; every chain vertex lies within a rounding
   tolerance of the segment line and strictly inside its span. */
int64_t orc_check_subsegments(const orc_mesh *m, const double *in_xy, const int32_t *in_seg,
                              char *err, int32_t errlen) {
  int64_t bad = 0;
  if (err && errlen > 0) err[0] = 0;
  int32_t ns = m->n_input_s;
  /* count subsegments per parent, and build successor map per parent */
  int32_t *cnt = calloc((size_t)ns + 1, sizeof(int32_t));
  for (int32_t k = 0; k < m->nS; k++) {
    int32_t p = m->sparent[k];
    if (p < 0 || p >= ns) { bad++; wr(err, errlen, "bad parent", k, p); continue; }
    cnt[p]++;
  }
  int32_t *start = calloc((size_t)ns + 1, sizeof(int32_t));
  for (int32_t s = 0; s < ns; s++) start[s + 1] = start[s] + cnt[s];
  int32_t *fill = calloc((size_t)ns + 1, sizeof(int32_t));
  int32_t *list = malloc(sizeof(int32_t) * ((size_t)m->nS + 1));
  for (int32_t k = 0; k < m->nS; k++) {
    int32_t p = m->sparent[k];
    if (p < 0 || p >= ns) continue;
    list[start[p] + fill[p]++] = k;
  }
  for (int32_t s = 0; s < ns; s++) {
    int32_t a = in_seg[2 * s], b = in_seg[2 * s + 1];
    double ax = in_xy[2 * a], ay = in_xy[2 * a + 1], bx = in_xy[2 * b], by = in_xy[2 * b + 1];
    double dx = bx - ax, dy = by - ay, L2 = dx * dx + dy * dy, L = sqrt(L2);
    int32_t cur = a, steps = 0;
    double last_t = 0.0;
    while (cur != b) {
      int32_t next = -1;
      for (int32_t q = start[s]; q < start[s + 1]; q++) {
        int32_t k = list[q];
        if (m->sv[2 * k] == cur) { next = m->sv[2 * k + 1]; break; }
      }
      if (next < 0) { bad++; wr(err, errlen, "subsegment chain broken", s, cur); break; }
      if (++steps > cnt[s]) { bad++; wr(err, errlen, "subsegment chain cycles", s, cur); break; }
      if (next != b) {
        double px = m->x[next] - ax, py = m->y[next] - ay;
        double tt = (px * dx + py * dy) / L2;
        double off = fabs(px * dy - py * dx) / L;
        if (!(tt > last_t && tt < 1.0)) { bad++; wr(err, errlen, "chain not monotone", s, next); }
        if (off > 8.0 * 0x1p-53 * (fabs(ax) + fabs(bx) + fabs(ay) + fabs(by) + L)) {
          bad++;
          wr(err, errlen, "chain vertex off the segment", s, next);
        }
        last_t = tt;
      }
      cur = next;
    }
    if (steps != cnt[s] && cur == b) { bad++; wr(err, errlen, "extra subsegments for segment", s, cnt[s]); }
  }
  free(cnt); free(start); free(fill); free(list);
  return bad;
}

/* Sum of triangle areas, Neumaier-compensated. */
double orc_area_sum(const orc_mesh *m) {
  double sum = 0.0, comp = 0.0;
  for (int32_t t = 0; t < m->nT; t++) {
    int32_t a = m->tv[3 * t], b = m->tv[3 * t + 1], c = m->tv[3 * t + 2];
    double bx = m->x[b] - m->x[a], by = m->y[b] - m->y[a];
    double cx = m->x[c] - m->x[a], cy = m->y[c] - m->y[a];
    double ar = 0.5 * (bx * cy - by * cx);
    double s = sum + ar;
    if (fabs(sum) >= fabs(ar)) comp += (sum - s) + ar;
    else comp += (ar - s) + sum;
    sum = s;
  }
  return sum + comp;
}

/*
 * orc_exact.c -- exact geometric signs and fixed-order FP64 formulas (oracle).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper evaluates its geometric tests with exact arithmetic (Section 7,
 * platform paragraph).  The oracle gets exact signs in the plainest way it
 * can: every FP64 input is converted to an integer scaled by a power of two
 * (x = m * 2^e, |m| < 2^53), and the determinants are evaluated with
 * schoolbook multi-precision integer arithmetic.  A conservative FP64 error
 * bound decides the easy cases first; the bound constants are derived below
 * and are loose on purpose (a loose bound only sends more cases to the exact
 * path, never a wrong sign).
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Multi-precision integers scaled by powers of two                          */
/* ------------------------------------------------------------------------- */

#define BQ_LIMBS 320 /* 10240 bits: covers products of four differences of any
                        doubles with |x| < 2^900 aligned at 2^-1074 */

typedef struct {
  int sign; /* -1, 0, +1 */
  int n;    /* used 32-bit limbs, little endian */
  int exp;  /* value = sign * mag * 2^exp */
  uint32_t d[BQ_LIMBS];
} bq;

static void bq_overflow(void) {
  fprintf(stderr, "oracle: multi-precision capacity exceeded\n");
  abort();
}

static void bq_trim(bq *a) {
  while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
  if (a->n == 0) { a->sign = 0; a->exp = 0; }
}

static void bq_set_double(bq *r, double x) {
  if (!isfinite(x)) {
    fprintf(stderr, "oracle: non-finite coordinate in a predicate\n");
    abort();
  }
  if (x == 0.0) { r->sign = 0; r->n = 0; r->exp = 0; return; }
  int e;
  double f = frexp(fabs(x), &e);          /* f in [0.5, 1) */
  uint64_t m = (uint64_t)ldexp(f, 53);     /* exact: 53-bit integer */
  r->sign = x < 0 ? -1 : 1;
  r->exp = e - 53;
  r->d[0] = (uint32_t)m;
  r->d[1] = (uint32_t)(m >> 32);
  r->n = 2;
  bq_trim(r);
}

/* out = a << s (bits); returns limb count. out must not alias a. */
static int mag_shl(uint32_t *out, const uint32_t *a, int n, int s) {
  int limbs = s / 32, bits = s % 32;
  if (n + limbs + 1 > BQ_LIMBS) bq_overflow();
  for (int i = 0; i < limbs; i++) out[i] = 0;
  if (bits == 0) {
    for (int i = 0; i < n; i++) out[limbs + i] = a[i];
    return n + limbs;
  }
  uint32_t carry = 0;
  for (int i = 0; i < n; i++) {
    out[limbs + i] = (a[i] << bits) | carry;
    carry = a[i] >> (32 - bits);
  }
  out[limbs + n] = carry;
  return n + limbs + 1;
}

static int mag_cmp(const uint32_t *a, int na, const uint32_t *b, int nb) {
  while (na > 0 && a[na - 1] == 0) na--;
  while (nb > 0 && b[nb - 1] == 0) nb--;
  if (na != nb) return na > nb ? 1 : -1;
  for (int i = na - 1; i >= 0; i--)
    if (a[i] != b[i]) return a[i] > b[i] ? 1 : -1;
  return 0;
}

static int mag_add(uint32_t *out, const uint32_t *a, int na, const uint32_t *b, int nb) {
  int n = na > nb ? na : nb;
  if (n + 1 > BQ_LIMBS) bq_overflow();
  uint64_t carry = 0;
  for (int i = 0; i < n; i++) {
    uint64_t s = carry;
    if (i < na) s += a[i];
    if (i < nb) s += b[i];
    out[i] = (uint32_t)s;
    carry = s >> 32;
  }
  out[n] = (uint32_t)carry;
  return n + 1;
}

/* out = a - b, requires a >= b */
static int mag_sub(uint32_t *out, const uint32_t *a, int na, const uint32_t *b, int nb) {
  int64_t borrow = 0;
  for (int i = 0; i < na; i++) {
    int64_t s = (int64_t)a[i] - borrow - (i < nb ? (int64_t)b[i] : 0);
    if (s < 0) { s += ((int64_t)1 << 32); borrow = 1; } else borrow = 0;
    out[i] = (uint32_t)s;
  }
  return na;
}

static void bq_add(bq *r, const bq *a, const bq *b) {
  if (a->sign == 0) { if (r != b) *r = *b; return; }
  if (b->sign == 0) { if (r != a) *r = *a; return; }
  static __thread uint32_t A[BQ_LIMBS], B[BQ_LIMBS];
  int sa = a->sign, sb = b->sign;
  int e = a->exp < b->exp ? a->exp : b->exp;
  int na = mag_shl(A, a->d, a->n, a->exp - e);
  int nb = mag_shl(B, b->d, b->n, b->exp - e);
  if (sa == sb) {
    r->n = mag_add(r->d, A, na, B, nb);
    r->sign = sa;
  } else {
    int c = mag_cmp(A, na, B, nb);
    if (c == 0) { r->sign = 0; r->n = 0; r->exp = 0; return; }
    if (c > 0) { r->n = mag_sub(r->d, A, na, B, nb); r->sign = sa; }
    else { r->n = mag_sub(r->d, B, nb, A, na); r->sign = sb; }
  }
  r->exp = e;
  bq_trim(r);
}

static void bq_neg(bq *r) { r->sign = -r->sign; }

static void bq_mul(bq *r, const bq *a, const bq *b) {
  if (a->sign == 0 || b->sign == 0) { r->sign = 0; r->n = 0; r->exp = 0; return; }
  static __thread uint32_t P[BQ_LIMBS];
  int n = a->n + b->n;
  if (n > BQ_LIMBS) bq_overflow();
  memset(P, 0, sizeof(uint32_t) * (size_t)n);
  for (int i = 0; i < a->n; i++) {
    uint64_t carry = 0;
    for (int j = 0; j < b->n; j++) {
      uint64_t t = (uint64_t)a->d[i] * b->d[j] + P[i + j] + carry;
      P[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    int k = i + b->n;
    while (carry) {
      uint64_t t = (uint64_t)P[k] + carry;
      P[k] = (uint32_t)t;
      carry = t >> 32;
      k++;
    }
  }
  int sign = a->sign * b->sign;
  int exp = a->exp + b->exp;
  memcpy(r->d, P, sizeof(uint32_t) * (size_t)n);
  r->n = n;
  r->sign = sign;
  r->exp = exp;
  bq_trim(r);
}

/* r = x - y, exactly */
static void bq_diff(bq *r, double x, double y) {
  bq X, Y;
  bq_set_double(&X, x);
  bq_set_double(&Y, y);
  bq_neg(&Y);
  bq_add(r, &X, &Y);
}

/* ------------------------------------------------------------------------- */
/* Exact determinants                                                        */
/* ------------------------------------------------------------------------- */

static int64_t g_exact_orient, g_exact_incircle, g_exact_indiam;

void orc_exact_counts(int64_t *o, int64_t *i, int64_t *d) {
  if (o) *o = g_exact_orient;
  if (i) *i = g_exact_incircle;
  if (d) *d = g_exact_indiam;
}

/* orient2d(a,b,c) = (ax-cx)(by-cy) - (ay-cy)(bx-cx): positive iff a,b,c CCW. */
static int orient_exact(const double *a, const double *b, const double *c) {
  bq acx, acy, bcx, bcy, l, r;
  bq_diff(&acx, a[0], c[0]);
  bq_diff(&acy, a[1], c[1]);
  bq_diff(&bcx, b[0], c[0]);
  bq_diff(&bcy, b[1], c[1]);
  bq_mul(&l, &acx, &bcy);
  bq_mul(&r, &acy, &bcx);
  bq_neg(&r);
  bq_add(&l, &l, &r);
  return l.sign;
}

/* incircle(a,b,c,d) = det | adx ady adx^2+ady^2 | (rows a, b, c; xdx = x - d)
   positive iff d lies strictly inside the circle through CCW a,b,c. */
static int incircle_exact(const double *a, const double *b, const double *c, const double *d) {
  bq adx, ady, bdx, bdy, cdx, cdy, t1, t2, alift, blift, clift, bc, ca, ab, det, term;
  bq_diff(&adx, a[0], d[0]);
  bq_diff(&ady, a[1], d[1]);
  bq_diff(&bdx, b[0], d[0]);
  bq_diff(&bdy, b[1], d[1]);
  bq_diff(&cdx, c[0], d[0]);
  bq_diff(&cdy, c[1], d[1]);
  bq_mul(&t1, &adx, &adx); bq_mul(&t2, &ady, &ady); bq_add(&alift, &t1, &t2);
  bq_mul(&t1, &bdx, &bdx); bq_mul(&t2, &bdy, &bdy); bq_add(&blift, &t1, &t2);
  bq_mul(&t1, &cdx, &cdx); bq_mul(&t2, &cdy, &cdy); bq_add(&clift, &t1, &t2);
  /* bc = bdx*cdy - cdx*bdy ; ca = cdx*ady - adx*cdy ; ab = adx*bdy - bdx*ady */
  bq_mul(&t1, &bdx, &cdy); bq_mul(&t2, &cdx, &bdy); bq_neg(&t2); bq_add(&bc, &t1, &t2);
  bq_mul(&t1, &cdx, &ady); bq_mul(&t2, &adx, &cdy); bq_neg(&t2); bq_add(&ca, &t1, &t2);
  bq_mul(&t1, &adx, &bdy); bq_mul(&t2, &bdx, &ady); bq_neg(&t2); bq_add(&ab, &t1, &t2);
  bq_mul(&det, &alift, &bc);
  bq_mul(&term, &blift, &ca); bq_add(&det, &det, &term);
  bq_mul(&term, &clift, &ab); bq_add(&det, &det, &term);
  return det.sign;
}

/* indiametral(a,b,c) = -((ax-cx)(bx-cx) + (ay-cy)(by-cy)): positive iff c lies
   strictly inside the circle with diameter ab (the angle acb is obtuse). */
static int indiam_exact(const double *a, const double *b, const double *c) {
  bq acx, acy, bcx, bcy, l, r;
  bq_diff(&acx, a[0], c[0]);
  bq_diff(&acy, a[1], c[1]);
  bq_diff(&bcx, b[0], c[0]);
  bq_diff(&bcy, b[1], c[1]);
  bq_mul(&l, &acx, &bcx);
  bq_mul(&r, &acy, &bcy);
  bq_add(&l, &l, &r);
  return -l.sign;
}

/* ------------------------------------------------------------------------- */
/* Filters                                                                   */
/*                                                                           */
/* u = 2^-53.  orient2d: each difference carries relative error <= u, each   */
/* product one more, the final subtraction one more; with l, r the computed  */
/* products, |det_fp - det| <= (4u + O(u^2)) (|l| + |r|).  We use 8u.        */
/* indiametral has the same shape.  incircle: the longest chain per monomial */
/* is 4 differences + 2 products + 1 sum (lift) + 1 product + 1 difference   */
/* (minor) + 1 product + 2 sums, i.e. about 11u of the permanent; we use 16u.*/
/* Below 2^-900 the relative model could meet underflow, so go exact.        */
/* ------------------------------------------------------------------------- */

#define ORC_U 0x1p-53
#define ORC_TINY 0x1p-900

int orc_orient2d(const double *a, const double *b, const double *c) {
  double acx = a[0] - c[0], bcx = b[0] - c[0];
  double acy = a[1] - c[1], bcy = b[1] - c[1];
  double l = acx * bcy, r = acy * bcx;
  double det = l - r;
  double perm = fabs(l) + fabs(r);
  double bound = 8.0 * ORC_U * perm;
  if (perm > ORC_TINY) {
    if (det > bound) return 1;
    if (-det > bound) return -1;
  }
  g_exact_orient++;
  return orient_exact(a, b, c);
}

int orc_incircle(const double *a, const double *b, const double *c, const double *d) {
  double adx = a[0] - d[0], ady = a[1] - d[1];
  double bdx = b[0] - d[0], bdy = b[1] - d[1];
  double cdx = c[0] - d[0], cdy = c[1] - d[1];
  double alift = adx * adx + ady * ady;
  double blift = bdx * bdx + bdy * bdy;
  double clift = cdx * cdx + cdy * cdy;
  double bc1 = bdx * cdy, bc2 = cdx * bdy;
  double ca1 = cdx * ady, ca2 = adx * cdy;
  double ab1 = adx * bdy, ab2 = bdx * ady;
  double det = alift * (bc1 - bc2) + blift * (ca1 - ca2) + clift * (ab1 - ab2);
  double perm = (fabs(bc1) + fabs(bc2)) * alift + (fabs(ca1) + fabs(ca2)) * blift +
                (fabs(ab1) + fabs(ab2)) * clift;
  double bound = 16.0 * ORC_U * perm;
  if (perm > ORC_TINY) {
    if (det > bound) return 1;
    if (-det > bound) return -1;
  }
  g_exact_incircle++;
  return incircle_exact(a, b, c, d);
}

int orc_indiametral(const double *a, const double *b, const double *c) {
  double acx = a[0] - c[0], bcx = b[0] - c[0];
  double acy = a[1] - c[1], bcy = b[1] - c[1];
  double l = acx * bcx, r = acy * bcy;
  double dot = l + r;
  double perm = fabs(l) + fabs(r);
  double bound = 8.0 * ORC_U * perm;
  if (perm > ORC_TINY) {
    if (dot > bound) return -1;
    if (-dot > bound) return 1;
  }
  g_exact_indiam++;
  return indiam_exact(a, b, c);
}

/* Symbolic perturbation of the lifting map: point i is lifted to
   x^2 + y^2 + eps^(i+1) for an infinitesimal eps > 0, so a smaller id carries
   the dominant perturbation.  The 4x4 lifted determinant (rows a,b,c,d with
   columns x, y, lift, 1) equals incircle(a,b,c,d); it is linear in each
   perturbation with cofactor (row a) +orient(b,c,d), (row b) -orient(a,c,d),
   (row c) +orient(a,b,d), (row d) -orient(a,b,c).  When the exact determinant
   vanishes, its sign is the sign of the first nonzero cofactor taken in
   increasing vertex id. */
int orc_incircle_sos(const double *a, const double *b, const double *c, const double *d,
                     int32_t ia, int32_t ib, int32_t ic, int32_t id) {
  int s = orc_incircle(a, b, c, d);
  if (s != 0) return s;
  int32_t ids[4] = {ia, ib, ic, id};
  int ord[4] = {0, 1, 2, 3};
  for (int i = 1; i < 4; i++)
    for (int j = i; j > 0 && ids[ord[j]] < ids[ord[j - 1]]; j--) {
      int t = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = t;
    }
  for (int k = 0; k < 4; k++) {
    int r = ord[k], cof;
    switch (r) {
      case 0: cof = orc_orient2d(b, c, d); break;
      case 1: cof = -orc_orient2d(a, c, d); break;
      case 2: cof = orc_orient2d(a, b, d); break;
      default: cof = -orc_orient2d(a, b, c); break;
    }
    if (cof != 0) return cof;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Priorities and fixed-order formulas                                       */
/* ------------------------------------------------------------------------- */

/* A fixed bijection on 32-bit words: the MurmurHash3 32-bit finalizer
   (xor-shift / odd-multiply rounds, each invertible) applied to id + 1, so
   that no element id maps to 0 (0 means "unmarked"). */
uint32_t orc_perm32(uint32_t x) {
  uint32_t h = x + 1u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* q(x): bits 62..32 of the IEEE-754 pattern of x >= 0 (monotone in x). */
static uint32_t q31(double x) {
  uint64_t b;
  memcpy(&b, &x, sizeof b);
  return (uint32_t)((b >> 32) & 0x7fffffffu);
}

/* Splitting point of subsegment k.  Midpoint, or with split_mode 1
   (concentric shells): when exactly one endpoint c is an input vertex, the
   point on the subsegment at distance 2^j from c, 2^j the power of two
   nearest to half its length (2^e if len/2 = f 2^e with f > 3/4, else
   2^(e-1)), so that subsegments meeting at a small input angle are cut on
   common circles around c. */
void orc_midpoint(const orc_mesh *m, int32_t k, double *mx, double *my, uint64_t *key,
                  int32_t priority_mode, int32_t split_mode) {
  int32_t ia = m->sv[2 * k], ib = m->sv[2 * k + 1];
  double ax = m->x[ia], ay = m->y[ia], bx = m->x[ib], by = m->y[ib];
  double dx = bx - ax, dy = by - ay;
  double len2 = dx * dx + dy * dy;
  int ina = m->vkind[ia] == ORC_VK_INPUT, inb = m->vkind[ib] == ORC_VK_INPUT;
  if (split_mode == 1 && ina != inb) {
    double cx = ina ? ax : bx, cy = ina ? ay : by;
    double ox = ina ? bx : ax, oy = ina ? by : ay;
    double len = sqrt(len2);
    int e;
    double f = frexp(len * 0.5, &e);
    double d = f > 0.75 ? ldexp(1.0, e) : ldexp(1.0, e - 1);
    double t = d / len;
    *mx = cx + (ox - cx) * t;
    *my = cy + (oy - cy) * t;
  } else {
    *mx = (ax + bx) * 0.5;
    *my = (ay + by) * 0.5;
  }
  uint64_t q = priority_mode == 1 ? 0 : (uint64_t)q31(len2);
  *key = ((uint64_t)1 << 63) | (q << 32) | (uint64_t)orc_perm32((uint32_t)k);
}

/* Circumcenter, radius-edge test and priority of triangle t.
   Vertices are rotated (keeping CCW order) so that a has the smallest id.
   Needle guard: if the FP64 doubled area d is not positive, or the computed
   circumcenter lies outside |x|,|y| <= 2^20, the triangle is bad, its measure
   is 0 and its splitting point is the midpoint of its longest edge (first of
   ab, ac, bc on ties). */
void orc_circumcenter(const orc_mesh *m, int32_t t, double ratio_bound_sq, double max_edge_len_sq,
                      double *px, double *py, int32_t *bad, uint64_t *key,
                      int32_t priority_mode) {
  int32_t v0 = m->tv[3 * t], v1 = m->tv[3 * t + 1], v2 = m->tv[3 * t + 2];
  int32_t ia, ib, ic;
  if (v0 < v1 && v0 < v2) { ia = v0; ib = v1; ic = v2; }
  else if (v1 < v2) { ia = v1; ib = v2; ic = v0; }
  else { ia = v2; ib = v0; ic = v1; }
  double ax = m->x[ia], ay = m->y[ia];
  double bx = m->x[ib] - ax, by = m->y[ib] - ay;
  double cx = m->x[ic] - ax, cy = m->y[ic] - ay;
  double b2 = bx * bx + by * by;
  double c2 = cx * cx + cy * cy;
  double d = bx * cy - by * cx;
  double ex = m->x[ic] - m->x[ib], ey = m->y[ic] - m->y[ib];
  double e2 = ex * ex + ey * ey;
  uint64_t q = 0;
  int needle = 1;
  if (d > 0.0) {
    double den = d + d;
    double ux = (cy * b2 - by * c2) / den;
    double uy = (bx * c2 - cx * b2) / den;
    double cxp = ax + ux, cyp = ay + uy;
    if (fabs(cxp) <= 0x1p20 && fabs(cyp) <= 0x1p20) {
      needle = 0;
      *px = cxp;
      *py = cyp;
      double r2 = ux * ux + uy * uy;
      double lmin2 = b2;
      if (c2 < lmin2) lmin2 = c2;
      if (e2 < lmin2) lmin2 = e2;
      *bad = r2 > ratio_bound_sq * lmin2 ? 1 : 0;
      if (max_edge_len_sq > 0.0) {
        /* edge-length criterion: the longest of the three edges against l^2 */
        double lmax2 = b2;
        if (c2 > lmax2) lmax2 = c2;
        if (e2 > lmax2) lmax2 = e2;
        if (lmax2 > max_edge_len_sq) *bad = 1;
      }
      q = (uint64_t)q31(d);
    }
  }
  if (needle) {
    /* longest edge: ab (b2), ac (c2), bc (e2) */
    int32_t u = ia, w = ib;
    double best = b2;
    if (c2 > best) { best = c2; u = ia; w = ic; }
    if (e2 > best) { best = e2; u = ib; w = ic; }
    *px = (m->x[u] + m->x[w]) * 0.5;
    *py = (m->y[u] + m->y[w]) * 0.5;
    *bad = 1;
    q = 0;
  }
  if (priority_mode == 1) q = 0;
  if (priority_mode == 2)
    *key = ((q >> 12) << 44) | ((uint64_t)ia << 22) | (uint64_t)ib;
  else
    *key = (q << 32) | (uint64_t)orc_perm32((uint32_t)t);
}

/* Encroachment of subsegment ab by p (Section 4.1: inside the diametric
   circle under Ruppert's algorithm, inside the diametric lens under Chew's).
   The paper does not give the lens angle.  The lens here is bounded by two
   circular arcs through a and b that meet ab at 60 degrees; its points see
   ab under an angle above 120 degrees, i.e. (a-p).(b-p) < 0 and
   4 ((a-p).(b-p))^2 > |a-p|^2 |b-p|^2.  (A flatter lens, arcs at 30 degrees,
   lets free vertices sit close to a subsegment whose circumcenters lie behind
   it; without vertex deletion the splits then feed each other.)  The lens
   lies inside the circle, so the exact circle test comes first; the angle
   test is the FP64 formula below in this order. */
int orc_encroaches(int32_t mode, const double *a, const double *b, const double *p) {
  if (orc_indiametral(a, b, p) <= 0) return 0;
  if (mode == 0) return 1;
  double dax = a[0] - p[0], day = a[1] - p[1];
  double dbx = b[0] - p[0], dby = b[1] - p[1];
  double dot = dax * dbx + day * dby;
  double la = dax * dax + day * day;
  double lb = dbx * dbx + dby * dby;
  return (dot * dot) * 4.0 > la * lb ? 1 : 0;
}

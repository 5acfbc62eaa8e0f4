// gdp_exact.h -- exact orientation / incircle / diametral-circle signs for
// FP64 points, usable from host code and from gfx950 kernels.
//
// The paper's geometric tests are exact (Section 7, platform paragraph:
// exact arithmetic and robust predicates).  Here each test runs in stages:
//   A. an FP64 evaluation with a forward error bound (most calls end here);
//   B. (incircle) if every coordinate difference is exact in FP64, the
//      determinant of the differences is evaluated exactly with
//      floating-point expansions;
//   C. otherwise the determinant is expanded in raw coordinates (the lifted
//      4x4 form for incircle) and evaluated exactly with expansions.
// Expansion arithmetic follows J. R. Shewchuk, "Adaptive Precision
// Floating-Point Arithmetic and Fast Robust Geometric Predicates" (1997):
// error-free sum and product of two doubles, growing an expansion by a
// double, scaling an expansion by a double, each with zero elimination; the
// sign of a nonoverlapping expansion is the sign of its largest component.
//
// Exactness needs every nonzero coordinate in [2^-100, 2^20] in magnitude
// (the library validates its inputs and guards computed points), so no
// product underflows or overflows.  Build with -ffp-contract=off: the filter
// bounds assume separately rounded operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GDP_HD __host__ __device__ __forceinline__

namespace gdp {

constexpr double kU = 0x1p-53;       // unit roundoff
constexpr double kTiny = 0x1p-900;   // below this the relative model is not trusted

// ---- error-free transformations -------------------------------------------
GDP_HD void two_sum(double a, double b, double &x, double &y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}

GDP_HD void two_prod(double a, double b, double &x, double &y) {
  x = a * b;
  y = fma(a, b, -x);
}

// h = e + b (e nonoverlapping, increasing magnitude).  h may alias e.
GDP_HD int grow_exp(int elen, const double *e, double b, double *h) {
  double q = b;
  int n = 0;
  for (int i = 0; i < elen; i++) {
    double s, t;
    two_sum(q, e[i], s, t);
    q = s;
    if (t != 0.0) h[n++] = t;
  }
  if (q != 0.0 || n == 0) h[n++] = q;
  return n;
}

// h = h + f, in place (h holds hlen terms and has room for hlen + flen).
GDP_HD int add_exp(int hlen, double *h, int flen, const double *f) {
  for (int i = 0; i < flen; i++) hlen = grow_exp(hlen, h, f[i], h);
  return hlen;
}

// h = e * b.  h must not alias e; room for 2 * elen.
GDP_HD int scale_exp(int elen, const double *e, double b, double *h) {
  double q, hh;
  two_prod(e[0], b, q, hh);
  int n = 0;
  if (hh != 0.0) h[n++] = hh;
  for (int i = 1; i < elen; i++) {
    double p1, p0, s, t, u;
    two_prod(e[i], b, p1, p0);
    two_sum(q, p0, s, t);
    if (t != 0.0) h[n++] = t;
    two_sum(p1, s, q, u);
    if (u != 0.0) h[n++] = u;
  }
  if (q != 0.0 || n == 0) h[n++] = q;
  return n;
}

GDP_HD int exp_sign(int n, const double *e) {
  for (int i = n - 1; i >= 0; i--) {
    if (e[i] > 0.0) return 1;
    if (e[i] < 0.0) return -1;
  }
  return 0;
}

// e = a*b (2 terms) appended into h via grow; helper for sums of products.
GDP_HD int add_prod(int hlen, double *h, double a, double b, bool negate) {
  double x, y;
  two_prod(a, b, x, y);
  if (negate) { x = -x; y = -y; }
  hlen = grow_exp(hlen, h, y, h);
  hlen = grow_exp(hlen, h, x, h);
  return hlen;
}

// raw orient2d expansion: px*qy - py*qx + qx*ry - qy*rx + rx*py - ry*px
GDP_HD int orient_raw(double px, double py, double qx, double qy, double rx, double ry, double *h) {
  int n = 1;
  h[0] = 0.0;
  n = add_prod(n, h, px, qy, false);
  n = add_prod(n, h, py, qx, true);
  n = add_prod(n, h, qx, ry, false);
  n = add_prod(n, h, qy, rx, true);
  n = add_prod(n, h, rx, py, false);
  n = add_prod(n, h, ry, px, true);
  return n;
}

// ---- exact slow paths (kept out of line on the device) ---------------------
#ifdef __HIP_DEVICE_COMPILE__
#define GDP_SLOW __device__ __noinline__
#else
#define GDP_SLOW __host__ inline
#endif

GDP_SLOW int orient_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  double h[16];
  int n = orient_raw(ax, ay, bx, by, cx, cy, h);
  return exp_sign(n, h);
}

// (a-c).(b-c) sign, raw: ax*bx - ax*cx - cx*bx + cx*cx + ay*by - ay*cy - cy*by + cy*cy
GDP_SLOW int dot_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  double h[24];
  int n = 1;
  h[0] = 0.0;
  n = add_prod(n, h, ax, bx, false);
  n = add_prod(n, h, ax, cx, true);
  n = add_prod(n, h, cx, bx, true);
  n = add_prod(n, h, cx, cx, false);
  n = add_prod(n, h, ay, by, false);
  n = add_prod(n, h, ay, cy, true);
  n = add_prod(n, h, cy, by, true);
  n = add_prod(n, h, cy, cy, false);
  return exp_sign(n, h);
}

// lift(x,y) * o  where lift = x^2 + y^2 (4 terms) and o has olen terms;
// accumulated into acc (negated if neg).
GDP_HD int add_lift_times(int alen, double *acc, double x, double y, int olen, const double *o,
                          bool neg, double *tmp) {
  double l[8];
  int ln = 1;
  l[0] = 0.0;
  ln = add_prod(ln, l, x, x, false);
  ln = add_prod(ln, l, y, y, false);
  for (int i = 0; i < ln; i++) {
    double c = neg ? -l[i] : l[i];
    if (c == 0.0) continue;
    int sn = scale_exp(olen, o, c, tmp);
    alen = add_exp(alen, acc, sn, tmp);
  }
  return alen;
}

// incircle, stage C: lifted 4x4 determinant in raw coordinates,
//   +|a|^2 orient(b,c,d) - |b|^2 orient(a,c,d) + |c|^2 orient(a,b,d) - |d|^2 orient(a,b,c)
GDP_SLOW int incircle_exact_raw(double ax, double ay, double bx, double by, double cx, double cy,
                                double dx, double dy) {
  double acc[544];  // <= 1 + 4 lifts * 5 terms * 26
  double o[16];
  double tmp[40];
  int alen = 1;
  acc[0] = 0.0;
  int on = orient_raw(bx, by, cx, cy, dx, dy, o);
  alen = add_lift_times(alen, acc, ax, ay, on, o, false, tmp);
  on = orient_raw(ax, ay, cx, cy, dx, dy, o);
  alen = add_lift_times(alen, acc, bx, by, on, o, true, tmp);
  on = orient_raw(ax, ay, bx, by, dx, dy, o);
  alen = add_lift_times(alen, acc, cx, cy, on, o, false, tmp);
  on = orient_raw(ax, ay, bx, by, cx, cy, o);
  alen = add_lift_times(alen, acc, dx, dy, on, o, true, tmp);
  return exp_sign(alen, acc);
}

// incircle, stage B: all six differences are exact doubles.
//   alift*(bdx*cdy - cdx*bdy) + blift*(cdx*ady - adx*cdy) + clift*(adx*bdy - bdx*ady)
GDP_SLOW int incircle_exact_diff(double adx, double ady, double bdx, double bdy, double cdx,
                                 double cdy) {
  double acc[160];  // <= 1 + 3 lifts * 5 terms * 10
  double m[8];
  double tmp[24];
  int alen = 1;
  acc[0] = 0.0;
  const double X[3] = {adx, bdx, cdx}, Y[3] = {ady, bdy, cdy};
  for (int r = 0; r < 3; r++) {
    int i = (r + 1) % 3, j = (r + 2) % 3;
    int mn = 1;
    m[0] = 0.0;
    mn = add_prod(mn, m, X[i], Y[j], false);
    mn = add_prod(mn, m, X[j], Y[i], true);
    alen = add_lift_times(alen, acc, X[r], Y[r], mn, m, false, tmp);
  }
  return exp_sign(alen, acc);
}

// ---- public predicates -------------------------------------------------------
// orient2d > 0 iff a, b, c are in counter-clockwise order.
GDP_HD int orient2d(double ax, double ay, double bx, double by, double cx, double cy) {
  double acx = ax - cx, bcx = bx - cx, acy = ay - cy, bcy = by - cy;
  double l = acx * bcy, r = acy * bcx;
  double det = l - r;
  double perm = fabs(l) + fabs(r);
  double bound = 6.0 * kU * perm;
  if (perm > kTiny) {
    if (det > bound) return 1;
    if (-det > bound) return -1;
  }
  return orient_exact(ax, ay, bx, by, cx, cy);
}

// incircle > 0 iff d lies strictly inside the circle through CCW a, b, c.
GDP_HD int incircle(double ax, double ay, double bx, double by, double cx, double cy, double dx,
                    double dy) {
  double adx = ax - dx, ady = ay - dy, bdx = bx - dx, bdy = by - dy, cdx = cx - dx, cdy = cy - dy;
  double bc1 = bdx * cdy, bc2 = cdx * bdy;
  double ca1 = cdx * ady, ca2 = adx * cdy;
  double ab1 = adx * bdy, ab2 = bdx * ady;
  double al = adx * adx + ady * ady;
  double bl = bdx * bdx + bdy * bdy;
  double cl = cdx * cdx + cdy * cdy;
  double det = al * (bc1 - bc2) + bl * (ca1 - ca2) + cl * (ab1 - ab2);
  double perm = (fabs(bc1) + fabs(bc2)) * al + (fabs(ca1) + fabs(ca2)) * bl + (fabs(ab1) + fabs(ab2)) * cl;
  double bound = 12.0 * kU * perm;
  if (perm > kTiny) {
    if (det > bound) return 1;
    if (-det > bound) return -1;
  }
  // Stage B applies when every difference is exact (zero tail).
  double s, t;
  bool exact = true;
  two_sum(ax, -dx, s, t); exact &= (t == 0.0);
  two_sum(ay, -dy, s, t); exact &= (t == 0.0);
  two_sum(bx, -dx, s, t); exact &= (t == 0.0);
  two_sum(by, -dy, s, t); exact &= (t == 0.0);
  two_sum(cx, -dx, s, t); exact &= (t == 0.0);
  two_sum(cy, -dy, s, t); exact &= (t == 0.0);
  if (exact) return incircle_exact_diff(adx, ady, bdx, bdy, cdx, cdy);
  return incircle_exact_raw(ax, ay, bx, by, cx, cy, dx, dy);
}

// indiametral > 0 iff c lies strictly inside the circle with diameter ab.
GDP_HD int indiametral(double ax, double ay, double bx, double by, double cx, double cy) {
  double acx = ax - cx, bcx = bx - cx, acy = ay - cy, bcy = by - cy;
  double l = acx * bcx, r = acy * bcy;
  double dot = l + r;
  double perm = fabs(l) + fabs(r);
  double bound = 6.0 * kU * perm;
  if (perm > kTiny) {
    if (dot > bound) return -1;
    if (-dot > bound) return 1;
  }
  return -dot_exact(ax, ay, bx, by, cx, cy);
}

}  // namespace gdp

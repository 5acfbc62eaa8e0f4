// gdp_exact.h -- exact orientation / incircle / diametral-circle signs for
// FP64 points, usable from host code and from gfx950 kernels.
//
// The paper's geometric tests are exact (Section 7, platform paragraph:
// exact arithmetic and robust predicates).  Here each test runs in stages:
//   A. an FP64 evaluation with a forward error bound (most calls end here);
//   B. (incircle) if every coordinate difference is exact in FP64, the
//      determinant of the differences is evaluated exactly;
//   C. otherwise the determinant is expanded in raw coordinates (the lifted
//      4x4 form for incircle) and evaluated exactly.
// The exact stages split every product into doubles without error (the
// error-free product of two doubles, with a fused multiply-add) and sum
// them in a fixed-point long accumulator (below), whose frame is a few
// hundred bytes: small enough that kernels calling these predicates need
// little scratch memory per lane.
//
// Exactness needs every nonzero coordinate in [2^-100, 2^20] in magnitude
// (the library validates its inputs and guards computed points).  Build
// with -ffp-contract=off: the filter bounds assume separately rounded
// operations.
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

// ---- exact slow paths: a fixed-point long accumulator ----------------------
// Every exact evaluation below is a signed sum of products of two or four
// coordinates (or of exact coordinate differences).  Each product is split
// into doubles without error (two_prod, twice for four factors), and every
// such double is added exactly into a fixed-point accumulator of 32-bit
// digits: the long accumulator of exact dot products (U. Kulisch, "Computer
// Arithmetic and Validity", 2008; one digit array wide enough for the whole
// exponent range of the terms).  The sign of the sum is read after one carry
// pass.  The digits are int64, so each can take more than 2^30 additions of
// a value below 2^32 before a carry is needed; an evaluation adds at most 384.
//
// Range: with every nonzero coordinate in [2^-100, 2^20], a coordinate's
// lowest set bit is at least 2^-152, so a product of four has no bit below
// 2^-608 and no term reaches 2^90; digit 0 weighs 2^-640 and 24 digits reach
// 2^128.  A term outside that window (an input that breaks the range
// precondition) is clamped into it: the evaluation then stays in bounds but
// may give a wrong sign, as expansion arithmetic would after an underflow.
constexpr int kAccBase = -640;
constexpr int kAccDigits = 24;

// Stage counters of the exact paths (optional): t points to a stripe array
// of kTallyStripes lines of kTallyStride 64-bit words; the evaluation adds 1
// to word kTally0 + stage of the line of its wave.
enum ExactStage { kExOrient = 0, kExDot = 1, kExInB = 2, kExInC = 3, kExStages = 4 };
constexpr int kTallyStride = 32;
constexpr int kTallyStripes = 64;
constexpr int kTally0 = 16;

struct LongAcc {
  int64_t d[kAccDigits];
};

GDP_HD void acc_clear(LongAcc &a) {
  for (int i = 0; i < kAccDigits; i++) a.d[i] = 0;
}

// a += v exactly (v a normal double inside the window above).
GDP_HD void acc_add(LongAcc &a, double v) {
  if (v == 0.0) return;
  uint64_t bits;
  __builtin_memcpy(&bits, &v, sizeof bits);
  const int be = (int)((bits >> 52) & 0x7ff);
  const uint64_t mant = (bits & 0xfffffffffffffull) | (be ? (1ull << 52) : 0ull);
  int sh = (be ? be : 1) - 1075 - kAccBase;  // weight of mant's lowest bit, above digit 0
  if (sh < 0) sh = 0;
  if (sh > 32 * (kAccDigits - 3) + 31) sh = 32 * (kAccDigits - 3) + 31;
  const int k = sh >> 5, r = sh & 31;
  const int64_t d0 = (int64_t)((mant << r) & 0xffffffffull);
  const uint64_t rest = (mant >> 1) >> (31 - r);  // mant * 2^r / 2^32, rounded down
  const int64_t d1 = (int64_t)(rest & 0xffffffffull), d2 = (int64_t)(rest >> 32);
  if (bits >> 63) {
    a.d[k] -= d0; a.d[k + 1] -= d1; a.d[k + 2] -= d2;
  } else {
    a.d[k] += d0; a.d[k + 1] += d1; a.d[k + 2] += d2;
  }
}

// Sign of the accumulated value: one carry pass from the lowest digit, after
// which value = carry * 2^(32 kAccDigits) + (nonnegative digits).
GDP_HD int acc_sign(const LongAcc &a) {
  int64_t carry = 0;
  bool nz = false;
  for (int i = 0; i < kAccDigits; i++) {
    const int64_t v = a.d[i] + carry;
    nz = nz || (v & 0xffffffffll) != 0;
    carry = v >> 32;  // arithmetic shift: floor division by 2^32
  }
  if (carry != 0) return carry > 0 ? 1 : -1;
  return nz ? 1 : 0;
}

// a += s * x * y (two factors), exactly.
GDP_HD void acc_prod2(LongAcc &a, double x, double y, bool neg) {
  double h, l;
  two_prod(x, y, h, l);
  acc_add(a, neg ? -h : h);
  acc_add(a, neg ? -l : l);
}

// a += s * (x1 * x2) * (y1 * y2) (four factors), exactly: each pair is split
// without error, then the four cross products are split again.
GDP_HD void acc_prod4(LongAcc &a, double x1, double x2, double y1, double y2, bool neg) {
  double xh, xl, yh, yl;
  two_prod(x1, x2, xh, xl);
  two_prod(y1, y2, yh, yl);
  acc_prod2(a, xh, yh, neg);
  acc_prod2(a, xh, yl, neg);
  acc_prod2(a, xl, yh, neg);
  acc_prod2(a, xl, yl, neg);
}

#ifdef __HIP_DEVICE_COMPILE__
#define GDP_SLOW __device__ __noinline__
GDP_HD void tally(uint64_t *t, int stage) {
  if (!t) return;
  const unsigned wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  atomicAdd((unsigned long long *)(t + (wave & (kTallyStripes - 1)) * kTallyStride + kTally0 + stage), 1ull);
}
#else
#define GDP_SLOW __host__ inline
inline void tally(uint64_t *t, int stage) {
  if (t) t[kTally0 + stage]++;
}
#endif

// orient2d, exact: px*qy - py*qx + qx*ry - qy*rx + rx*py - ry*px
GDP_SLOW int orient_exact(double ax, double ay, double bx, double by, double cx, double cy, uint64_t *t) {
  tally(t, kExOrient);
  LongAcc a;
  acc_clear(a);
  acc_prod2(a, ax, by, false);
  acc_prod2(a, ay, bx, true);
  acc_prod2(a, bx, cy, false);
  acc_prod2(a, by, cx, true);
  acc_prod2(a, cx, ay, false);
  acc_prod2(a, cy, ax, true);
  return acc_sign(a);
}

// (a-c).(b-c), exact: ax*bx - ax*cx - cx*bx + cx*cx + ay*by - ay*cy - cy*by + cy*cy
GDP_SLOW int dot_exact(double ax, double ay, double bx, double by, double cx, double cy, uint64_t *t) {
  tally(t, kExDot);
  LongAcc a;
  acc_clear(a);
  acc_prod2(a, ax, bx, false);
  acc_prod2(a, ax, cx, true);
  acc_prod2(a, cx, bx, true);
  acc_prod2(a, cx, cx, false);
  acc_prod2(a, ay, by, false);
  acc_prod2(a, ay, cy, true);
  acc_prod2(a, cy, by, true);
  acc_prod2(a, cy, cy, false);
  return acc_sign(a);
}

// a += s * (px^2 + py^2) * orient(q, r, u), expanded into four-factor terms.
GDP_HD void acc_lift_orient(LongAcc &a, double px, double py, double qx, double qy, double rx, double ry,
                            double ux, double uy, bool neg) {
  const double L[2] = {px, py};
  for (int i = 0; i < 2; i++) {
    const double l = L[i];
    acc_prod4(a, l, l, qx, ry, neg);
    acc_prod4(a, l, l, qy, rx, !neg);
    acc_prod4(a, l, l, rx, uy, neg);
    acc_prod4(a, l, l, ry, ux, !neg);
    acc_prod4(a, l, l, ux, qy, neg);
    acc_prod4(a, l, l, uy, qx, !neg);
  }
}

// incircle, stage C: the lifted 4x4 determinant in raw coordinates,
//   |a|^2 orient(b,c,d) - |b|^2 orient(a,c,d) + |c|^2 orient(a,b,d) - |d|^2 orient(a,b,c)
GDP_SLOW int incircle_exact_raw(double ax, double ay, double bx, double by, double cx, double cy,
                                double dx, double dy, uint64_t *t) {
  tally(t, kExInC);
  LongAcc a;
  acc_clear(a);
  acc_lift_orient(a, ax, ay, bx, by, cx, cy, dx, dy, false);
  acc_lift_orient(a, bx, by, ax, ay, cx, cy, dx, dy, true);
  acc_lift_orient(a, cx, cy, ax, ay, bx, by, dx, dy, false);
  acc_lift_orient(a, dx, dy, ax, ay, bx, by, cx, cy, true);
  return acc_sign(a);
}

// incircle, stage B: all six differences are exact doubles.
//   alift*(bdx*cdy - cdx*bdy) + blift*(cdx*ady - adx*cdy) + clift*(adx*bdy - bdx*ady)
GDP_SLOW int incircle_exact_diff(double adx, double ady, double bdx, double bdy, double cdx,
                                 double cdy, uint64_t *t) {
  tally(t, kExInB);
  LongAcc a;
  acc_clear(a);
  const double X[3] = {adx, bdx, cdx}, Y[3] = {ady, bdy, cdy};
  for (int r = 0; r < 3; r++) {
    const int i = (r + 1) % 3, j = (r + 2) % 3;
    acc_prod4(a, X[r], X[r], X[i], Y[j], false);
    acc_prod4(a, X[r], X[r], X[j], Y[i], true);
    acc_prod4(a, Y[r], Y[r], X[i], Y[j], false);
    acc_prod4(a, Y[r], Y[r], X[j], Y[i], true);
  }
  return acc_sign(a);
}

// ---- stage A alone ------------------------------------------------------------
// The FP64 filters by themselves: the sign when the forward error bound
// decides it, else kUndecided.  Kernels whose register budget matters call
// these and hand the rare undecided case to a path that evaluates exactly.
constexpr int kUndecided = 2;

GDP_HD int orient2d_filter(double ax, double ay, double bx, double by, double cx, double cy) {
  double acx = ax - cx, bcx = bx - cx, acy = ay - cy, bcy = by - cy;
  double l = acx * bcy, r = acy * bcx;
  double det = l - r;
  double perm = fabs(l) + fabs(r);
  double bound = 6.0 * kU * perm;
  if (perm > kTiny) {
    if (det > bound) return 1;
    if (-det > bound) return -1;
  }
  return kUndecided;
}

GDP_HD int incircle_filter(double ax, double ay, double bx, double by, double cx, double cy, double dx,
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
  return kUndecided;
}

// sign of -(a-c).(b-c): > 0 iff c lies strictly inside the circle with diameter ab
GDP_HD int indiametral_filter(double ax, double ay, double bx, double by, double cx, double cy) {
  double acx = ax - cx, bcx = bx - cx, acy = ay - cy, bcy = by - cy;
  double l = acx * bcx, r = acy * bcy;
  double dot = l + r;
  double perm = fabs(l) + fabs(r);
  double bound = 6.0 * kU * perm;
  if (perm > kTiny) {
    if (dot > bound) return -1;
    if (-dot > bound) return 1;
  }
  return kUndecided;
}

// ---- public predicates -------------------------------------------------------
// orient2d > 0 iff a, b, c are in counter-clockwise order.
GDP_HD int orient2d(double ax, double ay, double bx, double by, double cx, double cy, uint64_t *t = nullptr) {
  const int s = orient2d_filter(ax, ay, bx, by, cx, cy);
  return s != kUndecided ? s : orient_exact(ax, ay, bx, by, cx, cy, t);
}

// incircle > 0 iff d lies strictly inside the circle through CCW a, b, c.
GDP_HD int incircle(double ax, double ay, double bx, double by, double cx, double cy, double dx,
                    double dy, uint64_t *tl = nullptr) {
  const int f = incircle_filter(ax, ay, bx, by, cx, cy, dx, dy);
  if (f != kUndecided) return f;
  double adx = ax - dx, ady = ay - dy, bdx = bx - dx, bdy = by - dy, cdx = cx - dx, cdy = cy - dy;
  // Stage B applies when every difference is exact (zero tail).
  double s, t;
  bool exact = true;
  two_sum(ax, -dx, s, t); exact &= (t == 0.0);
  two_sum(ay, -dy, s, t); exact &= (t == 0.0);
  two_sum(bx, -dx, s, t); exact &= (t == 0.0);
  two_sum(by, -dy, s, t); exact &= (t == 0.0);
  two_sum(cx, -dx, s, t); exact &= (t == 0.0);
  two_sum(cy, -dy, s, t); exact &= (t == 0.0);
  if (exact) return incircle_exact_diff(adx, ady, bdx, bdy, cdx, cdy, tl);
  return incircle_exact_raw(ax, ay, bx, by, cx, cy, dx, dy, tl);
}

// incircle under the symbolic perturbation of the lifting map (Section 7's
// simulation of simplicity): on an exact tie the cofactors of the lifted
// determinant (+o(b,c,d), -o(a,c,d), +o(a,b,d), -o(a,b,c), one per point)
// decide, taken in the order of increasing vertex id; equal ids keep their
// argument order.  Nonzero for four distinct ids of points in general
// position or on one circle.
GDP_HD int incircle_sos(double ax, double ay, double bx, double by, double cx, double cy, double dx, double dy,
                        int ia, int ib, int ic, int id, uint64_t *tl = nullptr) {
  const int s = incircle(ax, ay, bx, by, cx, cy, dx, dy, tl);
  if (s != 0) return s;
  // argument positions ordered by id (a sorting network on scalars, so the
  // tie path needs no indexed private array); equal ids keep argument order
  int p0 = 0, p1 = 1, p2 = 2, p3 = 3;
  int k0 = ia, k1 = ib, k2 = ic, k3 = id;
#define GDP_SOS_SWAP(pa, ka, pb, kb) \
  if (kb < ka) { int tp = pa; pa = pb; pb = tp; int tk = ka; ka = kb; kb = tk; }
  GDP_SOS_SWAP(p0, k0, p1, k1)
  GDP_SOS_SWAP(p2, k2, p3, k3)
  GDP_SOS_SWAP(p1, k1, p2, k2)
  GDP_SOS_SWAP(p0, k0, p1, k1)
  GDP_SOS_SWAP(p2, k2, p3, k3)
  GDP_SOS_SWAP(p1, k1, p2, k2)
#undef GDP_SOS_SWAP
  for (int r = 0; r < 4; r++) {
    int cof;
    switch (r == 0 ? p0 : (r == 1 ? p1 : (r == 2 ? p2 : p3))) {
      case 0: cof = orient2d(bx, by, cx, cy, dx, dy, tl); break;
      case 1: cof = -orient2d(ax, ay, cx, cy, dx, dy, tl); break;
      case 2: cof = orient2d(ax, ay, bx, by, dx, dy, tl); break;
      default: cof = -orient2d(ax, ay, bx, by, cx, cy, tl); break;
    }
    if (cof != 0) return cof;
  }
  return 0;
}

// indiametral > 0 iff c lies strictly inside the circle with diameter ab.
GDP_HD int indiametral(double ax, double ay, double bx, double by, double cx, double cy, uint64_t *t = nullptr) {
  const int s = indiametral_filter(ax, ay, bx, by, cx, cy);
  return s != kUndecided ? s : -dot_exact(ax, ay, bx, by, cx, cy, t);
}

// Encroachment of subsegment ab by p (Section 4.1): strictly inside the
// diametric circle (mode 0, exact), or strictly inside the diametric lens
// (mode 1): the points that see ab under more than 120 degrees, bounded by
// two circular arcs through a and b meeting ab at 60 degrees.  The lens lies
// in the circle; after the exact circle test the angle is tested by the FP64
// formula (a-p).(b-p) < 0 and 4 ((a-p).(b-p))^2 > |a-p|^2 |b-p|^2 in this
// operation order.
GDP_HD bool in_lens_angle(double ax, double ay, double bx, double by, double px, double py) {
  const double dax = ax - px, day = ay - py;
  const double dbx = bx - px, dby = by - py;
  const double dot = dax * dbx + day * dby;
  const double la = dax * dax + day * day;
  const double lb = dbx * dbx + dby * dby;
  return (dot * dot) * 4.0 > la * lb;
}

GDP_HD bool encroaches(int mode, double ax, double ay, double bx, double by, double px, double py,
                       uint64_t *t = nullptr) {
  if (indiametral(ax, ay, bx, by, px, py, t) <= 0) return false;
  if (mode == 0) return true;
  return in_lens_angle(ax, ay, bx, by, px, py);
}

// encroaches() from the filter alone: 1 or 0, or kUndecided when the circle
// test needs the exact evaluation.
GDP_HD int encroaches_filter(int mode, double ax, double ay, double bx, double by, double px, double py) {
  const int s = indiametral_filter(ax, ay, bx, by, px, py);
  if (s == kUndecided) return kUndecided;
  if (s <= 0) return 0;
  if (mode == 0) return 1;
  return in_lens_angle(ax, ay, bx, by, px, py) ? 1 : 0;
}

}  // namespace gdp

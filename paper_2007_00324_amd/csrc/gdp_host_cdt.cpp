// gdp_host_cdt.cpp -- Line 1 of Algorithm 1 (gDP2d): the constrained Delaunay
// triangulation of the input PSLG, built on the host before the refinement
// loop (the paper also computes it on the CPU and leaves it out of the timed
// region, Section 7.1).
//
// Method (independent of any other builder in this repository):
//   * Bowyer-Watson insertion of all points, in Morton order, into a large
//     enclosing triangle; cocircular ties are broken by the symbolic
//     perturbation of the lifting map in which a smaller vertex id carries
//     the dominant perturbation (so the CDT is unique);
//   * each segment is recovered by deleting the triangles it crosses and
//     retriangulating the two pseudo-polygons on either side with their
//     constrained Delaunay triangulation (recursive choice of the apex whose
//     circle holds no other polygon vertex);
//   * triangles outside the convex hull are removed by a flood fill from the
//     enclosing triangle that stops at segments, so every hull edge must be a
//     segment;
//   * canonical form: each triangle rotated so its smallest vertex id comes
//     first, triangles sorted lexicographically; subsegment id = segment index.
#include "gdp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

namespace {

using gdp::incircle;
using gdp::orient2d;

struct Builder {
  int n = 0;                 // input vertices; n, n+1, n+2 are the enclosing triangle
  std::vector<double> X, Y;  // n + 3
  std::vector<int> V;        // 3 per triangle
  std::vector<int> N;        // 3 per triangle (-1 = none)
  std::vector<int> Cn;       // 3 per triangle: segment id or -1
  std::vector<char> dead;
  std::vector<int> freeslots;
  std::vector<int> vt;       // vertex -> a live incident triangle
  std::string err;

  int orient(int a, int b, int c) const { return orient2d(X[a], Y[a], X[b], Y[b], X[c], Y[c]); }

  // incircle with the symbolic tie-break (smaller id dominant); the four
  // cofactors of the lifted determinant are +o(b,c,d), -o(a,c,d), +o(a,b,d), -o(a,b,c).
  int incircle_sos(int a, int b, int c, int d) const {
    int s = incircle(X[a], Y[a], X[b], Y[b], X[c], Y[c], X[d], Y[d]);
    if (s != 0) return s;
    int ids[4] = {a, b, c, d};
    int order[4] = {0, 1, 2, 3};
    std::sort(order, order + 4, [&](int p, int q) { return ids[p] < ids[q]; });
    for (int k = 0; k < 4; k++) {
      int cof;
      switch (order[k]) {
        case 0: cof = orient(b, c, d); break;
        case 1: cof = -orient(a, c, d); break;
        case 2: cof = orient(a, b, d); break;
        default: cof = -orient(a, b, c); break;
      }
      if (cof != 0) return cof;
    }
    return 0;
  }

  int alloc_tri() {
    if (!freeslots.empty()) {
      int t = freeslots.back();
      freeslots.pop_back();
      dead[t] = 0;
      return t;
    }
    int t = (int)dead.size();
    V.resize(3 * (size_t)(t + 1));
    N.resize(3 * (size_t)(t + 1));
    Cn.resize(3 * (size_t)(t + 1));
    dead.push_back(0);
    return t;
  }
  void kill(int t) {
    dead[t] = 1;
    freeslots.push_back(t);
  }
  int eidx(int t, int u, int v) const {
    for (int i = 0; i < 3; i++)
      if (V[3 * t + i] == u && V[3 * t + (i + 1) % 3] == v) return i;
    return -1;
  }

  // straight walk from t towards point p; returns the triangle containing p
  int locate(int t, int p) const {
    for (long long step = 0; step < (1LL << 32); step++) {
      int moved = -1;
      for (int i = 0; i < 3; i++) {
        int u = V[3 * t + i], v = V[3 * t + (i + 1) % 3];
        if (orient(u, v, p) < 0) { moved = i; break; }
      }
      if (moved < 0) return t;
      t = N[3 * t + moved];
      if (t < 0) return -1;
    }
    return -1;
  }

  struct Fan { int u, v, o, oe, c; };

  // Replaces the triangles in `cav` by the fan of p over the cavity boundary.
  void refan(const std::vector<int> &cav, int p, std::vector<Fan> &fan, std::vector<int> &slots) {
    fan.clear();
    for (int t : cav) {
      for (int i = 0; i < 3; i++) {
        int o = N[3 * t + i];
        if (o >= 0 && dead[o] == 2) continue;  // inside the cavity
        Fan f;
        f.u = V[3 * t + i];
        f.v = V[3 * t + (i + 1) % 3];
        f.o = o;
        f.oe = o >= 0 ? eidx(o, f.v, f.u) : -1;
        f.c = Cn[3 * t + i];
        fan.push_back(f);
      }
    }
    for (int t : cav) kill(t);
    slots.clear();
    for (size_t j = 0; j < fan.size(); j++) slots.push_back(alloc_tri());
    for (size_t j = 0; j < fan.size(); j++) {
      int s = slots[j];
      const Fan &f = fan[j];
      V[3 * s] = f.u; V[3 * s + 1] = f.v; V[3 * s + 2] = p;
      N[3 * s] = f.o; Cn[3 * s] = f.c;
      Cn[3 * s + 1] = -1; Cn[3 * s + 2] = -1;
      if (f.o >= 0) N[3 * f.o + f.oe] = s;
      vt[f.u] = s; vt[f.v] = s; vt[p] = s;
    }
    for (size_t j = 0; j < fan.size(); j++) {
      int s = slots[j];
      N[3 * s + 1] = -1;
      N[3 * s + 2] = -1;
      for (size_t k = 0; k < fan.size(); k++) {
        if (fan[k].u == fan[j].v) N[3 * s + 1] = slots[k];
        if (fan[k].v == fan[j].u) N[3 * s + 2] = slots[k];
      }
    }
  }

  bool insert(int p, int &hint, std::vector<int> &cav, std::vector<Fan> &fan, std::vector<int> &slots) {
    int t = locate(hint, p);
    if (t < 0) { err = "point location failed"; return false; }
    for (int i = 0; i < 3; i++) {
      int u = V[3 * t + i];
      if (X[u] == X[p] && Y[u] == Y[p]) { err = "duplicate point"; return false; }
    }
    cav.clear();
    cav.push_back(t);
    dead[t] = 2;
    for (size_t h = 0; h < cav.size(); h++) {
      int c = cav[h];
      for (int i = 0; i < 3; i++) {
        int o = N[3 * c + i];
        if (o < 0 || dead[o] == 2) continue;
        if (incircle_sos(V[3 * o], V[3 * o + 1], V[3 * o + 2], p) > 0) {
          dead[o] = 2;
          cav.push_back(o);
        }
      }
    }
    refan(cav, p, fan, slots);
    hint = slots[0];
    return true;
  }

  // CDT of the pseudo-polygon with base edge (p,q) and chain c[lo..hi) to the left of p->q.
  void tri_poly(int p, int q, const std::vector<int> &c, int lo, int hi, std::vector<int> &made) {
    if (lo >= hi) return;
    int best = lo;
    for (int k = lo + 1; k < hi; k++)
      if (incircle_sos(p, q, c[best], c[k]) > 0) best = k;
    int t = alloc_tri();
    V[3 * t] = p; V[3 * t + 1] = q; V[3 * t + 2] = c[best];
    for (int i = 0; i < 3; i++) { N[3 * t + i] = -1; Cn[3 * t + i] = -1; }
    made.push_back(t);
    tri_poly(p, c[best], c, lo, best, made);
    tri_poly(c[best], q, c, best + 1, hi, made);
  }

  bool find_edge(int a, int b, int &t, int &i) const {
    // rotate around a starting at vt[a]
    int start = vt[a], cur = start;
    for (int dir = 0; dir < 2; dir++) {
      cur = start;
      for (int guard = 0; guard < (1 << 26); guard++) {
        int k = -1;
        for (int q = 0; q < 3; q++)
          if (V[3 * cur + q] == a) k = q;
        if (V[3 * cur + (k + 1) % 3] == b) { t = cur; i = k; return true; }
        int nx = dir == 0 ? N[3 * cur + (k + 2) % 3] : N[3 * cur + k];
        if (nx < 0 || nx == start) break;
        cur = nx;
      }
    }
    return false;
  }

  bool insert_segment(int a, int b, int s) {
    int t, i;
    if (find_edge(a, b, t, i) || find_edge(b, a, t, i)) {
      int t2 = N[3 * t + i];
      Cn[3 * t + i] = s;
      if (t2 >= 0) Cn[3 * t2 + eidx(t2, V[3 * t + (i + 1) % 3], V[3 * t + i])] = s;
      return true;
    }
    // triangle around a whose wedge holds b
    int start = vt[a], cur = start, found = -1;
    for (int dir = 0; dir < 2 && found < 0; dir++) {
      cur = start;
      for (int guard = 0; guard < (1 << 26); guard++) {
        int k = -1;
        for (int q = 0; q < 3; q++)
          if (V[3 * cur + q] == a) k = q;
        int u = V[3 * cur + (k + 1) % 3], w = V[3 * cur + (k + 2) % 3];
        int ou = orient(a, u, b), ow = orient(a, w, b);
        if (ou == 0 && (X[u] - X[a]) * (X[b] - X[a]) + (Y[u] - Y[a]) * (Y[b] - Y[a]) > 0) {
          err = "a vertex lies in the interior of a segment";
          return false;
        }
        if (ou > 0 && ow < 0) { found = cur; break; }
        int nx = dir == 0 ? N[3 * cur + (k + 2) % 3] : N[3 * cur + k];
        if (nx < 0 || nx == start) break;
        cur = nx;
      }
    }
    if (found < 0) { err = "segment direction not found"; return false; }
    std::vector<int> crossed, left, right;
    int k = -1;
    for (int q = 0; q < 3; q++)
      if (V[3 * found + q] == a) k = q;
    int R = V[3 * found + (k + 1) % 3], L = V[3 * found + (k + 2) % 3];
    left.push_back(L);
    right.push_back(R);
    int cur_t = found;
    for (long long guard = 0;; guard++) {
      if (guard > (1LL << 30)) { err = "segment walk did not end"; return false; }
      crossed.push_back(cur_t);
      int e = eidx(cur_t, R, L);
      if (Cn[3 * cur_t + e] >= 0) { err = "segments cross"; return false; }
      int nx = N[3 * cur_t + e];
      if (nx < 0) { err = "segment leaves the domain"; return false; }
      int j = eidx(nx, L, R);
      int w = V[3 * nx + (j + 2) % 3];
      if (w == b) { crossed.push_back(nx); break; }
      int o = orient(a, b, w);
      if (o == 0) { err = "a vertex lies in the interior of a segment"; return false; }
      if (o > 0) { L = w; left.push_back(w); } else { R = w; right.push_back(w); }
      cur_t = nx;
    }
    // outside neighbours of the region, keyed by directed edge
    std::unordered_map<long long, std::pair<int, int>> outside;
    std::unordered_map<long long, int> slit;  // uncrossed edges between two crossed triangles
    auto key = [](int u, int v) { return ((long long)u << 32) | (unsigned)v; };
    for (int c : crossed) dead[c] = 2;
    for (int c : crossed)
      for (int q = 0; q < 3; q++) {
        int o = N[3 * c + q];
        int u = V[3 * c + q], v = V[3 * c + (q + 1) % 3];
        if (o >= 0 && dead[o] == 2) {
          slit[key(u, v)] = Cn[3 * c + q];
          continue;
        }
        outside[key(u, v)] = {o, Cn[3 * c + q]};
      }
    for (int c : crossed) kill(c);
    std::vector<int> made;
    tri_poly(a, b, left, 0, (int)left.size(), made);
    std::vector<int> rrev(right.rbegin(), right.rend());
    tri_poly(b, a, rrev, 0, (int)rrev.size(), made);
    std::unordered_map<long long, std::pair<int, int>> inner;
    for (int t2 : made)
      for (int q = 0; q < 3; q++) inner[key(V[3 * t2 + q], V[3 * t2 + (q + 1) % 3])] = {t2, q};
    for (int t2 : made)
      for (int q = 0; q < 3; q++) {
        int u = V[3 * t2 + q], v = V[3 * t2 + (q + 1) % 3];
        auto it = inner.find(key(v, u));
        if (it != inner.end()) {
          N[3 * t2 + q] = it->second.first;
          auto sl = slit.find(key(u, v));
          Cn[3 * t2 + q] = ((u == a && v == b) || (u == b && v == a)) ? s : (sl != slit.end() ? sl->second : -1);
        } else {
          auto ot = outside.find(key(u, v));
          if (ot == outside.end()) { err = "segment recovery left an unmatched edge"; return false; }
          int o = ot->second.first;
          N[3 * t2 + q] = o;
          Cn[3 * t2 + q] = ot->second.second;
          if (o >= 0) N[3 * o + eidx(o, v, u)] = t2;
        }
        vt[u] = t2;
      }
    return true;
  }
};

struct CTri { int v[3]; int old; };

}  // namespace

namespace gdp {

int host_cdt_build(int32_t nv, const double *xy, int32_t ns, const int32_t *seg, HostMesh &out,
                   std::string &err) {
  if (nv < 3 || !xy || ns < 0 || (ns > 0 && !seg)) { err = "bad arguments"; return GDP_E_ARG; }
  for (int64_t i = 0; i < 2 * (int64_t)nv; i++) {
    double a = std::fabs(xy[i]);
    if (!std::isfinite(xy[i]) || a > 0x1p20 || (a != 0.0 && a < 0x1p-100)) {
      err = "coordinate not finite, or nonzero with magnitude outside [2^-100, 2^20]";
      return GDP_E_INPUT;
    }
  }
  {
    std::vector<int> ord(nv);
    for (int i = 0; i < nv; i++) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int p, int q) {
      if (xy[2 * p] != xy[2 * q]) return xy[2 * p] < xy[2 * q];
      return xy[2 * p + 1] < xy[2 * q + 1];
    });
    for (int i = 1; i < nv; i++)
      if (xy[2 * ord[i]] == xy[2 * ord[i - 1]] && xy[2 * ord[i] + 1] == xy[2 * ord[i - 1] + 1]) {
        err = "duplicate point";
        return GDP_E_INPUT;
      }
    std::vector<std::pair<int, int>> sk(ns);
    for (int s = 0; s < ns; s++) {
      int a = seg[2 * s], b = seg[2 * s + 1];
      if (a < 0 || b < 0 || a >= nv || b >= nv || a == b) { err = "segment endpoint out of range or zero length"; return GDP_E_INPUT; }
      sk[s] = {std::min(a, b), std::max(a, b)};
    }
    std::sort(sk.begin(), sk.end());
    for (int s = 1; s < ns; s++)
      if (sk[s] == sk[s - 1]) { err = "repeated segment"; return GDP_E_INPUT; }
  }
  Builder B;
  B.n = nv;
  B.X.resize(nv + 3);
  B.Y.resize(nv + 3);
  double mx = 1.0;
  for (int i = 0; i < nv; i++) {
    B.X[i] = xy[2 * i];
    B.Y[i] = xy[2 * i + 1];
    mx = std::max(mx, std::max(std::fabs(B.X[i]), std::fabs(B.Y[i])));
  }
  double Lb = std::exp2(std::ceil(std::log2(mx)) + 1.0);  // box [-Lb, Lb]^2 holds every point
  B.X[nv] = -4 * Lb; B.Y[nv] = -4 * Lb;
  B.X[nv + 1] = 8 * Lb; B.Y[nv + 1] = -4 * Lb;
  B.X[nv + 2] = -4 * Lb; B.Y[nv + 2] = 8 * Lb;
  B.vt.assign(nv + 3, -1);
  int t0 = B.alloc_tri();
  B.V[0] = nv; B.V[1] = nv + 1; B.V[2] = nv + 2;
  for (int i = 0; i < 3; i++) { B.N[i] = -1; B.Cn[i] = -1; }
  B.vt[nv] = B.vt[nv + 1] = B.vt[nv + 2] = t0;
  // Morton order of the points
  {
    double lox = B.X[0], hix = B.X[0], loy = B.Y[0], hiy = B.Y[0];
    for (int i = 0; i < nv; i++) {
      lox = std::min(lox, B.X[i]); hix = std::max(hix, B.X[i]);
      loy = std::min(loy, B.Y[i]); hiy = std::max(hiy, B.Y[i]);
    }
    double sx = hix > lox ? 1048575.0 / (hix - lox) : 0.0, sy = hiy > loy ? 1048575.0 / (hiy - loy) : 0.0;
    std::vector<std::pair<uint64_t, int>> mk(nv);
    for (int i = 0; i < nv; i++) {
      uint32_t gx = (uint32_t)std::min(1048575.0, (B.X[i] - lox) * sx);
      uint32_t gy = (uint32_t)std::min(1048575.0, (B.Y[i] - loy) * sy);
      uint64_t m = 0;
      for (int b = 0; b < 20; b++) m |= ((uint64_t)((gx >> b) & 1) << (2 * b)) | ((uint64_t)((gy >> b) & 1) << (2 * b + 1));
      mk[i] = {m, i};
    }
    std::sort(mk.begin(), mk.end());
    std::vector<int> cav, slots;
    std::vector<Builder::Fan> fan;
    int hint = t0;
    for (int k = 0; k < nv; k++)
      if (!B.insert(mk[k].second, hint, cav, fan, slots)) { err = B.err; return GDP_E_INPUT; }
  }
  for (int s = 0; s < ns; s++)
    if (!B.insert_segment(seg[2 * s], seg[2 * s + 1], s)) { err = B.err; return GDP_E_INPUT; }
  // remove everything reachable from the enclosing triangle without crossing a segment
  int nt_all = (int)B.dead.size();
  std::vector<char> outside(nt_all, 0);
  std::vector<int> stack;
  for (int t = 0; t < nt_all; t++) {
    if (B.dead[t]) continue;
    for (int i = 0; i < 3; i++)
      if (B.V[3 * t + i] >= nv) { outside[t] = 1; stack.push_back(t); break; }
  }
  while (!stack.empty()) {
    int t = stack.back();
    stack.pop_back();
    for (int i = 0; i < 3; i++) {
      int o = B.N[3 * t + i];
      if (o < 0 || outside[o] || B.Cn[3 * t + i] >= 0) continue;
      outside[o] = 1;
      stack.push_back(o);
    }
  }
  std::vector<CTri> ct;
  std::vector<int> rot(nt_all, 0);
  for (int t = 0; t < nt_all; t++) {
    if (B.dead[t] || outside[t]) continue;
    int r = 0;
    for (int i = 1; i < 3; i++)
      if (B.V[3 * t + i] < B.V[3 * t + r]) r = i;
    rot[t] = r;
    CTri c;
    for (int i = 0; i < 3; i++) c.v[i] = B.V[3 * t + (r + i) % 3];
    c.old = t;
    ct.push_back(c);
  }
  std::sort(ct.begin(), ct.end(), [](const CTri &p, const CTri &q) {
    if (p.v[0] != q.v[0]) return p.v[0] < q.v[0];
    if (p.v[1] != q.v[1]) return p.v[1] < q.v[1];
    return p.v[2] < q.v[2];
  });
  std::vector<int> newid(nt_all, -1);
  for (size_t k = 0; k < ct.size(); k++) newid[ct[k].old] = (int)k;
  const int nt = (int)ct.size();
  out.nV = nv;
  out.nT = nt;
  out.nS = ns;
  out.xy.assign(xy, xy + 2 * (size_t)nv);
  out.tv.resize(3 * (size_t)nt);
  out.tn.resize(3 * (size_t)nt);
  out.ts.resize(3 * (size_t)nt);
  std::vector<char> used(nv, 0);
  int64_t hull_edges = 0;
  for (int k = 0; k < nt; k++) {
    int t = ct[k].old, r = rot[t];
    for (int i = 0; i < 3; i++) {
      int src = (r + i) % 3;
      out.tv[3 * k + i] = B.V[3 * t + src];
      used[B.V[3 * t + src]] = 1;
      int o = B.N[3 * t + src];
      int no = (o >= 0 && !outside[o] && !B.dead[o]) ? newid[o] : -1;
      out.tn[3 * k + i] = no;
      out.ts[3 * k + i] = B.Cn[3 * t + src];
      if (no < 0) {
        hull_edges++;
        if (out.ts[3 * k + i] < 0) { err = "a convex hull edge is not covered by a segment"; return GDP_E_INPUT; }
      }
    }
  }
  // The kept region must be the whole convex hull: every vertex used, Euler
  // for a disk, and a convex boundary.
  for (int i = 0; i < nv; i++)
    if (!used[i]) { err = "a convex hull edge is not covered by a segment"; return GDP_E_INPUT; }
  if ((int64_t)nt != 2 * (int64_t)nv - hull_edges - 2) { err = "the kept region is not a disk"; return GDP_E_INPUT; }
  for (int k = 0; k < nt; k++)
    for (int i = 0; i < 3; i++) {
      if (out.tn[3 * k + i] >= 0) continue;
      // boundary edge (u,v); the next boundary edge leaves v: rotate around v
      int u = out.tv[3 * k + i], v = out.tv[3 * k + (i + 1) % 3];
      int t = k, e = (i + 1) % 3;  // edge (v, w) of t
      for (int guard = 0; guard < (1 << 26); guard++) {
        int o = out.tn[3 * t + e];
        if (o < 0) break;
        int j = -1;
        for (int q = 0; q < 3; q++)
          if (out.tv[3 * o + q] == v) j = q;
        t = o;
        e = j;
      }
      int w = out.tv[3 * t + (e + 1) % 3];
      if (orient2d(B.X[u], B.Y[u], B.X[v], B.Y[v], B.X[w], B.Y[w]) < 0) {
        err = "a convex hull edge is not covered by a segment";
        return GDP_E_INPUT;
      }
    }
  out.sv.assign(seg, seg + 2 * (size_t)ns);
  out.sparent.resize(ns);
  for (int s = 0; s < ns; s++) out.sparent[s] = s;
  return GDP_OK;
}

}  // namespace gdp

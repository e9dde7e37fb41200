// Delaunay triangulation of a keyframe's tracked pixels (Sec. III-A), the
// host half of the point-cloud densification.
//
// Readings: the tracked pixels have distinct integer coordinates in
// [0, 32768), not all collinear; the triangulation is a Delaunay
// triangulation of their convex hull, built by Bowyer-Watson insertion with
// exact integer predicates (64-bit orientation, 128-bit in-circle) and ghost
// triangles for the hull, so it is exact; where four points are cocircular
// it is one of the valid triangulations.  A point's conflicting triangles are
// looked up in a bucket grid of circumcircles.
//
// Plain C++ (no device code), so it also builds with a host compiler alone,
// under the address and undefined-behaviour sanitizers.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "gs.h"

namespace gs {

gs_status fail(gs_status s, const std::string& msg);  // records the error text (api.hip)

struct IPt {
  int64_t x, y;
};
static inline int64_t orient2(const IPt& a, const IPt& b, const IPt& c) {
  return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}
// > 0 when d is strictly inside the circumcircle of the positively oriented a, b, c
static inline __int128 incircle(const IPt& a, const IPt& b, const IPt& c, const IPt& d) {
  const __int128 ax = a.x - d.x, ay = a.y - d.y, bx = b.x - d.x, by = b.y - d.y, cx = c.x - d.x, cy = c.y - d.y;
  const __int128 a2 = ax * ax + ay * ay, b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
  return ax * (by * c2 - b2 * cy) - ay * (bx * c2 - b2 * cx) + a2 * (bx * cy - by * cx);
}

struct DTri {
  int v[3];          // v[2] == -1: ghost triangle of the hull edge v0 -> v1 (outside on its left)
  double cx, cy, r2;  // circumcircle of a real triangle (a filter before the exact test)
  bool filter;        // false for a sliver, whose circumcircle in doubles is not trusted
};

static bool in_conflict(const DTri& t, const std::vector<IPt>& P, const IPt& p) {
  if (t.v[2] >= 0) {
    if (t.filter) {
      // the filter only decides far from the circle; near it the exact predicate does
      const double dx = (double)p.x - t.cx, dy = (double)p.y - t.cy, d2 = dx * dx + dy * dy;
      if (d2 > t.r2 * (1.0 + 1e-6) + 1e-3) return false;
      if (d2 < t.r2 * (1.0 - 1e-6) - 1e-3) return true;
    }
    return incircle(P[t.v[0]], P[t.v[1]], P[t.v[2]], p) > 0;
  }
  const IPt &a = P[t.v[0]], &b = P[t.v[1]];
  const int64_t o = orient2(a, b, p);
  if (o != 0) return o > 0;
  // on the hull edge's line: in conflict when strictly between its ends
  return std::min(a.x, b.x) <= p.x && p.x <= std::max(a.x, b.x) && std::min(a.y, b.y) <= p.y &&
         p.y <= std::max(a.y, b.y) && !(p.x == a.x && p.y == a.y) && !(p.x == b.x && p.y == b.y);
}

static DTri make_tri(int a, int b, int c, const std::vector<IPt>& P) {
  DTri t{{a, b, c}, 0.0, 0.0, 0.0, false};
  if (c >= 0) {
    const double ax = (double)P[a].x, ay = (double)P[a].y, bx = (double)P[b].x - ax, by = (double)P[b].y - ay;
    const double cx = (double)P[c].x - ax, cy = (double)P[c].y - ay;
    const double d = 2.0 * (bx * cy - by * cx);
    const double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
    const double ux = (cy * b2 - by * c2) / d, uy = (bx * c2 - cx * b2) / d;
    t.cx = ax + ux;
    t.cy = ay + uy;
    t.r2 = ux * ux + uy * uy;
    // twice the area against the squared edges: the centre's rounding error grows as this shrinks
    t.filter = std::fabs(d) >= 1e-3 * (b2 + c2);
  }
  return t;
}

static gs_status delaunay(const int32_t* xy, int n, std::vector<DTri>& out) {
  std::vector<IPt> P(n);
  for (int i = 0; i < n; ++i) {
    P[i] = IPt{xy[2 * i], xy[2 * i + 1]};
    if (P[i].x < 0 || P[i].y < 0 || P[i].x >= 32768 || P[i].y >= 32768)
      return fail(GS_ERR_INVALID_VALUE, "point " + std::to_string(i) + " outside [0, 32768)^2");
  }
  {
    std::vector<int64_t> keys(n);
    for (int i = 0; i < n; ++i) keys[i] = P[i].y * 32768 + P[i].x;
    std::sort(keys.begin(), keys.end());
    for (int i = 1; i < n; ++i)
      if (keys[i] == keys[i - 1]) return fail(GS_ERR_INVALID_VALUE, "points must be distinct");
  }
  int i2 = -1;
  for (int k = 2; k < n && i2 < 0; ++k)
    if (orient2(P[0], P[1], P[k]) != 0) i2 = k;
  if (i2 < 0) return fail(GS_ERR_INVALID_VALUE, "the points are collinear");
  int a = 0, b = 1, c = i2;
  if (orient2(P[a], P[b], P[c]) < 0) std::swap(b, c);
  // Triangles live in slots that are never reused.  A bucket grid over the points' bounding box
  // lists, per cell, the real triangles whose (filtered) circumcircle's box meets the cell; ghost
  // triangles, slivers and circles spanning much of the grid sit in one global list.  A point's
  // conflicts are then among its cell's list and the global list; dead slots are dropped from the
  // lists as they are scanned.
  int64_t bx0 = P[0].x, bx1 = P[0].x, by0 = P[0].y, by1 = P[0].y;
  for (const IPt& q : P) {
    bx0 = std::min(bx0, q.x);
    bx1 = std::max(bx1, q.x);
    by0 = std::min(by0, q.y);
    by1 = std::max(by1, q.y);
  }
  const int G = std::max(1, (int)std::sqrt((double)n / 2.0));
  const double cw = std::max(1.0, (double)(bx1 - bx0 + 1) / G), ch = std::max(1.0, (double)(by1 - by0 + 1) / G);
  std::vector<std::vector<int>> cells((size_t)G * G);
  std::vector<int> global;
  std::vector<DTri> T;
  std::vector<char> alive;
  auto cell_x = [&](double x) { return std::min(G - 1, std::max(0, (int)std::floor((x - (double)bx0) / cw))); };
  auto cell_y = [&](double y) { return std::min(G - 1, std::max(0, (int)std::floor((y - (double)by0) / ch))); };
  auto add = [&](const DTri& t) {
    const int id = (int)T.size();
    T.push_back(t);
    alive.push_back(1);
    if (t.v[2] < 0 || !t.filter) {
      global.push_back(id);
      return;
    }
    const double r = std::sqrt(t.r2) + 1.0;  // the filter's margin is far below a pixel
    const int cx0 = cell_x(t.cx - r), cx1 = cell_x(t.cx + r), cy0 = cell_y(t.cy - r), cy1 = cell_y(t.cy + r);
    if ((int64_t)(cx1 - cx0 + 1) * (cy1 - cy0 + 1) * 4 > (int64_t)G * G) {
      global.push_back(id);
      return;
    }
    for (int yy = cy0; yy <= cy1; ++yy)
      for (int xx = cx0; xx <= cx1; ++xx) cells[(size_t)yy * G + xx].push_back(id);
  };
  add(make_tri(a, b, c, P));
  add(make_tri(b, a, -1, P));
  add(make_tri(c, b, -1, P));
  add(make_tri(a, c, -1, P));
  std::vector<int> bad;
  std::vector<std::pair<int, int>> edges, boundary;
  auto scan = [&](std::vector<int>& list, const IPt& p) {
    size_t w = 0;
    for (size_t k = 0; k < list.size(); ++k) {
      const int id = list[k];
      if (!alive[id]) continue;
      list[w++] = id;
      if (in_conflict(T[id], P, p)) bad.push_back(id);
    }
    list.resize(w);
  };
  for (int ip = 2; ip < n; ++ip) {
    if (ip == i2) continue;
    const IPt& p = P[ip];
    bad.clear();
    scan(cells[(size_t)cell_y((double)p.y) * G + cell_x((double)p.x)], p);
    scan(global, p);
    if (bad.empty()) return fail(GS_ERR_INVALID_VALUE, "delaunay: a point in no triangle's circle");
    edges.clear();
    for (int t : bad)
      for (int e = 0; e < 3; ++e) edges.emplace_back(T[t].v[e], T[t].v[(e + 1) % 3]);
    boundary.clear();
    for (const auto& e : edges) {
      bool shared = false;
      for (const auto& f : edges)
        if (f.first == e.second && f.second == e.first) {
          shared = true;
          break;
        }
      if (!shared) boundary.push_back(e);
    }
    for (int t : bad) alive[t] = 0;
    for (const auto& e : boundary) {
      if (e.first == -1) {
        add(make_tri(e.second, ip, -1, P));
      } else if (e.second == -1) {
        add(make_tri(ip, e.first, -1, P));
      } else {
        if (orient2(P[e.first], P[e.second], p) <= 0) return fail(GS_ERR_INVALID_VALUE, "delaunay: degenerate cavity");
        add(make_tri(e.first, e.second, ip, P));
      }
    }
  }
  out.clear();
  for (size_t t = 0; t < T.size(); ++t)
    if (alive[t] && T[t].v[2] >= 0) out.push_back(T[t]);
  return GS_OK;
}

}  // namespace gs

extern "C" gs_status gs_delaunay(const int32_t* xy, int32_t n, int32_t* tris, int32_t max_tris, int32_t* n_tris) {
  using namespace gs;
  if (!xy || !n_tris) return fail(GS_ERR_INVALID_VALUE, "xy and n_tris are required");
  if (n < 3) return fail(GS_ERR_INVALID_VALUE, "at least three points are needed");
  std::vector<DTri> T;
  gs_status s;
  if ((s = delaunay(xy, n, T)) != GS_OK) return s;
  std::vector<std::array<int, 3>> out;
  out.reserve(T.size());
  for (const DTri& t : T) {
    // smallest index first, orientation kept
    int k = 0;
    for (int e = 1; e < 3; ++e)
      if (t.v[e] < t.v[k]) k = e;
    out.push_back({t.v[k], t.v[(k + 1) % 3], t.v[(k + 2) % 3]});
  }
  std::sort(out.begin(), out.end());
  *n_tris = (int32_t)out.size();
  if (!tris || max_tris < (int32_t)out.size())
    return fail(GS_ERR_CAPACITY, "tris holds too few triangles: need " + std::to_string(out.size()));
  for (size_t i = 0; i < out.size(); ++i)
    for (int e = 0; e < 3; ++e) tris[3 * i + e] = out[i][e];
  return GS_OK;
}

// Host mesh builder: Delaunay triangulation of the support points, plane fit
// per triangle, and the raster records the GPU consumes (Section III-A: a
// Delaunay mesh of the support points defines the slanted-plane prior;
// Section IV: the triangulation is the sequential step the paper leaves on
// the CPU; Section VI-D: the mesh is remapped to an image-sized prior
// matrix, which the raster kernel does on the GPU from these records).
//
// Uniqueness: support points lie on a lattice, so four or more co-circular
// points are common. The mesh is the Delaunay triangulation under a
// "pulling" perturbation: the point smallest in (v, u) order is pushed below
// the paraboloid the most, so a co-circular cell is split as a fan from its
// smallest vertex. As a local rule: an edge ab with apexes p and q is legal
// iff q is strictly outside circle(p, a, b), or exactly on it and the
// (v, u)-smallest of p, a, b, q is a or b. Any flip-based construction that
// ends with every edge legal yields this triangulation.
//
// Construction: incremental insertion with a visibility walk for point
// location and Lawson flips, exact 64-bit predicates (coordinates < 2^13).
#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <vector>

#include "elas_internal.h"

namespace elas {

namespace {

struct Pt {
  int32_t u, v;
};

inline int64_t orient(Pt a, Pt b, Pt c) {
  return (int64_t)(b.u - a.u) * (c.v - a.v) - (int64_t)(b.v - a.v) * (c.u - a.u);
}

// > 0 iff d is strictly inside the circle through a, b, c (orient(a,b,c) > 0).
inline int64_t incircle(Pt a, Pt b, Pt c, Pt d) {
  const int64_t ax = a.u - d.u, ay = a.v - d.v;
  const int64_t bx = b.u - d.u, by = b.v - d.v;
  const int64_t cx = c.u - d.u, cy = c.v - d.v;
  const int64_t a2 = ax * ax + ay * ay, b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
  return a2 * (bx * cy - by * cx) + b2 * (cx * ay - cy * ax) + c2 * (ax * by - ay * bx);
}

inline bool vu_less(Pt a, Pt b) { return a.v < b.v || (a.v == b.v && a.u < b.u); }

// v[k] are vertex ids in positive orientation; nb[k] is the triangle across
// the edge opposite v[k] (-1 on the image border).
struct Tri {
  int32_t v[3];
  int32_t nb[3];
};

}  // namespace

struct MeshScratch {
  std::vector<Pt> pts;
  std::vector<int32_t> disp;
  std::vector<Tri> tris;
  std::vector<std::pair<int32_t, int32_t>> todo;  // (triangle, index of the new point)
  std::vector<std::array<int32_t, 9>> recs;
  std::vector<int32_t> rank, order, bucket, sorted;
  std::vector<std::pair<int32_t, int64_t>> key;
  int32_t last = 0;
};

MeshScratch* mesh_scratch_create() { return new MeshScratch(); }
void mesh_scratch_destroy(MeshScratch* s) { delete s; }

namespace {

inline void replace_neighbour(std::vector<Tri>& T, int32_t t, int32_t from, int32_t to) {
  if (t < 0) return;
  for (int k = 0; k < 3; ++k)
    if (T[t].nb[k] == from) {
      T[t].nb[k] = to;
      return;
    }
}

// Walks from s.last towards point p; returns a triangle containing p in the
// closed sense, or -1 if p lies outside the mesh. A walk that does not settle
// within its step budget falls back to a scan of every triangle.
int32_t locate(MeshScratch& s, Pt p) {
  auto& T = s.tris;
  int32_t t = s.last;
  const int32_t limit = 4 * (int32_t)T.size() + 16;
  int rot = 0;
  for (int32_t step = 0; step < limit; ++step) {
    int k_out = -1;
    for (int kk = 0; kk < 3 && k_out < 0; ++kk) {
      const int k = (kk + rot) % 3;
      const Pt a = s.pts[T[t].v[(k + 1) % 3]], b = s.pts[T[t].v[(k + 2) % 3]];
      if (orient(a, b, p) < 0) k_out = k;
    }
    if (k_out < 0) return t;            // no edge separates t from p: p is in t
    const int32_t next = T[t].nb[k_out];
    if (next < 0) return -1;            // p is outside the image rectangle
    t = next;
    rot = (rot + 1) % 3;
  }
  for (int32_t i = 0; i < (int32_t)T.size(); ++i) {
    bool inside = true;
    for (int k = 0; k < 3; ++k)
      if (orient(s.pts[T[i].v[(k + 1) % 3]], s.pts[T[i].v[(k + 2) % 3]], p) < 0) inside = false;
    if (inside) return i;
  }
  return -1;
}

// Flips until every edge opposite a newly created corner of `ip` is legal.
void legalize(MeshScratch& s, int32_t ip) {
  auto& T = s.tris;
  while (!s.todo.empty()) {
    const auto [t, i] = s.todo.back();
    s.todo.pop_back();
    if (T[t].v[i] != ip) continue;  // triangle was rewritten since it was queued
    const int32_t o = T[t].nb[i];
    if (o < 0) continue;
    const int32_t a = T[t].v[(i + 1) % 3], b = T[t].v[(i + 2) % 3];
    int j = 0;
    while (T[o].nb[j] != t) ++j;
    const int32_t q = T[o].v[j];
    const Pt P = s.pts[ip], A = s.pts[a], B = s.pts[b], Q = s.pts[q];
    const int64_t ic = incircle(P, A, B, Q);
    bool flip = ic > 0;
    if (ic == 0) {
      Pt m = P;
      for (Pt x : {A, B, Q})
        if (vu_less(x, m)) m = x;
      const bool on_edge = (m.u == A.u && m.v == A.v) || (m.u == B.u && m.v == B.v);
      flip = !on_edge;
    }
    if (!flip) continue;
    const int32_t t_bp = T[t].nb[(i + 1) % 3];  // across (b, p)
    const int32_t t_pa = T[t].nb[(i + 2) % 3];  // across (p, a)
    const int32_t o_aq = T[o].nb[(j + 1) % 3];  // across (a, q)
    const int32_t o_qb = T[o].nb[(j + 2) % 3];  // across (q, b)
    T[t] = Tri{{ip, a, q}, {o_aq, o, t_pa}};
    T[o] = Tri{{ip, q, b}, {o_qb, t_bp, t}};
    replace_neighbour(T, o_aq, o, t);
    replace_neighbour(T, t_bp, t, o);
    s.todo.push_back({t, 0});
    s.todo.push_back({o, 0});
  }
}

bool insert(MeshScratch& s, int32_t ip) {
  auto& T = s.tris;
  const Pt p = s.pts[ip];
  const int32_t t = locate(s, p);
  if (t < 0) return false;
  int on = -1, zeros = 0;
  for (int k = 0; k < 3; ++k)
    if (orient(s.pts[T[t].v[(k + 1) % 3]], s.pts[T[t].v[(k + 2) % 3]], p) == 0) {
      on = k;
      ++zeros;
    }
  if (zeros > 1) return false;  // coincides with a vertex: points must be distinct
  if (on < 0) {
    const Tri old = T[t];
    const int32_t v0 = old.v[0], v1 = old.v[1], v2 = old.v[2];
    const int32_t t1 = (int32_t)T.size(), t2 = t1 + 1;
    T.push_back(Tri{});
    T.push_back(Tri{});
    T[t] = Tri{{ip, v1, v2}, {old.nb[0], t1, t2}};
    T[t1] = Tri{{ip, v2, v0}, {old.nb[1], t2, t}};
    T[t2] = Tri{{ip, v0, v1}, {old.nb[2], t, t1}};
    replace_neighbour(T, old.nb[1], t, t1);
    replace_neighbour(T, old.nb[2], t, t2);
    s.todo.push_back({t, 0});
    s.todo.push_back({t1, 0});
    s.todo.push_back({t2, 0});
  } else {
    const Tri ot = T[t];
    const int32_t a = ot.v[on], b = ot.v[(on + 1) % 3], c = ot.v[(on + 2) % 3];
    const int32_t t2 = ot.nb[on];
    if (t2 < 0) return false;  // on the border: points must lie strictly inside
    const int32_t na_b = ot.nb[(on + 2) % 3];  // across (a, b)
    const int32_t na_c = ot.nb[(on + 1) % 3];  // across (c, a)
    const Tri oo = T[t2];
    int j = 0;
    while (oo.nb[j] != t) ++j;
    const int32_t q = oo.v[j];
    // oo = (q, c, b) up to rotation: the edge opposite b is (q, c), the edge
    // opposite c is (b, q)
    const int32_t n_qc = oo.nb[(j + 2) % 3];
    const int32_t n_bq = oo.nb[(j + 1) % 3];
    const int32_t A2 = (int32_t)T.size(), B2 = A2 + 1;
    T.push_back(Tri{});
    T.push_back(Tri{});
    T[t] = Tri{{a, b, ip}, {B2, A2, na_b}};
    T[A2] = Tri{{a, ip, c}, {t2, na_c, t}};
    T[t2] = Tri{{q, c, ip}, {A2, B2, n_qc}};
    T[B2] = Tri{{q, ip, b}, {t, n_bq, t2}};
    replace_neighbour(T, na_c, t, A2);
    replace_neighbour(T, n_bq, t2, B2);
    s.todo.push_back({t, 2});
    s.todo.push_back({A2, 1});
    s.todo.push_back({t2, 2});
    s.todo.push_back({B2, 1});
  }
  legalize(s, ip);
  s.last = t;
  return true;
}

}  // namespace

int32_t build_mesh(MeshScratch* sp, const int32_t* list, int32_t n, const int32_t* corners,
                   int32_t w, int32_t h, RasterTri* tri_out, int32_t* recs_out,
                   float* planes_out) {
  MeshScratch& s = *sp;
  const int32_t total = n + 4;
  s.pts.resize(total);
  s.disp.resize(total);
  const int32_t cu[4] = {0, w - 1, 0, w - 1}, cv[4] = {0, 0, h - 1, h - 1};
  for (int k = 0; k < 4; ++k) {
    s.pts[k] = Pt{cu[k], cv[k]};
    s.disp[k] = corners[k];
  }
  for (int32_t i = 0; i < n; ++i) {
    s.pts[4 + i] = Pt{list[3 * i], list[3 * i + 1]};
    s.disp[4 + i] = list[3 * i + 2];
    if (list[3 * i] <= 0 || list[3 * i] >= w - 1 || list[3 * i + 1] <= 0 ||
        list[3 * i + 1] >= h - 1)
      return -1;
  }
  s.tris.clear();
  s.tris.reserve(2 * total);
  // the four corners are co-circular: fan from (0, 0), the (v, u)-smallest
  s.tris.push_back(Tri{{0, 1, 3}, {-1, 1, -1}});
  s.tris.push_back(Tri{{0, 3, 2}, {-1, -1, 0}});
  s.last = 0;
  s.todo.clear();
  for (int32_t i = 4; i < total; ++i)
    if (!insert(s, i)) return -1;
  const int32_t ntri = (int32_t)s.tris.size();
  if (ntri != 2 * total - 6) return -1;

  // canonical records: vertices by (v, u), triangles by their vertex triples.
  // Rank every vertex in (v, u) order, then order triangles by their sorted
  // rank triples: a counting sort on the smallest rank, and an insertion sort
  // of the few triangles that share it.
  const int32_t nv = total;
  s.rank.resize(nv);
  s.order.resize(nv);
  for (int32_t i = 0; i < nv; ++i) s.order[i] = i;
  std::sort(s.order.begin(), s.order.end(),
            [&](int32_t x, int32_t y) { return vu_less(s.pts[x], s.pts[y]); });
  for (int32_t i = 0; i < nv; ++i) s.rank[s.order[i]] = i;
  s.key.resize(ntri);
  s.bucket.assign(nv + 1, 0);
  for (int32_t t = 0; t < ntri; ++t) {
    int32_t r0 = s.rank[s.tris[t].v[0]], r1 = s.rank[s.tris[t].v[1]], r2 = s.rank[s.tris[t].v[2]];
    if (r0 > r1) std::swap(r0, r1);
    if (r1 > r2) std::swap(r1, r2);
    if (r0 > r1) std::swap(r0, r1);
    s.key[t] = {r0, ((int64_t)r1 << 32) | (uint32_t)r2};
    ++s.bucket[r0 + 1];
  }
  for (int32_t i = 0; i < nv; ++i) s.bucket[i + 1] += s.bucket[i];
  s.sorted.resize(ntri);
  for (int32_t t = 0; t < ntri; ++t) s.sorted[s.bucket[s.key[t].first]++] = t;
  for (int32_t lo = 0, i = 0; i <= ntri; ++i) {
    if (i == ntri || s.key[s.sorted[i]].first != s.key[s.sorted[lo]].first) {
      for (int32_t a = lo + 1; a < i; ++a)
        for (int32_t b = a; b > lo && s.key[s.sorted[b]].second < s.key[s.sorted[b - 1]].second; --b)
          std::swap(s.sorted[b], s.sorted[b - 1]);
      lo = i;
    }
  }
  s.recs.resize(ntri);
  for (int32_t t = 0; t < ntri; ++t) {
    std::array<int32_t, 9>& r = s.recs[t];
    const auto& k = s.key[s.sorted[t]];
    const int32_t ids[3] = {s.order[k.first], s.order[(int32_t)(k.second >> 32)],
                            s.order[(int32_t)(k.second & 0xFFFFFFFF)]};
    for (int q = 0; q < 3; ++q) {
      r[3 * q] = s.pts[ids[q]].u;
      r[3 * q + 1] = s.pts[ids[q]].v;
      r[3 * q + 2] = s.disp[ids[q]];
    }
  }

  for (int32_t t = 0; t < ntri; ++t) {
    const std::array<int32_t, 9>& r = s.recs[t];
    // plane through the three points: exact Cramer numerators relative to the
    // first vertex, one correctly rounded double division, rounded to float
    const int64_t u1 = r[0], v1 = r[1], d1 = r[2];
    const int64_t du2 = r[3] - u1, dv2 = r[4] - v1, dd2 = r[5] - d1;
    const int64_t du3 = r[6] - u1, dv3 = r[7] - v1, dd3 = r[8] - d1;
    const int64_t den = du2 * dv3 - du3 * dv2;
    const int64_t na = dd2 * dv3 - dd3 * dv2;
    const int64_t nbv = du2 * dd3 - du3 * dd2;
    const int64_t nc = d1 * den - na * u1 - nbv * v1;
    if (den == 0) return -1;
    const float a = (float)((double)na / (double)den);
    const float b = (float)((double)nbv / (double)den);
    const float c = (float)((double)nc / (double)den);
    RasterTri rt;
    int o1 = 1, o2 = 2;
    const Pt P0{r[0], r[1]}, P1{r[3], r[4]}, P2{r[6], r[7]};
    if (orient(P0, P1, P2) < 0) std::swap(o1, o2);
    rt.u[0] = (int16_t)r[0];
    rt.v[0] = (int16_t)r[1];
    rt.u[1] = (int16_t)r[3 * o1];
    rt.v[1] = (int16_t)r[3 * o1 + 1];
    rt.u[2] = (int16_t)r[3 * o2];
    rt.v[2] = (int16_t)r[3 * o2 + 1];
    rt.a = a;
    rt.b = b;
    rt.c = c;
    tri_out[t] = rt;
    if (recs_out) std::memcpy(recs_out + 9 * t, r.data(), 9 * sizeof(int32_t));
    if (planes_out) {
      planes_out[3 * t] = a;
      planes_out[3 * t + 1] = b;
      planes_out[3 * t + 2] = c;
    }
  }
  return ntri;
}

}  // namespace elas

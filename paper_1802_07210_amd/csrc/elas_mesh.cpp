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

namespace {
int32_t finish_mesh(MeshScratch& s, int32_t nv, RasterTri* tri_out, int32_t* recs_out,
                    float* planes_out);
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
  return finish_mesh(s, total, tri_out, recs_out, planes_out);
}

namespace {

// Canonical records, planes and raster records of the triangles in s.tris
// over the nv vertices in s.pts / s.disp; returns the triangle count or -1.
int32_t finish_mesh(MeshScratch& s, int32_t nv, RasterTri* tri_out, int32_t* recs_out,
                    float* planes_out) {
  const int32_t ntri = (int32_t)s.tris.size();
  // canonical records: vertices by (v, u), triangles by their vertex triples.
  // Rank every vertex in (v, u) order, then order triangles by their sorted
  // rank triples: a counting sort on the smallest rank, and an insertion sort
  // of the few triangles that share it.
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

// The triangle across edge k of t, flipped when the edge is illegal under the
// canonical rule; returns whether it flipped. t = (p, a, b) with p = v[k]
// and o = (q, b, a) across (a, b) become (p, a, q) and (p, q, b).
bool flip_if_illegal(MeshScratch& s, int32_t t, int k) {
  auto& T = s.tris;
  const int32_t o = T[t].nb[k];
  if (o < 0) return false;
  const int32_t p = T[t].v[k], a = T[t].v[(k + 1) % 3], b = T[t].v[(k + 2) % 3];
  int j = 0;
  while (T[o].nb[j] != t) ++j;
  const int32_t q = T[o].v[j];
  const Pt P = s.pts[p], A = s.pts[a], B = s.pts[b], Q = s.pts[q];
  const int64_t ic = incircle(P, A, B, Q);
  bool flip = ic > 0;
  if (ic == 0) {
    Pt m = P;
    for (Pt x : {A, B, Q})
      if (vu_less(x, m)) m = x;
    flip = !((m.u == A.u && m.v == A.v) || (m.u == B.u && m.v == B.v));
  }
  if (!flip) return false;
  const int32_t t_bp = T[t].nb[(k + 1) % 3];  // across (b, p)
  const int32_t t_pa = T[t].nb[(k + 2) % 3];  // across (p, a)
  const int32_t o_aq = T[o].nb[(j + 1) % 3];  // across (a, q)
  const int32_t o_qb = T[o].nb[(j + 2) % 3];  // across (q, b)
  T[t] = Tri{{p, a, q}, {o_aq, o, t_pa}};
  T[o] = Tri{{p, q, b}, {o_qb, t_bp, t}};
  replace_neighbour(T, o_aq, o, t);
  replace_neighbour(T, t_bp, t, o);
  return true;
}

}  // namespace

// The mesh of the support points alone (no corners). A sweep in (v, u) order
// joins each new point to every hull edge it sees (the new point is the
// largest so far, so it lies outside the hull and sees a contiguous chain of
// edges around the previous point); collinear points that start the sweep are
// fanned from the first point off their line. Lawson flips under the
// canonical rule then make every edge legal. Returns the triangle count
// (2n - 2 - hull points; 0 for collinear or fewer than three points), or -1.
int32_t build_mesh_points(MeshScratch* sp, const int32_t* list, int32_t n, int32_t w,
                          int32_t h, RasterTri* tri_out, int32_t* recs_out,
                          float* planes_out) {
  MeshScratch& s = *sp;
  s.pts.resize(n);
  s.disp.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    s.pts[i] = Pt{list[3 * i], list[3 * i + 1]};
    s.disp[i] = list[3 * i + 2];
    if (list[3 * i] < 0 || list[3 * i] > w - 1 || list[3 * i + 1] < 0 || list[3 * i + 1] > h - 1)
      return -1;
  }
  s.tris.clear();
  if (n < 3) return 0;
  std::vector<int32_t> ord(n);
  for (int32_t i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return vu_less(s.pts[x], s.pts[y]); });
  for (int32_t i = 1; i < n; ++i)
    if (!vu_less(s.pts[ord[i - 1]], s.pts[ord[i]])) return -1;  // duplicate points
  // the first point off the line of the first two
  int32_t k = 2;
  while (k < n && orient(s.pts[ord[0]], s.pts[ord[1]], s.pts[ord[k]]) == 0) ++k;
  if (k == n) return 0;
  auto& T = s.tris;
  // the hull as a cycle nxt / prv in positive orientation; etri[x], eopp[x]:
  // the triangle holding the hull edge x -> nxt[x] and the local index of
  // the vertex opposite that edge
  std::vector<int32_t> nxt(n, -1), prv(n, -1), etri(n, -1), eopp(n, -1);
  const int32_t pk = ord[k];
  const bool pos = orient(s.pts[ord[0]], s.pts[ord[1]], s.pts[pk]) > 0;
  for (int32_t i = 0; i + 1 < k; ++i) {
    const int32_t a = ord[i], b = ord[i + 1];
    const int32_t t = (int32_t)T.size();
    if (pos)
      T.push_back(Tri{{a, b, pk}, {-1, -1, -1}});  // edge a->b opposite pk (index 2)
    else
      T.push_back(Tri{{b, a, pk}, {-1, -1, -1}});  // edge b->a opposite pk
    if (i > 0) {  // shares (a, pk) with the previous triangle
      const int32_t tp = t - 1;
      if (pos) {  // t = (a, b, pk): edge (pk, a) opposite b (1); tp = (a', a, pk): edge (a, pk) opposite a' (0)
        T[t].nb[1] = tp;
        T[tp].nb[0] = t;
      } else {    // t = (b, a, pk): edge (a, pk) opposite b (0); tp = (a, a', pk): edge (pk, a) opposite a' (1)
        T[t].nb[0] = tp;
        T[tp].nb[1] = t;
      }
    }
  }
  const int32_t t0 = 0, tl = (int32_t)T.size() - 1;
  if (pos) {  // o0 -> o1 -> ... -> o(k-1) -> pk -> o0
    for (int32_t i = 0; i + 1 < k; ++i) {
      nxt[ord[i]] = ord[i + 1];
      etri[ord[i]] = i;
      eopp[ord[i]] = 2;
    }
    nxt[ord[k - 1]] = pk;
    etri[ord[k - 1]] = tl;   // (o(k-2), o(k-1), pk): edge o(k-1) -> pk opposite o(k-2)
    eopp[ord[k - 1]] = 0;
    nxt[pk] = ord[0];
    etri[pk] = t0;           // (o0, o1, pk): edge pk -> o0 opposite o1
    eopp[pk] = 1;
  } else {    // o(k-1) -> ... -> o1 -> o0 -> pk -> o(k-1)
    for (int32_t i = k - 1; i > 0; --i) {
      nxt[ord[i]] = ord[i - 1];
      etri[ord[i]] = i - 1;
      eopp[ord[i]] = 2;
    }
    nxt[ord[0]] = pk;
    etri[ord[0]] = t0;       // (o1, o0, pk): edge o0 -> pk opposite o1
    eopp[ord[0]] = 0;
    nxt[pk] = ord[k - 1];
    etri[pk] = tl;           // (o(k-1), o(k-2), pk): edge pk -> o(k-1) opposite o(k-2)
    eopp[pk] = 1;
  }
  for (int32_t i = 0; i < n; ++i)
    if (nxt[i] >= 0) prv[nxt[i]] = i;
  // the remaining points in (v, u) order, each outside the hull so far
  int32_t last = pk;
  for (int32_t ii = k + 1; ii < n; ++ii) {
    const int32_t p = ord[ii];
    const Pt P = s.pts[p];
    auto visible = [&](int32_t x) { return orient(s.pts[x], s.pts[nxt[x]], P) < 0; };
    // The visible edges form one chain first -> ... -> end on the hull, and
    // it holds an edge at `last`: the hull lies in the points (v, u)-smaller
    // than `last`, a vertex with an angle below 180 degrees, and p lies
    // beyond it in that order.
    int32_t first = last, end = last;
    if (visible(last)) end = nxt[last];
    if (visible(prv[last])) first = prv[last];
    if (first == end) return -1;
    for (int32_t steps = 0; visible(prv[first]); first = prv[first])
      if (++steps > n) return -1;
    for (int32_t steps = 0; visible(end); end = nxt[end])
      if (++steps > n) return -1;
    // one triangle (y, x, p) per visible edge x -> y, chained along p
    int32_t prev_t = -1, first_t = -1;
    for (int32_t x = first; x != end; x = nxt[x]) {
      const int32_t y = nxt[x];
      const int32_t t = (int32_t)T.size();
      T.push_back(Tri{{y, x, p}, {-1, -1, etri[x]}});  // edge (y, x) opposite p
      T[etri[x]].nb[eopp[x]] = t;
      if (prev_t >= 0) {  // (x, x_prev, p) and (y, x, p) share (x, p)
        T[prev_t].nb[1] = t;  // in (x, x_prev, p) it is (p, x), opposite x_prev
        T[t].nb[0] = prev_t;  // in (y, x, p) it is (x, p), opposite y
      }
      if (first_t < 0) first_t = t;
      prev_t = t;
    }
    // hull: first -> p -> end; the chain's inner vertices leave it
    for (int32_t x = nxt[first]; x != end;) {
      const int32_t nx = nxt[x];
      nxt[x] = prv[x] = -1;
      x = nx;
    }
    nxt[first] = p;
    prv[p] = first;
    nxt[p] = end;
    prv[end] = p;
    etri[first] = first_t;   // (x1, first, p): edge first -> p opposite x1
    eopp[first] = 0;
    etri[p] = prev_t;        // (end, x_last, p): edge p -> end opposite x_last
    eopp[p] = 1;
    last = p;
  }
  // Lawson flips until every interior edge is legal
  std::vector<std::pair<int32_t, int>> stack;
  for (int32_t t = 0; t < (int32_t)T.size(); ++t)
    for (int k2 = 0; k2 < 3; ++k2)
      if (T[t].nb[k2] > t) stack.push_back({t, k2});
  const int64_t limit = 64ll * (int64_t)T.size() * (int64_t)T.size() + 1024;
  for (int64_t guard = 0; !stack.empty(); ++guard) {
    if (guard > limit) return -1;
    const auto [t, kk] = stack.back();
    stack.pop_back();
    const int32_t o = T[t].nb[kk];
    if (!flip_if_illegal(s, t, kk)) continue;
    for (int q = 0; q < 3; ++q) {
      stack.push_back({t, q});
      stack.push_back({o, q});
    }
  }
  int32_t nhull = 0;
  for (int32_t i = 0; i < n; ++i) nhull += nxt[i] >= 0 ? 1 : 0;
  if ((int32_t)T.size() != 2 * n - 2 - nhull) return -1;
  return finish_mesh(s, n, tri_out, recs_out, planes_out);
}

}  // namespace elas

/*
 * Oracle, mesh stages: Delaunay triangulation of the support points, the
 * slanted plane of each triangle, and the remap of the mesh into a per-pixel
 * matrix of plane priors (Section III-A, Fig. 1(g); Section VI-D).
 * TEST INFRASTRUCTURE ONLY (see elas_oracle.h).
 *
 * The paper names Delaunay triangulation and nothing more. Support points
 * sit on a lattice, so four or more co-circular points are common and the
 * triangulation must be made unique. Reading: the Delaunay subdivision in
 * which every cell of >= 4 co-circular points is split as a fan from its
 * smallest vertex in (v, u) order. This is the Delaunay triangulation of the
 * points lifted to the paraboloid with an infinitesimal downward push that is
 * largest for the (v, u)-smallest point ("pulling" it), so it is unique and
 * does not depend on the algorithm or insertion order. Here it is built by
 * Bowyer-Watson insertion with that perturbed in-circle test, exact int64.
 */
#include "elas_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_orient(const int32_t* a, const int32_t* b, const int32_t* c) {
  return (int64_t)(b[0] - a[0]) * (c[1] - a[1]) - (int64_t)(b[1] - a[1]) * (c[0] - a[0]);
}

/* Positive iff d lies strictly inside the circle through a, b, c when
 * orient(a, b, c) > 0. Exact: coordinates below 2^13 keep every term below
 * 2^55. */
int64_t orc_incircle(const int32_t* a, const int32_t* b, const int32_t* c,
                     const int32_t* d) {
  int64_t adx = a[0] - d[0], ady = a[1] - d[1];
  int64_t bdx = b[0] - d[0], bdy = b[1] - d[1];
  int64_t cdx = c[0] - d[0], cdy = c[1] - d[1];
  int64_t al = adx * adx + ady * ady;
  int64_t bl = bdx * bdx + bdy * bdy;
  int64_t cl = cdx * cdx + cdy * cdy;
  return al * (bdx * cdy - cdx * bdy) - bl * (adx * cdy - cdx * ady) +
         cl * (adx * bdy - bdx * ady);
}

/* (v, u) order */
static int lex_less(const int32_t* a, const int32_t* b) {
  return a[1] < b[1] || (a[1] == b[1] && a[0] < b[0]);
}

/* In-circle under the pulling perturbation. Exactly co-circular case: the
 * (v, u)-smallest of the four points is pushed down the most. If that is p,
 * p is inside. If it is a triangle vertex m, the circle through the pushed
 * triangle shrinks away from the side opposite m, so p counts as inside iff
 * it lies across the edge opposite m. */
static int inside_perturbed(const int32_t* P, const int32_t* t, int32_t ip) {
  const int32_t *a = P + 2 * t[0], *b = P + 2 * t[1], *c = P + 2 * t[2], *p = P + 2 * ip;
  int64_t det = orc_incircle(a, b, c, p);
  if (det != 0) return det > 0;
  const int32_t* m = p;
  int mi = -1;
  const int32_t* vs[3] = {a, b, c};
  for (int i = 0; i < 3; ++i)
    if (lex_less(vs[i], m)) {
      m = vs[i];
      mi = i;
    }
  if (mi < 0) return 1;
  const int32_t* e1 = vs[(mi + 1) % 3];
  const int32_t* e2 = vs[(mi + 2) % 3];
  int64_t op = orc_orient(e1, e2, p), om = orc_orient(e1, e2, m);
  return (op > 0) != (om > 0);
}

int32_t orc_delaunay(const int32_t* pts, int32_t n, int32_t* tris) {
  if (n < 4) return -1;
  int32_t W1 = pts[2], H1 = pts[5];
  if (pts[0] != 0 || pts[1] != 0 || pts[3] != 0 || pts[4] != 0 || pts[6] != W1 ||
      pts[7] != H1 || W1 <= 0 || H1 <= 0)
    return -1;
  for (int32_t i = 4; i < n; ++i)
    if (pts[2 * i] <= 0 || pts[2 * i] >= W1 || pts[2 * i + 1] <= 0 || pts[2 * i + 1] >= H1)
      return -1;
  int32_t cap = 2 * n + 8;
  int32_t* live = (int32_t*)malloc(sizeof(int32_t) * 3 * cap);
  int32_t* bad = (int32_t*)malloc(sizeof(int32_t) * cap);
  int32_t* edges = (int32_t*)malloc(sizeof(int32_t) * 2 * 3 * cap);
  int32_t nt = 0;
  /* The four corners are co-circular: fan from (0,0), the smallest. */
  const int32_t init[2][3] = {{0, 1, 3}, {0, 3, 2}};
  for (int k = 0; k < 2; ++k) {
    memcpy(live + 3 * nt, init[k], sizeof(init[k]));
    ++nt;
  }
  int32_t status = 0;
  for (int32_t ip = 4; ip < n && status == 0; ++ip) {
    int32_t nb = 0;
    for (int32_t t = 0; t < nt; ++t)
      if (inside_perturbed(pts, live + 3 * t, ip)) bad[nb++] = t;
    /* cavity boundary: edges of bad triangles whose reverse is not an edge of
     * another bad triangle */
    int32_t ne = 0;
    for (int32_t i = 0; i < nb; ++i) {
      const int32_t* t = live + 3 * bad[i];
      for (int e = 0; e < 3; ++e) {
        int32_t a = t[e], b = t[(e + 1) % 3];
        int shared = 0;
        for (int32_t j = 0; j < nb && !shared; ++j) {
          if (j == i) continue;
          const int32_t* s = live + 3 * bad[j];
          for (int f = 0; f < 3; ++f)
            if (s[f] == b && s[(f + 1) % 3] == a) shared = 1;
        }
        if (!shared) {
          edges[2 * ne] = a;
          edges[2 * ne + 1] = b;
          ++ne;
        }
      }
    }
    /* remove bad triangles (descending order keeps indices valid) */
    for (int32_t i = nb - 1; i >= 0; --i) {
      int32_t t = bad[i];
      --nt;
      if (t != nt) memcpy(live + 3 * t, live + 3 * nt, 3 * sizeof(int32_t));
    }
    for (int32_t i = 0; i < ne; ++i) {
      int32_t a = edges[2 * i], b = edges[2 * i + 1];
      if (orc_orient(pts + 2 * a, pts + 2 * b, pts + 2 * ip) <= 0 || nt >= cap) {
        status = -1;
        break;
      }
      live[3 * nt] = a;
      live[3 * nt + 1] = b;
      live[3 * nt + 2] = ip;
      ++nt;
    }
  }
  if (status == 0) memcpy(tris, live, sizeof(int32_t) * 3 * nt);
  free(live);
  free(bad);
  free(edges);
  return status == 0 ? nt : -1;
}

/* ------------------------------------------------------------------------
 * Delaunay triangulation of the points alone (no image corners), by gift
 * wrapping: every hull edge and every edge of a Delaunay triangle is a
 * Delaunay edge, and the triangle on the left of a Delaunay edge (a, b) has
 * as apex the point left of it whose circle through a and b holds no other
 * candidate (under the same perturbed in-circle test, the points are in
 * general position, so that point is unique). Starting from one hull edge,
 * each triangle's two new edges are wrapped in turn; each directed edge is
 * taken once. Plain O(n^2): n scans of the points per triangle pair.
 * Returns the triangle count (0 for fewer than three points or collinear
 * ones), -1 for bad input.
 * ---------------------------------------------------------------------- */
typedef struct {
  int64_t* keys;  /* directed edge a * n + b, or -1 */
  int64_t cap;
} edge_set;

static int edge_set_add(edge_set* s, int64_t key) { /* 1 if newly added */
  uint64_t h = (uint64_t)key * 0x9E3779B97F4A7C15ull;
  int64_t i = (int64_t)(h % (uint64_t)s->cap);
  while (s->keys[i] >= 0) {
    if (s->keys[i] == key) return 0;
    i = (i + 1) % s->cap;
  }
  s->keys[i] = key;
  return 1;
}

static int edge_set_has(const edge_set* s, int64_t key) {
  uint64_t h = (uint64_t)key * 0x9E3779B97F4A7C15ull;
  int64_t i = (int64_t)(h % (uint64_t)s->cap);
  while (s->keys[i] >= 0) {
    if (s->keys[i] == key) return 1;
    i = (i + 1) % s->cap;
  }
  return 0;
}

int32_t orc_delaunay_points(const int32_t* pts, int32_t n, int32_t* tris) {
  if (n < 0) return -1;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j)
      if (pts[2 * i] == pts[2 * j] && pts[2 * i + 1] == pts[2 * j + 1]) return -1;
  if (n < 3) return 0;
  /* a: the (v, u)-smallest point; b: the next hull vertex, the point with
   * every other point on its positive side or on the line beyond it */
  int32_t a = 0;
  for (int32_t i = 1; i < n; ++i)
    if (lex_less(pts + 2 * i, pts + 2 * a)) a = i;
  int32_t b = -1;
  for (int32_t i = 0; i < n; ++i) {
    if (i == a) continue;
    if (b < 0) {
      b = i;
      continue;
    }
    int64_t o = orc_orient(pts + 2 * a, pts + 2 * b, pts + 2 * i);
    if (o < 0) {
      b = i;
    } else if (o == 0) { /* collinear: the nearer point is the hull neighbour */
      int64_t db = (int64_t)(pts[2 * b] - pts[2 * a]) * (pts[2 * b] - pts[2 * a]) +
                   (int64_t)(pts[2 * b + 1] - pts[2 * a + 1]) * (pts[2 * b + 1] - pts[2 * a + 1]);
      int64_t di = (int64_t)(pts[2 * i] - pts[2 * a]) * (pts[2 * i] - pts[2 * a]) +
                   (int64_t)(pts[2 * i + 1] - pts[2 * a + 1]) * (pts[2 * i + 1] - pts[2 * a + 1]);
      if (di < db) b = i;
    }
  }
  int collinear = 1;
  for (int32_t i = 0; i < n && collinear; ++i)
    if (orc_orient(pts + 2 * a, pts + 2 * b, pts + 2 * i) != 0) collinear = 0;
  if (collinear) return 0;
  edge_set done = {NULL, 16 * (int64_t)n + 64};
  done.keys = (int64_t*)malloc(sizeof(int64_t) * done.cap);
  for (int64_t i = 0; i < done.cap; ++i) done.keys[i] = -1;
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * 2 * (6 * (size_t)n + 8));
  int32_t top = 0, nt = 0, cap = 2 * n;
  stack[top++] = a;
  stack[top++] = b;
  int32_t status = 0;
  while (top > 0 && status == 0) {
    const int32_t y = stack[--top], x = stack[--top];
    if (edge_set_has(&done, (int64_t)x * n + y)) continue;
    /* the apex: the left point whose circle through x, y holds no other */
    int32_t c = -1;
    for (int32_t i = 0; i < n; ++i) {
      if (orc_orient(pts + 2 * x, pts + 2 * y, pts + 2 * i) <= 0) continue;
      if (c < 0) {
        c = i;
        continue;
      }
      const int32_t t[3] = {x, y, c};
      if (inside_perturbed(pts, t, i)) c = i;
    }
    if (c < 0) continue; /* a hull edge: nothing on its left */
    if (nt >= cap) {
      status = -1;
      break;
    }
    tris[3 * nt] = x;
    tris[3 * nt + 1] = y;
    tris[3 * nt + 2] = c;
    ++nt;
    edge_set_add(&done, (int64_t)x * n + y);
    edge_set_add(&done, (int64_t)y * n + c);
    edge_set_add(&done, (int64_t)c * n + x);
    /* the triangles across its two other edges */
    if (!edge_set_has(&done, (int64_t)c * n + y)) {
      stack[top++] = c;
      stack[top++] = y;
    }
    if (!edge_set_has(&done, (int64_t)x * n + c)) {
      stack[top++] = x;
      stack[top++] = c;
    }
  }
  free(done.keys);
  free(stack);
  return status == 0 ? nt : -1;
}

/* ------------------------------------------------------------------------
 * Canonical triangle records: vertices sorted by (v, u), triangles sorted by
 * their sorted vertex triples. The record order is the tie rule for pixels
 * on shared edges and vertices (the earlier record owns them).
 * ---------------------------------------------------------------------- */
static int cmp_vertex(const int32_t* a, const int32_t* b) {
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  return 0;
}

static int cmp_record(const void* x, const void* y) {
  const int32_t* a = (const int32_t*)x;
  const int32_t* b = (const int32_t*)y;
  for (int k = 0; k < 3; ++k) {
    int c = cmp_vertex(a + 3 * k, b + 3 * k);
    if (c) return c;
  }
  return 0;
}

void orc_canonical_triangles(const int32_t* pts, const int32_t* tris, int32_t ntri,
                             int32_t* recs) {
  for (int32_t t = 0; t < ntri; ++t) {
    int32_t* r = recs + 9 * t;
    for (int k = 0; k < 3; ++k) memcpy(r + 3 * k, pts + 3 * tris[3 * t + k], 3 * sizeof(int32_t));
    /* insertion sort of three vertices */
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && cmp_vertex(r + 3 * j, r + 3 * (j - 1)) < 0; --j) {
        int32_t tmp[3];
        memcpy(tmp, r + 3 * j, sizeof(tmp));
        memcpy(r + 3 * j, r + 3 * (j - 1), sizeof(tmp));
        memcpy(r + 3 * (j - 1), tmp, sizeof(tmp));
      }
  }
  qsort(recs, (size_t)ntri, 9 * sizeof(int32_t), cmp_record);
}

/* ------------------------------------------------------------------------
 * Slanted plane d = a*u + b*v + c through a triangle's three support points
 * (Section III-A). Exact integer Cramer numerators relative to the first
 * vertex, then one correctly rounded double division each, rounded to FP32.
 * The quotients are exact rationals of the plane, so the result does not
 * depend on the vertex order.
 * ---------------------------------------------------------------------- */
void orc_plane(const int32_t* rec, float* abc) {
  int64_t u1 = rec[0], v1 = rec[1], d1 = rec[2];
  int64_t du2 = rec[3] - u1, dv2 = rec[4] - v1, dd2 = rec[5] - d1;
  int64_t du3 = rec[6] - u1, dv3 = rec[7] - v1, dd3 = rec[8] - d1;
  int64_t det = du2 * dv3 - du3 * dv2;
  int64_t an = dd2 * dv3 - dd3 * dv2;
  int64_t bn = du2 * dd3 - du3 * dd2;
  int64_t cn = d1 * det - an * u1 - bn * v1;
  abc[0] = (float)((double)an / (double)det);
  abc[1] = (float)((double)bn / (double)det);
  abc[2] = (float)((double)cn / (double)det);
}

/* ------------------------------------------------------------------------
 * Remap of the mesh into an image-sized matrix of disparity priors
 * (Section VI-D). A pixel belongs to the first triangle in canonical order
 * that contains it in the closed sense (edge functions >= 0). Plane mean in
 * FP32, fixed order ((a*u) + (b*v)) + c, no fused multiply-add; d_plane is
 * floor(mean + 0.5) clamped to [dmin, dmax]; -1 where no triangle covers.
 * ---------------------------------------------------------------------- */
void orc_plane_map(const orc_params* p, const int32_t* recs, const float* planes,
                   int32_t ntri, int32_t w, int32_t h, int32_t* owner,
                   int16_t* dplane) {
  for (size_t i = 0; i < (size_t)w * h; ++i) owner[i] = -1;
  for (int32_t t = 0; t < ntri; ++t) {
    const int32_t* r = recs + 9 * t;
    int32_t A[2] = {r[0], r[1]}, B[2] = {r[3], r[4]}, C[2] = {r[6], r[7]};
    if (orc_orient(A, B, C) < 0) {
      int32_t tmp[2] = {B[0], B[1]};
      B[0] = C[0];
      B[1] = C[1];
      C[0] = tmp[0];
      C[1] = tmp[1];
    }
    int32_t umin = A[0], umax = A[0], vmin = A[1], vmax = A[1];
    const int32_t* vs[2] = {B, C};
    for (int k = 0; k < 2; ++k) {
      if (vs[k][0] < umin) umin = vs[k][0];
      if (vs[k][0] > umax) umax = vs[k][0];
      if (vs[k][1] < vmin) vmin = vs[k][1];
      if (vs[k][1] > vmax) vmax = vs[k][1];
    }
    if (umin < 0) umin = 0;
    if (vmin < 0) vmin = 0;
    if (umax > w - 1) umax = w - 1;
    if (vmax > h - 1) vmax = h - 1;
    for (int32_t v = vmin; v <= vmax; ++v)
      for (int32_t u = umin; u <= umax; ++u) {
        size_t i = (size_t)v * w + u;
        if (owner[i] >= 0) continue;
        int32_t X[2] = {u, v};
        if (orc_orient(A, B, X) >= 0 && orc_orient(B, C, X) >= 0 && orc_orient(C, A, X) >= 0)
          owner[i] = t;
      }
  }
  for (int32_t v = 0; v < h; ++v)
    for (int32_t u = 0; u < w; ++u) {
      size_t i = (size_t)v * w + u;
      if (owner[i] < 0) {
        dplane[i] = -1;
        continue;
      }
      const float* abc = planes + 3 * owner[i];
      float au = abc[0] * (float)u;
      float bv = abc[1] * (float)v;
      float mu = au + bv;
      mu = mu + abc[2];
      float f = floorf(mu + 0.5f);
      int32_t d;
      if (f < (float)p->disp_min)
        d = p->disp_min;
      else if (f > (float)p->disp_max)
        d = p->disp_max;
      else
        d = (int32_t)f;
      dplane[i] = (int16_t)d;
    }
}

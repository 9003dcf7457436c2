// Device-resident mesh step (Section III-A: Delaunay triangulation of the
// support points, one slanted plane per triangle). The paper's CPU/FPGA split
// (Section IV) leaves this sequential step to the CPU; here it runs on the
// GPU so that a frame needs no host round trip.
//
// One 1024-thread workgroup per view:
//  1. gather the per-row support lists into points in (v, u) rank order:
//     rank 0 = (0,0), 1 = (w-1,0), 2..n+1 = the lists, n+2 = (0,h-1),
//     n+3 = (w-1,h-1); each corner takes the d of the nearest list point.
//     A point is one 32-bit key v<<20 | u<<8 | (d - dmin): key order is rank
//     order, so triangles carry keys and need no vertex ids.
//  2. initial triangulation. Support points lie on lattice rows, so the
//     region between two consecutive non-empty rows (the image's top and
//     bottom edges act as extra rows) is a trapezoid, triangulated by the
//     in-circle zipper over the two sorted rows, which for two horizontal
//     rows is a merge of their edge u-sums (one lane per row edge). On a tie
//     (four co-circular points, e.g. every lattice rectangle) the lower edge's
//     triangle comes first, which gives the diagonal from the (v, u)-smallest
//     of the four: the canonical fan, so such cells need no flip. The two side
//     pockets between the rows' end points and the image border are
//     polygons monotone in v with one straight side. Their stack
//     triangulation has a closed form that is evaluated in parallel: the
//     point below a chain point on the stack is the earlier point at the
//     extreme angle seen from it (the later one on ties); the point that pops
//     it is the first later chain point strictly across that segment (none:
//     the bottom corner). Each chain point gives one triangle.
//  3. adjacency: a neighbour is stored as 4 * triangle + local vertex index.
//     The bands set the neighbours their construction fixes (row edges and
//     band diagonals); the other half-edges are matched with their reverse
//     through buckets by origin vertex.
//  4. Lawson flips in synchronous rounds until every edge is legal under the
//     canonical rule (strictly outside the circumcircle, or exactly on it and
//     the (v, u)-smallest of the four points is an endpoint of the edge).
//     A round tests the edges of the triangles flipped in the previous round
//     and keeps the previous candidates whose two triangles did not change
//     (an edge with unchanged triangles keeps its verdict). Each candidate
//     claims its two triangles with an atomic max of a round-stamped,
//     inverted edge key, so the smallest key wins and no claim is ever
//     reset; winners flip, then every flipped triangle re-links its outer
//     neighbours. The canonical rule is a consistent perturbation of the
//     lifted points, so the flips end at the unique canonical triangulation
//     whatever the starting mesh.
//  5. canonical order (bucket by smallest vertex, position within the
//     bucket), exact planes and raster records.
// The predicates are exact: orientation in int32, and the in-circle
// determinant in fp64 from int32 minors below 2^26, so every product and sum
// is an integer below 2^53; this needs coordinates below 4096.
// Arrays live in LDS (16-bit indices) when they fit, else in a global
// scratch area (32-bit indices); both paths run the same template.
#include <algorithm>
#include <climits>

#include <hip/hip_ext.h>

#include "elas_internal.h"
#include "elas_wave.h"

namespace elas {
namespace {

constexpr int kMT = 1024;          // threads per mesh workgroup
constexpr int kPocketG = 4;        // lanes per side pocket point
constexpr int kTwinUnknown = -2;   // neighbour code of a half-edge not yet matched

// ---- point keys and exact predicates --------------------------------------
__device__ __forceinline__ int key_u(uint32_t k) { return (int)((k >> 8) & 0xFFFu); }
__device__ __forceinline__ int key_v(uint32_t k) { return (int)(k >> 20); }
__device__ __forceinline__ int key_dd(uint32_t k) { return (int)(k & 0xFFu); }
__device__ __forceinline__ uint32_t make_key(int u, int v, int dd) {
  return ((uint32_t)v << 20) | ((uint32_t)u << 8) | (uint32_t)dd;
}

// > 0 if (a, b, c) turns counter-clockwise in (u, v); |value| < 2^25.
__device__ __forceinline__ int orient_k(uint32_t a, uint32_t b, uint32_t c) {
  const int au = key_u(a), av = key_v(a);
  return (key_u(b) - au) * (key_v(c) - av) - (key_v(b) - av) * (key_u(c) - au);
}

// > 0 if d lies inside the circle through the counter-clockwise a, b, c.
__device__ __forceinline__ double incircle_k(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const int du = key_u(d), dv = key_v(d);
  const int ax = key_u(a) - du, ay = key_v(a) - dv;
  const int bx = key_u(b) - du, by = key_v(b) - dv;
  const int cx = key_u(c) - du, cy = key_v(c) - dv;
  const int la = ax * ax + ay * ay, lb = bx * bx + by * by, lc = cx * cx + cy * cy;
  const int xa = bx * cy - by * cx, xb = cx * ay - cy * ax, xc = ax * by - ay * bx;
  return (double)la * (double)xa + (double)lb * (double)xb + (double)lc * (double)xc;
}

// Edge (a, b) of the counter-clockwise triangle (p, a, b) against the apex q
// of the triangle across it.
__device__ __forceinline__ bool edge_illegal(uint32_t p, uint32_t a, uint32_t b, uint32_t q) {
  const double ic = incircle_k(p, a, b, q);
  if (ic != 0.0) return ic > 0.0;
  // co-circular: legal iff the (v, u)-smallest point is an endpoint
  const uint32_t mn = min(min(p, q), min(a, b));
  return !(mn == a || mn == b);
}

__device__ __forceinline__ void sort3(uint32_t& a, uint32_t& b, uint32_t& c) {
  if (a > b) { const uint32_t t = a; a = b; b = t; }
  if (b > c) { const uint32_t t = b; b = c; c = t; }
  if (a > b) { const uint32_t t = a; a = b; b = t; }
}

// ---- workgroup scans --------------------------------------------------------
// Exclusive scan over the workgroup; *total receives the sum.
__device__ int scan_excl(int x, int* total, int* wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int incl = wave_scan_incl(x);
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kMT / 64; ++w) {
    const int s = wsum[w];
    before += w < wid ? s : 0;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// In-place exclusive scan of a[0..n); returns the total.
__device__ int scan_array(int32_t* a, int n, int* wsum) {
  int base = 0;
  for (int c0 = 0; c0 < n; c0 += kMT) {
    const int i = c0 + threadIdx.x;
    const int x = i < n ? a[i] : 0;
    int tot;
    const int e = scan_excl(x, &tot, wsum);
    if (i < n) a[i] = base + e;
    base += tot;
  }
  __syncthreads();
  return base;
}

// ---- memory layout ----------------------------------------------------------
// Claim words: round << shift | (mask - edge key). The 16-bit variant has
// fewer than 8192 triangles (keys below 2^15) and fewer than 2^15 rounds.
template <typename I>
struct ClaimT;
template <>
struct ClaimT<int16_t> {
  typedef uint32_t T;
  static constexpr int kShift = 17;
};
template <>
struct ClaimT<int32_t> {
  typedef unsigned long long T;
  static constexpr int kShift = 32;
};

template <typename I>
__device__ __forceinline__ typename ClaimT<I>::T claim_stamp(int round, int key) {
  typedef typename ClaimT<I>::T C;
  const C mask = (C(1) << ClaimT<I>::kShift) - 1;
  return (C(round) << ClaimT<I>::kShift) | (mask - (C)(unsigned)key);
}

template <typename I>
struct MeshMem {
  typedef typename ClaimT<I>::T C;
  // rows and side chains (sized by the lattice height only)
  int32_t* rowStart;     // lh + 1: first point of each lattice row, then n
  int32_t* rowNE;        // lh + 1: non-empty lattice rows in order
  int32_t* rowRank;      // lh + 1: index of a non-empty lattice row among them
  int32_t* stripOff;     // lh + 2: first triangle of each strip
  uint32_t *chainK0, *chainK1;  // lh + 1: key of the first / last point of each non-empty row
  int32_t *chainI0, *chainI1;   // lh + 1: its rank
  // points and triangles
  uint32_t* pk;          // NP keys in rank order
  uint32_t* tk;          // 3 NT vertex keys, counter-clockwise
  I* tn;                 // 3 NT neighbour across the edge opposite vertex k: 4 t + k', or -1
  // construction and adjacency (aliases: hbuck in tk, the rest in the flip state)
  I* hbuck;              // 3 NT half-edges grouped by origin vertex
  I* tv;                 // 3 NT vertex ranks
  int32_t* vcnt;         // NP + 1 bucket starts
  int32_t* vcur;         // NP + 1 fill cursors
  // flip state
  C* claim;              // NT
  I* partner;            // NT flip partner of the last flip
  uint16_t* flipr;       // NT round of the last flip (0: none)
  I *lf0, *lf1;          // NT flipped triangles of a round, by round parity
  I *cl0, *cl1;          // ncand candidate edge keys of a round, by round parity
  // canonical order (aliases of the flip state)
  int32_t* scnt;         // NP + 1 bucket starts by smallest vertex rank
  int32_t* scur;         // NP + 1 fill cursors
  I* slist;              // NT triangles grouped by smallest vertex
  int32_t* smin;         // NT: rank of each triangle's smallest vertex
  int NP, NT, ncand;
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

struct Carver {
  char* base;
  size_t off;
  __host__ __device__ __forceinline__ char* take(size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += a16(bytes);
    return p;
  }
};

// Lays the arrays of one view out from base (base == nullptr: sizes only)
// into m; returns the bytes used. The row arrays come first, at offsets that do not
// depend on n.
template <typename I>
__host__ __device__ __forceinline__ size_t carve(char* base, int n, int lh, MeshMem<I>& m) {
  typedef typename ClaimT<I>::T C;
  const size_t NP = (size_t)n + 4, NT = 2 * (size_t)n + 2, L = (size_t)lh + 2;
  const size_t ncand = 3 * NT / 2 + 2;
  Carver c{base, 0};
  MeshMem<I> t{};
  t.rowStart = reinterpret_cast<int32_t*>(c.take(L * 4));
  t.rowNE = reinterpret_cast<int32_t*>(c.take(L * 4));
  t.rowRank = reinterpret_cast<int32_t*>(c.take(L * 4));
  t.stripOff = reinterpret_cast<int32_t*>(c.take(L * 4));
  t.chainK0 = reinterpret_cast<uint32_t*>(c.take(L * 4));
  t.chainI0 = reinterpret_cast<int32_t*>(c.take(L * 4));
  t.chainK1 = reinterpret_cast<uint32_t*>(c.take(L * 4));
  t.chainI1 = reinterpret_cast<int32_t*>(c.take(L * 4));
  t.pk = reinterpret_cast<uint32_t*>(c.take(NP * 4));
  char* r1 = c.take(3 * NT * 4);
  t.tk = reinterpret_cast<uint32_t*>(r1);
  t.hbuck = reinterpret_cast<I*>(r1);
  t.tn = reinterpret_cast<I*>(c.take(3 * NT * sizeof(I)));
  // region of the flip state, shared with construction and final order
  const size_t flip_bytes = a16(NT * sizeof(C)) + a16(NT * sizeof(I)) + a16(NT * 2) +
                            2 * a16(NT * sizeof(I)) + 2 * a16(ncand * sizeof(I));
  const size_t adj_bytes = a16(3 * NT * sizeof(I)) + 2 * a16((NP + 1) * 4);
  const size_t fin_bytes = 2 * a16((NP + 1) * 4) + a16(NT * sizeof(I)) + a16(NT * 4);
  size_t d_bytes = flip_bytes;
  if (adj_bytes > d_bytes) d_bytes = adj_bytes;
  if (fin_bytes > d_bytes) d_bytes = fin_bytes;
  char* rd = c.take(d_bytes);
  {
    Carver d{rd, 0};
    t.claim = reinterpret_cast<C*>(d.take(NT * sizeof(C)));
    t.partner = reinterpret_cast<I*>(d.take(NT * sizeof(I)));
    t.flipr = reinterpret_cast<uint16_t*>(d.take(NT * 2));
    t.lf0 = reinterpret_cast<I*>(d.take(NT * sizeof(I)));
    t.lf1 = reinterpret_cast<I*>(d.take(NT * sizeof(I)));
    t.cl0 = reinterpret_cast<I*>(d.take(ncand * sizeof(I)));
    t.cl1 = reinterpret_cast<I*>(d.take(ncand * sizeof(I)));
  }
  {
    Carver d{rd, 0};
    t.tv = reinterpret_cast<I*>(d.take(3 * NT * sizeof(I)));
    t.vcnt = reinterpret_cast<int32_t*>(d.take((NP + 1) * 4));
    t.vcur = reinterpret_cast<int32_t*>(d.take((NP + 1) * 4));
  }
  {
    Carver d{rd, 0};
    t.scnt = reinterpret_cast<int32_t*>(d.take((NP + 1) * 4));
    t.scur = reinterpret_cast<int32_t*>(d.take((NP + 1) * 4));
    t.slist = reinterpret_cast<I*>(d.take(NT * sizeof(I)));
    t.smin = reinterpret_cast<int32_t*>(d.take(NT * 4));
  }
  t.NP = (int)NP;
  t.NT = (int)NT;
  t.ncand = (int)ncand;
  m = t;
  return c.off;
}

struct MeshShared {
  int wsum[kMT / 64];
  unsigned long long corner[4];
  int ncand[2];   // candidates appended in a round, by parity
  int nflip[2];   // flipped triangles appended in a round, by parity
  int err;        // 2: the initial triangulation failed a consistency check
  int border;     // half-edges without a twin (4 for a valid mesh)
};

// Writes triangle k with ranks (a, b, c) and keys (ka, kb, kc), turned
// counter-clockwise.
template <typename I>
__device__ __forceinline__ void put_tri(I* tv, int NT, int k, int a, int b, int c, uint32_t ka,
                                        uint32_t kb, uint32_t kc, int* err) {
  const int o = orient_k(ka, kb, kc);
  if (k < 0 || k >= NT || o == 0) {
    *err = 2;
    return;
  }
  if (o < 0) {
    const int t = b;
    b = c;
    c = t;
  }
  tv[3 * k] = (I)a;
  tv[3 * k + 1] = (I)b;
  tv[3 * k + 2] = (I)c;
}

// One side pocket point: chain index k in 1..m of side s (0: the rows' first
// points against the left border, 1: last points against the right border),
// evaluated by a group of G lanes (l: this lane's index in the group; the
// group's lanes are consecutive and run this call together).
template <typename I, int G>
__device__ __forceinline__ void pocket_point(const uint32_t* pk, const uint32_t* ck,
                                             const int32_t* ci, I* tv, int NT, int s, int k, int m,
                                             int n, int slot0, int l, int* err) {
  const int T = s == 0 ? 0 : 1, B = s == 0 ? n + 2 : n + 3;
  const uint32_t c = ck[k - 1];
  // below c on the stack: the earlier point at the extreme angle from c, the
  // later one on ties. All earlier points (and the top corner, index 0 here)
  // lie strictly above c's row, so the angle order is total and the choice
  // is an argmax: each lane takes every G-th point, then the lanes combine.
  uint32_t q = pk[T];
  int qx = l == 0 ? 0 : -1;  // -1: none yet
#pragma unroll 2
  for (int x = 1 + l; x < k; x += G) {
    const uint32_t kx = ck[x - 1];
    const int o = orient_k(q, c, kx);
    if (qx < 0 || (s == 0 ? o >= 0 : o <= 0)) {
      q = kx;
      qx = x;
    }
  }
  static_assert(G == 4, "a pocket point's lanes are the lanes of a quad");
#pragma unroll
  for (int off = 2; off >= 1; off >>= 1) {
    const uint32_t q2 = (uint32_t)(off == 2 ? quad_xor2((int)q) : quad_xor1((int)q));
    const int x2 = off == 2 ? quad_xor2(qx) : quad_xor1(qx);
    const int o = orient_k(q, c, q2);
    const bool take =
        x2 >= 0 && (qx < 0 || (s == 0 ? o > 0 : o < 0) || (o == 0 && x2 > qx));
    if (take) {
      q = q2;
      qx = x2;
    }
  }
  // the point that pops c: the first later point strictly across (q, c),
  // found G points at a time
  const int gbase = (threadIdx.x & 63) - l;
  const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
  int py = m + 1;  // none: the bottom corner
  for (int base = k + 1; base <= m; base += G) {
    const int y = base + l;
    bool hit = false;
    if (y <= m) {
      const int o = orient_k(q, c, ck[y - 1]);
      hit = s == 0 ? o > 0 : o < 0;
    }
    const unsigned long long gm = (__ballot(hit) >> gbase) & gmask;
    if (gm) {
      py = base + __ffsll((long long)gm) - 1;
      break;
    }
  }
  if (l != 0) return;
  const int qi = qx == 0 ? T : ci[qx - 1];
  const int pi = py > m ? B : ci[py - 1];
  const uint32_t p = py > m ? pk[B] : ck[py - 1];
  put_tri(tv, NT, slot0 + k - 1, qi, ci[k - 1], pi, q, c, p, err);
}

// Strip triangles. Within the band between two consecutive non-empty rows
// (upper row A, lower row B, both sorted by u and each on one lattice row)
// a zipper that takes the in-circle choice of the diagonal at every step is
// a merge: for points on two horizontal lines, B[j+1] lies strictly inside
// the circle through A[i], A[i+1], B[j] exactly when
// u(B[j]) + u(B[j+1]) < u(A[i]) + u(A[i+1]). So the top edge i takes the
// triangle (A[i], A[i+1], B[j]) with j the number of lower edge sums below
// its sum, and the bottom edge j the triangle (A[i], B[j+1], B[j]) with i
// the number of upper edge sums at or below its sum (ties: the upper edge
// first); either sits at slot i + j of the band. Rows of band s: the upper
// one is the top corners for s = 0, the lower one the bottom corners for
// s = m.
struct BandRow {
  int first, count;  // rank of its first point, number of points
};

__device__ __forceinline__ BandRow band_upper(int s, const int32_t* rowStart,
                                              const int32_t* rowNE) {
  if (s == 0) return {0, 2};
  const int l = rowNE[s - 1];
  return {2 + rowStart[l], rowStart[l + 1] - rowStart[l]};
}

__device__ __forceinline__ BandRow band_lower(int s, int m, int n, const int32_t* rowStart,
                                              const int32_t* rowNE) {
  if (s == m) return {n + 2, 2};
  const int l = rowNE[s];
  return {2 + rowStart[l], rowStart[l + 1] - rowStart[l]};
}

// Number of edges of row r whose u-sum is below sum (or_equal: at or below).
__device__ __forceinline__ int edges_below(const uint32_t* pk, BandRow r, int sum,
                                           bool or_equal) {
  int lo = 0, hi = r.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int t = key_u(pk[r.first + mid]) + key_u(pk[r.first + mid + 1]);
    if (t < sum || (or_equal && t == sum))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The one or two band triangles of edge (ga, ga + 1), with the twins known
// from the construction: the row edge joins them, and each is joined to the
// next triangle of its band across their diagonal (local vertex 0 of a top
// edge triangle or 2 of a bottom edge one, against 1 of the next). q = 0: the top
// corners (top edge of band 0); q = 1: the bottom corners (bottom edge of
// band m); q >= 2: the points of rank q and q + 1 if they share a row (the
// top edge of the band below, the bottom edge of the band above).
template <typename I>
__device__ __forceinline__ void strip_edge(int q, const uint32_t* pk, const int32_t* rowStart,
                                           const int32_t* rowNE, const int32_t* rowRank,
                                           const int32_t* stripOff, const Geometry& g, int m,
                                           int n, I* tv, I* tn, int NT, int* err,
                                           int* border) {
  int ga, idx, below, above;  // band below / above the edge, -1: none
  if (q == 0) {
    ga = 0, idx = 0, below = 0, above = -1;
  } else if (q == 1) {
    ga = n + 2, idx = 0, below = -1, above = m;
  } else {
    if (q + 1 > n + 1) return;
    ga = q;
    if (key_v(pk[q]) != key_v(pk[q + 1])) return;  // q ends its row
    const int l = (key_v(pk[q]) - g.lv0) / g.step;
    const int rho = rowRank[l];
    idx = q - (2 + rowStart[l]);
    below = rho + 1;
    above = rho;
  }
  const int sum = key_u(pk[ga]) + key_u(pk[ga + 1]);
  int kb = -1, ka = -1;
  if (below >= 0) {
    const BandRow B = band_lower(below, m, n, rowStart, rowNE);
    const int j = edges_below(pk, B, sum, true);
    const int k = stripOff[below] + idx + j;
    if (k < 0 || k + 1 > NT) {
      *err = 2;
    } else {
      tv[3 * k] = (I)ga;
      tv[3 * k + 1] = (I)(ga + 1);
      tv[3 * k + 2] = (I)(B.first + j);
      kb = k;
      // the next triangle of the band shares the diagonal (A[i+1], B[j])
      if (k + 1 < stripOff[below + 1]) {
        tn[3 * k] = (I)(4 * (k + 1) + 1);
        tn[3 * (k + 1) + 1] = (I)(4 * k);
      }
    }
  }
  if (above >= 0) {
    const BandRow A = band_upper(above, rowStart, rowNE);
    const int i = edges_below(pk, A, sum, false);
    const int k = stripOff[above] + i + idx;
    if (k < 0 || k + 1 > NT) {
      *err = 2;
    } else {
      tv[3 * k] = (I)(A.first + i);
      tv[3 * k + 1] = (I)(ga + 1);
      tv[3 * k + 2] = (I)ga;
      ka = k;
      // the next triangle of the band shares the diagonal (A[i], B[j+1])
      if (k + 1 < stripOff[above + 1]) {
        tn[3 * k + 2] = (I)(4 * (k + 1) + 1);
        tn[3 * (k + 1) + 1] = (I)(4 * k + 2);
      }
    }
  }
  // a row edge joins its two band triangles; the corner rows' edges are the
  // image's top and bottom sides
  if (kb >= 0 && ka >= 0) {
    tn[3 * kb + 2] = (I)(4 * ka);
    tn[3 * ka] = (I)(4 * kb + 2);
  } else if (kb >= 0 || ka >= 0) {
    if (kb >= 0) tn[3 * kb + 2] = (I)-1;
    if (ka >= 0) tn[3 * ka] = (I)-1;
    atomicAdd(border, 1);
  }
}

// Rank of key s in the sorted point keys (s is present).
__device__ __forceinline__ int rank_of(const uint32_t* pk, int np, uint32_t s) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pk[mid] < s)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// A view that fails leaves no triangles, so raster and dense run without a
// plane prior; the failure is recorded in the header and, when the frame has
// one, in its pinned host report word, which the host turns into an error.
template <typename I>
__device__ void mesh_fail(MeshHeader* hdr, int32_t* mfail, int view, int status) {
  if (threadIdx.x == 0) {
    hdr->status[view] = status;
    hdr->ntri[view] = 0;
    if (mfail) __hip_atomic_store(mfail, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// An empty asm that reads its operands: the loads that produce them are
// issued before it and waited for together there, instead of one by one in
// the branches that use them.
__device__ __forceinline__ void pin(int v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void pin(uint32_t v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void pin(unsigned long long v) { asm volatile("" ::"v"(v)); }

// Re-links outer edge k of triangle x, flipped in round r, and tests it for
// round r + 1 (one lane per edge: the three edges of x touch disjoint
// entries). An unflipped neighbour is pointed back at x; across a flipped
// one the edge now lies in that triangle or its partner. The entries any
// case may need are loaded up front from indices kept in range.
template <typename I>
__device__ __forceinline__ void relink_edge(int x, int k, int r, int NT, const uint32_t* tk,
                                            I* tn, const uint16_t* flipr, const I* partner,
                                            typename ClaimT<I>::T* claim, I* cl, int* count,
                                            int ncand, int* err) {
  const int px = partner[x];
  const uint32_t k0 = tk[3 * x], k1 = tk[3 * x + 1], k2 = tk[3 * x + 2];
  int e = tn[3 * x + k];
  if (e < 0) return;
  const uint32_t p = k == 0 ? k0 : (k == 1 ? k1 : k2);
  const uint32_t ea = k == 0 ? k1 : (k == 1 ? k2 : k0);
  const uint32_t eb = k == 0 ? k2 : (k == 1 ? k0 : k1);
  int z = e >> 2;
  const int fz = flipr[z];
  const int pz = min(max((int)partner[z], 0), NT - 1);
  uint32_t z0 = tk[3 * z], z1 = tk[3 * z + 1], z2 = tk[3 * z + 2];
  const uint32_t q0 = tk[3 * pz], q1 = tk[3 * pz + 1], q2 = tk[3 * pz + 2];
  int fo = fz;
  if (z != px) {
    if (fz != r) {
      tn[3 * z + (e & 3)] = (I)(4 * x + k);
    } else {
      const bool has_a = z0 == ea || z1 == ea || z2 == ea;
      const bool has_b = z0 == eb || z1 == eb || z2 == eb;
      if (!(has_a && has_b)) {
        z = pz;
        z0 = q0;
        z1 = q1;
        z2 = q2;
      }
      const int jj = (z0 != ea && z0 != eb) ? 0 : ((z1 != ea && z1 != eb) ? 1 : 2);
      e = 4 * z + jj;
      tn[3 * x + k] = (I)e;
      fo = r;
    }
  }
  // the triangle across is o = e >> 2 with keys z0..z2; an edge between two
  // triangles flipped in round r is tested by the one with the smaller index
  const int o = e >> 2, j = e & 3;
  if (o < x && fo == r) return;
  const uint32_t q = j == 0 ? z0 : (j == 1 ? z1 : z2);
  if (!edge_illegal(p, ea, eb, q)) return;
  const int key = x < o ? 4 * x + k : e;
  const typename ClaimT<I>::T st = claim_stamp<I>(r + 1, key);
  atomicMax(&claim[x], st);
  atomicMax(&claim[o], st);
  const int slot = atomicAdd(count, 1);
  if (slot < ncand)
    cl[slot] = (I)key;
  else
    *err = 2;
}

template <typename I>
__device__ __forceinline__ void mesh_run(char* base, const int32_t* __restrict__ rows,
                         const int32_t* __restrict__ cnt_view, int c_first, int n, int tri_base,
                         const Geometry& g, int dmin, MeshHeader* hdr, int32_t* mfail,
                         int max_rounds, int view, int32_t* out_pts, int32_t* out_recs,
                         float* out_planes, RasterTri* out_tris, MeshShared& sh) {
  typedef typename ClaimT<I>::T C;
  const int tid = threadIdx.x;
  MeshMem<I> M;
  carve<I>(base, n, g.lh, M);
  int32_t* const rowStart = M.rowStart;
  int32_t* const rowNE = M.rowNE;
  int32_t* const rowRank = M.rowRank;
  int32_t* const stripOff = M.stripOff;
  uint32_t* const chainK0 = M.chainK0;
  uint32_t* const chainK1 = M.chainK1;
  int32_t* const chainI0 = M.chainI0;
  int32_t* const chainI1 = M.chainI1;
  uint32_t* const pk = M.pk;
  uint32_t* const tk = M.tk;
  I* const tn = M.tn;
  I* const hbuck = M.hbuck;
  I* const tv = M.tv;
  int32_t* const vcnt = M.vcnt;
  int32_t* const vcur = M.vcur;
  C* const claim = M.claim;
  I* const partner = M.partner;
  uint16_t* const flipr = M.flipr;
  I* const lf0 = M.lf0;
  I* const lf1 = M.lf1;
  I* const cl0 = M.cl0;
  I* const cl1 = M.cl1;
  int32_t* const scnt = M.scnt;
  int32_t* const scur = M.scur;
  I* const slist = M.slist;
  int32_t* const smin = M.smin;
  const int NP = M.NP, NT = M.NT, ncand = M.ncand;

  // ---- 1. points in rank order, corners ----------------------------------
  // neighbours not known from the construction keep this mark until step 3
  for (int e = tid; e < 3 * NT; e += kMT) tn[e] = (I)kTwinUnknown;
  for (int l = tid; l < g.lh; l += kMT) rowStart[l] = l < kMT ? c_first : cnt_view[l];
  if (tid == 0) rowStart[g.lh] = 0;
  if (tid < 4) sh.corner[tid] = ~0ull;
  __syncthreads();
  scan_array(rowStart, g.lh + 1, sh.wsum);
  {
    const int cu[4] = {0, g.w - 1, 0, g.w - 1}, cv[4] = {0, 0, g.h - 1, g.h - 1};
    unsigned long long best[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    for (int k = tid; k < n; k += kMT) {
      // lattice row of point k: the last row starting at or before k
      int lo = 0, hi = g.lh - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rowStart[mid] <= k)
          lo = mid;
        else
          hi = mid - 1;
      }
      const int e = rows[(size_t)lo * g.lw + (k - rowStart[lo])];
      const int u = e & 0xFFFF, d = e >> 16, v = g.lv0 + lo * g.step;
      pk[2 + k] = make_key(u, v, d - dmin);
      out_pts[3 * k] = u;
      out_pts[3 * k + 1] = v;
      out_pts[3 * k + 2] = d;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const long long du = u - cu[c], dv = v - cv[c];
        const unsigned long long key =
            ((unsigned long long)(du * du + dv * dv) << 32) | (unsigned long long)(unsigned)k;
        best[c] = key < best[c] ? key : best[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const unsigned long long b = wave_min_u64(best[c]);
      if ((tid & 63) == 0) atomicMin(&sh.corner[c], b);
    }
  }
  // non-empty rows, in order
  int m = 0;
  for (int c0 = 0; c0 < g.lh; c0 += kMT) {
    const int l = c0 + tid;
    const int f = (l < g.lh && rowStart[l + 1] > rowStart[l]) ? 1 : 0;
    int tot;
    const int e = scan_excl(f, &tot, sh.wsum);
    if (f) {
      rowNE[m + e] = l;
      rowRank[l] = m + e;
    }
    m += tot;
  }
  if (tid < 4) {
    const int src = (int)(sh.corner[tid] & 0xFFFFFFFFull);
    const int dd = key_dd(pk[2 + src]);
    const int rank = tid < 2 ? tid : n + tid;  // ranks 0, 1, n+2, n+3
    const int cu = (tid & 1) ? g.w - 1 : 0, cv = tid < 2 ? 0 : g.h - 1;
    pk[rank] = make_key(cu, cv, dd);
    hdr->corners[4 * view + tid] = dd + dmin;
  }
  __syncthreads();
  for (int r = tid; r < m; r += kMT) {
    const int l = rowNE[r];
    const int i0 = 2 + rowStart[l], i1 = 1 + rowStart[l + 1];
    chainI0[r] = i0;
    chainI1[r] = i1;
    chainK0[r] = pk[i0];
    chainK1[r] = pk[i1];
  }
  // strips: s = 0 between the top corners and the first row, s = m between
  // the last row and the bottom corners
  for (int s = tid; s <= m; s += kMT) {
    const int ca = s == 0 ? 2 : rowStart[rowNE[s - 1] + 1] - rowStart[rowNE[s - 1]];
    const int cb = s == m ? 2 : rowStart[rowNE[s] + 1] - rowStart[rowNE[s]];
    stripOff[s] = ca + cb - 2;
  }
  if (tid == 0) stripOff[m + 1] = 0;
  __syncthreads();
  const int strip_tris = scan_array(stripOff, m + 2, sh.wsum);

  // ---- 2. initial triangulation: strips and both pockets concurrently ------
  // every thread takes its band edges (one lane per row edge and per corner
  // edge), then its share of the pockets (kPocketG lanes per chain point,
  // half of the workgroup per side); the two write disjoint triangles
  for (int q = tid; q < n + 2; q += kMT)
    strip_edge(q, pk, rowStart, rowNE, rowRank, stripOff, g, m, n, tv, tn, NT, &sh.err,
               &sh.border);
  {
    const int side = tid / (kMT / 2), lt = tid % (kMT / 2);
    const int groups = kMT / 2 / kPocketG;
    for (int k = 1 + lt / kPocketG; k <= m; k += groups)
      pocket_point<I, kPocketG>(pk, side == 0 ? chainK0 : chainK1,
                                side == 0 ? chainI0 : chainI1, tv, NT, side, k, m, n,
                                strip_tris + side * m, lt % kPocketG, &sh.err);
  }
  if (tid == 0 && strip_tris + 2 * m != NT) sh.err = 2;
  __syncthreads();
  if (sh.err) {
    mesh_fail<I>(hdr, mfail, view, 2);
    return;
  }

  // ---- 3. adjacency -------------------------------------------------------
  // every half-edge is bucketed by origin vertex. The bands set every twin
  // but their two side edges, whose twins are pocket half-edges; so the
  // pockets' half-edges (one contiguous range, all unmatched) are matched,
  // each also linking the band side it finds
  for (int v = tid; v <= NP; v += kMT) vcnt[v] = 0;
  __syncthreads();
  for (int e = tid; e < 3 * NT; e += kMT) {
    const int t = e / 3, k = e - 3 * t;
    atomicAdd(&vcnt[(int)tv[3 * t + (k == 2 ? 0 : k + 1)]], 1);
  }
  __syncthreads();
  scan_array(vcnt, NP + 1, sh.wsum);
  for (int v = tid; v <= NP; v += kMT) vcur[v] = vcnt[v];
  __syncthreads();
  for (int e = tid; e < 3 * NT; e += kMT) {
    const int t = e / 3, k = e - 3 * t;
    const int a = tv[3 * t + (k == 2 ? 0 : k + 1)];
    hbuck[atomicAdd(&vcur[a], 1)] = (I)e;
  }
  __syncthreads();
  for (int e = 3 * strip_tris + tid; e < 3 * NT; e += kMT) {
    // half-edge a -> b opposite vertex k; its twin runs b -> a. The twin's
    // triangle holds a half-edge leaving b (the twin) and one leaving a (the
    // one after the twin, whose opposite vertex is b), so the smaller of the
    // two buckets is searched: the corners' buckets are long.
    const int t = e / 3, k = e - 3 * t;
    const int a = tv[3 * t + (k == 2 ? 0 : k + 1)], b = tv[3 * t + (k == 0 ? 2 : k - 1)];
    // with any list point, the starting mesh joins two corners only along the
    // image sides (bands and pockets each hold a list point otherwise): those
    // are the border, whose search would run through two long buckets
    if (n > 0 && (a < 2 || a >= n + 2) && (b < 2 || b >= n + 2)) {
      tn[e] = (I)-1;
      atomicAdd(&sh.border, 1);
      continue;
    }
    const int sa = vcnt[a], sa1 = vcnt[a + 1], sb = vcnt[b], sb1 = vcnt[b + 1];
    const bool from_b = sb1 - sb <= sa1 - sa;
    const int want = from_b ? a : b;
    int nb = -1;
    for (int s = from_b ? sb : sa, s1 = from_b ? sb1 : sa1; s < s1; ++s) {
      const int e2 = hbuck[s];
      const int t2 = e2 / 3, k2 = e2 - 3 * t2;
      // from b: the end of b -> x; from a: the vertex before a in a -> x
      const int probe = from_b ? (k2 == 0 ? 2 : k2 - 1) : k2;
      if ((int)tv[3 * t2 + probe] == want) {
        nb = 4 * t2 + (from_b ? k2 : (k2 == 0 ? 2 : k2 - 1));
        break;
      }
    }
    tn[e] = (I)nb;
    if (nb < 0)
      atomicAdd(&sh.border, 1);
    else if ((nb >> 2) < strip_tris)  // a band side: its only twin is this one
      tn[3 * (nb >> 2) + (nb & 3)] = (I)(4 * t + k);
  }
  __syncthreads();
  if (sh.border != 4) {  // only the four image sides lack a twin
    mesh_fail<I>(hdr, mfail, view, 2);
    return;
  }
  // vertex keys (over the buckets, which are no longer needed)
  for (int e = tid; e < 3 * NT; e += kMT) tk[e] = pk[(int)tv[e]];
  __syncthreads();
  // flip state (over the vertex ranks, which are no longer needed)
  for (int t = tid; t < NT; t += kMT) {
    claim[t] = C(0);
    flipr[t] = 0;
  }
  if (tid == 0) {
    sh.ncand[0] = sh.ncand[1] = 0;
    sh.nflip[0] = sh.nflip[1] = 0;
  }
  __syncthreads();

  // ---- 4. Lawson flips in synchronous rounds ------------------------------
  // round 1 tests every edge, from the triangle with the smaller index; the
  // three apexes across are loaded together
  for (int t = tid; t < NT; t += kMT) {
    const uint32_t kk[3] = {tk[3 * t], tk[3 * t + 1], tk[3 * t + 2]};
    int e[3];
    uint32_t q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) e[i] = tn[3 * t + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = tk[e[i] >= 0 ? 3 * (e[i] >> 2) + (e[i] & 3) : 3 * t];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (e[i] < 0) {
        if (e[i] == kTwinUnknown) sh.err = 2;  // left unmatched by the adjacency step
        continue;
      }
      const int o = e[i] >> 2;
      if (o < t || !edge_illegal(kk[i], kk[(i + 1) % 3], kk[(i + 2) % 3], q[i])) continue;
      const int key = 4 * t + i;
      const C st = claim_stamp<I>(1, key);
      atomicMax(&claim[t], st);
      atomicMax(&claim[o], st);
      const int slot = atomicAdd(&sh.ncand[1], 1);
      if (slot < ncand)
        cl1[slot] = (I)key;
      else
        sh.err = 2;
    }
  }
  __syncthreads();
  int nflips = 0;  // thread 0's count of the view's flips
  for (int r = 1;; ++r) {
    const int cur = r & 1, nxt = cur ^ 1;
    I* const lf_cur = cur ? lf1 : lf0;
    I* const cl_cur = cur ? cl1 : cl0;
    I* const cl_nxt = cur ? cl0 : cl1;
    const int nc = sh.ncand[cur];
    if (sh.err || (nc > 0 && r >= max_rounds)) {
      mesh_fail<I>(hdr, mfail, view, sh.err ? sh.err : 1);
      return;
    }
    if (nc == 0) {
      if (tid == 0) {
        hdr->rounds[view] = r - 1;
        hdr->flips[view] = nflips;
      }
      break;
    }
    if (tid == 0) sh.ncand[nxt] = 0;  // appended to only after the next barrier
    // winners flip: (p, a, b) + (q, b, a) -> (p, a, q) + (p, q, b). Both
    // triangles' entries are loaded before the claims are compared, from
    // indices kept in range, so one wait covers them; they are used only by
    // the winner, which alone writes them in this phase.
    for (int idx = tid; idx < nc; idx += kMT) {
      const int key = cl_cur[idx];
      const int t = key >> 2, i = key & 3;
      const C st = claim_stamp<I>(r, key);
      const C ct = claim[t];
      const uint32_t t0 = tk[3 * t], t1 = tk[3 * t + 1], t2 = tk[3 * t + 2];
      const I n0 = tn[3 * t], n1 = tn[3 * t + 1], n2 = tn[3 * t + 2];
      const int e = i == 0 ? (int)n0 : (i == 1 ? (int)n1 : (int)n2);
      const int o = e < 0 ? t : e >> 2, j = e & 3;
      const int j1 = j == 2 ? 0 : j + 1, j2 = j == 0 ? 2 : j - 1;
      const C co = claim[o];
      const uint32_t q = tk[3 * o + j];
      const I o_aq = tn[3 * o + j1], o_qb = tn[3 * o + j2];
      pin(t0);
      pin(t1);
      pin(t2);
      pin((int)n0);
      pin((int)n1);
      pin((int)n2);
      pin(q);
      pin((int)o_aq);
      pin((int)o_qb);
      pin(co);
      if (ct != st || co != st) continue;
      const uint32_t p = i == 0 ? t0 : (i == 1 ? t1 : t2);
      const uint32_t a = i == 0 ? t1 : (i == 1 ? t2 : t0);
      const uint32_t b = i == 0 ? t2 : (i == 1 ? t0 : t1);
      const I t_bp = i == 0 ? n1 : (i == 1 ? n2 : n0);
      const I t_pa = i == 0 ? n2 : (i == 1 ? n0 : n1);
      tk[3 * t] = p;
      tk[3 * t + 1] = a;
      tk[3 * t + 2] = q;
      tn[3 * t] = o_aq;
      tn[3 * t + 1] = (I)(4 * o + 2);
      tn[3 * t + 2] = t_pa;
      tk[3 * o] = p;
      tk[3 * o + 1] = q;
      tk[3 * o + 2] = b;
      tn[3 * o] = o_qb;
      tn[3 * o + 1] = t_bp;
      tn[3 * o + 2] = (I)(4 * t + 1);
      flipr[t] = (uint16_t)r;
      flipr[o] = (uint16_t)r;
      partner[t] = (I)o;
      partner[o] = (I)t;
      const int slot = atomicAdd(&sh.nflip[cur], 2);
      lf_cur[slot] = (I)t;
      lf_cur[slot + 1] = (I)o;
    }
    __syncthreads();
    // Items [0, 3 nf): edge idx % 3 of flipped triangle idx / 3 is re-linked
    // and at once tested for round r + 1. Items [3 nf, 3 nf + nc): round r's
    // candidates whose two triangles did not flip carry over. Both kinds run
    // side by side on different threads.
    const int nf = sh.nflip[cur];
    nflips += nf >> 1;
    if (tid == 0) sh.nflip[nxt] = 0;  // appended to only after the next barrier
    for (int idx = tid; idx < 3 * nf + nc; idx += kMT) {
      if (idx < 3 * nf) {
        const int item = idx / 3;
        relink_edge<I>(lf_cur[item], idx - 3 * item, r, NT, tk, tn, flipr, partner, claim,
                       cl_nxt, &sh.ncand[nxt], ncand, &sh.err);
        continue;
      }
      const int key = cl_cur[idx - 3 * nf];
      const int t = key >> 2, i = key & 3;
      const int ft = flipr[t];
      const int o = (int)tn[3 * t + i] >> 2;
      const int fo = flipr[o];
      if ((ft == r) | (fo == r)) continue;
      const C st = claim_stamp<I>(r + 1, key);
      atomicMax(&claim[t], st);
      atomicMax(&claim[o], st);
      const int slot = atomicAdd(&sh.ncand[nxt], 1);
      if (slot < ncand)
        cl_nxt[slot] = (I)key;
      else
        sh.err = 2;
    }
    __syncthreads();
  }

  // ---- 5. canonical order, planes, raster records -------------------------
  for (int v = tid; v <= NP; v += kMT) scnt[v] = 0;
  __syncthreads();
  // the rank of each triangle's smallest vertex is searched once
  for (int t = tid; t < NT; t += kMT) {
    uint32_t s0 = tk[3 * t], s1 = tk[3 * t + 1], s2 = tk[3 * t + 2];
    sort3(s0, s1, s2);
    const int a = rank_of(pk, NP, s0);
    smin[t] = a;
    atomicAdd(&scnt[a], 1);
  }
  __syncthreads();
  scan_array(scnt, NP + 1, sh.wsum);
  for (int v = tid; v <= NP; v += kMT) scur[v] = scnt[v];
  __syncthreads();
  for (int t = tid; t < NT; t += kMT) slist[atomicAdd(&scur[smin[t]], 1)] = (I)t;
  __syncthreads();
  for (int t = tid; t < NT; t += kMT) {
    uint32_t s0 = tk[3 * t], s1 = tk[3 * t + 1], s2 = tk[3 * t + 2];
    sort3(s0, s1, s2);
    const int a = smin[t];
    // position: bucket start + triangles of the bucket with a smaller
    // (middle, largest) vertex pair
    int pos = scnt[a];
    for (int qq = scnt[a], q1 = scnt[a + 1]; qq < q1; ++qq) {
      const int t2 = slist[qq];
      if (t2 == t) continue;
      uint32_t r0 = tk[3 * t2], r1 = tk[3 * t2 + 1], r2 = tk[3 * t2 + 2];
      sort3(r0, r1, r2);
      pos += (r1 < s1 || (r1 == s1 && r2 < s2)) ? 1 : 0;
    }
    const uint32_t sv[3] = {s0, s1, s2};
    int32_t* rec = out_recs + 9 * (size_t)pos;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      rec[3 * q] = key_u(sv[q]);
      rec[3 * q + 1] = key_v(sv[q]);
      rec[3 * q + 2] = key_dd(sv[q]) + dmin;
    }
    // plane through the three points: exact Cramer numerators relative to the
    // first vertex, one correctly rounded double division each, then FP32
    const long long u1 = key_u(s0), v1 = key_v(s0), d1 = key_dd(s0) + dmin;
    const long long du2 = key_u(s1) - u1, dv2 = key_v(s1) - v1, dd2 = key_dd(s1) + dmin - d1;
    const long long du3 = key_u(s2) - u1, dv3 = key_v(s2) - v1, dd3 = key_dd(s2) + dmin - d1;
    const long long den = du2 * dv3 - du3 * dv2;
    const long long na = dd2 * dv3 - dd3 * dv2;
    const long long nb = du2 * dd3 - du3 * dd2;
    const long long nc = d1 * den - na * u1 - nb * v1;
    const float pa = (float)__ddiv_rn((double)na, (double)den);
    const float pb = (float)__ddiv_rn((double)nb, (double)den);
    const float pc = (float)__ddiv_rn((double)nc, (double)den);
    out_planes[3 * (size_t)pos] = pa;
    out_planes[3 * (size_t)pos + 1] = pb;
    out_planes[3 * (size_t)pos + 2] = pc;
    uint32_t o1 = s1, o2 = s2;
    if (orient_k(s0, s1, s2) < 0) {
      o1 = s2;
      o2 = s1;
    }
    RasterTri rt;
    rt.u[0] = (int16_t)key_u(s0);
    rt.v[0] = (int16_t)key_v(s0);
    rt.u[1] = (int16_t)key_u(o1);
    rt.v[1] = (int16_t)key_v(o1);
    rt.u[2] = (int16_t)key_u(o2);
    rt.v[2] = (int16_t)key_v(o2);
    rt.a = pa;
    rt.b = pb;
    rt.c = pc;
    out_tris[tri_base + pos] = rt;
  }
}

__device__ __forceinline__ void mesh_body(const Frame& F, int view) {
  extern __shared__ __align__(16) char smem[];
  __shared__ MeshShared sh;
  __shared__ int part[3][kMT / 64];
  const Geometry g = F.g;
  const int32_t* __restrict__ cnt = F.cnt;
  MeshHeader* hdr = F.hdr;
  const int tid = threadIdx.x;
  // point counts of both views and the support evaluations in one pass
  int x = 0, xl = 0, ev = 0, c_first = 0;
  for (int l = tid; l < g.lh; l += kMT) {
    const int cv = cnt[view * g.lh + l];
    if (l == tid) c_first = cv;
    x += cv;
    xl += cnt[l];
    ev += cnt[2 * g.lh + l];
  }
  const int lane = tid & 63, wid = tid >> 6;
  x = wave_sum_i32(x);
  xl = wave_sum_i32(xl);
  ev = wave_sum_i32(ev);
  if (lane == 0) {
    part[0][wid] = x;
    part[1][wid] = xl;
    part[2][wid] = ev;
  }
  if (tid == 0) {
    sh.err = 0;
    sh.border = 0;
  }
  __syncthreads();
  int n = 0, nL = 0, evals = 0;
#pragma unroll
  for (int w = 0; w < kMT / 64; ++w) {
    n += part[0][w];
    nL += part[1][w];
    evals += part[2][w];
  }
  if (tid == 0) {
    hdr->n[view] = n;
    hdr->ntri[view] = n > 0 ? 2 * n + 2 : 0;
    hdr->status[view] = 0;
    hdr->rounds[view] = 0;
    hdr->flips[view] = 0;
    if (view == 0) hdr->support_evals = evals;
    if (n == 0) {
      for (int c = 0; c < 4; ++c) hdr->corners[4 * view + c] = -1;
    }
  }
  if (n == 0) return;
  const int tri_base = view ? 2 * nL + 2 : 0;
  const int32_t* rows = view ? F.rowsR : F.rowsL;
  int32_t* pts = view ? F.ptsR : F.ptsL;
  int32_t* recs = view ? F.recsR : F.recsL;
  float* planes = view ? F.planesR : F.planesL;
  const int dmin = F.p.dmin;
  int32_t* const mfail = F.mfail;
  const int max_rounds = min(F.p.mesh_max_rounds, kMeshMaxRounds);
  MeshMem<int16_t> probe;
  if (2 * n + 2 < 8192 && carve<int16_t>(nullptr, n, g.lh, probe) <= (size_t)kMeshLdsBytes)
    mesh_run<int16_t>(smem, rows, cnt + view * g.lh, c_first, n, tri_base, g, dmin, hdr, mfail,
                      max_rounds, view, pts, recs, planes, F.tris, sh);
  else
    mesh_run<int32_t>(F.mesh_scratch + view * F.mesh_scratch_per_view, rows,
                      cnt + view * g.lh, c_first, n, tri_base, g, dmin, hdr, mfail, max_rounds,
                      view, pts, recs, planes, F.tris, sh);
}

__global__ __launch_bounds__(kMT) void k_mesh(Frame F) { mesh_body(F, blockIdx.x); }

__global__ __launch_bounds__(kMT) void k_mesh_batch(const Frame* __restrict__ frames, int nf) {
  const int f = blockIdx.x >> 1;
  if (f >= nf) return;
  const Frame F = global_frame(frames[f], reinterpret_cast<const char*>(frames));
  mesh_body(F, blockIdx.x & 1);
}

}  // namespace

size_t mesh_global_scratch_per_view(const Geometry& g) {
  const int nmax = std::max(1, g.lw * g.lh);
  MeshMem<int32_t> probe;
  return a16(carve<int32_t>(nullptr, nmax, g.lh, probe));
}

hipError_t launch_mesh_frame(const Frame& f, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  if (f.g.w > kDeviceMeshMaxSide || f.g.h > kDeviceMeshMaxSide) return hipErrorInvalidValue;
  if (start || stop)
    hipExtLaunchKernelGGL(k_mesh, dim3(2), dim3(kMT), kMeshLdsBytes, s, start, stop, 0u, f);
  else
    hipLaunchKernelGGL(k_mesh, dim3(2), dim3(kMT), kMeshLdsBytes, s, f);
  return hipGetLastError();
}

hipError_t launch_mesh_batch(const Frame* frames, int32_t nf, hipStream_t s, hipEvent_t start,
                             hipEvent_t stop) {
  if (nf <= 0) return hipSuccess;
  if (start || stop)
    hipExtLaunchKernelGGL(k_mesh_batch, dim3(2 * nf), dim3(kMT), kMeshLdsBytes, s, start, stop,
                          0u, frames, nf);
  else
    hipLaunchKernelGGL(k_mesh_batch, dim3(2 * nf), dim3(kMT), kMeshLdsBytes, s, frames, nf);
  return hipGetLastError();
}

}  // namespace elas

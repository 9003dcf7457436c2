// Device-resident mesh step (Section III-A: Delaunay triangulation of the
// support points, one slanted plane per triangle; Section IV leaves this
// sequential step on the CPU, here it runs on the GPU so the frame needs no
// host round trip).
//
// One 1024-thread workgroup per view:
//  1. gather the per-row support lists into points ranked in (v, u) order:
//     index 0 = (0,0), 1 = (w-1,0), 2..n+1 = the list, n+2 = (0,h-1),
//     n+3 = (w-1,h-1); the corners take the d of the nearest list point;
//  2. initial triangulation: the support points lie on lattice rows, so the
//     region between two consecutive non-empty rows (with the image's top and
//     bottom edges as extra rows) is a trapezoid, triangulated by a zipper
//     over the two sorted rows (one thread per strip); the two side pockets
//     between the rows' end points and the image border are v-monotone
//     polygons, triangulated by the stack method (one thread per side);
//  3. adjacency from vertex-to-triangle incidence lists;
//  4. Lawson flips in synchronous rounds until every edge is legal under the
//     canonical rule (strictly outside the circumcircle, or exactly on it and
//     the (v, u)-smallest of the four points is an endpoint of the edge):
//     each illegal edge claims its two triangles (atomicMin of the edge key),
//     winners flip from the round's state, then every triangle re-points the
//     neighbours it had across edges that moved to the flip partner. Only
//     edges of triangles changed in the previous round are re-tested. The
//     canonical rule is a consistent symbolic perturbation of the lifted
//     points, so the flips terminate at the unique canonical triangulation,
//     whatever the starting mesh;
//  5. canonical order (counting sort on the smallest vertex rank, insertion
//     sort inside each bucket), exact planes, raster records.
// Arrays live in LDS (16-bit indices) when they fit, else in a global
// scratch area (32-bit indices); both paths run the same template.
#include <algorithm>
#include <climits>

#include "elas_internal.h"

namespace elas {
namespace {

constexpr int kMT = 1024;  // threads per mesh workgroup

__device__ __forceinline__ long long orient2(int au, int av, int bu, int bv, int cu, int cv) {
  return (long long)(bu - au) * (cv - av) - (long long)(bv - av) * (cu - au);
}

__device__ __forceinline__ long long incircle2(int au, int av, int bu, int bv, int cu, int cv,
                                               int du, int dv) {
  const long long ax = au - du, ay = av - dv, bx = bu - du, by = bv - dv;
  const long long cx = cu - du, cy = cv - dv;
  return (ax * ax + ay * ay) * (bx * cy - by * cx) + (bx * bx + by * by) * (cx * ay - cy * ax) +
         (cx * cx + cy * cy) * (ax * by - ay * bx);
}

// Exclusive scan over the workgroup (kMT threads); *total receives the sum.
__device__ int scan_excl(int x, int* total, int* wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
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

// In-place exclusive scan of a[0..n) (int32); returns the total.
__device__ int scan_array(int* a, int n, int* wsum) {
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

__device__ int block_sum(int x, int* wsum) {
  int tot;
  (void)scan_excl(x, &tot, wsum);
  return tot;
}

template <typename I>
struct MeshMem {
  int16_t *pu, *pv, *pd;   // NP points in rank order
  I* tv;                   // 3*NT vertex ids, positive orientation
  I* tn;                   // 3*NT neighbour across the edge opposite vertex k (-1: border)
  int32_t* claim;          // NT
  I* partner;              // NT flip partner of the current round (-1: none)
  uint8_t* cand;           // NT candidate-edge bits of the current round
  uint8_t* dirty;          // NT changed in the previous round
  int32_t* cnt;            // NP+1 slot starts (incidence lists, sort buckets)
  int32_t* cur;            // NP+1 fill cursors
  I* inc;                  // 3*NT incidence lists, then the canonical order
  int32_t* rowStart;       // lh+1
  int32_t* rowNE;          // lh   non-empty lattice rows
  int32_t* stripOff;       // lh+2
  int32_t* stack;          // 2*(lh+2)
  int NT;                  // triangle count 2n + 2
  int* overflow;           // set if construction would write past NT
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

template <typename I>
__host__ __device__ inline size_t mesh_bytes(int n, int lh) {
  const size_t NP = (size_t)n + 4, NT = 2 * (size_t)n + 2, L = (size_t)lh;
  return 3 * align16(NP * 2) + 2 * align16(3 * NT * sizeof(I)) + align16(NT * 4) +
         align16(NT * sizeof(I)) + 2 * align16(NT) + 2 * align16((NP + 1) * 4) +
         align16(3 * NT * sizeof(I)) + align16((L + 1) * 4) + align16(L * 4 + 4) +
         align16((L + 2) * 4) + align16(2 * (L + 2) * 4);
}

template <typename I>
__device__ MeshMem<I> carve(char* base, int n, int lh) {
  const size_t NP = (size_t)n + 4, NT = 2 * (size_t)n + 2, L = (size_t)lh;
  MeshMem<I> m;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base + o;
    o += align16(bytes);
    return p;
  };
  m.pu = reinterpret_cast<int16_t*>(take(NP * 2));
  m.pv = reinterpret_cast<int16_t*>(take(NP * 2));
  m.pd = reinterpret_cast<int16_t*>(take(NP * 2));
  m.tv = reinterpret_cast<I*>(take(3 * NT * sizeof(I)));
  m.tn = reinterpret_cast<I*>(take(3 * NT * sizeof(I)));
  m.claim = reinterpret_cast<int32_t*>(take(NT * 4));
  m.partner = reinterpret_cast<I*>(take(NT * sizeof(I)));
  m.cand = reinterpret_cast<uint8_t*>(take(NT));
  m.dirty = reinterpret_cast<uint8_t*>(take(NT));
  m.cnt = reinterpret_cast<int32_t*>(take((NP + 1) * 4));
  m.cur = reinterpret_cast<int32_t*>(take((NP + 1) * 4));
  m.inc = reinterpret_cast<I*>(take(3 * NT * sizeof(I)));
  m.rowStart = reinterpret_cast<int32_t*>(take((L + 1) * 4));
  m.rowNE = reinterpret_cast<int32_t*>(take(L * 4 + 4));
  m.stripOff = reinterpret_cast<int32_t*>(take((L + 2) * 4));
  m.stack = reinterpret_cast<int32_t*>(take(2 * (L + 2) * 4));
  return m;
}

template <typename I>
__device__ __forceinline__ void put_tri(MeshMem<I>& M, int k, int a, int b, int c) {
  if (k < 0 || k >= M.NT) {
    *M.overflow = 1;
    return;
  }
  if (orient2(M.pu[a], M.pv[a], M.pu[b], M.pv[b], M.pu[c], M.pv[c]) < 0) {
    const int t = b;
    b = c;
    c = t;
  }
  M.tv[3 * k] = (I)a;
  M.tv[3 * k + 1] = (I)b;
  M.tv[3 * k + 2] = (I)c;
}

// Stack triangulation of one side pocket: the v-monotone polygon between the
// end points of the non-empty rows (top to bottom) and the image border from
// corner `top` to corner `bottom`. side < 0: left pocket (rows' first
// points), side > 0: right pocket (last points). Emits exactly m triangles
// from index k.
template <typename I>
__device__ void pocket(MeshMem<I>& M, int m, int top, int bottom, int side, int* S, int k) {
  int L = 0;
  S[L++] = top;
  for (int r = 0; r < m; ++r) {
    const int l = M.rowNE[r];
    const int p = side < 0 ? 2 + M.rowStart[l] : 2 + M.rowStart[l + 1] - 1;
    while (L >= 2) {
      const int a = S[L - 2], b = S[L - 1];
      const long long o = orient2(M.pu[a], M.pv[a], M.pu[b], M.pv[b], M.pu[p], M.pv[p]);
      if ((side < 0 && o > 0) || (side > 0 && o < 0)) {
        put_tri(M, k++, a, b, p);
        --L;
      } else {
        break;
      }
    }
    S[L++] = p;
  }
  // the remaining chain is reflex as seen from the pocket: fan from the
  // bottom corner, except that chain points collinear with that corner at the
  // end of the chain are fanned from the last point before them
  int j = L - 1;
  while (j >= 1 && orient2(M.pu[S[j - 1]], M.pv[S[j - 1]], M.pu[S[j]], M.pv[S[j]], M.pu[bottom],
                           M.pv[bottom]) == 0)
    --j;
  for (int i = 0; i < j; ++i) put_tri(M, k++, S[i], S[i + 1], bottom);
  if (j < L - 1) {
    for (int i = j; i + 1 < L; ++i) put_tri(M, k++, S[j - 1], S[i], S[i + 1]);
    put_tri(M, k++, S[j - 1], S[L - 1], bottom);
  }
}

template <typename I>
__device__ __forceinline__ bool has_vertex(const MeshMem<I>& M, int t, int v) {
  return (int)M.tv[3 * t] == v || (int)M.tv[3 * t + 1] == v || (int)M.tv[3 * t + 2] == v;
}

template <typename I>
__device__ __forceinline__ int back_index(const MeshMem<I>& M, int o, int t) {
  return (int)M.tn[3 * o] == t ? 0 : ((int)M.tn[3 * o + 1] == t ? 1 : 2);
}

// Edge i of triangle t (apex p) against neighbour o (apex q at index j).
template <typename I>
__device__ bool edge_illegal(const MeshMem<I>& M, int t, int i, int o, int j) {
  const int p = M.tv[3 * t + i], a = M.tv[3 * t + (i + 1) % 3], b = M.tv[3 * t + (i + 2) % 3];
  const int q = M.tv[3 * o + j];
  const long long ic = incircle2(M.pu[p], M.pv[p], M.pu[a], M.pv[a], M.pu[b], M.pv[b], M.pu[q],
                                 M.pv[q]);
  if (ic != 0) return ic > 0;
  // co-circular: indices are ranks in (v, u) order, so the smallest index is
  // the (v, u)-smallest point; the edge is legal iff it is an endpoint
  const int mn = min(min(p, q), min(a, b));
  return !(mn == a || mn == b);
}

__device__ __forceinline__ void sort3(int& a, int& b, int& c) {
  if (a > b) { const int t = a; a = b; b = t; }
  if (b > c) { const int t = b; b = c; c = t; }
  if (a > b) { const int t = a; a = b; b = t; }
}

template <typename I>
__device__ void mesh_run(char* base, const int32_t* __restrict__ rows,
                         const int32_t* __restrict__ cnt_view, int n, int tri_base,
                         const Geometry& g, MeshHeader* hdr, int view, int32_t* out_pts,
                         int32_t* out_recs, float* out_planes, RasterTri* out_tris, int* wsum,
                         unsigned long long* s_corner, int* s_flag) {
  const int tid = threadIdx.x;
  const int NP = n + 4, NT = 2 * n + 2;
  MeshMem<I> M = carve<I>(base, n, g.lh);
  M.NT = NT;
  M.overflow = s_flag;
  if (tid == 0) *s_flag = 0;

  // ---- 1. points in rank order, corners --------------------------------
  for (int l = tid; l < g.lh; l += kMT) M.rowStart[l] = cnt_view[l];
  if (tid == 0) M.rowStart[g.lh] = 0;
  if (tid < 4) s_corner[tid] = ~0ull;
  __syncthreads();
  scan_array(M.rowStart, g.lh + 1, wsum);
  for (int l = tid; l < g.lh; l += kMT) {
    const int s0 = M.rowStart[l], c = M.rowStart[l + 1] - s0;
    const int v = g.lv0 + l * g.step;
    for (int j = 0; j < c; ++j) {
      const int e = rows[(size_t)l * g.lw + j];
      const int idx = 2 + s0 + j;
      M.pu[idx] = (int16_t)(e & 0xFFFF);
      M.pv[idx] = (int16_t)v;
      M.pd[idx] = (int16_t)(e >> 16);
      out_pts[3 * (s0 + j)] = e & 0xFFFF;
      out_pts[3 * (s0 + j) + 1] = v;
      out_pts[3 * (s0 + j) + 2] = e >> 16;
    }
  }
  if (tid == 0) {
    M.pu[0] = 0;
    M.pv[0] = 0;
    M.pu[1] = (int16_t)(g.w - 1);
    M.pv[1] = 0;
    M.pu[n + 2] = 0;
    M.pv[n + 2] = (int16_t)(g.h - 1);
    M.pu[n + 3] = (int16_t)(g.w - 1);
    M.pv[n + 3] = (int16_t)(g.h - 1);
  }
  __syncthreads();
  {
    const int cu[4] = {0, g.w - 1, 0, g.w - 1}, cvv[4] = {0, 0, g.h - 1, g.h - 1};
    unsigned long long best[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    for (int i = tid; i < n; i += kMT) {
      const int u = M.pu[2 + i], v = M.pv[2 + i];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const long long du = u - cu[c], dv = v - cvv[c];
        const unsigned long long key =
            ((unsigned long long)(du * du + dv * dv) << 32) | (unsigned long long)(unsigned)i;
        best[c] = key < best[c] ? key : best[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      unsigned long long b = best[c];
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(b, off, 64);
        b = o < b ? o : b;
      }
      if ((tid & 63) == 0) atomicMin(&s_corner[c], b);
    }
  }
  // non-empty rows, in order
  int m = 0;
  for (int c0 = 0; c0 < g.lh; c0 += kMT) {
    const int l = c0 + tid;
    const int f = (l < g.lh && M.rowStart[l + 1] > M.rowStart[l]) ? 1 : 0;
    int tot;
    const int e = scan_excl(f, &tot, wsum);
    if (f) M.rowNE[m + e] = l;
    m += tot;
  }
  if (tid < 4) {
    const int src = 2 + (int)(s_corner[tid] & 0xFFFFFFFFull);
    const int ci = tid < 2 ? tid : n + tid;  // corner ranks 0, 1, n+2, n+3
    M.pd[ci] = M.pd[src];
    hdr->corners[4 * view + tid] = M.pd[src];
  }
  __syncthreads();

  // ---- 2. initial triangulation ------------------------------------------
  // rows r = 0 (top edge: ranks 0, 1), 1..m (non-empty lattice rows),
  // m + 1 (bottom edge: ranks n+2, n+3); ranks inside a row are contiguous
  for (int s = tid; s <= m; s += kMT) {
    const int ca = s == 0 ? 2 : M.rowStart[M.rowNE[s - 1] + 1] - M.rowStart[M.rowNE[s - 1]];
    const int cb = s == m ? 2 : M.rowStart[M.rowNE[s] + 1] - M.rowStart[M.rowNE[s]];
    M.stripOff[s] = ca + cb - 2;
  }
  if (tid == 0) M.stripOff[m + 1] = 0;
  __syncthreads();
  const int strip_tris = scan_array(M.stripOff, m + 2, wsum);
  for (int s = tid; s <= m; s += kMT) {
    const int fa = s == 0 ? 0 : 2 + M.rowStart[M.rowNE[s - 1]];
    const int ca = s == 0 ? 2 : M.rowStart[M.rowNE[s - 1] + 1] - M.rowStart[M.rowNE[s - 1]];
    const int fb = s == m ? n + 2 : 2 + M.rowStart[M.rowNE[s]];
    const int cb = s == m ? 2 : M.rowStart[M.rowNE[s] + 1] - M.rowStart[M.rowNE[s]];
    int i = 0, j = 0, k = M.stripOff[s];
    while (i + 1 < ca || j + 1 < cb) {
      bool adv_i;
      if (i + 1 >= ca) {
        adv_i = false;
      } else if (j + 1 >= cb) {
        adv_i = true;
      } else {
        const int a0 = fa + i, a1 = fa + i + 1, b0 = fb + j, b1 = fb + j + 1;
        adv_i = !(incircle2(M.pu[a0], M.pv[a0], M.pu[a1], M.pv[a1], M.pu[b0], M.pv[b0], M.pu[b1],
                            M.pv[b1]) > 0);
      }
      // the upper row is above the lower one and both are sorted by u, so
      // these vertex orders are positively oriented
      if (k >= NT) {
        *s_flag = 1;
        break;
      }
      if (adv_i) {
        M.tv[3 * k] = (I)(fa + i);
        M.tv[3 * k + 1] = (I)(fa + i + 1);
        M.tv[3 * k + 2] = (I)(fb + j);
        ++i;
      } else {
        M.tv[3 * k] = (I)(fa + i);
        M.tv[3 * k + 1] = (I)(fb + j + 1);
        M.tv[3 * k + 2] = (I)(fb + j);
        ++j;
      }
      ++k;
    }
  }
  if (tid == 0) pocket(M, m, 0, n + 2, -1, M.stack, strip_tris);
  if (tid == 64) pocket(M, m, 1, n + 3, +1, M.stack + (g.lh + 2), strip_tris + m);
  __syncthreads();
  if (*s_flag) {  // cannot happen for valid lists; report, and leave no triangles
    if (tid == 0) {
      hdr->status[view] = 2;
      hdr->ntri[view] = 0;
    }
    return;
  }
  __syncthreads();

  // ---- 3. adjacency through vertex incidence lists ------------------------
  for (int v = tid; v <= NP; v += kMT) M.cnt[v] = 0;
  __syncthreads();
  for (int e = tid; e < 3 * NT; e += kMT) atomicAdd(&M.cnt[(int)M.tv[e]], 1);
  __syncthreads();
  scan_array(M.cnt, NP + 1, wsum);
  for (int v = tid; v <= NP; v += kMT) M.cur[v] = M.cnt[v];
  __syncthreads();
  for (int e = tid; e < 3 * NT; e += kMT) M.inc[atomicAdd(&M.cur[(int)M.tv[e]], 1)] = (I)(e / 3);
  __syncthreads();
  for (int e = tid; e < 3 * NT; e += kMT) {
    const int t = e / 3, k = e - 3 * t;
    const int a = M.tv[3 * t + (k + 1) % 3], b = M.tv[3 * t + (k + 2) % 3];
    int nb = -1;
    for (int s = M.cnt[b], s1 = M.cnt[b + 1]; s < s1; ++s) {
      const int x = M.inc[s];
      if (x != t && has_vertex(M, x, a)) {
        nb = x;
        break;
      }
    }
    M.tn[e] = (I)nb;
  }
  for (int t = tid; t < NT; t += kMT) {
    M.claim[t] = INT_MAX;
    M.partner[t] = (I)-1;
    M.cand[t] = 0;
    M.dirty[t] = 1;
  }
  __syncthreads();

  // ---- 4. Lawson flips in synchronous rounds ------------------------------
  int rounds = 0;
  const int max_rounds = 4 * NT + 64;
  for (;;) {
    if (tid == 0) *s_flag = 0;
    __syncthreads();
    for (int t = tid; t < NT; t += kMT) {
      M.partner[t] = (I)-1;
      uint8_t cb = 0;
      for (int i = 0; i < 3; ++i) {
        const int o = M.tn[3 * t + i];
        if (o <= t || (!M.dirty[t] && !M.dirty[o])) continue;
        if (edge_illegal(M, t, i, o, back_index(M, o, t))) {
          cb |= (uint8_t)(1u << i);
          const int key = 4 * t + i;
          atomicMin(&M.claim[t], key);
          atomicMin(&M.claim[o], key);
        }
      }
      M.cand[t] = cb;
      if (cb) *s_flag = 1;
    }
    __syncthreads();
    if (*s_flag == 0) break;
    if (++rounds > max_rounds) {
      if (tid == 0) hdr->status[view] = 1;
      break;
    }
    for (int t = tid; t < NT; t += kMT) {
      const uint8_t cb = M.cand[t];
      if (!cb) continue;
      for (int i = 0; i < 3; ++i) {
        if (!((cb >> i) & 1u)) continue;
        const int key = 4 * t + i;
        const int o = M.tn[3 * t + i];
        if (M.claim[t] != key || M.claim[o] != key) continue;
        const int j = back_index(M, o, t);
        const int p = M.tv[3 * t + i], a = M.tv[3 * t + (i + 1) % 3];
        const int b = M.tv[3 * t + (i + 2) % 3], q = M.tv[3 * o + j];
        const int t_bp = M.tn[3 * t + (i + 1) % 3], t_pa = M.tn[3 * t + (i + 2) % 3];
        const int o_aq = M.tn[3 * o + (j + 1) % 3], o_qb = M.tn[3 * o + (j + 2) % 3];
        M.tv[3 * t] = (I)p;
        M.tv[3 * t + 1] = (I)a;
        M.tv[3 * t + 2] = (I)q;
        M.tn[3 * t] = (I)o_aq;
        M.tn[3 * t + 1] = (I)o;
        M.tn[3 * t + 2] = (I)t_pa;
        M.tv[3 * o] = (I)p;
        M.tv[3 * o + 1] = (I)q;
        M.tv[3 * o + 2] = (I)b;
        M.tn[3 * o] = (I)o_qb;
        M.tn[3 * o + 1] = (I)t_bp;
        M.tn[3 * o + 2] = (I)t;
        M.partner[t] = (I)o;
        M.partner[o] = (I)t;
        break;
      }
    }
    __syncthreads();
    // neighbours across edges that moved to the flip partner
    for (int x = tid; x < NT; x += kMT) {
      for (int k = 0; k < 3; ++k) {
        const int y = M.tn[3 * x + k];
        if (y < 0 || (int)M.partner[y] < 0) continue;
        const int a = M.tv[3 * x + (k + 1) % 3], b = M.tv[3 * x + (k + 2) % 3];
        if (!(has_vertex(M, y, a) && has_vertex(M, y, b))) M.tn[3 * x + k] = M.partner[y];
      }
      M.dirty[x] = (int)M.partner[x] >= 0 ? 1 : 0;
      M.claim[x] = INT_MAX;
    }
    __syncthreads();
  }

  // ---- 5. canonical order, planes, raster records --------------------------
  for (int v = tid; v <= NP; v += kMT) M.cnt[v] = 0;
  __syncthreads();
  for (int t = tid; t < NT; t += kMT) {
    int a = M.tv[3 * t], b = M.tv[3 * t + 1], c = M.tv[3 * t + 2];
    sort3(a, b, c);
    atomicAdd(&M.cnt[a], 1);
  }
  __syncthreads();
  scan_array(M.cnt, NP + 1, wsum);
  for (int v = tid; v <= NP; v += kMT) M.cur[v] = M.cnt[v];
  __syncthreads();
  for (int t = tid; t < NT; t += kMT) {
    int a = M.tv[3 * t], b = M.tv[3 * t + 1], c = M.tv[3 * t + 2];
    sort3(a, b, c);
    M.inc[atomicAdd(&M.cur[a], 1)] = (I)t;
  }
  __syncthreads();
  for (int v = tid; v < NP; v += kMT) {
    const int s0 = M.cnt[v], s1 = M.cnt[v + 1];
    for (int x = s0 + 1; x < s1; ++x) {
      for (int y = x; y > s0; --y) {
        int a1 = M.tv[3 * (int)M.inc[y]], b1 = M.tv[3 * (int)M.inc[y] + 1],
            c1 = M.tv[3 * (int)M.inc[y] + 2];
        int a0 = M.tv[3 * (int)M.inc[y - 1]], b0 = M.tv[3 * (int)M.inc[y - 1] + 1],
            c0 = M.tv[3 * (int)M.inc[y - 1] + 2];
        sort3(a1, b1, c1);
        sort3(a0, b0, c0);
        if (b1 < b0 || (b1 == b0 && c1 < c0)) {
          const I tmp = M.inc[y];
          M.inc[y] = M.inc[y - 1];
          M.inc[y - 1] = tmp;
        } else {
          break;
        }
      }
    }
  }
  __syncthreads();
  for (int r = tid; r < NT; r += kMT) {
    const int t = M.inc[r];
    int i0 = M.tv[3 * t], i1 = M.tv[3 * t + 1], i2 = M.tv[3 * t + 2];
    sort3(i0, i1, i2);
    const int vid[3] = {i0, i1, i2};
    int32_t* rec = out_recs + 9 * (size_t)r;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      rec[3 * q] = M.pu[vid[q]];
      rec[3 * q + 1] = M.pv[vid[q]];
      rec[3 * q + 2] = M.pd[vid[q]];
    }
    // plane through the three points: exact Cramer numerators relative to the
    // first vertex, one correctly rounded double division each, then FP32
    const long long u1 = M.pu[i0], v1 = M.pv[i0], d1 = M.pd[i0];
    const long long du2 = M.pu[i1] - u1, dv2 = M.pv[i1] - v1, dd2 = M.pd[i1] - d1;
    const long long du3 = M.pu[i2] - u1, dv3 = M.pv[i2] - v1, dd3 = M.pd[i2] - d1;
    const long long den = du2 * dv3 - du3 * dv2;
    const long long na = dd2 * dv3 - dd3 * dv2;
    const long long nb = du2 * dd3 - du3 * dd2;
    const long long nc = d1 * den - na * u1 - nb * v1;
    const float pa = (float)__ddiv_rn((double)na, (double)den);
    const float pb = (float)__ddiv_rn((double)nb, (double)den);
    const float pc = (float)__ddiv_rn((double)nc, (double)den);
    out_planes[3 * (size_t)r] = pa;
    out_planes[3 * (size_t)r + 1] = pb;
    out_planes[3 * (size_t)r + 2] = pc;
    int o1 = i1, o2 = i2;
    if (orient2(M.pu[i0], M.pv[i0], M.pu[i1], M.pv[i1], M.pu[i2], M.pv[i2]) < 0) {
      o1 = i2;
      o2 = i1;
    }
    RasterTri rt;
    rt.u[0] = M.pu[i0];
    rt.v[0] = M.pv[i0];
    rt.u[1] = M.pu[o1];
    rt.v[1] = M.pv[o1];
    rt.u[2] = M.pu[o2];
    rt.v[2] = M.pv[o2];
    rt.a = pa;
    rt.b = pb;
    rt.c = pc;
    out_tris[tri_base + r] = rt;
  }
}

__global__ __launch_bounds__(kMT) void k_mesh(const int32_t* __restrict__ rowsL,
                                              const int32_t* __restrict__ rowsR,
                                              const int32_t* __restrict__ cnt, Geometry g,
                                              MeshHeader* hdr, int32_t* ptsL, int32_t* ptsR,
                                              int32_t* recsL, int32_t* recsR, float* planesL,
                                              float* planesR, RasterTri* tris, char* gscratch,
                                              size_t gscratch_per_view, int lds_bytes) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int wsum[kMT / 64];
  __shared__ unsigned long long s_corner[4];
  __shared__ int s_flag;
  const int view = blockIdx.x;
  const int tid = threadIdx.x;
  int x = 0, xl = 0, ev = 0;
  for (int l = tid; l < g.lh; l += kMT) {
    x += cnt[view * g.lh + l];
    xl += cnt[l];
    ev += cnt[2 * g.lh + l];
  }
  const int n = block_sum(x, wsum);
  const int nL = block_sum(xl, wsum);
  const int evals = block_sum(ev, wsum);
  if (tid == 0) {
    hdr->n[view] = n;
    hdr->ntri[view] = n > 0 ? 2 * n + 2 : 0;
    hdr->status[view] = 0;
    if (view == 0) hdr->support_evals = evals;
    if (n == 0)
      for (int c = 0; c < 4; ++c) hdr->corners[4 * view + c] = -1;
  }
  if (n == 0) return;
  const int tri_base = view ? 2 * nL + 2 : 0;
  const int32_t* rows = view ? rowsR : rowsL;
  int32_t* pts = view ? ptsR : ptsL;
  int32_t* recs = view ? recsR : recsL;
  float* planes = view ? planesR : planesL;
  if (2 * n + 2 <= 32767 && mesh_bytes<int16_t>(n, g.lh) <= (size_t)lds_bytes)
    mesh_run<int16_t>(smem, rows, cnt + view * g.lh, n, tri_base, g, hdr, view, pts, recs,
                      planes, tris, wsum, s_corner, &s_flag);
  else
    mesh_run<int32_t>(gscratch + view * gscratch_per_view, rows, cnt + view * g.lh, n, tri_base,
                      g, hdr, view, pts, recs, planes, tris, wsum, s_corner, &s_flag);
}

}  // namespace

size_t mesh_global_scratch_per_view(const Geometry& g) {
  const int nmax = std::max(1, g.lw * g.lh);
  return align16(mesh_bytes<int32_t>(nmax, g.lh));
}

hipError_t launch_mesh(const int32_t* rowsL, const int32_t* rowsR, const int32_t* cnt,
                       const Geometry& g, MeshHeader* hdr, int32_t* ptsL, int32_t* ptsR,
                       int32_t* recsL, int32_t* recsR, float* planesL, float* planesR,
                       RasterTri* tris, char* gscratch, hipStream_t s) {
  const int lds = kMeshLdsBytes;
  hipLaunchKernelGGL(k_mesh, dim3(2), dim3(kMT), lds, s, rowsL, rowsR, cnt, g, hdr, ptsL, ptsR,
                     recsL, recsR, planesL, planesR, tris, gscratch,
                     mesh_global_scratch_per_view(g), lds);
  return hipGetLastError();
}

}  // namespace elas

// HIP kernels of the ELAS hot path for gfx950 (MI355X).
//
// Data layout in HBM, per image size (one handle, one size):
//   images       uint8  [h][stride]            caller-owned
//   descriptors  uint8  [h][w][16]             one 16-byte descriptor per pixel
//   lattice      int16  [lh][lw]               support disparity per candidate
//   grid masks   uint32 [gh][gw][ceil(D/32)]   one-hot grid vectors
//   owner        int32  [h][w]                 owning triangle rank
//   maps         int16  [h][w]                 prior, raw and final disparities
// All matching arithmetic is integer; byte SADs use v_sad_u8 (four absolute
// byte differences accumulated per instruction). Minima over disparities use
// packed keys (energy << 8 | d - dmin), so any evaluation order gives the
// smallest energy with the smallest disparity on ties.
#include "elas_internal.h"

namespace elas {
namespace {

__device__ __forceinline__ uint4 ld16(const uint8_t* p) {
  return *reinterpret_cast<const uint4*>(p);
}

__device__ __forceinline__ uint32_t sad16(const uint4 a, const uint4 b) {
  uint32_t s = __builtin_amdgcn_sad_u8(a.x, b.x, 0u);
  s = __builtin_amdgcn_sad_u8(a.y, b.y, s);
  s = __builtin_amdgcn_sad_u8(a.z, b.z, s);
  return __builtin_amdgcn_sad_u8(a.w, b.w, s);
}

// Texture: distance of a descriptor from the flat descriptor (all bytes 128).
__device__ __forceinline__ uint32_t texture16(const uint4 a) {
  return sad16(a, make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u));
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, off, 64));
  return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Gradient quantisation: divide by 4 truncating toward zero, clamp to
// [-127, 127], offset by 128 (bytes 1..255; a negated gradient maps b to 256-b).
__device__ __forceinline__ uint32_t quantise(int g) {
  int q = g / 4;
  q = q > 127 ? 127 : (q < -127 ? -127 : q);
  return (uint32_t)(128 + q);
}

// ---------------------------------------------------------------------------
// Stage 1: 3x3 Sobel gradients and the 16-byte descriptor (Section III-A,
// Fig. 1(b); Section VI-A: a 16-byte subset of the window's gradients).
// Block = 64 x 4 pixels. The image tile with a 3-pixel halo is staged in LDS,
// the quantised gradients of the tile with a 2-pixel halo are computed once
// into LDS, and each thread gathers its 16 bytes and writes one 16-byte
// store (a wave writes 1 KiB contiguous). Also resets the pixel's owner.
// Sample pattern (column, row offsets): du at (-2,0) (-1,0) (1,0) (2,0)
// (-1,-2) (1,-2) (-1,2) (1,2); dv at (0,-2) (0,-1) (0,1) (0,2) (-2,-1) (2,-1)
// (-2,1) (2,1). Descriptors are defined for 2 <= u <= w-3, 2 <= v <= h-3 and
// all-zero elsewhere.
// ---------------------------------------------------------------------------
constexpr int kDescW = 64, kDescH = 4;

__global__ __launch_bounds__(256) void k_descriptor(const uint8_t* __restrict__ left,
                                                    const uint8_t* __restrict__ right,
                                                    int32_t stride, Geometry g,
                                                    uint8_t* __restrict__ descL,
                                                    uint8_t* __restrict__ descR,
                                                    int32_t* __restrict__ ownerL,
                                                    int32_t* __restrict__ ownerR) {
  const uint8_t* img = blockIdx.z ? right : left;
  uint8_t* desc = blockIdx.z ? descR : descL;
  int32_t* owner = blockIdx.z ? ownerR : ownerL;
  __shared__ uint8_t tile[kDescH + 6][kDescW + 8];
  __shared__ uint8_t qdu[kDescH + 4][kDescW + 4];
  __shared__ uint8_t qdv[kDescH + 4][kDescW + 4];
  const int u0 = blockIdx.x * kDescW, v0 = blockIdx.y * kDescH;
  const int tid = threadIdx.y * kDescW + threadIdx.x;
  for (int i = tid; i < (kDescH + 6) * (kDescW + 6); i += 256) {
    const int r = i / (kDescW + 6), c = i - r * (kDescW + 6);
    const int y = v0 - 3 + r, x = u0 - 3 + c;
    tile[r][c] = (x >= 0 && x < g.w && y >= 0 && y < g.h) ? img[(size_t)y * stride + x] : 0;
  }
  __syncthreads();
  for (int i = tid; i < (kDescH + 4) * (kDescW + 4); i += 256) {
    const int r = i / (kDescW + 4), c = i - r * (kDescW + 4);
    const int y = v0 - 2 + r, x = u0 - 2 + c;
    int gx = 0, gy = 0;
    if (x >= 1 && x <= g.w - 2 && y >= 1 && y <= g.h - 2) {
      const int tr = r + 1, tc = c + 1;  // (x, y) in tile coordinates
      const int a = tile[tr - 1][tc - 1], b = tile[tr - 1][tc], cc = tile[tr - 1][tc + 1];
      const int l = tile[tr][tc - 1], rr = tile[tr][tc + 1];
      const int d = tile[tr + 1][tc - 1], e = tile[tr + 1][tc], f = tile[tr + 1][tc + 1];
      gx = (cc + 2 * rr + f) - (a + 2 * l + d);
      gy = (d + 2 * e + f) - (a + 2 * b + cc);
    }
    qdu[r][c] = (uint8_t)quantise(gx);
    qdv[r][c] = (uint8_t)quantise(gy);
  }
  __syncthreads();
  const int u = u0 + threadIdx.x, v = v0 + threadIdx.y;
  if (u >= g.w || v >= g.h) return;
  uint4 out = make_uint4(0u, 0u, 0u, 0u);
  if (u >= 2 && u <= g.w - 3 && v >= 2 && v <= g.h - 3) {
    const int r = threadIdx.y + 2, c = threadIdx.x + 2;
    out.x = qdu[r][c - 2] | (qdu[r][c - 1] << 8) | (qdu[r][c + 1] << 16) |
            ((uint32_t)qdu[r][c + 2] << 24);
    out.y = qdu[r - 2][c - 1] | (qdu[r - 2][c + 1] << 8) | (qdu[r + 2][c - 1] << 16) |
            ((uint32_t)qdu[r + 2][c + 1] << 24);
    out.z = qdv[r - 2][c] | (qdv[r - 1][c] << 8) | (qdv[r + 1][c] << 16) |
            ((uint32_t)qdv[r + 2][c] << 24);
    out.w = qdv[r - 1][c - 2] | (qdv[r - 1][c + 2] << 8) | (qdv[r + 1][c - 2] << 16) |
            ((uint32_t)qdv[r + 1][c + 2] << 24);
  }
  const size_t px = (size_t)v * g.w + u;
  *reinterpret_cast<uint4*>(desc + px * 16) = out;
  owner[px] = kNoOwner;
}

// ---------------------------------------------------------------------------
// Stage 2: support matching (Section III-A; ambiguity test of Section VI-B,
// eq. 1-2) with a reverse check. One wavefront per lattice point; lane k
// evaluates d = dmin + k + 64 j. The 512-bit support descriptor is the four
// 16-byte descriptors at (u-2, v-2), (u+2, v-2), (u-2, v+2), (u+2, v+2).
// ---------------------------------------------------------------------------
struct Desc64 {
  uint4 q[4];
};

__device__ __forceinline__ Desc64 load_support(const uint8_t* desc, int w, int u, int v) {
  Desc64 r;
  r.q[0] = ld16(desc + ((size_t)(v - 2) * w + (u - 2)) * 16);
  r.q[1] = ld16(desc + ((size_t)(v - 2) * w + (u + 2)) * 16);
  r.q[2] = ld16(desc + ((size_t)(v + 2) * w + (u - 2)) * 16);
  r.q[3] = ld16(desc + ((size_t)(v + 2) * w + (u + 2)) * 16);
  return r;
}

__device__ __forceinline__ uint32_t sad64(const Desc64& a, const Desc64& b) {
  return sad16(a.q[0], b.q[0]) + sad16(a.q[1], b.q[1]) + sad16(a.q[2], b.q[2]) +
         sad16(a.q[3], b.q[3]);
}

__device__ __forceinline__ uint32_t texture64(const Desc64& a) {
  return texture16(a.q[0]) + texture16(a.q[1]) + texture16(a.q[2]) + texture16(a.q[3]);
}

// Full search of one point over d = dmin..dhi (at least two values); the
// partner column is u + dir*d. Returns whether the ratio test accepts and the
// best disparity. Control flow is wavefront-uniform.
__device__ bool support_search(const Desc64& self, const uint8_t* __restrict__ other, int w,
                               int u, int v, int dir, int dhi, const KParams& p, int lane,
                               int* d_best) {
  uint32_t cost[kMaxD / 64];
  uint32_t best = 0xFFFFFFFFu;
  const int nj = (dhi - p.dmin + 64) >> 6;
#pragma unroll
  for (int j = 0; j < kMaxD / 64; ++j) {
    cost[j] = 0xFFFFFFFFu;
    const int d = p.dmin + lane + 64 * j;
    if (j < nj && d <= dhi) {
      const uint32_t c = sad64(self, load_support(other, w, u + dir * d, v));
      cost[j] = c;
      best = min(best, (c << 8) | (uint32_t)(d - p.dmin));
    }
  }
  best = wave_min(best);
  const int d1 = p.dmin + (int)(best & 0xFFu);
  const uint32_t m1 = best >> 8;
  uint32_t m2 = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < kMaxD / 64; ++j) {
    const int d = p.dmin + lane + 64 * j;
    if (d != d1) m2 = min(m2, cost[j]);
  }
  m2 = wave_min(m2);
  *d_best = d1;
  return (float)m1 < __fmul_rn(p.support_threshold, (float)m2);
}

__global__ __launch_bounds__(256) void k_support(const uint8_t* __restrict__ descL,
                                                 const uint8_t* __restrict__ descR, Geometry g,
                                                 KParams p, int16_t* __restrict__ dcan,
                                                 int32_t* __restrict__ evals) {
  const int lane = threadIdx.x & 63;
  const int pt = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (pt >= g.lw * g.lh) return;
  const int l = pt / g.lw, k = pt - l * g.lw;
  const int u = g.lu0 + k * g.step, v = g.lv0 + l * g.step;
  int result = -1, ev = 0;
  const Desc64 ls = load_support(descL, g.w, u, v);
  if ((int)texture64(ls) >= p.support_texture) {
    const int dhi = min(p.dmax, u - 4);
    if (dhi - p.dmin + 1 >= 2) {
      ev += dhi - p.dmin + 1;
      int d1;
      if (support_search(ls, descR, g.w, u, v, -1, dhi, p, lane, &d1)) {
        const int ur = u - d1;
        const Desc64 rs = load_support(descR, g.w, ur, v);
        const int dhi2 = min(p.dmax, g.w - 5 - ur);
        if ((int)texture64(rs) >= p.support_texture && dhi2 - p.dmin + 1 >= 2) {
          ev += dhi2 - p.dmin + 1;
          int d2;
          if (support_search(rs, descL, g.w, ur, v, +1, dhi2, p, lane, &d2) &&
              abs(d2 - d1) <= p.lr_threshold)
            result = d1;
        }
      }
    }
  }
  if (lane == 0) {
    dcan[pt] = (int16_t)result;
    evals[pt] = ev;
  }
}

// ---------------------------------------------------------------------------
// Stage 3a: inconsistency filter (Section III-A, Fig. 1(e)). A point survives
// iff at least incon_min_support other points within +-incon_window lattice
// steps have |d' - d| <= incon_threshold. Reads only the unfiltered lattice.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_incon(const int16_t* __restrict__ in, Geometry g,
                                               KParams p, int16_t* __restrict__ out) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= g.lw * g.lh) return;
  const int l = idx / g.lw, k = idx - l * g.lw;
  const int d = in[idx];
  int res = -1;
  if (d >= 0) {
    const int r = p.incon_window;
    const int l0 = max(l - r, 0), l1 = min(l + r, g.lh - 1);
    const int k0 = max(k - r, 0), k1 = min(k + r, g.lw - 1);
    int count = 0;
    for (int ll = l0; ll <= l1; ++ll) {
      const int16_t* row = in + (size_t)ll * g.lw;
      for (int kk = k0; kk <= k1; ++kk) {
        const int e = row[kk];
        count += (e >= 0 && abs(e - d) <= p.incon_threshold) ? 1 : 0;
      }
    }
    count -= 1;  // the point itself was counted
    res = count >= p.incon_min_support ? d : -1;
  }
  out[idx] = (int16_t)res;
}

// ---------------------------------------------------------------------------
// Stage 3b: redundancy filter, support lists, corners and grid vectors, in
// one workgroup of 1024 threads (the lattice is a few thousand to tens of
// thousands of points; this stage is latency-, not throughput-bound).
//  * redundancy (Section III-A: identical values along a row or column;
//    Fig. 7A: look both backwards and forwards): a point goes iff within
//    redun_max_dist steps on both sides along the pass there is a point with
//    |d' - d| <= redun_threshold; vertical pass, then horizontal pass.
//  * left list: survivors in lattice order. Right list: each survivor seen at
//    (u - d, v); on collisions the larger d wins; ordered by (v, u).
//  * corners: each image corner takes the d of the nearest list point
//    (squared distance, earlier point on ties).
//  * grid vectors (Fig. 2; Section VI-D one-hot): region mask bits d-1..d+1
//    of every list point in the region.
// The lists go to device memory and to host-mapped memory for the host mesh.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int redundant(const int16_t* in, const Geometry& g, const KParams& p,
                                         int idx, bool vertical) {
  const int l = idx / g.lw, k = idx - l * g.lw;
  const int d = in[idx];
  if (d < 0) return -1;
  bool before = false, after = false;
  for (int j = 1; j <= p.redun_max_dist; ++j) {
    if (vertical) {
      if (l - j >= 0) {
        const int e = in[idx - j * g.lw];
        before |= e >= 0 && abs(e - d) <= p.redun_threshold;
      }
      if (l + j < g.lh) {
        const int e = in[idx + j * g.lw];
        after |= e >= 0 && abs(e - d) <= p.redun_threshold;
      }
    } else {
      if (k - j >= 0) {
        const int e = in[idx - j];
        before |= e >= 0 && abs(e - d) <= p.redun_threshold;
      }
      if (k + j < g.lw) {
        const int e = in[idx + j];
        after |= e >= 0 && abs(e - d) <= p.redun_threshold;
      }
    }
  }
  return (before && after) ? -1 : d;
}

// Exclusive prefix sum over the 1024 threads of the block; *total gets the sum.
__device__ int block_exclusive_scan(int x, int* total, int* wsum) {
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
  for (int w2 = 0; w2 < kListsThreads / 64; ++w2) {
    const int s = wsum[w2];
    before += w2 < wid ? s : 0;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

__global__ __launch_bounds__(kListsThreads) void k_lists(
    Geometry g, KParams p, const int16_t* __restrict__ incon, int16_t* __restrict__ vert,
    int16_t* __restrict__ fin, const int32_t* __restrict__ evals, int32_t* row_scratch,
    int32_t* flag_scratch, ListHeader* dev_hdr, int32_t* dev_ptsL, int32_t* dev_ptsR,
    ListHeader* host_hdr, int32_t* host_ptsL, int32_t* host_ptsR, uint32_t* gridL,
    uint32_t* gridR, unsigned long long* dense_counter) {
  __shared__ int wsum[kListsThreads / 64];
  __shared__ unsigned long long s_corner[8];
  __shared__ unsigned long long s_evals;
  const int tid = threadIdx.x;
  const int N = g.lw * g.lh;
  const int gcount = g.gw * g.gh * g.gwords;
  for (int i = tid; i < gcount; i += kListsThreads) {
    gridL[i] = 0u;
    gridR[i] = 0u;
  }
  if (tid < 8) s_corner[tid] = ~0ull;
  if (tid == 0) {
    s_evals = 0ull;
    *dense_counter = 0ull;
  }
  for (int i = tid; i < N; i += kListsThreads) vert[i] = (int16_t)redundant(incon, g, p, i, true);
  __syncthreads();
  for (int i = tid; i < N; i += kListsThreads) fin[i] = (int16_t)redundant(vert, g, p, i, false);
  __syncthreads();

  // left list: compaction in lattice order; rowStartL[l] = first index of row l
  int32_t* rowStartL = row_scratch;               // lh + 1 entries
  int32_t* rowStartR = row_scratch + (g.lh + 1);  // lh + 1 entries
  int base = 0;
  for (int c0 = 0; c0 < N; c0 += kListsThreads) {
    const int idx = c0 + tid;
    const int d = idx < N ? fin[idx] : -1;
    int total;
    const int excl = block_exclusive_scan(d >= 0 ? 1 : 0, &total, wsum);
    if (idx < N) {
      const int l = idx / g.lw, k = idx - l * g.lw;
      if (k == 0) rowStartL[l] = base + excl;
      if (d >= 0) {
        const int pos = base + excl;
        const int u = g.lu0 + k * g.step, v = g.lv0 + l * g.step;
        dev_ptsL[3 * pos] = u;
        dev_ptsL[3 * pos + 1] = v;
        dev_ptsL[3 * pos + 2] = d;
        host_ptsL[3 * pos] = u;
        host_ptsL[3 * pos + 1] = v;
        host_ptsL[3 * pos + 2] = d;
      }
    }
    base += total;
  }
  const int nL = base;
  if (tid == 0) rowStartL[g.lh] = nL;
  for (int l = tid; l <= g.lh; l += kListsThreads) rowStartR[l] = 0;
  __syncthreads();

  // right list: a point is dropped if another point of its row lands on the
  // same right-view pixel with a larger disparity
  for (int i = tid; i < nL; i += kListsThreads) {
    const int u = dev_ptsL[3 * i], v = dev_ptsL[3 * i + 1], d = dev_ptsL[3 * i + 2];
    const int ur = u - d, l = (v - g.lv0) / g.step;
    bool keep = true;
    for (int j = rowStartL[l]; j < rowStartL[l + 1]; ++j) {
      const int dj = dev_ptsL[3 * j + 2];
      if (j != i && dev_ptsL[3 * j] - dj == ur && dj > d) keep = false;
    }
    flag_scratch[i] = keep ? 1 : 0;
    if (keep) atomicAdd(&rowStartR[l], 1);
  }
  __syncthreads();
  // exclusive scan of the per-row counts (in place)
  int baseR = 0;
  for (int c0 = 0; c0 <= g.lh; c0 += kListsThreads) {
    const int idx = c0 + tid;
    const int x = idx <= g.lh ? rowStartR[idx] : 0;
    int total;
    const int excl = block_exclusive_scan(x, &total, wsum);
    if (idx <= g.lh) rowStartR[idx] = baseR + excl;
    baseR += total;
  }
  const int nR = baseR;
  __syncthreads();
  for (int i = tid; i < nL; i += kListsThreads) {
    if (!flag_scratch[i]) continue;
    const int u = dev_ptsL[3 * i], v = dev_ptsL[3 * i + 1], d = dev_ptsL[3 * i + 2];
    const int ur = u - d, l = (v - g.lv0) / g.step;
    int rank = 0;
    for (int j = rowStartL[l]; j < rowStartL[l + 1]; ++j)
      rank += (flag_scratch[j] && dev_ptsL[3 * j] - dev_ptsL[3 * j + 2] < ur) ? 1 : 0;
    const int pos = rowStartR[l] + rank;
    dev_ptsR[3 * pos] = ur;
    dev_ptsR[3 * pos + 1] = v;
    dev_ptsR[3 * pos + 2] = d;
    host_ptsR[3 * pos] = ur;
    host_ptsR[3 * pos + 1] = v;
    host_ptsR[3 * pos + 2] = d;
  }
  __syncthreads();

  // corners and grid vectors of both views
  const int cu[4] = {0, g.w - 1, 0, g.w - 1}, cv[4] = {0, 0, g.h - 1, g.h - 1};
  for (int f = 0; f < 2; ++f) {
    const int n = f ? nR : nL;
    const int32_t* pts = f ? dev_ptsR : dev_ptsL;
    uint32_t* grid = f ? gridR : gridL;
    for (int i = tid; i < n; i += kListsThreads) {
      const int u = pts[3 * i], v = pts[3 * i + 1], d = pts[3 * i + 2];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const long long du = u - cu[c], dv = v - cv[c];
        const unsigned long long key =
            ((unsigned long long)(du * du + dv * dv) << 32) | (unsigned long long)i;
        atomicMin(&s_corner[4 * f + c], key);
      }
      const int cell = (v / p.grid_size) * g.gw + u / p.grid_size;
      for (int dd = d - 1; dd <= d + 1; ++dd) {
        if (dd < p.dmin || dd > p.dmax) continue;
        const int bit = dd - p.dmin;
        atomicOr(&grid[cell * g.gwords + (bit >> 5)], 1u << (bit & 31));
      }
    }
  }
  unsigned long long ev = 0;
  for (int i = tid; i < N; i += kListsThreads) ev += (unsigned long long)evals[i];
  atomicAdd(&s_evals, ev);
  __syncthreads();
  if (tid == 0) {
    ListHeader hd;
    hd.nL = nL;
    hd.nR = nR;
    for (int c = 0; c < 4; ++c) {
      hd.cornersL[c] = nL > 0 ? dev_ptsL[3 * (int)(s_corner[c] & 0xFFFFFFFFull) + 2] : -1;
      hd.cornersR[c] = nR > 0 ? dev_ptsR[3 * (int)(s_corner[4 + c] & 0xFFFFFFFFull) + 2] : -1;
    }
    hd.support_evals = (int64_t)s_evals;
    *dev_hdr = hd;
    *host_hdr = hd;
  }
}

// ---------------------------------------------------------------------------
// Prior raster (Section VI-D: the mesh becomes an image-sized matrix of
// priors). One workgroup per kRasterChunk pixels of a triangle's bounding
// box; a pixel inside the closed triangle takes the smallest canonical rank
// of the triangles containing it (atomicMin, order-independent).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_raster(const RasterTri* __restrict__ tris,
                                                const RasterUnit* __restrict__ units,
                                                int32_t ntL, Geometry g,
                                                int32_t* __restrict__ ownerL,
                                                int32_t* __restrict__ ownerR) {
  const RasterUnit wu = units[blockIdx.x];
  const RasterTri t = tris[wu.tri];
  const bool right = wu.tri >= ntL;
  const int rank = right ? wu.tri - ntL : wu.tri;
  int32_t* owner = right ? ownerR : ownerL;
  const int au = t.u[0], av = t.v[0], bu = t.u[1], bv = t.v[1], cu = t.u[2], cv = t.v[2];
  const int umin = min(au, min(bu, cu)), umax = max(au, max(bu, cu));
  const int vmin = min(av, min(bv, cv)), vmax = max(av, max(bv, cv));
  const int bw = umax - umin + 1;
  const int area = bw * (vmax - vmin + 1);
  const int start = wu.chunk * kRasterChunk;
  const int end = min(start + kRasterChunk, area);
  for (int i = start + (int)threadIdx.x; i < end; i += 256) {
    const int y = i / bw, x = i - y * bw;
    const int u = umin + x, v = vmin + y;
    const int e0 = (bu - au) * (v - av) - (bv - av) * (u - au);
    const int e1 = (cu - bu) * (v - bv) - (cv - bv) * (u - bu);
    const int e2 = (au - cu) * (v - cv) - (av - cv) * (u - cu);
    if (e0 >= 0 && e1 >= 0 && e2 >= 0) atomicMin(&owner[(size_t)v * g.w + u], rank);
  }
}

// ---------------------------------------------------------------------------
// Dense matching (Section III-A, Fig. 1(h)). One thread per pixel; blockIdx.y
// selects the view. The prior disparity is the owning triangle's plane mean
// ((a*u) + (b*v)) + c in FP32 without contraction, rounded as
// floor(mean + 0.5) and clamped. Candidates: the plane window, the grid
// region's one-hot mask (or every d with full_search), restricted to
// partners with a defined descriptor. Energy: descriptor SAD plus the prior
// table at |d - d_plane|. Argmin by packed key.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bits_between(int a, int b) {
  a = max(a, 0);
  b = min(b, 31);
  if (a > b) return 0u;
  const uint32_t hi = b == 31 ? 0xFFFFFFFFu : ((2u << b) - 1u);
  return hi & ~((1u << a) - 1u);
}

__global__ __launch_bounds__(256) void k_dense(
    const uint8_t* __restrict__ descL, const uint8_t* __restrict__ descR,
    const int32_t* __restrict__ ownerL, const int32_t* __restrict__ ownerR,
    const RasterTri* __restrict__ tris, int32_t ntL, const uint32_t* __restrict__ gridL,
    const uint32_t* __restrict__ gridR, const int32_t* __restrict__ lut, int32_t has_list,
    Geometry g, KParams p, int16_t* __restrict__ dplaneL, int16_t* __restrict__ dplaneR,
    int16_t* __restrict__ rawL, int16_t* __restrict__ rawR,
    unsigned long long* __restrict__ dense_counter) {
  __shared__ int32_t s_lut[kMaxD];
  __shared__ int s_cnt[4];
  for (int i = threadIdx.x; i < p.D; i += 256) s_lut[i] = lut[i];
  __syncthreads();
  const bool right = blockIdx.y != 0;
  const int npx = g.w * g.h;
  const int px = blockIdx.x * 256 + threadIdx.x;
  int cnt = 0;
  if (px < npx) {
    const int v = px / g.w, u = px - v * g.w;
    const uint8_t* self_desc = right ? descR : descL;
    const uint8_t* other_desc = right ? descL : descR;
    int dp = -1;
    if (has_list) {
      const int o = (right ? ownerR : ownerL)[px];
      if (o != kNoOwner) {
        const RasterTri t = tris[o + (right ? ntL : 0)];
        const float au = __fmul_rn(t.a, (float)u);
        const float bv = __fmul_rn(t.b, (float)v);
        const float mu = __fadd_rn(__fadd_rn(au, bv), t.c);
        const float f = floorf(__fadd_rn(mu, 0.5f));
        dp = f < (float)p.dmin ? p.dmin : (f > (float)p.dmax ? p.dmax : (int)f);
      }
    }
    (right ? dplaneR : dplaneL)[px] = (int16_t)dp;
    int res = -1;
    if (u >= 2 && u <= g.w - 3 && v >= 2 && v <= g.h - 3) {
      const uint4 s = ld16(self_desc + (size_t)px * 16);
      const int lim = (right ? (g.w - 3 - u) : (u - 2)) - p.dmin;  // largest admissible d-dmin
      if ((int)texture16(s) >= p.match_texture && lim >= 0) {
        const int lo = dp >= 0 ? max(dp - p.sradius, p.dmin) - p.dmin : 1;
        const int hi = dp >= 0 ? min(dp + p.sradius, p.dmax) - p.dmin : 0;
        const int top = min(lim, p.D - 1);
        const uint32_t* cell =
            has_list ? (right ? gridR : gridL) +
                           ((size_t)(v / p.grid_size) * g.gw + u / p.grid_size) * g.gwords
                     : nullptr;
        uint32_t best = 0xFFFFFFFFu;
        const uint8_t* orow = other_desc + (size_t)v * g.w * 16;
        for (int j = 0; j < g.gwords && 32 * j <= top; ++j) {
          const int base = 32 * j;
          uint32_t m = p.full_search ? 0xFFFFFFFFu : 0u;
          if (cell) m |= cell[j];
          m |= bits_between(lo - base, hi - base);
          m &= bits_between(0, top - base);
          while (m) {
            const int b = __builtin_ctz(m);
            m &= m - 1u;
            const int dd = base + b;
            const int d = p.dmin + dd;
            const int uo = right ? u + d : u - d;
            int E = (int)sad16(s, ld16(orow + (size_t)uo * 16));
            if (dp >= 0) E += s_lut[abs(d - dp)];
            best = min(best, ((uint32_t)(E + p.lut_bias) << 8) | (uint32_t)dd);
            ++cnt;
          }
        }
        if (best != 0xFFFFFFFFu) res = p.dmin + (int)(best & 0xFFu);
      }
    }
    (right ? rawR : rawL)[px] = (int16_t)res;
  }
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    if (tot) atomicAdd(dense_counter, (unsigned long long)tot);
  }
}

// ---------------------------------------------------------------------------
// Final left/right consistency check (Section III-A: occlusions invalidated).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lrcheck(const int16_t* __restrict__ rawL,
                                                 const int16_t* __restrict__ rawR, Geometry g,
                                                 KParams p, int16_t* __restrict__ outL,
                                                 int16_t* __restrict__ outR) {
  const int px = blockIdx.x * 256 + threadIdx.x;
  if (px >= g.w * g.h) return;
  const int v = px / g.w, u = px - v * g.w;
  const size_t row = (size_t)v * g.w;
  if (blockIdx.y == 0) {
    const int d = rawL[px];
    int r = -1;
    if (d >= 0 && u - d >= 0) {
      const int e = rawR[row + u - d];
      if (e >= 0 && abs(e - d) <= p.lr_threshold) r = d;
    }
    outL[px] = (int16_t)r;
  } else {
    const int d = rawR[px];
    int r = -1;
    if (d >= 0 && u + d < g.w) {
      const int e = rawL[row + u + d];
      if (e >= 0 && abs(e - d) <= p.lr_threshold) r = d;
    }
    outR[px] = (int16_t)r;
  }
}

inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_descriptor(const uint8_t* left, const uint8_t* right, int32_t stride,
                             const Geometry& g, uint8_t* descL, uint8_t* descR,
                             int32_t* ownerL, int32_t* ownerR, hipStream_t s) {
  dim3 grid(cdiv(g.w, kDescW), cdiv(g.h, kDescH), 2), block(kDescW, kDescH, 1);
  hipLaunchKernelGGL(k_descriptor, grid, block, 0, s, left, right, stride, g, descL, descR,
                     ownerL, ownerR);
  return hipGetLastError();
}

hipError_t launch_support(const uint8_t* descL, const uint8_t* descR, const Geometry& g,
                          const KParams& p, int16_t* dcan, int32_t* evals, hipStream_t s) {
  const int n = g.lw * g.lh;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_support, dim3(cdiv(n, 4)), dim3(256), 0, s, descL, descR, g, p, dcan,
                     evals);
  return hipGetLastError();
}

hipError_t launch_incon(const int16_t* in, const Geometry& g, const KParams& p, int16_t* out,
                        hipStream_t s) {
  const int n = g.lw * g.lh;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_incon, dim3(cdiv(n, 256)), dim3(256), 0, s, in, g, p, out);
  return hipGetLastError();
}

hipError_t launch_lists(const Geometry& g, const KParams& p, const int16_t* dcan_incon,
                        int16_t* dcan_vert, int16_t* dcan_final, const int32_t* evals,
                        int32_t* row_scratch, int32_t* flag_scratch, ListHeader* dev_hdr,
                        int32_t* dev_ptsL, int32_t* dev_ptsR, ListHeader* host_hdr,
                        int32_t* host_ptsL, int32_t* host_ptsR, uint32_t* gridL,
                        uint32_t* gridR, unsigned long long* dense_counter, hipStream_t s) {
  hipLaunchKernelGGL(k_lists, dim3(1), dim3(kListsThreads), 0, s, g, p, dcan_incon, dcan_vert,
                     dcan_final, evals, row_scratch, flag_scratch, dev_hdr, dev_ptsL, dev_ptsR,
                     host_hdr, host_ptsL, host_ptsR, gridL, gridR, dense_counter);
  return hipGetLastError();
}

hipError_t launch_raster(const RasterTri* tris, const RasterUnit* units, int32_t nunits,
                         int32_t ntL, const Geometry& g, int32_t* ownerL, int32_t* ownerR,
                         hipStream_t s) {
  if (nunits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster, dim3(nunits), dim3(256), 0, s, tris, units, ntL, g, ownerL,
                     ownerR);
  return hipGetLastError();
}

hipError_t launch_dense(const uint8_t* descL, const uint8_t* descR, const int32_t* ownerL,
                        const int32_t* ownerR, const RasterTri* tris, int32_t ntL,
                        const uint32_t* gridL, const uint32_t* gridR, const int32_t* lut,
                        int32_t has_list, const Geometry& g, const KParams& p,
                        int16_t* dplaneL, int16_t* dplaneR, int16_t* rawL, int16_t* rawR,
                        unsigned long long* dense_counter, hipStream_t s) {
  dim3 grid(cdiv((long long)g.w * g.h, 256), 2);
  hipLaunchKernelGGL(k_dense, grid, dim3(256), 0, s, descL, descR, ownerL, ownerR, tris, ntL,
                     gridL, gridR, lut, has_list, g, p, dplaneL, dplaneR, rawL, rawR,
                     dense_counter);
  return hipGetLastError();
}

hipError_t launch_lrcheck(const int16_t* rawL, const int16_t* rawR, const Geometry& g,
                          const KParams& p, int16_t* outL, int16_t* outR, hipStream_t s) {
  dim3 grid(cdiv((long long)g.w * g.h, 256), 2);
  hipLaunchKernelGGL(k_lrcheck, grid, dim3(256), 0, s, rawL, rawR, g, p, outL, outR);
  return hipGetLastError();
}

}  // namespace elas

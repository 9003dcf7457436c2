// HIP kernels of the ELAS hot path for gfx950 (MI355X).
//
// Data layout in HBM, per frame (arrays carved from one allocation):
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
//
// Every stage is a device function of (frame, frame-local block index). Two
// kernels call it: one for a single frame (the frame passed by value), one
// for a batch of frames in a single launch (frames in a device table; a
// block finds its frame in the prefix of the per-frame block counts).
#include <algorithm>

#include <hip/hip_ext.h>

#include "elas_internal.h"
#include "elas_wave.h"

namespace elas {
namespace {

extern __shared__ __align__(16) char dyn_smem[];

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

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b % 8), and each XCD has its own L2. Remapping the launch order so that XCD
// x gets the x-th contiguous eighth of the logical blocks keeps each image
// row band, and the descriptors written and read for it, in one L2 across
// the descriptor, support, dense and check kernels. Bijective on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Frame of logical block b in a batch: the last frame starting at or before b.
__device__ __forceinline__ int frame_of(const int32_t* __restrict__ starts, int nf, int b) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
__host__ __device__ __forceinline__ int cdivd(int a, int b) { return (a + b - 1) / b; }

// Stages count elements into LDS: element i = load(i) goes to store(i, .).
// A plain strided loop waits for each global load before its LDS write, one
// memory round trip per iteration; here the first N * THREADS loads are all
// issued before the first write (a loop finishes any remainder).
template <int N, int THREADS, class Load, class Store>
__device__ __forceinline__ void stage_copy(int count, const Load& load, const Store& store) {
  decltype(load(0)) v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int i = (int)threadIdx.x + k * THREADS;
    if (i < count) v[k] = load(i);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int i = (int)threadIdx.x + k * THREADS;
    if (i < count) store(i, v[k]);
  }
  for (int i = (int)threadIdx.x + N * THREADS; i < count; i += THREADS) store(i, load(i));
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
// Block = 128 columns x TH rows, 256 threads; a thread works on 4 adjacent
// columns at a time, so that every LDS access moves a word or two instead of
// a byte. The image tile with its halo is staged in LDS, the quantised
// gradients of the tile with a 2-pixel halo are computed once into LDS (4
// per thread step, from two words per image row), and each thread assembles
// the descriptors of its 4 pixels from two words per gradient row with byte
// permutes; they leave through an LDS buffer in 1 KiB contiguous stores.
// Sample pattern (column, row offsets): du at (-2,0) (-1,0) (1,0) (2,0)
// (-1,-2) (1,-2) (-1,2) (1,2); dv at (0,-2) (0,-1) (0,1) (0,2) (-2,-1) (2,-1)
// (-2,1) (2,1). Descriptors are defined for 2 <= u <= w-3, 2 <= v <= h-3 and
// all-zero elsewhere.
// ---------------------------------------------------------------------------
constexpr int kDescW = 128;                  // columns per Sobel block
constexpr int kDescGroups = kDescW / 4;      // 4-column groups per block row
constexpr int kDescTW = kDescW / 4 + 2;      // tile words per row: image u0-4 .. u0+kDescW+3
constexpr int kDescQW = kDescW / 4 + 2;      // gradient words per row: image u0-2 .. u0+kDescW+5
constexpr int kCensusW = 64;                 // columns per census block
constexpr int kDescRows[kDescVariants] = {4, 8, 16};

__host__ __device__ __forceinline__ int desc_block_width(const KParams& p) {
  return p.descriptor == 0 ? kDescW : kCensusW;
}

// Byte k (0..7) of the little-endian pair (lo, hi), k a compile-time constant.
template <int K>
__device__ __forceinline__ uint32_t byte_of(uint32_t lo, uint32_t hi) {
  return K < 4 ? (lo >> (8 * K)) & 0xFFu : (hi >> (8 * (K - 4))) & 0xFFu;
}

// Selector of v_perm_b32(hi, lo, sel): result byte n = byte sel_n of the
// pair, 0x0C = zero byte.
__host__ __device__ constexpr uint32_t perm_sel(int b0, int b1, int b2, int b3) {
  return (uint32_t)b0 | ((uint32_t)b1 << 8) | ((uint32_t)b2 << 16) | ((uint32_t)b3 << 24);
}
constexpr int kZ = 0x0C;  // v_perm: a zero byte

// NT: the descriptors leave with non-temporal stores (a template argument:
// a runtime choice between two stores of the same value to the same address
// is merged into one ordinary store by the compiler).
template <int TH, bool NT>
__device__ __forceinline__ void descriptor_body(const Frame& F, int lb) {
  const Geometry g = F.g;
  const int nbx = cdivd(g.w, kDescW);
  const int view = lb & 1, tile_id = lb >> 1;  // views interleaved
  const uint8_t* img = view ? F.right : F.left;
  uint8_t* desc = view ? F.descR : F.descL;
  const int stride = F.stride;
  // tile word j of row r: image columns u0-4+4j .. +3 of image row v0-3+r;
  // gradient word j of row r: image columns u0-2+4j .. +3 of image row v0-2+r
  __shared__ uint32_t tile[TH + 6][kDescTW];
  __shared__ uint32_t qdu[TH + 4][kDescQW];
  __shared__ uint32_t qdv[TH + 4][kDescQW];
  const int u0 = (tile_id % nbx) * kDescW, v0 = (tile_id / nbx) * TH;
  const int tid = threadIdx.x;
  // rows of 4-byte aligned words whole in the image load as words; the rest
  // byte by byte (zero outside the image)
  const bool words_ok = ((reinterpret_cast<uintptr_t>(img) | (uintptr_t)stride) & 3u) == 0;
  constexpr int kTile = (TH + 6) * kDescTW;
  stage_copy<(kTile + 255) / 256, 256>(
      kTile,
      [&](int i) -> uint32_t {
        const int r = i / kDescTW, j = i - r * kDescTW;
        const int y = v0 - 3 + r, x = u0 - 4 + 4 * j;
        if (y < 0 || y >= g.h) return 0u;
        const uint8_t* row = img + (size_t)y * stride;
        if (words_ok && x >= 0 && x + 3 < g.w) return *reinterpret_cast<const uint32_t*>(row + x);
        uint32_t wv = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (x + b >= 0 && x + b < g.w) wv |= (uint32_t)row[x + b] << (8 * b);
        return wv;
      },
      [&](int i, uint32_t x) {
        const int r = i / kDescTW, j = i - r * kDescTW;
        tile[r][j] = x;
      });
  __syncthreads();
  // gradients: word j of gradient row r (image columns x0 .. x0+3, x0 =
  // u0-2+4j, image row y = v0-2+r) from tile words j, j+1 of tile rows r,
  // r+1, r+2 (image columns x0-1 .. x0+4 are bytes 1..6 of the pair)
  for (int i = tid; i < (TH + 4) * kDescQW; i += 256) {
    const int r = i / kDescQW, j = i - r * kDescQW;
    const int y = v0 - 2 + r, x0 = u0 - 2 + 4 * j;
    const uint32_t t0 = tile[r][j], t1 = tile[r][min(j + 1, kDescTW - 1)];
    const uint32_t m0 = tile[r + 1][j], m1 = tile[r + 1][min(j + 1, kDescTW - 1)];
    const uint32_t b0 = tile[r + 2][j], b1 = tile[r + 2][min(j + 1, kDescTW - 1)];
    int colS[6], colD[6];  // per column x0-1+k: top + 2 mid + bottom, bottom - top
#define ELAS_SOBEL_COL(K)                                                             \
  {                                                                                   \
    const int tt = (int)byte_of<K + 1>(t0, t1), mm = (int)byte_of<K + 1>(m0, m1),     \
              bb = (int)byte_of<K + 1>(b0, b1);                                       \
    colS[K] = tt + 2 * mm + bb;                                                       \
    colD[K] = bb - tt;                                                                \
  }
    ELAS_SOBEL_COL(0) ELAS_SOBEL_COL(1) ELAS_SOBEL_COL(2) ELAS_SOBEL_COL(3)
    ELAS_SOBEL_COL(4) ELAS_SOBEL_COL(5)
#undef ELAS_SOBEL_COL
    const bool yin = y >= 1 && y <= g.h - 2;
    uint32_t wu = 0u, wv = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int x = x0 + k;
      int gx = colS[k + 2] - colS[k];
      int gy = colD[k] + 2 * colD[k + 1] + colD[k + 2];
      if (!(yin && x >= 1 && x <= g.w - 2)) gx = gy = 0;
      wu |= quantise(gx) << (8 * k);
      wv |= quantise(gy) << (8 * k);
    }
    qdu[r][j] = wu;
    qdv[r][j] = wv;
  }
  __syncthreads();
  // descriptors: pixels u = u0+4c .. u0+4c+3 of image row v = v0+ty take
  // gradient words c, c+1 (image columns u-2 .. u+5 as bytes k = 0..7 for
  // the first pixel, shifted by one per pixel) of gradient rows ty .. ty+4.
  // Four rows at a time (a smaller buffer, more workgroups per CU); the 4
  // descriptors of a thread go through LDS so that each store instruction
  // writes 1 KiB contiguous. A descriptor's slot
  // in a row of the buffer is swizzled (pixel 4c+k at 4c + (k ^ (c/4 % 4)))
  // so that neither the writes nor the reads conflict on LDS banks.
  constexpr int kOutRows = 4;
  __shared__ uint4 obuf[kOutRows][kDescW];
  const int c = tid & (kDescGroups - 1), orow = tid / kDescGroups;
  const int ug = u0 + 4 * c;
  for (int pass = 0; pass < TH; pass += kOutRows) {
    const int ty = pass + orow;
    if (orow < kOutRows && ty < TH) {
      const int v = v0 + ty;
      const int r = ty + 2;  // gradient row of image row v
      const uint32_t a0 = qdu[r][c], a1 = qdu[r][c + 1];          // du, row v
      const uint32_t n0 = qdu[r - 2][c], n1 = qdu[r - 2][c + 1];  // du, row v-2
      const uint32_t s0 = qdu[r + 2][c], s1 = qdu[r + 2][c + 1];  // du, row v+2
      const uint32_t e0 = qdv[r - 2][c], e1 = qdv[r - 2][c + 1];  // dv, row v-2
      const uint32_t f0 = qdv[r - 1][c], f1 = qdv[r - 1][c + 1];  // dv, row v-1
      const uint32_t h0 = qdv[r + 1][c], h1 = qdv[r + 1][c + 1];  // dv, row v+1
      const uint32_t k0 = qdv[r + 2][c], k1 = qdv[r + 2][c + 1];  // dv, row v+2
      const bool vin = v >= 2 && v <= g.h - 3;
      const int sw = (c >> 2) & 3;
#define ELAS_DESC_PIXEL(I)                                                                     \
  {                                                                                            \
    uint4 o;                                                                                   \
    o.x = __builtin_amdgcn_perm(a1, a0, perm_sel(I, I + 1, I + 3, I + 4));                     \
    o.y = __builtin_amdgcn_perm(n1, n0, perm_sel(I + 1, I + 3, kZ, kZ)) |                      \
          __builtin_amdgcn_perm(s1, s0, perm_sel(kZ, kZ, I + 1, I + 3));                       \
    o.z = __builtin_amdgcn_perm(e1, e0, perm_sel(I + 2, kZ, kZ, kZ)) |                         \
          __builtin_amdgcn_perm(f1, f0, perm_sel(kZ, I + 2, kZ, kZ)) |                         \
          __builtin_amdgcn_perm(h1, h0, perm_sel(kZ, kZ, I + 2, kZ)) |                         \
          __builtin_amdgcn_perm(k1, k0, perm_sel(kZ, kZ, kZ, I + 2));                          \
    o.w = __builtin_amdgcn_perm(f1, f0, perm_sel(I, I + 4, kZ, kZ)) |                          \
          __builtin_amdgcn_perm(h1, h0, perm_sel(kZ, kZ, I, I + 4));                           \
    const int u = ug + I;                                                                      \
    if (!(vin && u >= 2 && u <= g.w - 3)) o = make_uint4(0u, 0u, 0u, 0u);                      \
    obuf[orow][4 * c + (I ^ sw)] = o;                                                          \
  }
      ELAS_DESC_PIXEL(0) ELAS_DESC_PIXEL(1) ELAS_DESC_PIXEL(2) ELAS_DESC_PIXEL(3)
#undef ELAS_DESC_PIXEL
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kOutRows * kDescW / 256; ++i) {
      const int q = tid + 256 * i, rr = q / kDescW, col = q & (kDescW - 1);
      const int v = v0 + pass + rr, u = u0 + col;
      if (pass + rr < TH && v < g.h && u < g.w) {
        const uint4 o = obuf[rr][(col & ~3) | ((col & 3) ^ ((col >> 4) & 3))];
        uint4* dst = reinterpret_cast<uint4*>(desc + ((size_t)v * g.w + u) * 16);
        if constexpr (NT) {  // straight to HBM, leaving no dirty lines in the caches
          __builtin_nontemporal_store(o.x, &dst->x);
          __builtin_nontemporal_store(o.y, &dst->y);
          __builtin_nontemporal_store(o.z, &dst->z);
          __builtin_nontemporal_store(o.w, &dst->w);
        } else {
          *dst = o;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Stage 1, census variant (Section VI-A: census descriptors over the whole
// window, compared by Hamming distance). Same 64 x TH tiling; the tile is
// staged with a 6-pixel halo (13 x 13 windows), positions outside the image
// holding 255 so that they never count as darker. Bit i of a descriptor is
// the i-th window offset in row-major order, set iff that neighbour is darker
// than the centre; a window row of W bits is placed at bit W*dy.
//  * dense census (window cd_win <= 7, at most 49 bits): one uint64 per pixel,
//    every pixel;
//  * support census (window cs_win <= 13, at most 169 bits): lattice rows
//    only (the support search never reads other rows), cs_q 16-byte words
//    per pixel, zero-padded.
// ---------------------------------------------------------------------------
constexpr int kCensusHalo = 6;

// Bits of rb (at most 13) moved to bit offset s of a 64-bit word (s may be
// negative: the part of a window row that spills into this word).
__device__ __forceinline__ uint64_t place_bits(uint32_t rb, int s) {
  if (s >= 64 || s <= -32) return 0ull;
  return s >= 0 ? ((uint64_t)rb << s) : (uint64_t)(rb >> (-s));
}

template <int TH>
__device__ __forceinline__ void census_body(const Frame& F, int lb) {
  const Geometry g = F.g;
  const KParams p = F.p;
  const int nbx = cdivd(g.w, kCensusW);
  const int view = lb & 1, tile_id = lb >> 1;
  const uint8_t* img = view ? F.right : F.left;
  uint64_t* dcen = reinterpret_cast<uint64_t*>(view ? F.descR : F.descL);
  uint4* scen = view ? F.csupR : F.csupL;
  const int stride = F.stride;
  constexpr int H = kCensusHalo, TW = kCensusW + 2 * H;
  __shared__ uint8_t tile[TH + 2 * H][TW];
  const int u0 = (tile_id % nbx) * kCensusW, v0 = (tile_id / nbx) * TH;
  const int tid = threadIdx.x;
  constexpr int kTile = (TH + 2 * H) * TW;
  stage_copy<(kTile + 255) / 256, 256>(
      kTile,
      [&](int i) -> uint32_t {
        const int r = i / TW, c = i - r * TW;
        const int y = v0 - H + r, x = u0 - H + c;
        return (x >= 0 && x < g.w && y >= 0 && y < g.h) ? img[(size_t)y * stride + x] : 255u;
      },
      [&](int i, uint32_t x) {
        const int r = i / TW, c = i - r * TW;
        tile[r][c] = (uint8_t)x;
      });
  __syncthreads();
  const int tx = tid & 63;
  const int u = u0 + tx;
  if (u >= g.w) return;
  for (int ty = tid >> 6; ty < TH; ty += 4) {
    const int v = v0 + ty;
    if (v >= g.h) break;
    const uint32_t c = tile[ty + H][tx + H];
    {
      const int W = p.cd_win, r = W >> 1;
      uint64_t acc = 0ull;
      for (int dy = 0; dy < W; ++dy) {
        const uint8_t* row = &tile[ty + H - r + dy][tx + H - r];
        uint32_t rb = 0u;
        for (int dx = 0; dx < W; ++dx) rb |= (uint32_t)(row[dx] < c) << dx;
        acc |= (uint64_t)rb << (dy * W);
      }
      dcen[(size_t)v * g.w + u] = acc;
    }
    const int dv = v - g.lv0;
    if (dv >= 0 && dv % g.step == 0 && dv / g.step < g.lh) {
      const int l = dv / g.step;
      const int W = p.cs_win, r = W >> 1;
      uint64_t a0 = 0ull, a1 = 0ull, a2 = 0ull;
      for (int dy = 0; dy < W; ++dy) {
        const uint8_t* row = &tile[ty + H - r + dy][tx + H - r];
        uint32_t rb = 0u;
        for (int dx = 0; dx < W; ++dx) rb |= (uint32_t)(row[dx] < c) << dx;
        const int o = dy * W;
        a0 |= place_bits(rb, o);
        a1 |= place_bits(rb, o - 64);
        a2 |= place_bits(rb, o - 128);
      }
      uint4* dst = scen + ((size_t)l * g.w + u) * p.cs_q;
      dst[0] = make_uint4((uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)a1, (uint32_t)(a1 >> 32));
      if (p.cs_q == 2) dst[1] = make_uint4((uint32_t)a2, (uint32_t)(a2 >> 32), 0u, 0u);
    }
  }
}

template <int TH, bool NT = false>
__device__ __forceinline__ void stage1_body(const Frame& F, int lb) {
  if (F.p.descriptor)
    census_body<TH>(F, lb);
  else
    descriptor_body<TH, NT>(F, lb);
}
template <int TH>
__device__ __forceinline__ void stage1_nt_body(const Frame& F, int lb) {
  stage1_body<TH, true>(F, lb);
}

// ---------------------------------------------------------------------------
// Stage 2: support matching (Section III-A) with a reverse check. A
// workgroup takes a run of up to 16 lattice points on one lattice row and
// stages, once, every descriptor column its searches can reach (both views,
// the rows the support descriptor samples) in LDS; each wavefront then takes
// every fourth point of the run, lane k evaluating d = dmin + k + 64 j with
// its candidates read from LDS and the point's own descriptor from scalar
// loads (one address for the whole wavefront).
// Ambiguity test: eq. 1-2 (m1 < t*m2 in FP32) or the shift-sum of eq. 3
// (m1 <= m2/2 + m2/4 + m2/8 + m2/32 with truncating shifts). Descriptors:
//  * gradient: the 512-bit support descriptor is the four 16-byte descriptors
//    at (u-2, v-2), (u+2, v-2), (u-2, v+2), (u+2, v+2); cost = SAD;
//  * census: the support-window census of the pixel; cost = Hamming distance;
//    texture = number of set bits.
// ---------------------------------------------------------------------------
struct Desc64 {
  uint4 q[4];
};

__device__ __forceinline__ uint32_t sad64(const Desc64& a, const Desc64& b) {
  return sad16(a.q[0], b.q[0]) + sad16(a.q[1], b.q[1]) + sad16(a.q[2], b.q[2]) +
         sad16(a.q[3], b.q[3]);
}

__device__ __forceinline__ bool support_accept(const KParams& p, uint32_t m1, uint32_t m2) {
  if (p.ambiguity) return m1 <= (m2 >> 1) + (m2 >> 2) + (m2 >> 3) + (m2 >> 5);
  return (float)m1 < __fmul_rn(p.support_threshold, (float)m2);
}

__device__ __forceinline__ uint32_t popc4(const uint4 a) {
  return __popc(a.x) + __popc(a.y) + __popc(a.z) + __popc(a.w);
}
__device__ __forceinline__ uint4 xor4(const uint4 a, const uint4 b) {
  return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
}

// A census support descriptor: NQ 16-byte words; cost = Hamming distance.
template <int NQ>
struct CensusDesc {
  uint4 q[NQ];
};
template <int NQ>
__device__ __forceinline__ uint32_t hamming(const CensusDesc<NQ>& a, const CensusDesc<NQ>& b) {
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) c += popc4(xor4(a.q[i], b.q[i]));
  return c;
}

// LDS copies of a view's descriptor columns c0.. (one plane of 16 bytes per
// column for each descriptor row or census word), the sources of the
// searches: load(x) = the descriptor of column x on the point's row (the
// gradient descriptor takes columns x - 2 and x + 2 of rows v - 2 and
// v + 2); cost(a, b). texture(x, lane) splits the point's own texture over the
// lanes of each 16-lane row: lane i takes 4 of its bytes, a row sum adds
// them, so the wavefront pays one SAD instead of sixteen.
__device__ __forceinline__ uint4 lds16(uint32_t off) {
  return *reinterpret_cast<const uint4*>(dyn_smem + off);
}
__device__ __forceinline__ uint32_t lds4(uint32_t off) {
  return *reinterpret_cast<const uint32_t*>(dyn_smem + off);
}

struct LdsGrad {
  typedef Desc64 T;
  __device__ __forceinline__ static uint32_t cost(const T& a, const T& b) { return sad64(a, b); }
  uint32_t base;     // plane 0: row v - 2; plane 1 (base + pstride): row v + 2
  uint32_t pstride;
  int c0;
  __device__ __forceinline__ T load(int x) const {
    const uint32_t o = base + (uint32_t)(x - 2 - c0) * 16u;  // columns x - 2 and x + 2
    Desc64 r;
    r.q[0] = lds16(o);
    r.q[1] = lds16(o + 64u);
    r.q[2] = lds16(o + pstride);
    r.q[3] = lds16(o + pstride + 64u);
    return r;
  }
  // lane i of a row: dword i & 3 of part (i >> 2) & 3 of the descriptor
  __device__ __forceinline__ uint32_t texture(int x, int lane) const {
    const int part = (lane >> 2) & 3;
    const uint32_t o = base + (uint32_t)(x - 2 - c0) * 16u + (uint32_t)(part & 1) * 64u +
                       (uint32_t)(part >> 1) * pstride + (uint32_t)(lane & 3) * 4u;
    const uint32_t t = __builtin_amdgcn_sad_u8(lds4(o), 0x80808080u, 0u);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)row_sum_u32(t));
  }
};

template <int NQ>
struct LdsCensus {
  typedef CensusDesc<NQ> T;
  __device__ __forceinline__ static uint32_t cost(const T& a, const T& b) { return hamming(a, b); }
  uint32_t base;     // plane i (base + i * pstride): word i of each column
  uint32_t pstride;
  int c0;
  __device__ __forceinline__ T load(int x) const {
    const uint32_t o = base + (uint32_t)(x - c0) * 16u;
    T r;
#pragma unroll
    for (int i = 0; i < NQ; ++i) r.q[i] = lds16(o + (uint32_t)i * pstride);
    return r;
  }
  // lane i < 4 NQ of a row: the set bits of dword i & 3 of word i >> 2
  __device__ __forceinline__ uint32_t texture(int x, int lane) const {
    const int i = lane & 15, wd = min(i >> 2, NQ - 1);
    const uint32_t o = base + (uint32_t)(x - c0) * 16u + (uint32_t)wd * pstride +
                       (uint32_t)(i & 3) * 4u;
    const uint32_t t = i < 4 * NQ ? (uint32_t)__popc(lds4(o)) : 0u;
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)row_sum_u32(t));
  }
};

// The point's own descriptor in global memory, one address for the whole
// wavefront: scalar loads into SGPRs, which each SAD takes as its scalar
// operand (no LDS bandwidth and no VGPRs for it).
struct GradSelf {
  const uint8_t* ra;  // row v - 2
  const uint8_t* rb;  // row v + 2
  __device__ __forceinline__ Desc64 load(int x) const {
    const uint32_t o = (uint32_t)(x - 2) * 16u;  // columns x - 2 and x + 2
    Desc64 r;
    r.q[0] = ld16(ra + o);
    r.q[1] = ld16(ra + o + 64u);
    r.q[2] = ld16(rb + o);
    r.q[3] = ld16(rb + o + 64u);
    return r;
  }
};

template <int NQ>
struct CensusSelf {
  const uint4* row;  // the lattice row's census, NQ words per column
  __device__ __forceinline__ CensusDesc<NQ> load(int x) const {
    CensusDesc<NQ> r;
#pragma unroll
    for (int i = 0; i < NQ; ++i) r.q[i] = row[(uint32_t)x * NQ + i];
    return r;
  }
};

// One search of a point with own descriptor `self`: the candidate columns
// u + dir*d, d = dmin + lane + 64 j for j < NJ (NJ 64-wide batches cover the
// disparity range), taken two batches at a time so that at most two
// candidate descriptors per lane are live. Lanes past dhi load column dhi
// instead (in the image like every searched column) and are masked out.
// FULL: every lane of every batch is in range (dhi = dmin + 64 NJ - 1), so a
// batch's columns are one lane-dependent base plus constants and its loads
// take immediate offsets. Argmin over d = dmin..dhi (smallest cost, smallest
// d on ties; at least two values) and the ambiguity test; returns whether it
// accepts. Control flow is wavefront-uniform.
template <int NJ, bool FULL, class C>
__device__ __forceinline__ bool search(const typename C::T& self, const C& other, int u, int dir,
                                       int dhi, const KParams& p, int lane, int* d_best) {
  uint32_t key[NJ];
  uint32_t best = 0xFFFFFFFFu;
  const int xb = dir < 0 ? u - p.dmin - lane : u + p.dmin + lane;  // column of batch 0
#pragma unroll
  for (int j0 = 0; j0 < NJ; j0 += 2) {
    typename C::T o[2];
#pragma unroll
    for (int jj = 0; jj < 2 && j0 + jj < NJ; ++jj) {
      const int j = j0 + jj;
      o[jj] = other.load(FULL ? xb + dir * 64 * j : u + dir * min(p.dmin + lane + 64 * j, dhi));
    }
#pragma unroll
    for (int jj = 0; jj < 2 && j0 + jj < NJ; ++jj) {
      const int j = j0 + jj, k = lane + 64 * j;  // k = d - dmin
      const uint32_t c = C::cost(self, o[jj]);
      key[j] = FULL || p.dmin + k <= dhi ? (c << 8) | (uint32_t)k : 0xFFFFFFFFu;
      best = min(best, key[j]);
    }
  }
  best = wave_min_u32(best);
  const int d1 = p.dmin + (int)(best & 0xFFu);
  const uint32_t m1 = best >> 8;
  uint32_t m2 = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < NJ; ++j) m2 = min(m2, key[j] != best ? key[j] : 0xFFFFFFFFu);
  m2 = wave_min_u32(m2) >> 8;
  *d_best = d1;
  return support_accept(p, m1, m2);
}

// The search (full or general form) and the texture test. The search runs
// whether or not the own descriptor is textured, so that its loads (scalar
// and LDS) all issue at once instead of waiting behind the texture test's
// branch; *d_best = -2 when the own descriptor is untextured (the search
// does not count as evaluated and never accepts).
template <int NJ, class G, class C>
__device__ __forceinline__ bool support_search(const G& self_src, const C& self_lds, int xs,
                                               const C& other, int u, int dir, int dhi,
                                               const KParams& p, int lane, int* d_best) {
  const typename C::T self = self_src.load(xs);
  const bool textured = (int)self_lds.texture(xs, lane) >= p.support_texture;
  const bool ok = dhi - p.dmin + 1 == 64 * NJ
                      ? search<NJ, true>(self, other, u, dir, dhi, p, lane, d_best)
                      : search<NJ, false>(self, other, u, dir, dhi, p, lane, d_best);
  if (!textured) *d_best = -2;
  return ok && textured;
}

// One lattice point: forward search, then the reverse search from the
// matched right column. gL, gR: the views in global memory (the own
// descriptors); cL, cR: the staged columns in LDS (candidates, texture).
template <int NJ, class G, class C>
__device__ __forceinline__ int support_point(const G& gL, const G& gR, const C& cL, const C& cR,
                                             int u, int w, const KParams& p, int lane,
                                             int* ev) {
  const int dhi = min(p.dmax, u - 4);
  if (dhi - p.dmin + 1 < 2) return -1;
  int d1;
  const bool fwd = support_search<NJ>(gL, cL, u, cR, u, -1, dhi, p, lane, &d1);
  if (d1 != -2) *ev += dhi - p.dmin + 1;  // textured: the search was evaluated
  if (!fwd) return -1;
  const int ur = u - d1;
  const int dhi2 = min(p.dmax, w - 5 - ur);
  if (dhi2 - p.dmin + 1 < 2) return -1;
  int d2;
  const bool rev = support_search<NJ>(gR, cR, ur, cL, ur, +1, dhi2, p, lane, &d2);
  if (d2 != -2) *ev += dhi2 - p.dmin + 1;
  return rev && abs(d2 - d1) <= p.lr_threshold ? d1 : -1;
}

// The batch count of the frame's disparity range, as a template argument.
template <class G, class C>
__device__ __forceinline__ int support_point_d(const G& gL, const G& gR, const C& cL,
                                               const C& cR, int u, int w, const KParams& p,
                                               int lane, int* ev) {
  switch ((p.D + 63) >> 6) {
    case 1: return support_point<1>(gL, gR, cL, cR, u, w, p, lane, ev);
    case 2: return support_point<2>(gL, gR, cL, cR, u, w, p, lane, ev);
    case 3: return support_point<3>(gL, gR, cL, cR, u, w, p, lane, ev);
    default: return support_point<4>(gL, gR, cL, cR, u, w, p, lane, ev);
  }
}

// Columns a run of q lattice points (step apart) can reach, per view: right
// view [max(u_first - dmax, 4), u_last - dmin], left view that range shifted
// by up to D - 1 (reverse candidates), each widened by the two columns the
// gradient descriptor samples on either side.
__host__ __device__ __forceinline__ int support_cols_right(int q, int step, int D) {
  return (q - 1) * step + D + 4;
}
__host__ __device__ __forceinline__ int support_cols_left(int q, int step, int D) {
  return (q - 1) * step + 2 * D + 3;
}
constexpr int kSupportRunMax = 32;          // lattice points per workgroup, at most
constexpr int kSupportLdsMax = 64 * 1024;   // 32 bytes per staged column
constexpr int kSupportStageCols = 512;      // columns per plane staged per round

// Points per workgroup: the geometry's run length, fewer when the staged
// columns would not fit.
__host__ __device__ __forceinline__ int support_run(const Geometry& g, const KParams& p) {
  int q = max(1, min(g.srun, kSupportRunMax));
  while (q > 1 && 32 * (support_cols_right(q, g.step, p.D) + support_cols_left(q, g.step, p.D)) >
                      kSupportLdsMax)
    --q;
  return q;
}

__device__ __forceinline__ void support_body(const Frame& F, int lb) {
  const Geometry g = F.g;
  const KParams p = F.p;
  const int q = support_run(g, p), runs = cdivd(g.lw, q);
  const int l = lb / runs, k0 = (lb - l * runs) * q, k1 = min(g.lw, k0 + q);
  const int v = g.lv0 + l * g.step;
  const int uf = g.lu0 + k0 * g.step, ul = g.lu0 + (k1 - 1) * g.step;
  // staged search columns (every searched column lies in them; clamped ends
  // keep an empty search range in the image)
  const int rlo = max(uf - p.dmax, 4), rhi = max(rlo, ul - p.dmin);
  const int llo = min(uf, rlo + p.dmin), lhi = max(ul, min(ul - p.dmin + p.dmax, g.w - 5));
  const int cR0 = rlo - 2, nR = rhi - rlo + 5, cL0 = llo - 2, nL = lhi - llo + 5;
  const int planes = p.descriptor == 0 ? 2 : p.cs_q;  // 16-byte planes per view
  // LDS: the right view's planes (nR columns each), then the left view's.
  // Each plane is a run of columns at a fixed pitch from a uniform base;
  // every thread issues its loads for all planes before its first store.
  const int tid = threadIdx.x;
  const uint8_t* pb[4];  // plane bases: right 0, right 1, left 0, left 1
  uint32_t pd[4];        // LDS byte offsets of the planes
  int pn[4];             // columns per plane
  const uint32_t pitch = p.descriptor == 0 ? 16u : 16u * (uint32_t)p.cs_q;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool right = k < 2;
    const int pl = k & 1, c0 = right ? cR0 : cL0;
    pn[k] = pl < planes ? (right ? nR : nL) : 0;
    pd[k] = (uint32_t)(right ? pl * nR : planes * nR + pl * nL) * 16u;
    if (p.descriptor == 0)
      pb[k] = (right ? F.descR : F.descL) + ((size_t)(v - 2 + 4 * pl) * g.w + c0) * 16;
    else
      pb[k] = reinterpret_cast<const uint8_t*>((right ? F.csupR : F.csupL) +
                                               ((size_t)l * g.w + c0) * p.cs_q + pl);
  }
  const int nmax = max(nR, nL);
  for (int c0 = 0; c0 < nmax; c0 += kSupportStageCols) {
    uint4 t[4][kSupportStageCols / 256];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int s2 = 0; s2 < kSupportStageCols / 256; ++s2) {
        const int c = min(c0 + s2 * 256 + tid, max(pn[k], 1) - 1);
        t[k][s2] = ld16(pb[k] + (uint32_t)c * pitch);
      }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int s2 = 0; s2 < kSupportStageCols / 256; ++s2) {
        const int c = c0 + s2 * 256 + tid;
        if (c < pn[k]) *reinterpret_cast<uint4*>(dyn_smem + pd[k] + (uint32_t)c * 16u) = t[k][s2];
      }
  }
  __syncthreads();
  // results go through LDS and out in one coalesced store per block: with no
  // global store in the kernel before them, the loads of each point's own
  // descriptor are known not to be clobbered and become scalar loads
  __shared__ int32_t s_res[kSupportRunMax], s_ev[kSupportRunMax];
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t bR = 0, bL = (uint32_t)(planes * nR) * 16u;
  for (int k = k0 + wv; k < k1; k += 4) {
    const int u = g.lu0 + k * g.step;
    int result, ev = 0;
    if (p.descriptor == 0) {
      const LdsGrad cR{bR, (uint32_t)nR * 16u, cR0}, cL{bL, (uint32_t)nL * 16u, cL0};
      const size_t ra = (size_t)(v - 2) * g.w * 16, rb = (size_t)(v + 2) * g.w * 16;
      result = support_point_d(GradSelf{F.descL + ra, F.descL + rb},
                               GradSelf{F.descR + ra, F.descR + rb}, cL, cR, u, g.w, p, lane,
                               &ev);
    } else {
      const size_t row = (size_t)l * g.w * p.cs_q;
      if (p.cs_q == 1) {
        const LdsCensus<1> cR{bR, (uint32_t)nR * 16u, cR0}, cL{bL, (uint32_t)nL * 16u, cL0};
        result = support_point_d(CensusSelf<1>{F.csupL + row}, CensusSelf<1>{F.csupR + row}, cL,
                                 cR, u, g.w, p, lane, &ev);
      } else {
        const LdsCensus<2> cR{bR, (uint32_t)nR * 16u, cR0}, cL{bL, (uint32_t)nL * 16u, cL0};
        result = support_point_d(CensusSelf<2>{F.csupL + row}, CensusSelf<2>{F.csupR + row}, cL,
                                 cR, u, g.w, p, lane, &ev);
      }
    }
    if (lane == 0) {
      s_res[k - k0] = result;
      s_ev[k - k0] = ev;
    }
  }
  __syncthreads();
  if (tid < k1 - k0) {
    F.dcan_raw[l * g.lw + k0 + tid] = (int16_t)s_res[tid];
    F.evals[l * g.lw + k0 + tid] = s_ev[tid];
  }
}

// ---------------------------------------------------------------------------
// Stage 3: support filtering (Section III-A, Fig. 1(e); Fig. 7A), three
// simultaneous-update passes fused in one kernel over 8 x 8 lattice tiles
// (16 x 16 in batches and on lattices with more than 256 such tiles; 1024
// threads per tile;
// a position's consistency count is split over four lanes, so that the
// longest per-thread chain is a quarter of the window):
//  * consistency: a point survives iff at least incon_min_support other
//    points within +-incon_window lattice steps have |d' - d| <=
//    incon_threshold;
//  * redundancy, vertical then horizontal: a point goes iff within
//    redun_max_dist steps on both sides along the pass there is a point with
//    |d' - d| <= redun_threshold.
// The tile's raw values are staged in LDS with a halo of incon_window +
// redun_max_dist; each pass is computed on the region the next pass reads
// (positions outside the lattice count as empty). The kernel also clears the
// grid masks that the rows stage fills. With past-only redundancy only the
// consistency pass runs here.
// ---------------------------------------------------------------------------
constexpr int kFiltParts = 4;    // lanes sharing one position's consistency count
constexpr int32_t kGridEmptyLo = 0x7FFF;  // smallest set bit of an empty region mask

// Tile side in lattice points (chosen with the frame's buffers: 8 for a
// single frame whose tiles can each have a CU, else 16).
__host__ __device__ __forceinline__ int filter_tile(const Geometry& g) { return g.ftile; }
__host__ __device__ __forceinline__ int filter_tiles_x(const Geometry& g) {
  return g.lw > 0 ? cdivd(g.lw, filter_tile(g)) : 1;
}
__host__ __device__ __forceinline__ int filter_tiles_y(const Geometry& g) {
  return g.lh > 0 ? cdivd(g.lh, filter_tile(g)) : 1;
}

// i / n for 2 <= n and 0 <= i < 2^32 / n by a multiply: m = ceil(2^32 / n)
// (the error term i * (m n - 2^32) / 2^32 stays below i n / 2^32 < 1)
__device__ __forceinline__ int div_small(int i, uint32_t m) { return (int)__umulhi((uint32_t)i, m); }

template <int RI, int RR, int T>
__device__ __forceinline__ void filter_windows(const Frame& F, int lb) {
  const Geometry g = F.g;
  const KParams p = F.p;
  int16_t* smem = reinterpret_cast<int16_t*>(dyn_smem);
  // window radii: compile-time when RI / RR > 0 (the loops then unroll and
  // every LDS read of a window row issues at once)
  const int ri = RI > 0 ? RI : p.incon_window, rr = RR > 0 ? RR : p.redun_max_dist;
  const int ft = filter_tile(g);
  const int SR = ft + 2 * (ri + rr), SI = ft + 2 * rr;
  int16_t* sraw = smem;            // SR x SR, origin (l0-ri-rr, k0-ri-rr)
  int16_t* sinc = sraw + SR * SR;  // SI x SI, origin (l0-rr, k0-rr)
  int16_t* svert = sinc + SI * SI; // ft x SI, origin (l0, k0-rr)
  // positions to (row, column) by multiplies (8 <= SI <= SR <= 80); with
  // compile-time windows the multipliers are constants for both tile sides
  auto mul_of = [](int n) { return (uint32_t)(((1ull << 32) + n - 1) / n); };
  uint32_t mSR, mSI;
  if constexpr (RI > 0 && RR > 0) {
    constexpr int kSR8 = 8 + 2 * (RI + RR), kSI8 = 8 + 2 * RR;
    constexpr int kSR16 = 16 + 2 * (RI + RR), kSI16 = 16 + 2 * RR;
    constexpr uint32_t mR8 = (uint32_t)(((1ull << 32) + kSR8 - 1) / kSR8);
    constexpr uint32_t mR16 = (uint32_t)(((1ull << 32) + kSR16 - 1) / kSR16);
    constexpr uint32_t mI8 = (uint32_t)(((1ull << 32) + kSI8 - 1) / kSI8);
    constexpr uint32_t mI16 = (uint32_t)(((1ull << 32) + kSI16 - 1) / kSI16);
    mSR = ft == 8 ? mR8 : (ft == 16 ? mR16 : mul_of(SR));
    mSI = ft == 8 ? mI8 : (ft == 16 ? mI16 : mul_of(SI));
  } else {
    mSR = mul_of(SR);
    mSI = mul_of(SI);
  }
  const int ntx = filter_tiles_x(g), nblk = ntx * filter_tiles_y(g);
  const int k0 = (lb % ntx) * ft, l0 = (lb / ntx) * ft;
  const int tid = threadIdx.x;
  const int16_t* raw = F.dcan_raw;
  // clear the grid masks and their bit ranges (grid-stride over the frame's
  // blocks)
  {
    const int gcount = g.gw * g.gh * g.gwords;
    uint32_t* gridL = F.gridL;
    uint32_t* gridR = F.gridR;
    for (int i = lb * T + tid; i < gcount; i += nblk * T) {
      gridL[i] = 0u;
      gridR[i] = 0u;
    }
    const int rcount = 2 * g.gw * g.gh;
    int32_t* grL = F.grangeL;
    int32_t* grR = F.grangeR;
    for (int i = lb * T + tid; i < rcount; i += nblk * T) {
      const int32_t init = (i & 1) ? -1 : kGridEmptyLo;
      grL[i] = init;
      grR[i] = init;
    }
  }
  stage_copy<T == 1024 ? 2 : 3, T>(
      SR * SR,
      [&](int i) -> int {
        const int y = div_small(i, mSR), x = i - y * SR;
        const int l = l0 - ri - rr + y, k = k0 - ri - rr + x;
        return (l >= 0 && l < g.lh && k >= 0 && k < g.lw) ? (int)raw[(size_t)l * g.lw + k] : -1;
      },
      [&](int i, int x) { sraw[i] = (int16_t)x; });
  __syncthreads();
  // consistency count of each position: kFiltParts consecutive lanes take
  // every kFiltParts-th window row and add their counts with shuffles (the
  // loop bound is a multiple of 64, so whole wavefronts take part)
  {
    const int npos = SI * SI;
    const int ntask = cdivd(npos * kFiltParts, 64) * 64;
    for (int task = tid; task < ntask; task += T) {
      const int i = min(task / kFiltParts, npos - 1), part = task % kFiltParts;
      const int y = div_small(i, mSI), x = i - y * SI;
      const int d = sraw[(y + ri) * SR + (x + ri)];
      // e counts iff e >= 0 and |e - d| <= threshold: for d >= 0 one unsigned
      // range test, e in [max(0, d - t), d + t] (e = -1 falls outside)
      const int t = min(p.incon_threshold, 1 << 12);  // disparities differ by < 2^9
      const int lo = max(0, d - t);
      const uint32_t span = (uint32_t)(d + t - lo);
      int count = 0;
      if (d >= 0) {
        if constexpr (RI > 0) {
#pragma unroll
          for (int q = 0; q < (2 * RI + kFiltParts) / kFiltParts; ++q) {
            const int yy = y + part + q * kFiltParts;
            if (yy > y + 2 * RI) break;
            const int16_t* row = sraw + yy * SR + x;
            int e[2 * RI + 1];
#pragma unroll
            for (int xx = 0; xx <= 2 * RI; ++xx) e[xx] = row[xx];
#pragma unroll
            for (int xx = 0; xx <= 2 * RI; ++xx) count += (uint32_t)(e[xx] - lo) <= span ? 1 : 0;
          }
        } else {
          for (int yy = y + part; yy <= y + 2 * ri; yy += kFiltParts) {
            const int16_t* row = sraw + yy * SR + x;
            for (int xx = 0; xx <= 2 * ri; ++xx) count += (uint32_t)(row[xx] - lo) <= span ? 1 : 0;
          }
        }
      }
      static_assert(kFiltParts == 4, "the parts of a count are the lanes of a quad");
      count += quad_xor1(count);
      count += quad_xor2(count);
      if (part == 0 && task / kFiltParts < npos)
        sinc[i] = (int16_t)((d >= 0 && count - 1 >= p.incon_min_support) ? d : -1);  // minus itself
    }
  }
  __syncthreads();
  if (p.redundancy) {  // past-only redundancy runs in its own stage
    if (tid < ft * ft) {
      const int y = tid / ft, x = tid - y * ft;
      const int l = l0 + y, k = k0 + x;
      if (l < g.lh && k < g.lw) F.dcan_incon[(size_t)l * g.lw + k] = sinc[(y + rr) * SI + x + rr];
    }
    return;
  }
  for (int i = tid; i < ft * SI; i += T) {
    const int y = div_small(i, mSI), x = i - y * SI;
    const int d = sinc[(y + rr) * SI + x];
    int res = d;
    if (d >= 0) {
      bool before = false, after = false;
      // e >= 0 and |e - d| <= threshold as one unsigned range test (d >= 0)
      const int t = min(p.redun_threshold, 1 << 12), lo = max(0, d - t);
      const uint32_t span = (uint32_t)(d + t - lo);
      auto probe = [&](int j) {
        const int eb = sinc[(y + rr - j) * SI + x], ea = sinc[(y + rr + j) * SI + x];
        before |= (uint32_t)(eb - lo) <= span;
        after |= (uint32_t)(ea - lo) <= span;
      };
      if constexpr (RR > 0) {
#pragma unroll
        for (int j = 1; j <= RR; ++j) probe(j);
      } else {
        for (int j = 1; j <= rr; ++j) probe(j);
      }
      if (before && after) res = -1;
    }
    svert[i] = (int16_t)res;
  }
  __syncthreads();
  if (tid < ft * ft) {
    const int y = tid / ft, x = tid - y * ft;
    const int l = l0 + y, k = k0 + x;
    if (l < g.lh && k < g.lw) {
      const int d = svert[y * SI + x + rr];
      int res = d;
      if (d >= 0) {
        bool before = false, after = false;
        const int t = min(p.redun_threshold, 1 << 12), lo = max(0, d - t);
        const uint32_t span = (uint32_t)(d + t - lo);
        auto probe = [&](int j) {
          const int eb = svert[y * SI + x + rr - j], ea = svert[y * SI + x + rr + j];
          before |= (uint32_t)(eb - lo) <= span;
          after |= (uint32_t)(ea - lo) <= span;
        };
        if constexpr (RR > 0) {
#pragma unroll
          for (int j = 1; j <= RR; ++j) probe(j);
        } else {
          for (int j = 1; j <= rr; ++j) probe(j);
        }
        if (before && after) res = -1;
      }
      const size_t idx = (size_t)l * g.lw + k;
      F.dcan_incon[idx] = sinc[(y + rr) * SI + x + rr];
      F.dcan_vert[idx] = (int16_t)d;
      F.dcan_final[idx] = (int16_t)res;
    }
  }
}

// The default windows (5 and 5 lattice steps) at compile time, else any.
// T threads per tile: 1024 for a single frame (few tiles, each alone on a
// CU), 512 in batches (four tiles share a CU, so one tile's barrier phases
// overlap another's work: 16 x 16 tiles over 32 pairs 34.4 -> 23.5 us)
template <int T>
__device__ __forceinline__ void filter_body(const Frame& F, int lb) {
  if (F.p.incon_window == 5 && F.p.redun_max_dist == 5)
    filter_windows<5, 5, T>(F, lb);
  else
    filter_windows<0, 0, T>(F, lb);
}

// ---------------------------------------------------------------------------
// Past-only redundancy (Section VI-C, Fig. 7B): along each lattice column from
// the top, then along each row from the left, a point is removed iff one of
// the previous redun_max_dist positions holds a point that survived the same
// pass with |d' - d| <= redun_threshold. Each line is a sequential chain, so
// one thread walks one line; the outputs of the last R positions are kept in
// a register shift ring (R a compile-time bound >= redun_max_dist, so the
// ring is never indexed at run time). One workgroup per frame: the vertical
// pass over every column, a barrier, the horizontal pass over every row.
// Inputs are prefetched eight positions at a time.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void redun_line(const int16_t* __restrict__ in,
                                           int16_t* __restrict__ out, int n, size_t step,
                                           int r, int t) {
  int last[R];
#pragma unroll
  for (int j = 0; j < R; ++j) last[j] = -1;
  for (int b0 = 0; b0 < n; b0 += 8) {
    int x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = b0 + i < n ? in[(size_t)(b0 + i) * step] : -1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (b0 + i >= n) break;
      const int d = x[i];
      bool hit = false;
#pragma unroll
      for (int j = 0; j < R; ++j) hit |= j < r && last[j] >= 0 && abs(last[j] - d) <= t;
      const int res = (d >= 0 && hit) ? -1 : d;
#pragma unroll
      for (int j = R - 1; j > 0; --j) last[j] = last[j - 1];
      last[0] = res;
      out[(size_t)(b0 + i) * step] = (int16_t)res;
    }
  }
}

template <int R>
__device__ __forceinline__ void redun_passes(const Frame& F) {
  const Geometry g = F.g;
  const int r = F.p.redun_max_dist, t = F.p.redun_threshold;
  const int16_t* inc = F.dcan_incon;
  int16_t* vert = F.dcan_vert;
  int16_t* fin = F.dcan_final;
  for (int k = threadIdx.x; k < g.lw; k += blockDim.x)
    redun_line<R>(inc + k, vert + k, g.lh, (size_t)g.lw, r, t);
  __syncthreads();
  for (int l = threadIdx.x; l < g.lh; l += blockDim.x)
    redun_line<R>(vert + (size_t)l * g.lw, fin + (size_t)l * g.lw, g.lw, 1, r, t);
}

__device__ __forceinline__ void redun_body(const Frame& F, int lb) {
  (void)lb;
  const int r = F.p.redun_max_dist;
  if (r <= 4)
    redun_passes<4>(F);
  else if (r <= 8)
    redun_passes<8>(F);
  else
    redun_passes<16>(F);
}

// ---------------------------------------------------------------------------
// Support lists per lattice row, one wavefront per row (for the mesh step;
// host-mapped memory when the host triangulates), plus the grid vectors.
//  * left list: the row's survivors in lattice order, packed u | d << 16;
//    with down-sampling by k (Section VII-B) only the survivors whose index
//    in the whole lattice-order list is a multiple of k (the row first counts
//    the survivors of the rows above);
//  * right list (each point seen from the right view at (u - d, v); on
//    collisions the larger d, the nearer surface, wins): an LDS slot per
//    right-view column takes atomicMax of d, then the occupied slots in
//    column order;
//  * grid vectors (Fig. 2; one-hot, Section VI-D): bits d-1..d+1 of every
//    list point are OR-ed into its region's mask, per view;
//  * the row's support-search evaluation count.
// ---------------------------------------------------------------------------
// Sets the grid bits d - 1 .. d + 1 (within the disparity range) of a cell:
// one atomic OR per 32-bit word they touch (one, or two across a word edge).
// The cell's bit range (smallest and largest set bit) follows by one atomic
// minimum and maximum.
__device__ __forceinline__ void grid_mark(uint32_t* cell, int32_t* range, int d,
                                          const KParams& p) {
  const int lo = max(d - 1, p.dmin) - p.dmin, hi = min(d + 1, p.dmax) - p.dmin;
  const int w0 = lo >> 5, w1 = hi >> 5;
  const uint32_t top0 = w1 == w0 ? hi & 31 : 31;
  atomicOr(&cell[w0], (top0 == 31 ? 0xFFFFFFFFu : ((2u << top0) - 1u)) & ~((1u << (lo & 31)) - 1u));
  if (w1 != w0) atomicOr(&cell[w1], (2u << (hi & 31)) - 1u);
  atomicMin(&range[0], lo);
  atomicMax(&range[1], hi);
}

__device__ __forceinline__ void rows_body(const Frame& F, int lb) {
  const Geometry g = F.g;
  const KParams p = F.p;
  int32_t* slot = reinterpret_cast<int32_t*>(dyn_smem);  // one per image column
  const int l = lb, lane = threadIdx.x;
  const int v = g.lv0 + l * g.step;
  const int grow = (v / p.grid_size) * g.gw;
  int32_t* hrowL = F.rowsL;
  int32_t* hrowR = F.rowsR;
  uint32_t* gridL = F.gridL;
  uint32_t* gridR = F.gridR;
  for (int x = lane; x < g.w; x += 64) slot[x] = -1;
  __syncthreads();
  int nL = 0, nV = 0, ev = 0;
  const int16_t* fin = F.dcan_final;
  const int16_t* frow = fin + (size_t)l * g.lw;
  const int32_t* erow = F.evals + (size_t)l * g.lw;
  const int ks = p.subsample;
  int base = 0;  // survivors in the rows above (global list index of this row's first)
  if (ks > 1) {
    const int n = l * g.lw;
    int c = 0;
    for (int i = lane; i < n; i += 64) c += fin[i] >= 0 ? 1 : 0;
    base = wave_sum_i32(c);
  }
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int k0 = 0; k0 < g.lw; k0 += 64) {
    const int k = k0 + lane;
    const int dv = k < g.lw ? frow[k] : -1;
    ev += k < g.lw ? erow[k] : 0;
    const unsigned long long vm = __ballot(dv >= 0);
    const int gi = base + nV + __popcll(vm & below);
    const int d = (dv >= 0 && (ks <= 1 || gi % ks == 0)) ? dv : -1;
    nV += __popcll(vm);
    const unsigned long long m = __ballot(d >= 0);
    if (d >= 0) {
      const int u = g.lu0 + k * g.step;
      const int pos = nL + __popcll(m & below);
      hrowL[(size_t)l * g.lw + pos] = u | (d << 16);
      atomicMax(&slot[u - d], d);
      const int cell = grow + u / p.grid_size;
      grid_mark(gridL + cell * g.gwords, F.grangeL + 2 * cell, d, p);
    }
    nL += __popcll(m);
  }
  __syncthreads();
  int nR = 0;
  for (int x0 = 0; x0 < g.w; x0 += 64) {
    const int x = x0 + lane;
    const int d = x < g.w ? slot[x] : -1;
    const unsigned long long m = __ballot(d >= 0);
    if (d >= 0) {
      const int pos = nR + __popcll(m & ((1ull << lane) - 1ull));
      hrowR[(size_t)l * g.lw + pos] = x | (d << 16);
      const int cell = grow + x / p.grid_size;
      grid_mark(gridR + cell * g.gwords, F.grangeR + 2 * cell, d, p);
    }
    nR += __popcll(m);
  }
  ev = wave_sum_i32(ev);
  if (lane == 0) {
    F.cnt[l] = nL;
    F.cnt[g.lh + l] = nR;
    F.cnt[2 * g.lh + l] = ev;
  }
}

// ---------------------------------------------------------------------------
// Prior raster (Section VI-D: the mesh becomes an image-sized matrix of
// priors). A pixel takes the smallest canonical rank of the triangles whose
// closed area contains it, or kNoOwner. One workgroup owns a band of pixel
// rows of one view and keeps its owners in an LDS tile: it gathers the
// triangles whose rows overlap the band (canonical order sorts triangles by
// their top vertex, so the scan stops at the first triangle starting below
// the band), computes the exact integer span of each of their band rows from
// the three edge functions, spreads all span pixels evenly over its
// threads, resolves each pixel with an LDS atomicMin, and finally writes the
// whole tile with coalesced stores, together with each pixel's prior
// disparity (the owning plane's mean). Every pixel is written.
// ---------------------------------------------------------------------------
// floor(a / b) for any int a and 0 < b <= 2^13, by a correctly rounded fp64
// division (no integer division sequence): a non-integral quotient lies at
// least 1/b >= 2^-13 from the nearest integer, and the rounding error of a
// quotient below 2^31 is at most 2^-22, so rounding cannot carry it across
// an integer.
__device__ __forceinline__ int floordiv_pos(int a, int b) {
  return (int)floor(__ddiv_rn((double)a, (double)b));
}

// Byte offset of record t (24 B each; a view has at most 2 * 8192^2 + 2
// triangles, so t * 24 < 2^32) as (t + 2t) << 3: two full-rate operations where a 32-bit multiply issues
// at a quarter of the rate. The addition is written out so that it is not
// folded back into a multiply.
__device__ __forceinline__ uint32_t times24(int t) {
  uint32_t x;
  asm("v_lshl_add_u32 %0, %1, 1, %1" : "=v"(x) : "v"(t));
  return x << 3;
}

// Narrows [lo, hi] to the u with k*u + c >= 0. One division whatever the
// sign of k, and selects after it: a wavefront's lanes see both signs, and a
// branch per sign would run both division sequences.
__device__ __forceinline__ void clip_edge(int k, int c, int* lo, int* hi) {
  const int x = floordiv_pos(c, k < 0 ? -k : (k > 0 ? k : 1));
  const int nlo = max(*lo, -x);  // k > 0: u >= ceil(-c / k) = -floor(c / k)
  const int nhi = min(*hi, x);   // k < 0: u <= floor(c / -k)
  if (k > 0)
    *lo = nlo;
  else if (k < 0)
    *hi = nhi;
  else if (c < 0)
    *hi = *lo - 1;
}

constexpr int kBandRowsMax = 4;
// per-wave span table in LDS: pixel offsets of the lanes, one packed span
// (first column | length << 16; 0 when empty) per lane and band row, ranks
constexpr int kWaveSpan = 64 * (2 + kBandRowsMax);

// Two workgroup sizes: 1024 threads (single frames whose bands all fit on
// the CUs at once), 256 threads (more bands per CU: larger frames, batches).
template <int kRasterThreads>
__device__ __forceinline__ void raster_body(const Frame& F, int lb) {
  // triangles per thread and gather step: 2048 per step with 1024 threads,
  // 768 with 256
  constexpr int kRasterScan = kRasterThreads == 1024 ? 2 : 3;
  constexpr int kRasterOut = 2048 / kRasterThreads < 4 ? 4 : 2048 / kRasterThreads;
  constexpr int kRasterWaves = kRasterThreads / 64;
  // ranks of gathered triangles per pass (a band of a few rows overlaps tens
  // of triangles; a pass ends when the list could overflow). The 256-thread
  // variant keeps its static LDS at 10 KB: with the 10 KB owner tile of a
  // 640-wide band of four rows a workgroup takes 20 KB, and eight of them
  // (32 wavefronts) share a CU's 160 KB.
  constexpr int kRasterSmall = 10240 - 4 * kRasterWaves * (kWaveSpan + 1) - 8;
  constexpr int kRasterList = kRasterThreads == 1024 ? 4096 : kRasterSmall / 4;
  static_assert(kRasterScan * kRasterThreads <= kRasterList, "a gather step must fit the list");
  int32_t* const tile = reinterpret_cast<int32_t*>(dyn_smem);  // band rows x width
  __shared__ int32_t rlist[kRasterList];
  __shared__ int32_t wspan[(kRasterThreads / 64) * kWaveSpan];
  __shared__ int32_t s_wtot[kRasterThreads / 64];  // span pixels per wave
  __shared__ int s_cnt, s_done;
  static_assert(kRasterThreads == 1024 ||
                    sizeof(rlist) + sizeof(wspan) + sizeof(s_wtot) + 2 * sizeof(int) == 10240,
                "static LDS of the 256-thread raster");
  const Geometry g = F.g;
  const int band_rows = F.raster_rows;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nb = cdivd(g.h, band_rows);
  const int view = lb >= nb ? 1 : 0, band = lb - view * nb;
  const int v0 = band * band_rows, v1 = min(g.h - 1, v0 + band_rows - 1);
  const int rows = v1 - v0 + 1;
  const int ntL = F.hdr->ntri[0], nt = view ? F.hdr->ntri[1] : ntL;
  const RasterTri* vt = F.tris + (view ? ntL : 0);
  // the view's records as a wavefront-uniform base with 32-bit byte offsets
  // (24 B per record)
  const uint8_t* const vtb = reinterpret_cast<const uint8_t*>(vt);
  for (int i = tid; i < rows * g.w; i += kRasterThreads) tile[i] = kNoOwner;
  int r0 = 0;
  for (;;) {
    // gather the ranks of the next triangles whose rows overlap the band
    if (tid == 0) {
      s_cnt = 0;
      s_done = 0;
    }
    __syncthreads();
    int cnt = 0, done = 0;
    while (r0 < nt) {
      int16_t tv[kRasterScan][3];
#pragma unroll
      for (int k = 0; k < kRasterScan; ++k) {
        const int r = min(r0 + k * kRasterThreads + tid, nt - 1);  // in bounds: nt > 0 here
        const RasterTri* T = reinterpret_cast<const RasterTri*>(vtb + times24(r));
        tv[k][0] = T->v[0];
        tv[k][1] = T->v[1];
        tv[k][2] = T->v[2];
      }
#pragma unroll
      for (int k = 0; k < kRasterScan; ++k) {
        const int r = r0 + k * kRasterThreads + tid;
        int vmin = min((int)tv[k][0], min((int)tv[k][1], (int)tv[k][2]));
        int vmax = max((int)tv[k][0], max((int)tv[k][1], (int)tv[k][2]));
        if (r >= nt) {  // past the list: neither listed nor a stop (v0 >= 0)
          vmin = 0;
          vmax = -1;
        }
        if (vmin > v1)
          s_done = 1;  // so does every later triangle
        else if (vmax >= v0)
          rlist[atomicAdd(&s_cnt, 1)] = r;
      }
      r0 += kRasterScan * kRasterThreads;
      __syncthreads();
      cnt = s_cnt;
      done = s_done;
      __syncthreads();
      if (done || cnt > kRasterList - kRasterScan * kRasterThreads) break;
    }
    // rasterise the gathered triangles into the tile: consecutive entries go
    // to consecutive lanes, so only the first ceil(cnt / 64) waves work out
    // spans (a wave's span setup costs the same for 1 entry as for 64), and
    // every thread then takes an equal share of all span pixels
    for (int e0 = 0; e0 < cnt; e0 += kRasterThreads) {
      const int e = e0 + tid;
      int lo[kBandRowsMax], len[kBandRowsMax], tot = 0, rank = 0;
#pragma unroll
      for (int q = 0; q < kBandRowsMax; ++q) {
        lo[q] = 0;
        len[q] = 0;
      }
      if (e < cnt) {
        rank = rlist[e];
        const RasterTri T = *reinterpret_cast<const RasterTri*>(vtb + times24(rank));
        // vertices lie in the image; the clamp only keeps every write inside it
        const int umin = max(0, min((int)T.u[0], min((int)T.u[1], (int)T.u[2])));
        const int umax = min(g.w - 1, max((int)T.u[0], max((int)T.u[1], (int)T.u[2])));
        const int vmin = min((int)T.v[0], min((int)T.v[1], (int)T.v[2]));
        const int vmax = max((int)T.v[0], max((int)T.v[1], (int)T.v[2]));
#pragma unroll
        for (int q = 0; q < kBandRowsMax; ++q) {
          const int v = v0 + q;
          if (q >= rows || v < vmin || v > vmax) continue;
          int slo = umin, shi = umax;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const int au = T.u[k], av = T.v[k], bu = T.u[(k + 1) % 3], bv = T.v[(k + 1) % 3];
            // orient(A, B, (u, v)) = (av - bv) * u + (bu - au)(v - av) + (bv - av) au
            clip_edge(av - bv, (bu - au) * (v - av) + (bv - av) * au, &slo, &shi);
          }
          lo[q] = slo;
          len[q] = max(0, shi - slo + 1);
          tot += len[q];
        }
      }
      // the spans of all waves, wave by wave, lane by lane and row by row,
      // form one pixel range; each thread takes a contiguous share of it,
      // finds its first span by a search over the waves' and the lanes'
      // offsets and walks on from there
      const int incl = wave_scan_incl(tot);
      int32_t* W = wspan + wid * kWaveSpan;  // [offsets 64][spans 64x4][rank 64]
      W[lane] = incl - tot;
#pragma unroll
      for (int q = 0; q < kBandRowsMax; ++q)  // a non-empty span lies in the row: 0 <= lo < w
        W[64 + 4 * lane + q] = len[q] > 0 ? lo[q] | (len[q] << 16) : 0;
      W[320 + lane] = rank;
      if (lane == 63) s_wtot[wid] = incl;
      __syncthreads();
      int P = 0;
#pragma unroll
      for (int w = 0; w < kRasterWaves; ++w) P += s_wtot[w];
      const int share = (P + kRasterThreads - 1) / kRasterThreads;
      int i = tid * share;
      const int iend = min(P, i + share);
      if (i < iend) {
        int w = 0, wbase = 0;  // the wave holding pixel i
        while (wbase + s_wtot[w] <= i) wbase += s_wtot[w++];
        const int32_t* Wt = wspan + w * kWaveSpan;
        const int li = i - wbase;
        int a = 0, b = 63;  // last lane whose pixels start at or before li
        while (a < b) {
          const int mid = (a + b + 1) >> 1;
          if (Wt[mid] <= li) a = mid; else b = mid - 1;
        }
        int j = a, off = li - Wt[a], q = 0, sp;
        while (off >= ((sp = Wt[64 + 4 * j + q]) >> 16)) {
          off -= sp >> 16;
          ++q;
        }
        // the rest of the current span from px on, then span after span
        int32_t* px = tile + q * g.w + (sp & 0xFFFF) + off;
        int R = Wt[320 + j];
        int left = (sp >> 16) - off;  // >= 1
        int n = iend - i;                       // >= 1
        // R comes from an LDS read: wait for it once per span, not before
        // every atomic of the loop (the atomics return nothing, so nothing
        // else in the loop waits)
        asm volatile("" ::"v"(R));
        for (;;) {
          atomicMin(px, R);
          if (--n == 0) break;
          ++px;
          if (--left == 0) {
            do {  // on to the next non-empty span (one exists: pixels remain)
              if (++q == kBandRowsMax) {
                q = 0;
                if (++j == 64) {
                  j = 0;
                  Wt += kWaveSpan;
                }
              }
              sp = Wt[64 + 4 * j + q];
            } while (sp == 0);
            px = tile + q * g.w + (sp & 0xFFFF);
            left = sp >> 16;
            R = Wt[320 + j];
            asm volatile("" ::"v"(R));
          }
        }
      }
      __syncthreads();  // the span tables are written again by the next entries
    }
    if (done || r0 >= nt) break;
  }
  __syncthreads();
  // owners and the prior disparity of every pixel: the owning triangle's
  // plane mean ((a*u) + (b*v)) + c in FP32 without contraction, rounded as
  // floor(mean + 0.5) and clamped to the disparity range; -1 without owner
  int32_t* ownL = F.ownerL;
  int32_t* ownR = F.ownerR;
  int16_t* dplL = F.dplaneL;
  int16_t* dplR = F.dplaneR;
  // band rows as wavefront-uniform bases with 32-bit byte offsets
  uint8_t* const owner = reinterpret_cast<uint8_t*>((view ? ownR : ownL) + (size_t)v0 * g.w);
  uint8_t* const dpl = reinterpret_cast<uint8_t*>((view ? dplR : dplL) + (size_t)v0 * g.w);
  const int dmin = F.p.dmin, dmax = F.p.dmax;
  const int npx = rows * g.w;
  // a thread's pixels are tid, tid + T, tid + 2T, ... (T threads): the column
  // u and band row q of each follow from the previous by adding T mod w and
  // T div w and one wrap (row of a band index by the width multiplier, exact
  // for T * w < 2^40)
  const int qstep = (int)(((uint64_t)kRasterThreads * g.rowmul) >> 40);
  const int ustep = kRasterThreads - qstep * g.w;
  int q = (int)(((uint64_t)tid * g.rowmul) >> 40), u = tid - q * g.w;
  // kRasterOut pixels per thread at a time: their plane loads (from an
  // in-bounds triangle even without an owner) are all in flight together
  for (int i0 = 0; i0 < npx; i0 += kRasterOut * kRasterThreads) {
    int o[kRasterOut];
    float a[kRasterOut], b[kRasterOut], c[kRasterOut];
#pragma unroll
    for (int k = 0; k < kRasterOut; ++k) {
      const int i = i0 + k * kRasterThreads + tid;
      o[k] = i < npx ? tile[i] : kNoOwner;
      const int t = (o[k] != kNoOwner) ? o[k] : 0;
      const RasterTri* T = reinterpret_cast<const RasterTri*>(vtb + times24(t));
      a[k] = T->a;
      b[k] = T->b;
      c[k] = T->c;
    }
#pragma unroll
    for (int k = 0; k < kRasterOut; ++k) {
      const int i = i0 + k * kRasterThreads + tid;
      if (i < npx) {
        int dp = -1;
        if (o[k] != kNoOwner) {
          const float mu = __fadd_rn(
              __fadd_rn(__fmul_rn(a[k], (float)u), __fmul_rn(b[k], (float)(v0 + q))), c[k]);
          const float f = floorf(__fadd_rn(mu, 0.5f));
          dp = f < (float)dmin ? dmin : (f > (float)dmax ? dmax : (int)f);
        }
        // the owner map is read by no later stage: it goes straight to HBM
        // (non-temporal), leaving the caches to the prior and the descriptors
        __builtin_nontemporal_store(o[k], reinterpret_cast<int32_t*>(owner + (uint32_t)i * 4u));
        *reinterpret_cast<int16_t*>(dpl + (uint32_t)i * 2u) = (int16_t)dp;
      }
      u += ustep;
      q += qstep;
      if (u >= g.w) {
        u -= g.w;
        ++q;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Dense matching (Section III-A, Fig. 1(h)). One thread per pixel; a block is
// a 256-pixel row segment of R rows of one view (R = 1, 2 or 4: the tile
// variant), views interleaved, with the other view's reachable descriptors
// staged in LDS. The prior disparity comes from the raster (the owning
// plane's rounded mean, -1 without a plane). Candidates: the plane window
// |d - d_plane| <= sradius and the grid region's one-hot mask (every d with
// full_search), restricted to partners with a defined descriptor. Energy:
// descriptor SAD (or census Hamming distance) plus the prior table at
// |d - d_plane|. Argmin by packed key (energy << 8 | d - dmin).
//
// Two facts keep a pixel's work short:
//  * window fast path: with sradius 2 and the whole window admissible for
//    every pixel of a wavefront, the five candidates of a pixel sit at fixed
//    offsets from one LDS address and their priors are the constants
//    prior[2], prior[1], prior[0], prior[1], prior[2];
//  * grid bits inside the window add nothing. The rows stage records each
//    region's smallest and largest set bit; a pixel whose admissible grid
//    bits all lie in its window never reads the mask words (the common case
//    on a smooth surface). The others walk the mask words for the bits
//    outside the window.
// A pixel's evaluation count is |window| + |grid bits outside it|.
// ---------------------------------------------------------------------------
// Dense descriptors: 16-byte gradient descriptors compared by SAD, or 64-bit
// census descriptors (Section VI-A) compared by Hamming distance; texture is
// the distance from the flat descriptor or the number of set bits. cost(a,
// b, acc) = acc + distance.
struct GradDense {
  typedef uint4 T;
  static constexpr uint32_t kBytes = 16;
  __device__ __forceinline__ static T load(const uint8_t* base, size_t px) {
    return ld16(base + px * 16);
  }
  // column c of a row whose first descriptor is at row (a wavefront-uniform
  // base); NT: a non-temporal load (the line is not kept in the caches)
  template <bool NT = false>
  __device__ __forceinline__ static T load_col(const uint8_t* row, uint32_t c) {
    if constexpr (NT) {
      typedef unsigned int v4u __attribute__((ext_vector_type(4)));
      const v4u x = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(row + c * 16u));
      return make_uint4(x.x, x.y, x.z, x.w);
    } else {
      return ld16(row + c * 16u);
    }
  }
  __device__ __forceinline__ static uint32_t cost(const T a, const T b, uint32_t acc) {
    uint32_t s = __builtin_amdgcn_sad_u8(a.x, b.x, acc);
    s = __builtin_amdgcn_sad_u8(a.y, b.y, s);
    s = __builtin_amdgcn_sad_u8(a.z, b.z, s);
    return __builtin_amdgcn_sad_u8(a.w, b.w, s);
  }
  __device__ __forceinline__ static uint32_t texture(const T a) { return texture16(a); }
};

struct CensusDense {
  typedef uint64_t T;
  static constexpr uint32_t kBytes = 8;
  __device__ __forceinline__ static T load(const uint8_t* base, size_t px) {
    return reinterpret_cast<const uint64_t*>(base)[px];
  }
  template <bool NT = false>
  __device__ __forceinline__ static T load_col(const uint8_t* row, uint32_t c) {
    const uint64_t* q = reinterpret_cast<const uint64_t*>(row + c * 8u);
    if constexpr (NT)
      return __builtin_nontemporal_load(q);
    else
      return *q;
  }
  __device__ __forceinline__ static uint32_t cost(const T a, const T b, uint32_t acc) {
    return (uint32_t)__popcll(a ^ b) + acc;
  }
  __device__ __forceinline__ static uint32_t texture(const T a) { return (uint32_t)__popcll(a); }
};

// A workgroup matches kDenseSeg consecutive pixels of R rows of one view.
// The other view's descriptors of every column the segment can reach
// (kDenseSeg + D - 1 per row) are staged in LDS once with coalesced loads, so
// each candidate costs an LDS read instead of a global gather.
constexpr int kDenseSeg = 256;
constexpr int kDenseRowsOf[kDenseVariants] = {1, 2, 4};
constexpr int kWinBatch = 5;   // window candidates per step of the general window loop
constexpr int kGridBatch = 2;  // grid candidates per step of the mask walk
constexpr int kDenseStage = kDenseSeg + kMaxD - 1;
// Prior table in LDS for the general paths, mirrored about its centre so
// that a candidate's entry is one add away, with the energy offset lut_bias
// already added: s_lut[kLutC + k] = s_lut[kLutC - k] = lut[k] + lut_bias (the
// prior of |d - dp| = k < D), then kMaxD entries lut_bias (pixels without a
// plane).
constexpr int kLutC = kMaxD - 1;
constexpr int kLutZero = 2 * kLutC + 1;
constexpr int kLutSize = kLutZero + kMaxD;

__host__ __device__ __forceinline__ int dense_segments(const Geometry& g) {
  return cdivd(g.w, kDenseSeg);
}

__device__ __forceinline__ int ctz_any(uint32_t m) { return __builtin_ctz(m); }
__device__ __forceinline__ int ctz_any(uint64_t m) { return __builtin_ctzll(m); }

__device__ __forceinline__ uint32_t bits32_between(int a, int b) {
  a = max(a, 0);
  b = min(b, 31);
  if (a > b) return 0u;
  const uint32_t hi = b == 31 ? 0xFFFFFFFFu : ((2u << b) - 1u);
  return hi & ~((1u << a) - 1u);
}

// x / grid_size for 0 <= x < 2^31 / grid_size.
__device__ __forceinline__ int grid_div(int x, const Geometry& g) {
  return (int)__umulhi(2u * (uint32_t)x, g.gdiv);
}

// The priors of the window fast path, energy bias included: prior[0..2].
struct WinPrior {
  uint32_t p0, p1, p2;
};

// Argmin over the candidates of one pixel (descriptors defined there); st
// holds the other view's descriptors of columns base .. base + n - 1; s_lut
// is the mirrored prior table (kLutC, kLutZero); gmin / gmax the pixel's
// grid region's bit range and cellw its mask words (global memory).
template <class DD, bool right>
__device__ __forceinline__ int dense_pixel(const Geometry& g, const KParams& p, int u, int dp,
                                           int gmin, int gmax, const uint32_t* cellw,
                                           bool has_list, const typename DD::T s,
                                           const typename DD::T* st, int base,
                                           const int32_t* s_lut, const WinPrior& wp, int* cnt) {
  const int lim = (right ? (g.w - 3 - u) : (u - 2)) - p.dmin;  // largest admissible d-dmin
  if ((int)DD::texture(s) < p.match_texture || lim < 0) return -1;
  const int top = min(lim, p.D - 1);
  const int c = dp - p.dmin;  // the plane disparity in d - dmin units (dp in [dmin, dmax])
  int wlo = 1, whi = 0;       // plane window clipped to [0, top]; empty without a plane
  if (dp >= 0) {
    wlo = max(c - p.sradius, 0);
    whi = min(c + p.sradius, top);
  }
  const int slot0 = (right ? u + p.dmin : u - p.dmin) - base;
  const int dir = right ? 1 : -1;
  uint32_t best = 0xFFFFFFFFu;
  int n = max(0, whi - wlo + 1);
  const bool full = dp >= 0 && p.sradius == 2 && c >= 2 && c + 2 <= top;
  if (__all(full)) {
    // slots c-2 .. c+2 from one address; priors are constants
    const typename DD::T* q = st + (slot0 + dir * (c - 2));
    typename DD::T o[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) o[t] = q[dir * t];
    const uint32_t pr[5] = {wp.p2, wp.p1, wp.p0, wp.p1, wp.p2};
#pragma unroll
    for (int t = 0; t < 5; ++t)
      best = min(best, (DD::cost(s, o[t], pr[t]) << 8) | (uint32_t)(c - 2 + t));
  } else if (dp >= 0) {
    // entry of candidate dd (d = dmin + dd): kLutC + dd - c, inside the table
    const int lidx = kLutC - c;
    // kWinBatch candidates at a time (the last batch repeats whi), every LDS
    // read of a batch issued before its arithmetic
    for (int b = wlo; b <= whi; b += kWinBatch) {
      int dd[kWinBatch];
      typename DD::T o[kWinBatch];
      int lv[kWinBatch];
#pragma unroll
      for (int t = 0; t < kWinBatch; ++t) dd[t] = min(b + t, whi);
#pragma unroll
      for (int t = 0; t < kWinBatch; ++t) {
        o[t] = st[slot0 + dir * dd[t]];
        lv[t] = s_lut[dd[t] + lidx];
      }
#pragma unroll
      for (int t = 0; t < kWinBatch; ++t) {
        const uint32_t E = DD::cost(s, o[t], (uint32_t)lv[t]);
        best = min(best, (E << 8) | (uint32_t)dd[t]);
      }
    }
  }
  // grid bits outside the window (every admissible d with full_search)
  const int ghi = min(gmax, top);  // the region's largest admissible bit
  const bool inside = dp >= 0 && gmin >= wlo && ghi <= whi;
  const int lidx = dp >= 0 ? kLutC - c : kLutZero;
  if (!p.full_search && has_list && !inside && gmin <= ghi && ghi - gmin < 64) {
    // the region's admissible bits in one 64-bit word, bit 0 = gmin (the
    // usual case: a region's support disparities lie close together)
    const int j0 = gmin >> 5, sh = gmin & 31, jl = g.gwords - 1;
    const uint32_t w0 = cellw[j0], w1 = cellw[min(j0 + 1, jl)], w2 = cellw[min(j0 + 2, jl)];
    uint64_t m = ((uint64_t)__builtin_amdgcn_alignbit(w2, w1, sh) << 32) |
                 __builtin_amdgcn_alignbit(w1, w0, sh);
    const int span = ghi - gmin;  // bits 0 .. span are admissible
    m &= span == 63 ? ~0ull : ((2ull << span) - 1ull);
    const int a = max(wlo - gmin, 0), b = min(whi - gmin, 63);  // the window's bits
    if (a <= b) m &= ~((b == 63 ? ~0ull : ((2ull << b) - 1ull)) & ~((1ull << a) - 1ull));
    n += __popcll(m);
    // the bits come two at a time; when no lane of the wavefront that walks
    // its bits has one past bit 31 (most of them: a region's support
    // disparities lie close together), from a 32-bit mask, whose lowest bit
    // costs one instruction instead of four
    auto walk = [&](auto mask) {
      while (mask) {
        int dd[kGridBatch];
        dd[0] = gmin + ctz_any(mask);
        mask &= mask - 1u;
#pragma unroll
        for (int t = 1; t < kGridBatch; ++t) {
          dd[t] = mask ? gmin + ctz_any(mask) : dd[0];
          mask &= mask - 1u;
        }
        typename DD::T o[kGridBatch];
        int lv[kGridBatch];
#pragma unroll
        for (int t = 0; t < kGridBatch; ++t) {
          o[t] = st[slot0 + dir * dd[t]];
          lv[t] = s_lut[dd[t] + lidx];
        }
#pragma unroll
        for (int t = 0; t < kGridBatch; ++t) {
          const uint32_t E = DD::cost(s, o[t], (uint32_t)lv[t]);
          best = min(best, (E << 8) | (uint32_t)dd[t]);
        }
      }
    };
    if (__all((uint32_t)(m >> 32) == 0u))
      walk((uint32_t)m);
    else
      walk(m);
  } else if (p.full_search || (has_list && gmax >= 0 && !inside && gmin <= ghi)) {
    const int nw = (top >> 5) + 1;  // 32-bit words in play
    // every word in play is loaded at once (one memory round trip)
    uint32_t words[kMaxD / 32];
#pragma unroll
    for (int j = 0; j < kMaxD / 32; ++j) words[j] = cellw[min(j, nw - 1)];
#pragma unroll
    for (int j = 0; j < kMaxD / 32; ++j) {
      if (j >= nw) break;
      const uint32_t grid = p.full_search ? 0xFFFFFFFFu : words[j];
      if (grid == 0u) continue;
      const int wb = 32 * j;
      uint32_t m = grid & bits32_between(0, top - wb) & ~bits32_between(wlo - wb, whi - wb);
      n += __popc(m);
      while (m) {
        int dd[kGridBatch];
        dd[0] = wb + __builtin_ctz(m);
        m &= m - 1u;
#pragma unroll
        for (int t = 1; t < kGridBatch; ++t) {
          dd[t] = m ? wb + __builtin_ctz(m) : dd[0];
          m &= m - 1u;
        }
        typename DD::T o[kGridBatch];
        int lv[kGridBatch];
#pragma unroll
        for (int t = 0; t < kGridBatch; ++t) {
          o[t] = st[slot0 + dir * dd[t]];
          lv[t] = s_lut[dd[t] + lidx];
        }
#pragma unroll
        for (int t = 0; t < kGridBatch; ++t) {
          const uint32_t E = DD::cost(s, o[t], (uint32_t)lv[t]);
          best = min(best, (E << 8) | (uint32_t)dd[t]);
        }
      }
    }
  }
  *cnt += n;
  return best != 0xFFFFFFFFu ? p.dmin + (int)(best & 0xFFu) : -1;
}

// Row of staged element i when each of the block's R rows holds nc elements:
// i / nc for i < R * nc, by comparisons instead of a division.
template <int R>
__device__ __forceinline__ int dense_row_of(int i, int nc) {
  int r = 0;
#pragma unroll
  for (int rr = 1; rr < R; ++rr) r += i >= rr * nc ? 1 : 0;
  return r;
}

// One workgroup: R rows x kDenseSeg columns of one view, a thread per column
// and row. Every global load (the other view's reachable descriptors, staged
// in LDS; the own descriptor, prior and grid-region bit range of each pixel)
// is issued before the one barrier, so a wave waits on memory once; only the
// pixels whose grid bits reach outside their window read mask words after
// it. The view is a template argument: the search direction is then a
// constant in every candidate's address.
template <class DD, bool right, int R, bool NT>
__device__ __forceinline__ void dense_rows(const Frame& F, const Geometry& g, const KParams& p,
                                           int v0, int u0, int32_t* s_lut,
                                           typename DD::T* st, int* cnt) {
  const int32_t* lut = F.lut;
  // fields copied to locals first, so that no pointer is selected by
  // indexing the frame struct (which would put it in scratch memory)
  const uint8_t* descL = F.descL;
  const uint8_t* descR = F.descR;
  const int16_t* dplL = F.dplaneL;
  const int16_t* dplR = F.dplaneR;
  const uint32_t* gridL = F.gridL;
  const uint32_t* gridR = F.gridR;
  const int32_t* grL = F.grangeL;
  const int32_t* grR = F.grangeR;
  int16_t* rawL = F.rawL;
  int16_t* rawR = F.rawR;
  const uint8_t* self_desc = right ? descR : descL;
  const uint8_t* other_desc = right ? descL : descR;
  const int16_t* dplane = right ? dplR : dplL;
  const uint32_t* grid = right ? gridR : gridL;
  const int32_t* grange = right ? grR : grL;
  int16_t* raw = right ? rawR : rawL;
  const bool has_list = F.hdr->n[0] > 0;
  // other-view columns a pixel of this segment can reach
  const int base = right ? u0 + p.dmin : u0 - p.dmax;
  const int n = kDenseSeg + p.D - 1;
  const int c0 = max(0, base), c1 = min(g.w - 1, base + n - 1);
  const int u = u0 + (int)threadIdx.x;
  const bool in_u = u < g.w;
  // issue every global load first, each from an in-bounds address whether
  // or not its value is used (a conditional load would make the compiler
  // wait for it at the branch join): the reachable other-view columns of the
  // block's rows (at most kDenseStage per row: two per thread and row, from
  // the row's uniform base; rows past the frame repeat its last row), the
  // prior table, then each pixel's prior, descriptor and region bit range
  typename DD::T sv[R * 2];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint8_t* row = other_desc + (size_t)min(v0 + r, g.h - 1) * g.w * DD::kBytes;
#pragma unroll
    for (int k = 0; k < 2; ++k)
      sv[2 * r + k] = DD::template load_col<NT>(row, (uint32_t)min(c0 + (int)threadIdx.x + 256 * k, c1));
  }
  int32_t lv[3];  // the mirrored table's entries tid, tid + 256, tid + 512
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int i = (int)threadIdx.x + 256 * q;
    const int32_t x = lut[min(abs(i - kLutC), p.D - 1)];
    lv[q] = (i <= 2 * kLutC ? x : 0) + p.lut_bias;
  }
  WinPrior wp;
  wp.p0 = (uint32_t)(lut[0] + p.lut_bias);
  wp.p1 = (uint32_t)(lut[min(1, p.D - 1)] + p.lut_bias);
  wp.p2 = (uint32_t)(lut[min(2, p.D - 1)] + p.lut_bias);
  const int uc = min(u, g.w - 1);
  const int cu = grid_div(uc, g);
  int dpv[R], cell[R];
  typename DD::T s[R];
  int2 rng[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int vc = min(v0 + r, g.h - 1);
    const int16_t* dprow = dplane + (size_t)vc * g.w;
    if constexpr (NT)
      dpv[r] = __builtin_nontemporal_load(&dprow[(uint32_t)uc]);
    else
      dpv[r] = dprow[(uint32_t)uc];
    s[r] = DD::template load_col<NT>(self_desc + (size_t)vc * g.w * DD::kBytes, (uint32_t)uc);
    const int crow = grid_div(vc, g) * g.gw;  // wavefront-uniform
    cell[r] = crow + cu;
    rng[r] = (reinterpret_cast<const int2*>(grange) + crow)[(uint32_t)cu];
  }
  // columns past c1 go to a spare slot after the rows (no branch)
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int c = c0 + (int)threadIdx.x + 256 * k;
      st[c <= c1 ? r * kDenseStage + (c - base) : R * kDenseStage] = sv[2 * r + k];
    }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int i = (int)threadIdx.x + 256 * q;
    if (i < kLutSize) s_lut[i] = lv[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int v = v0 + r;
    if (!in_u || v >= g.h) continue;
    int res = -1;
    if (u >= 2 && u <= g.w - 3 && v >= 2 && v <= g.h - 3)
      res = dense_pixel<DD, right>(g, p, u, dpv[r], rng[r].x, rng[r].y,
                                   grid + (size_t)cell[r] * g.gwords, has_list, s[r],
                                   st + r * kDenseStage, base, s_lut, wp, cnt);
    raw[(size_t)v * g.w + u] = (int16_t)res;
  }
}

// NT: the descriptors and the prior map are read with non-temporal loads (a
// batch whose descriptors were written past the last-level cache: no line
// of the reused descriptor buffers stays cached for the next batch's
// non-temporal writes to meet).
template <int R, bool NT = false>
__device__ __forceinline__ void dense_body(const Frame& F, int lb) {
  __shared__ int32_t s_lut[kLutSize];  // mirrored prior table, then zeros
  __shared__ int s_cnt[4];
  __shared__ uint4 s_stage[R * kDenseStage + 1];  // + a spare slot for unused lanes
  const Geometry g = F.g;
  const KParams p = F.p;
  const bool right = (lb & 1) != 0;
  const int nseg = dense_segments(g);
  const int rs = lb >> 1, band = rs / nseg, u0 = (rs - band * nseg) * kDenseSeg;
  const int v0 = band * R;
  int cnt = 0;
  uint64_t* const s_stage64 = reinterpret_cast<uint64_t*>(s_stage);
  if (p.descriptor) {
    if (right)
      dense_rows<CensusDense, true, R, NT>(F, g, p, v0, u0, s_lut, s_stage64, &cnt);
    else
      dense_rows<CensusDense, false, R, NT>(F, g, p, v0, u0, s_lut, s_stage64, &cnt);
  } else {
    if (right)
      dense_rows<GradDense, true, R, NT>(F, g, p, v0, u0, s_lut, s_stage, &cnt);
    else
      dense_rows<GradDense, false, R, NT>(F, g, p, v0, u0, s_lut, s_stage, &cnt);
  }
  cnt = wave_sum_i32(cnt);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) F.dense_counts[lb] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

template <int R>
__device__ __forceinline__ void dense_nt_body(const Frame& F, int lb) {
  dense_body<R, true>(F, lb);
}

// ---------------------------------------------------------------------------
// Final left/right consistency check (Section III-A: occlusions invalidated).
// ---------------------------------------------------------------------------
constexpr int kCheckPx = 4;  // pixels per thread (fewer, longer waves)

// MED: the checked maps go to the median stage's inputs (ordinary stores,
// read back next); otherwise they are the outputs, which no later stage
// reads, and leave with non-temporal stores.
template <bool MED>
__device__ __forceinline__ void check_rows(const Frame& F, int lb) {
  const Geometry g = F.g;
  const int thr = F.p.lr_threshold;
  constexpr bool med = MED;
  const int16_t* rawL = F.rawL;
  const int16_t* rawR = F.rawR;
  int16_t* outL = F.outL;
  int16_t* outR = F.outR;
  int16_t* chkL = F.chkL;
  int16_t* chkR = F.chkR;
  const bool right = (lb & 1) != 0;
  const int npx = g.w * g.h;
  const int16_t* self = right ? rawR : rawL;
  const int16_t* other = right ? rawL : rawR;
  int16_t* dst = right ? (med ? chkR : outR) : (med ? chkL : outL);
  const int px0 = (lb >> 1) * (256 * kCheckPx) + (int)threadIdx.x;
  // row of a pixel index by a multiply: v = floor(px * m / 2^40), m =
  // ceil(2^40 / w), exact for px < 2^27 and w < 2^13 (the error term stays
  // below px * w / 2^40 < 1/2 of a step)
  const uint64_t m = g.rowmul;
  int d[kCheckPx], e[kCheckPx];
#pragma unroll
  for (int k = 0; k < kCheckPx; ++k) d[k] = self[min(px0 + 256 * k, npx - 1)];
#pragma unroll
  for (int k = 0; k < kCheckPx; ++k) {
    const int px = min(px0 + 256 * k, npx - 1);
    const int v = (int)(((uint64_t)(uint32_t)px * m) >> 40), u = px - v * g.w;
    const int x = right ? u + d[k] : u - d[k];  // partner column
    const int ev = other[(size_t)v * g.w + min(max(x, 0), g.w - 1)];  // in bounds always
    e[k] = (d[k] >= 0 && x >= 0 && x < g.w) ? ev : -1;
  }
  // e >= 0 and |e - d| <= threshold as one unsigned range test (for d >= 0)
  const int t = min(thr, 1 << 12);
#pragma unroll
  for (int k = 0; k < kCheckPx; ++k) {
    const int px = px0 + 256 * k;
    if (px >= npx) break;
    const int lo = max(0, d[k] - t);
    const bool ok = d[k] >= 0 && (uint32_t)(e[k] - lo) <= (uint32_t)(d[k] + t - lo);
    const int16_t res = (int16_t)(ok ? d[k] : -1);
    if constexpr (MED)
      dst[px] = res;
    else
      __builtin_nontemporal_store(res, &dst[px]);
  }
  // keeps the two instantiations' last stores apart (the compiler would
  // otherwise sink them into one ordinary store)
  if constexpr (!MED) asm volatile("" ::: "memory");
}

__device__ __forceinline__ void check_body(const Frame& F, int lb) {
  if (F.p.median)
    check_rows<true>(F, lb);
  else
    check_rows<false>(F, lb);
}

// ---------------------------------------------------------------------------
// Median post-filter (Section VIII) of the checked maps, window 3 or 5
// clipped to the image: an invalid pixel stays invalid, a valid one takes
// the lower median of the valid values in its window. Block = 64 x 4 pixels
// of one view with a 2-pixel halo in LDS (outside the image reads as
// invalid). The window's values, invalid ones replaced by a sentinel above
// every disparity, are sorted by a Batcher odd-even merge network over the
// next power of two (fully unrolled: the values stay in registers), and the
// ((n-1)/2)-th of the n valid values is selected.
// ---------------------------------------------------------------------------
constexpr int kMedW = 64, kMedH = 4, kMedHalo = 2;

template <int N>
__device__ __forceinline__ void oddeven_merge_sort(int (&a)[N]) {
#pragma unroll
  for (int p = 1; p < N; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k; ++i)
          if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            const int x = a[i + j], y = a[i + j + k];
            a[i + j] = min(x, y);
            a[i + j + k] = max(x, y);
          }
}

template <int W, int N>
__device__ __forceinline__ int median_pixel(const int16_t (*t)[kMedW + 2 * kMedHalo], int ty,
                                            int tx) {
  constexpr int r = W / 2;
  constexpr int kInvalid = 0x7FFF;
  int a[N];
  int n = 0;
#pragma unroll
  for (int dy = 0; dy < W; ++dy)
#pragma unroll
    for (int dx = 0; dx < W; ++dx) {
      const int e = t[ty + kMedHalo - r + dy][tx + kMedHalo - r + dx];
      a[dy * W + dx] = e >= 0 ? e : kInvalid;
      n += e >= 0 ? 1 : 0;
    }
#pragma unroll
  for (int i = W * W; i < N; ++i) a[i] = kInvalid;
  oddeven_merge_sort<N>(a);
  const int k = (n - 1) >> 1;
  int res = -1;
#pragma unroll
  for (int i = 0; i < W * W; ++i) res = i == k ? a[i] : res;
  return res;
}

__device__ __forceinline__ void median_body(const Frame& F, int lb) {
  const Geometry g = F.g;
  const int win = F.p.median;
  const int nbx = cdivd(g.w, kMedW);
  const int view = lb & 1, tile_id = lb >> 1;
  const int16_t* in = view ? F.chkR : F.chkL;
  int16_t* out = view ? F.outR : F.outL;
  constexpr int TW = kMedW + 2 * kMedHalo;
  __shared__ int16_t t[kMedH + 2 * kMedHalo][TW];
  const int u0 = (tile_id % nbx) * kMedW, v0 = (tile_id / nbx) * kMedH;
  const int tid = threadIdx.x;
  constexpr int kTile = (kMedH + 2 * kMedHalo) * TW;
  stage_copy<(kTile + 255) / 256, 256>(
      kTile,
      [&](int i) -> int {
        const int r = i / TW, c = i - r * TW;
        const int y = v0 - kMedHalo + r, x = u0 - kMedHalo + c;
        return (x >= 0 && x < g.w && y >= 0 && y < g.h) ? (int)in[(size_t)y * g.w + x] : -1;
      },
      [&](int i, int x) {
        const int r = i / TW, c = i - r * TW;
        t[r][c] = (int16_t)x;
      });
  __syncthreads();
  const int tx = tid & 63, ty = tid >> 6;
  const int u = u0 + tx, v = v0 + ty;
  if (u >= g.w || v >= g.h) return;
  int res = t[ty + kMedHalo][tx + kMedHalo];
  if (res >= 0) res = win == 3 ? median_pixel<3, 16>(t, ty, tx) : median_pixel<5, 32>(t, ty, tx);
  out[(size_t)v * g.w + u] = (int16_t)res;
}

// ---- kernels: one frame, or a batch in one launch --------------------------
// ATTR: extra kernel attributes (an occupancy target where measured faster).
// A batch launch finds a block's frame as floor(b / bpf) = umulhi(b, bmul)
// when every frame has bpf blocks (bmul = ceil(2^32 / bpf), exact for
// b * bpf < 2^32, which the launcher checks), else by binary search.
// ELAS_BATCH_KERNEL_ATTR alone: the batch launch only (the non-temporal
// variants: plain calls never need them).
#define ELAS_BATCH_KERNEL_ATTR(NAME, BODY, THREADS, ATTR)                                \
  __global__ __launch_bounds__(THREADS) ATTR void NAME##_batch(                         \
      const Frame* __restrict__ frames, const int32_t* __restrict__ starts, int nf,      \
      int bpf, uint32_t bmul) {                                                          \
    const int b = xcd_remap(blockIdx.x, gridDim.x);                                     \
    int f, lb;                                                                           \
    if (bpf > 0) {                                                                       \
      f = (int)__umulhi((uint32_t)b, bmul);                                              \
      lb = b - f * bpf;                                                                  \
    } else {                                                                             \
      f = frame_of(starts, nf, b);                                                       \
      lb = b - starts[f];                                                                \
    }                                                                                    \
    const Frame F = global_frame(frames[f], reinterpret_cast<const char*>(frames));     \
    BODY(F, lb);                                                                         \
  }
#define ELAS_FRAME_KERNEL_ATTR(NAME, BODY, THREADS, ATTR)                              \
  __global__ __launch_bounds__(THREADS) ATTR void NAME(Frame F) {                       \
    BODY(F, xcd_remap(blockIdx.x, gridDim.x));                                          \
  }
#define ELAS_STAGE_KERNELS_ATTR(NAME, BODY, THREADS, ATTR)                              \
  ELAS_FRAME_KERNEL_ATTR(NAME, BODY, THREADS, ATTR)                                     \
  ELAS_BATCH_KERNEL_ATTR(NAME, BODY, THREADS, ATTR)
#define ELAS_NO_ATTR
#define ELAS_STAGE_KERNELS(NAME, BODY, THREADS) \
  ELAS_STAGE_KERNELS_ATTR(NAME, BODY, THREADS, ELAS_NO_ATTR)
// Eight wavefronts per SIMD: the register budget that lets the 1- and 2-row
// dense tiles fill the SIMDs (their LDS allows it; the compiler would
// otherwise take a few more VGPRs and stop at seven)
#define ELAS_OCC8 __attribute__((amdgpu_waves_per_eu(8, 8)))

ELAS_STAGE_KERNELS(k_descriptor4, stage1_body<4>, 256)
ELAS_STAGE_KERNELS(k_descriptor8, stage1_body<8>, 256)
ELAS_STAGE_KERNELS(k_descriptor16, stage1_body<16>, 256)
ELAS_BATCH_KERNEL_ATTR(k_descriptor4nt, stage1_nt_body<4>, 256, ELAS_NO_ATTR)
ELAS_BATCH_KERNEL_ATTR(k_descriptor8nt, stage1_nt_body<8>, 256, ELAS_NO_ATTR)
ELAS_BATCH_KERNEL_ATTR(k_descriptor16nt, stage1_nt_body<16>, 256, ELAS_NO_ATTR)
ELAS_STAGE_KERNELS(k_support, support_body, 256)
ELAS_FRAME_KERNEL_ATTR(k_filter, filter_body<1024>, 1024, ELAS_NO_ATTR)
ELAS_BATCH_KERNEL_ATTR(k_filter, filter_body<512>, 512, ELAS_NO_ATTR)
ELAS_STAGE_KERNELS(k_rows, rows_body, 64)
ELAS_STAGE_KERNELS(k_raster, raster_body<1024>, 1024)
ELAS_STAGE_KERNELS(k_raster256, raster_body<256>, 256)
ELAS_STAGE_KERNELS_ATTR(k_dense_r1, dense_body<1>, 256, ELAS_OCC8)
ELAS_STAGE_KERNELS_ATTR(k_dense_r2, dense_body<2>, 256, ELAS_OCC8)
ELAS_STAGE_KERNELS(k_dense_r4, dense_body<4>, 256)
ELAS_BATCH_KERNEL_ATTR(k_dense_r1nt, dense_nt_body<1>, 256, ELAS_OCC8)
ELAS_BATCH_KERNEL_ATTR(k_dense_r2nt, dense_nt_body<2>, 256, ELAS_OCC8)
ELAS_BATCH_KERNEL_ATTR(k_dense_r4nt, dense_nt_body<4>, 256, ELAS_NO_ATTR)
ELAS_STAGE_KERNELS(k_check, check_body, 256)
ELAS_STAGE_KERNELS(k_redun, redun_body, 1024)
ELAS_STAGE_KERNELS(k_median, median_body, 256)

#undef ELAS_STAGE_KERNELS
#undef ELAS_STAGE_KERNELS_ATTR
#undef ELAS_BATCH_KERNEL_ATTR
#undef ELAS_FRAME_KERNEL_ATTR
#undef ELAS_NO_ATTR
#undef ELAS_OCC8

size_t filter_lds_bytes(const Geometry& g, const KParams& p) {
  const int ft = filter_tile(g);
  const int SR = ft + 2 * (p.incon_window + p.redun_max_dist), SI = ft + 2 * p.redun_max_dist;
  return sizeof(int16_t) * (size_t)(SR * SR + SI * SI + ft * SI);
}

int stage_threads(int32_t stage) {
  switch (stage) {
    case kStageFilter: return 512;  // the batched launch; single frames take 1024
    case kStageRedun: return 1024;
    case kStageRows: return 64;
    case kStageRaster: return 256;  // the batched launch; single frames choose in launch_stage
    default: return 256;
  }
}

}  // namespace

int32_t raster_band_rows(int32_t w) { return std::max(1, std::min(kBandRowsMax, 4096 / w)); }

int32_t dense_blocks(const Geometry& g, int variant) {
  return 2 * cdiv(g.h, kDenseRowsOf[std::min(std::max(variant, 0), kDenseVariants - 1)]) *
         dense_segments(g);
}

int32_t dense_blocks_max(const Geometry& g) { return dense_blocks(g, 0); }

int32_t stage_blocks(int32_t stage, const Geometry& g, const KParams& p, int dv) {
  switch (stage) {
    case kStageDescriptor:
      return 2 * cdiv(g.w, desc_block_width(p)) * cdiv(g.h, kDescRows[std::min(std::max(dv, 0), 2)]);
    case kStageSupport: return g.lw > 0 ? g.lh * cdiv(g.lw, support_run(g, p)) : 0;
    case kStageFilter: return filter_tiles_x(g) * filter_tiles_y(g);
    case kStageRedun: return p.redundancy ? 1 : 0;
    case kStageRows: return g.lh;
    case kStageMesh: return 2;
    case kStageRaster: return 2 * cdiv(g.h, raster_band_rows(g.w));
    case kStageDense: return dense_blocks(g, dv);
    case kStageCheck: return 2 * cdiv((long long)g.w * g.h, 256 * kCheckPx);
    case kStageMedian: return p.median ? 2 * cdiv(g.w, kMedW) * cdiv(g.h, kMedH) : 0;
    default: return 0;
  }
}

size_t stage_lds(int32_t stage, const Geometry& g, const KParams& p) {
  switch (stage) {
    case kStageFilter: return filter_lds_bytes(g, p);
    case kStageRows: return sizeof(int32_t) * (size_t)g.w;
    case kStageRaster: return sizeof(int32_t) * (size_t)raster_band_rows(g.w) * g.w;
    case kStageMesh: return kMeshLdsBytes;
    case kStageSupport: {
      const int q = support_run(g, p);
      return 32 * (size_t)(support_cols_right(q, g.step, p.D) + support_cols_left(q, g.step, p.D));
    }
    default: return 0;
  }
}

hipError_t launch_stage(int32_t stage, const Frame& f, int variant, hipStream_t s,
                        hipEvent_t start, hipEvent_t stop) {
  if (stage == kStageMesh) return launch_mesh_frame(f, s, start, stop);
  const int nb = stage_blocks(stage, f.g, f.p, variant);
  if (nb <= 0) return hipSuccess;
  // the wide raster workgroup when every band of the frame gets a CU
  const bool wide_raster = stage == kStageRaster && nb <= 256;
  const dim3 grid(nb),
      block(wide_raster || stage == kStageFilter ? 1024 : stage_threads(stage));
  const uint32_t lds = (uint32_t)stage_lds(stage, f.g, f.p);
  const bool timed = start || stop;
  auto go = [&](auto kernel) {
    if (timed)
      hipExtLaunchKernelGGL(kernel, grid, block, lds, s, start, stop, 0u, f);
    else
      hipLaunchKernelGGL(kernel, grid, block, lds, s, f);
  };
  switch (stage) {
    case kStageDescriptor:
      if (variant == 1)
        go(k_descriptor8);
      else if (variant == 2)
        go(k_descriptor16);
      else
        go(k_descriptor4);
      break;
    case kStageSupport: go(k_support); break;
    case kStageFilter: go(k_filter); break;
    case kStageRedun: go(k_redun); break;
    case kStageRows: go(k_rows); break;
    case kStageRaster:
      if (wide_raster)
        go(k_raster);
      else
        go(k_raster256);
      break;
    case kStageDense:
      if (variant == 0)
        go(k_dense_r1);
      else if (variant == 2)
        go(k_dense_r4);
      else
        go(k_dense_r2);
      break;
    case kStageCheck: go(k_check); break;
    case kStageMedian: go(k_median); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int32_t uniform_blocks(const int32_t* starts, int32_t nf) {
  if (nf <= 0) return 0;
  const int32_t d = starts[1] - starts[0];
  for (int32_t i = 1; i < nf; ++i)
    if (starts[i + 1] - starts[i] != d) return 0;
  return d;
}

hipError_t launch_stage_batch(int32_t stage, const Frame* frames, const int32_t* starts,
                              int32_t nf, int32_t total_blocks, int32_t bpf, size_t lds,
                              int variant, bool desc_nt, hipStream_t s, hipEvent_t start,
                              hipEvent_t stop) {
  if (stage == kStageMesh) return launch_mesh_batch(frames, nf, s, start, stop);
  if (total_blocks <= 0 || nf <= 0) return hipSuccess;
  // the multiply path needs bpf >= 2 (bmul < 2^32), bpf * nf == total and
  // b * bpf < 2^32 for every block b
  if (bpf < 2 || (int64_t)bpf * nf != total_blocks ||
      (uint64_t)total_blocks * (uint64_t)bpf >= (1ull << 32))
    bpf = 0;
  const uint32_t bmul = bpf ? (uint32_t)(((1ull << 32) + (uint64_t)bpf - 1) / (uint64_t)bpf) : 0u;
  const dim3 grid(total_blocks), block(stage_threads(stage));
  const uint32_t shm = (uint32_t)lds;
  const bool timed = start || stop;
  auto go = [&](auto kernel, uint32_t bytes) {
    if (timed)
      hipExtLaunchKernelGGL(kernel, grid, block, bytes, s, start, stop, 0u, frames, starts, nf,
                            bpf, bmul);
    else
      hipLaunchKernelGGL(kernel, grid, block, bytes, s, frames, starts, nf, bpf, bmul);
  };
  switch (stage) {
    case kStageDescriptor:
      if (variant == 1)
        desc_nt ? go(k_descriptor8nt_batch, 0u) : go(k_descriptor8_batch, 0u);
      else if (variant == 2)
        desc_nt ? go(k_descriptor16nt_batch, 0u) : go(k_descriptor16_batch, 0u);
      else
        desc_nt ? go(k_descriptor4nt_batch, 0u) : go(k_descriptor4_batch, 0u);
      break;
    case kStageSupport: go(k_support_batch, shm); break;
    case kStageFilter: go(k_filter_batch, shm); break;
    case kStageRows: go(k_rows_batch, shm); break;
    case kStageRaster: go(k_raster256_batch, shm); break;
    case kStageDense:
      if (variant == 0)
        desc_nt ? go(k_dense_r1nt_batch, 0u) : go(k_dense_r1_batch, 0u);
      else if (variant == 2)
        desc_nt ? go(k_dense_r4nt_batch, 0u) : go(k_dense_r4_batch, 0u);
      else
        desc_nt ? go(k_dense_r2nt_batch, 0u) : go(k_dense_r2_batch, 0u);
      break;
    case kStageCheck: go(k_check_batch, 0u); break;
    case kStageRedun: go(k_redun_batch, 0u); break;
    case kStageMedian: go(k_median_batch, 0u); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace elas

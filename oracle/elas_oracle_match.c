/*
 * Oracle, matching stages: descriptors, prior table, support matching,
 * support filtering, support lists, grid vectors, dense matching and the
 * final left/right check. Plain loops, one thread, no intrinsics.
 * TEST INFRASTRUCTURE ONLY (see elas_oracle.h).
 */
#include "elas_oracle.h"

#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
static int32_t iabs(int32_t a) { return a < 0 ? -a : a; }

/* ------------------------------------------------------------------------
 * Sobel gradients (Section III-A: support matching works on the horizontal
 * and vertical gradient images, Fig. 1(b)). The paper names the operator
 * only; reading: the standard 3x3 Sobel pair, defined on the interior
 * 1 <= u <= w-2, 1 <= v <= h-2, and 0 on the one-pixel border.
 * du = right column minus left column (weights 1,2,1),
 * dv = bottom row minus top row (weights 1,2,1).
 * ---------------------------------------------------------------------- */
void orc_sobel(const uint8_t* img, int32_t w, int32_t h, int32_t stride,
               int16_t* du, int16_t* dv) {
  for (int32_t v = 0; v < h; ++v) {
    for (int32_t u = 0; u < w; ++u) {
      int32_t gx = 0, gy = 0;
      if (u >= 1 && u <= w - 2 && v >= 1 && v <= h - 2) {
#define I(x, y) ((int32_t)img[(size_t)(y) * stride + (x)])
        gx = (I(u + 1, v - 1) + 2 * I(u + 1, v) + I(u + 1, v + 1)) -
             (I(u - 1, v - 1) + 2 * I(u - 1, v) + I(u - 1, v + 1));
        gy = (I(u - 1, v + 1) + 2 * I(u, v + 1) + I(u + 1, v + 1)) -
             (I(u - 1, v - 1) + 2 * I(u, v - 1) + I(u + 1, v - 1));
#undef I
      }
      du[(size_t)v * w + u] = (int16_t)gx;
      dv[(size_t)v * w + u] = (int16_t)gy;
    }
  }
}

/* Quantisation of a gradient to one descriptor byte. Reading: divide by 4
 * with C truncation toward zero, clamp to [-127, 127], store 128 + q, so a
 * byte is in [1, 255] and negating the gradient maps byte b to 256 - b. */
static uint8_t quantise(int32_t g) {
  int32_t q = g / 4;
  if (q > 127) q = 127;
  if (q < -127) q = -127;
  return (uint8_t)(128 + q);
}

/* ------------------------------------------------------------------------
 * 16-byte descriptor per pixel (Section VI-A: the original ELAS matches a
 * 16-byte SIMD-width subset of the window's gradient samples; 128 bits per
 * dense descriptor). Reading of the subset: du at column/row offsets
 * (-2,0) (-1,0) (1,0) (2,0) (-1,-2) (1,-2) (-1,2) (1,2), then dv at
 * (0,-2) (0,-1) (0,1) (0,2) (-2,-1) (2,-1) (-2,1) (2,1). Defined for
 * 2 <= u <= w-3, 2 <= v <= h-3; other pixels are all-zero (a value no
 * defined descriptor can take, since every defined byte is >= 1).
 * ---------------------------------------------------------------------- */
static const int32_t kDuOff[8][2] = {{-2, 0}, {-1, 0}, {1, 0}, {2, 0},
                                     {-1, -2}, {1, -2}, {-1, 2}, {1, 2}};
static const int32_t kDvOff[8][2] = {{0, -2}, {0, -1}, {0, 1}, {0, 2},
                                     {-2, -1}, {2, -1}, {-2, 1}, {2, 1}};

void orc_descriptors(const uint8_t* img, int32_t w, int32_t h, int32_t stride,
                     uint8_t* desc) {
  size_t n = (size_t)w * h;
  int16_t* du = (int16_t*)malloc(n * sizeof(int16_t));
  int16_t* dv = (int16_t*)malloc(n * sizeof(int16_t));
  orc_sobel(img, w, h, stride, du, dv);
  memset(desc, 0, n * 16);
  for (int32_t v = 2; v <= h - 3; ++v) {
    for (int32_t u = 2; u <= w - 3; ++u) {
      uint8_t* o = desc + ((size_t)v * w + u) * 16;
      for (int k = 0; k < 8; ++k) {
        int32_t x = u + kDuOff[k][0], y = v + kDuOff[k][1];
        o[k] = quantise(du[(size_t)y * w + x]);
      }
      for (int k = 0; k < 8; ++k) {
        int32_t x = u + kDvOff[k][0], y = v + kDvOff[k][1];
        o[8 + k] = quantise(dv[(size_t)y * w + x]);
      }
    }
  }
  free(du);
  free(dv);
}

/* Texture of a descriptor: sum of |byte - 128| (distance from a flat patch). */
static int32_t texture16(const uint8_t* d) {
  int32_t t = 0;
  for (int k = 0; k < 16; ++k) t += iabs((int32_t)d[k] - 128);
  return t;
}

static int32_t sad16(const uint8_t* a, const uint8_t* b) {
  int32_t s = 0;
  for (int k = 0; k < 16; ++k) s += iabs((int32_t)a[k] - (int32_t)b[k]);
  return s;
}

/* ------------------------------------------------------------------------
 * Prior table. The paper keeps ELAS's slanted-plane prior but does not print
 * it. Reading (the ELAS generative model: likelihood ~ exp(-beta*SAD), prior
 * ~ gamma + exp(-(d-mu)^2 / (2 sigma^2))): the energy of a disparity at
 * distance k from the plane mean is -log(gamma + exp(-k^2/(2 sigma^2)))
 * scaled by 1/beta; the constant log(gamma)/beta is added so that far
 * candidates cost 0. Computed in double and rounded to the nearest integer.
 * ---------------------------------------------------------------------- */
void orc_prior_lut(const orc_params* p, int32_t* lut) {
  int32_t D = p->disp_max - p->disp_min + 1;
  double g = (double)p->gamma, s = (double)p->sigma, b = (double)p->beta;
  for (int32_t k = 0; k < D; ++k) {
    double kk = (double)k * (double)k;
    double e = -(log(g + exp(-kk / (2.0 * s * s))) - log(g)) / b;
    lut[k] = (int32_t)lround(e);
  }
}

/* ------------------------------------------------------------------------
 * Support candidate lattice: every s-th column and row, with the 9x9
 * support window (Section VII-A) inside the region where descriptors are
 * defined: 4 <= u <= w-5 and 4 <= v <= h-5, u and v multiples of s.
 * ---------------------------------------------------------------------- */
void orc_lattice(const orc_params* p, int32_t w, int32_t h, int32_t* lw,
                 int32_t* lh, int32_t* u0, int32_t* v0) {
  int32_t s = p->candidate_stepsize;
  int32_t kmin = (4 + s - 1) / s;
  int32_t kumax = (w - 5) / s, kvmax = (h - 5) / s;
  *u0 = kmin * s;
  *v0 = kmin * s;
  *lw = kumax >= kmin ? kumax - kmin + 1 : 0;
  *lh = kvmax >= kmin ? kvmax - kmin + 1 : 0;
}

/* Support descriptor (512 bits, Section VI-A): the four dense descriptors at
 * (u-2, v-2), (u+2, v-2), (u-2, v+2), (u+2, v+2), covering the 9x9 window. */
static const int32_t kCorner[4][2] = {{-2, -2}, {2, -2}, {-2, 2}, {2, 2}};

static int32_t texture64(const uint8_t* desc, int32_t w, int32_t u, int32_t v) {
  int32_t t = 0;
  for (int c = 0; c < 4; ++c)
    t += texture16(desc + ((size_t)(v + kCorner[c][1]) * w + u + kCorner[c][0]) * 16);
  return t;
}

static int32_t sad64(const uint8_t* da, int32_t ua, const uint8_t* db, int32_t ub,
                     int32_t v, int32_t w) {
  int32_t s = 0;
  for (int c = 0; c < 4; ++c) {
    size_t row = (size_t)(v + kCorner[c][1]) * w;
    s += sad16(da + (row + ua + kCorner[c][0]) * 16, db + (row + ub + kCorner[c][0]) * 16);
  }
  return s;
}

/* Ambiguity test (Section VI-B, eq. 1-2): a match is kept when the best cost
 * m1 is clearly below the second-best m2. Reading: strict m1 < thr*m2 with
 * one FP32 product, so m1 = m2 = 0 (flat or periodic texture) is rejected. */
int32_t orc_ratio_accept(float thr, int32_t m1, int32_t m2) {
  float lhs = (float)m1;
  float rhs = thr * (float)m2;
  return lhs < rhs ? 1 : 0;
}

/* Exhaustive search of one support point over d = dmin..dhi. self is the
 * image the point lies in; the partner column is u + dir*d. Costs: SAD of
 * the 64-byte support descriptors. m1/d1 = smallest cost, smallest d on
 * ties; m2 = smallest cost over every other admissible d. */
static int search(const orc_params* p, const uint8_t* dself, const uint8_t* dother,
                  int32_t u, int32_t v, int32_t w, int32_t dir, int32_t dhi,
                  int64_t* evals, int32_t* d_out) {
  int32_t n = dhi - p->disp_min + 1;
  if (n < 2) return 0;
  int32_t cost[256];
  int32_t m1 = INT_MAX, d1 = -1;
  for (int32_t d = p->disp_min; d <= dhi; ++d) {
    int32_t c = sad64(dself, u, dother, u + dir * d, v, w);
    cost[d - p->disp_min] = c;
    if (c < m1) {
      m1 = c;
      d1 = d;
    }
  }
  int32_t m2 = INT_MAX;
  for (int32_t d = p->disp_min; d <= dhi; ++d)
    if (d != d1 && cost[d - p->disp_min] < m2) m2 = cost[d - p->disp_min];
  *evals += n;
  if (!orc_support_accept(p, m1, m2)) return 0;
  *d_out = d1;
  return 1;
}

/* ------------------------------------------------------------------------
 * Support matching (Section III-A: sparse SAD matching over the gradient
 * images across the disparity range, kept only where the first and second
 * minima are far enough apart). Per lattice point:
 *   1. texture of the left support descriptor >= support_texture;
 *   2. left-to-right search over d in [dmin, min(dmax, u-4)] (at least 2);
 *   3. ratio test -> d1;
 *   4. right-to-left search from u_r = u - d1 (texture test on the right
 *      descriptor, d in [dmin, min(dmax, w-5-u_r)], ratio test) -> d2;
 *   5. keep d1 iff |d2 - d1| <= lr_threshold.
 * The left/right check of step 4-5 is not described in the paper; reading:
 * the same search mirrored, with the final check's tolerance.
 * ---------------------------------------------------------------------- */
void orc_support_match(const orc_params* p, const uint8_t* descL,
                       const uint8_t* descR, int32_t w, int32_t h,
                       int16_t* dcan, int64_t* evals) {
  int32_t lw, lh, u0, v0;
  orc_lattice(p, w, h, &lw, &lh, &u0, &v0);
  int32_t s = p->candidate_stepsize;
  for (int32_t l = 0; l < lh; ++l) {
    for (int32_t k = 0; k < lw; ++k) {
      int32_t u = u0 + k * s, v = v0 + l * s;
      int16_t result = -1;
      int32_t d1, d2;
      if (texture64(descL, w, u, v) >= p->support_texture &&
          search(p, descL, descR, u, v, w, -1, imin(p->disp_max, u - 4), evals, &d1)) {
        int32_t ur = u - d1;
        if (texture64(descR, w, ur, v) >= p->support_texture &&
            search(p, descR, descL, ur, v, w, +1, imin(p->disp_max, w - 5 - ur), evals,
                   &d2) &&
            iabs(d2 - d1) <= p->lr_threshold)
          result = (int16_t)d1;
      }
      dcan[(size_t)l * lw + k] = result;
    }
  }
}

/* ------------------------------------------------------------------------
 * Inconsistency filter (Section III-A, Fig. 1(e): support points are compared
 * with neighbours in a window and implausible ones removed). Reading: window
 * of +-incon_window_size lattice steps; a point survives iff at least
 * incon_min_support other valid points in it have |d' - d| <=
 * incon_threshold. All points read the unfiltered input (simultaneous
 * update).
 * ---------------------------------------------------------------------- */
void orc_filter_incon(const orc_params* p, const int16_t* in, int32_t lw,
                      int32_t lh, int16_t* out) {
  int32_t r = p->incon_window_size;
  for (int32_t l = 0; l < lh; ++l) {
    for (int32_t k = 0; k < lw; ++k) {
      int32_t d = in[(size_t)l * lw + k];
      int16_t res = -1;
      if (d >= 0) {
        int32_t count = 0;
        for (int32_t ll = l - r; ll <= l + r; ++ll) {
          if (ll < 0 || ll >= lh) continue;
          for (int32_t kk = k - r; kk <= k + r; ++kk) {
            if (kk < 0 || kk >= lw || (ll == l && kk == k)) continue;
            int32_t e = in[(size_t)ll * lw + kk];
            if (e >= 0 && iabs(e - d) <= p->incon_threshold) ++count;
          }
        }
        if (count >= p->incon_min_support) res = (int16_t)d;
      }
      out[(size_t)l * lw + k] = res;
    }
  }
}

/* ------------------------------------------------------------------------
 * Redundancy filter (Section III-A: identical values along the same row or
 * column are removed; Section VI-C and Fig. 7A: the original looks both
 * backwards and forwards). Reading: a point is removed iff within
 * redun_max_dist lattice steps on BOTH sides along the pass direction there
 * is a valid point with |d' - d| <= redun_threshold. Simultaneous update; the
 * vertical pass runs first and the horizontal pass reads its output.
 * ---------------------------------------------------------------------- */
void orc_filter_redun(const orc_params* p, const int16_t* in, int32_t lw,
                      int32_t lh, int32_t vertical, int16_t* out) {
  int32_t r = p->redun_max_dist, t = p->redun_threshold;
  for (int32_t l = 0; l < lh; ++l) {
    for (int32_t k = 0; k < lw; ++k) {
      int32_t d = in[(size_t)l * lw + k];
      int16_t res = (int16_t)d;
      if (d >= 0) {
        int before = 0, after = 0;
        for (int32_t j = 1; j <= r; ++j) {
          int32_t lb = vertical ? l - j : l, kb = vertical ? k : k - j;
          int32_t la = vertical ? l + j : l, ka = vertical ? k : k + j;
          if (lb >= 0 && kb >= 0) {
            int32_t e = in[(size_t)lb * lw + kb];
            if (e >= 0 && iabs(e - d) <= t) before = 1;
          }
          if (la < lh && ka < lw) {
            int32_t e = in[(size_t)la * lw + ka];
            if (e >= 0 && iabs(e - d) <= t) after = 1;
          }
        }
        if (before && after) res = -1;
      }
      out[(size_t)l * lw + k] = res;
    }
  }
}

/* ------------------------------------------------------------------------
 * Support lists. Left list: surviving lattice points (u, v, d) in row-major
 * lattice order. Right list (the paper does not describe the right view's
 * prior; reading): each left point seen from the right view at (u - d, v);
 * where two land on the same pixel the larger disparity (the nearer surface)
 * is kept; ordered by (v, u). Image corners (reading): each corner takes the
 * d of the nearest list point by squared distance, the earlier point in list
 * order on ties. With an empty list the corners are -1. Down-sampling
 * (orc_subsample) thins the left list first; everything after uses the kept
 * points only.
 * ---------------------------------------------------------------------- */
static int cmp_right(const void* a, const void* b) {
  const int32_t* x = (const int32_t*)a;
  const int32_t* y = (const int32_t*)b;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;   /* v */
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;   /* u */
  if (x[2] != y[2]) return x[2] > y[2] ? -1 : 1;   /* larger d first */
  return 0;
}

static void nearest_corners(const int32_t* pts, int32_t n, int32_t w, int32_t h,
                            int32_t* corners) {
  const int32_t cu[4] = {0, w - 1, 0, w - 1};
  const int32_t cv[4] = {0, 0, h - 1, h - 1};
  for (int c = 0; c < 4; ++c) {
    int64_t best = -1;
    int32_t bi = -1;
    for (int32_t i = 0; i < n; ++i) {
      int64_t du = pts[3 * i] - cu[c], dv = pts[3 * i + 1] - cv[c];
      int64_t dist = du * du + dv * dv;
      if (bi < 0 || dist < best) {
        best = dist;
        bi = i;
      }
    }
    corners[c] = bi >= 0 ? pts[3 * bi + 2] : -1;
  }
}

void orc_support_lists(const orc_params* p, const int16_t* dcan, int32_t lw,
                       int32_t lh, int32_t w, int32_t h,
                       int32_t* ptsL, int32_t* nL, int32_t* cornersL,
                       int32_t* ptsR, int32_t* nR, int32_t* cornersR) {
  int32_t lw2, lh2, u0, v0;
  orc_lattice(p, w, h, &lw2, &lh2, &u0, &v0);
  int32_t s = p->candidate_stepsize;
  int32_t n = 0;
  for (int32_t l = 0; l < lh; ++l)
    for (int32_t k = 0; k < lw; ++k) {
      int32_t d = dcan[(size_t)l * lw + k];
      if (d < 0) continue;
      ptsL[3 * n] = u0 + k * s;
      ptsL[3 * n + 1] = v0 + l * s;
      ptsL[3 * n + 2] = d;
      ++n;
    }
  n = orc_subsample(ptsL, n, p->support_subsample);
  *nL = n;
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * 3 * (n > 0 ? n : 1));
  for (int32_t i = 0; i < n; ++i) {
    tmp[3 * i] = ptsL[3 * i] - ptsL[3 * i + 2];
    tmp[3 * i + 1] = ptsL[3 * i + 1];
    tmp[3 * i + 2] = ptsL[3 * i + 2];
  }
  qsort(tmp, (size_t)n, 3 * sizeof(int32_t), cmp_right);
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (m > 0 && ptsR[3 * (m - 1)] == tmp[3 * i] && ptsR[3 * (m - 1) + 1] == tmp[3 * i + 1])
      continue;  /* same pixel, smaller d */
    memcpy(ptsR + 3 * m, tmp + 3 * i, 3 * sizeof(int32_t));
    ++m;
  }
  *nR = m;
  free(tmp);
  nearest_corners(ptsL, n, w, h, cornersL);
  nearest_corners(ptsR, m, w, h, cornersR);
}

/* ------------------------------------------------------------------------
 * Grid vectors (Section III-A and Fig. 2: the support disparities of each
 * grid region are pooled and widened by +-1; Section VI-D: one-hot encoded
 * into a fixed-width bit vector). Bit (d - dmin) of a region's D-bit mask is
 * set iff some support point of the region has |d' - d| <= 1. Reading: each
 * region pools only its own points; image corners do not count.
 * ---------------------------------------------------------------------- */
void orc_grid_dims(const orc_params* p, int32_t w, int32_t h, int32_t* gw,
                   int32_t* gh, int32_t* words) {
  int32_t g = p->grid_size;
  *gw = (w + g - 1) / g;
  *gh = (h + g - 1) / g;
  *words = (p->disp_max - p->disp_min + 1 + 63) / 64;
}

void orc_grid(const orc_params* p, const int32_t* pts, int32_t n, int32_t w,
              int32_t h, uint64_t* grid) {
  int32_t gw, gh, words;
  orc_grid_dims(p, w, h, &gw, &gh, &words);
  memset(grid, 0, sizeof(uint64_t) * (size_t)gw * gh * words);
  for (int32_t i = 0; i < n; ++i) {
    int32_t cell = (pts[3 * i + 1] / p->grid_size) * gw + pts[3 * i] / p->grid_size;
    for (int32_t dd = pts[3 * i + 2] - 1; dd <= pts[3 * i + 2] + 1; ++dd) {
      if (dd < p->disp_min || dd > p->disp_max) continue;
      int32_t bit = dd - p->disp_min;
      grid[(size_t)cell * words + bit / 64] |= (uint64_t)1 << (bit % 64);
    }
  }
}

/* ------------------------------------------------------------------------
 * Dense matching (Section III-A, Fig. 1(h): every pixel is matched over the
 * disparities the prior allows; the slanted-plane prior both weights and
 * restricts the search, widened by the grid vectors). For a pixel with a
 * defined descriptor of texture >= match_texture, the candidates are
 *   {d : |d - d_plane| <= sradius} (when the pixel has a plane)
 *   union {d : bit d of its grid region}   (when there are support points)
 * (every d when full_search), restricted to dmin..dmax and to partners with a
 * defined descriptor (left view: u-d >= 2; right view: u+d <= w-3).
 * Energy E(d) = SAD of the 16-byte descriptors + lut[|d - d_plane|] (prior
 * term only when there is a plane). Result: argmin, smallest d on ties, or
 * -1 when there are no candidates.
 * ---------------------------------------------------------------------- */
int64_t orc_dense(const orc_params* p, const uint8_t* desc_self,
                  const uint8_t* desc_other, const int16_t* dplane,
                  const uint64_t* grid, int32_t has_list, const int32_t* lut,
                  int32_t w, int32_t h, int32_t right_frame, int16_t* out) {
  int32_t gw, gh, words;
  orc_grid_dims(p, w, h, &gw, &gh, &words);
  int64_t evals = 0;
  for (int32_t v = 0; v < h; ++v) {
    for (int32_t u = 0; u < w; ++u) {
      int16_t res = -1;
      out[(size_t)v * w + u] = -1;
      if (u < 2 || u > w - 3 || v < 2 || v > h - 3) continue;
      const uint8_t* self = desc_self + ((size_t)v * w + u) * 16;
      if (texture16(self) < p->match_texture) continue;
      int32_t dp = has_list ? dplane[(size_t)v * w + u] : -1;
      int plane = dp >= 0;
      const uint64_t* cell =
          has_list ? grid + ((size_t)(v / p->grid_size) * gw + u / p->grid_size) * words : 0;
      int32_t bestE = 0;
      for (int32_t d = p->disp_min; d <= p->disp_max; ++d) {
        int32_t uo = right_frame ? u + d : u - d;
        if (uo < 2 || uo > w - 3) continue;
        int in = p->full_search;
        if (plane && iabs(d - dp) <= p->sradius) in = 1;
        if (cell) {
          int32_t bit = d - p->disp_min;
          if ((cell[bit / 64] >> (bit % 64)) & 1u) in = 1;
        }
        if (!in) continue;
        ++evals;
        int32_t E = sad16(self, desc_other + ((size_t)v * w + uo) * 16);
        if (plane) E += lut[iabs(d - dp)];
        if (res < 0 || E < bestE) {
          res = (int16_t)d;
          bestE = E;
        }
      }
      out[(size_t)v * w + u] = res;
    }
  }
  return evals;
}

/* ------------------------------------------------------------------------
 * Final left/right consistency check (Section III-A: occluded pixels are
 * invalidated). A left disparity d at (u, v) survives iff the right map at
 * (u - d, v) is valid and within lr_threshold of d; symmetrically for the
 * right map at (u + d, v). Both read the unchecked maps.
 * ---------------------------------------------------------------------- */
void orc_lrcheck(const orc_params* p, const int16_t* rawL, const int16_t* rawR,
                 int32_t w, int32_t h, int16_t* outL, int16_t* outR) {
  for (int32_t v = 0; v < h; ++v) {
    for (int32_t u = 0; u < w; ++u) {
      size_t i = (size_t)v * w + u;
      int32_t d = rawL[i];
      int16_t r = -1;
      if (d >= 0 && u - d >= 0) {
        int32_t e = rawR[(size_t)v * w + (u - d)];
        if (e >= 0 && iabs(e - d) <= p->lr_threshold) r = (int16_t)d;
      }
      outL[i] = r;
      d = rawR[i];
      r = -1;
      if (d >= 0 && u + d < w) {
        int32_t e = rawL[(size_t)v * w + (u + d)];
        if (e >= 0 && iabs(e - d) <= p->lr_threshold) r = (int16_t)d;
      }
      outR[i] = r;
    }
  }
}

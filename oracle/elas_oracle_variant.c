/*
 * Oracle, the paper's platform-conscious variant (Section VI) and the
 * optional steps of Section VII-VIII: census descriptors with Hamming
 * distance (Section VI-A), the shift-sum ambiguity threshold (Section VI-B,
 * eq. 3), past-only redundancy filtering (Section VI-C, Fig. 7B), support
 * point down-sampling (Section VII-B) and the median post-filter (Section
 * VIII). Plain loops, one thread, no intrinsics.
 * TEST INFRASTRUCTURE ONLY (see elas_oracle.h).
 */
#include "elas_oracle.h"

#include <limits.h>
#include <stdlib.h>
#include <string.h>

static int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
static int32_t iabs(int32_t a) { return a < 0 ? -a : a; }

static int32_t popcount32(uint32_t x) {
  int32_t c = 0;
  while (x) {
    c += (int32_t)(x & 1u);
    x >>= 1;
  }
  return c;
}

/* ------------------------------------------------------------------------
 * Census transform (Section VI-A: the FPGA variant replaces the gradient
 * descriptors by census descriptors over the whole W x W window, 81 bits for
 * 9 x 9, 25 bits for 5 x 5, compared by Hamming distance). The paper gives
 * the window sizes only; readings: bit i, for the i-th window offset
 * (dx, dy) in row-major order (dy outer, dx inner, the centre included and
 * always 0), is 1 iff the neighbour's intensity is strictly smaller than the
 * centre's; a neighbour outside the image counts as not smaller.
 * ---------------------------------------------------------------------- */
void orc_census(const uint8_t* img, int32_t w, int32_t h, int32_t stride, int32_t win,
                uint32_t* out, int32_t words) {
  int32_t r = win / 2;
  for (int32_t v = 0; v < h; ++v) {
    for (int32_t u = 0; u < w; ++u) {
      uint32_t* o = out + ((size_t)v * w + u) * words;
      memset(o, 0, sizeof(uint32_t) * words);
      int32_t c = img[(size_t)v * stride + u];
      int32_t bit = 0;
      for (int32_t dy = -r; dy <= r; ++dy) {
        for (int32_t dx = -r; dx <= r; ++dx, ++bit) {
          int32_t x = u + dx, y = v + dy;
          if (x < 0 || x >= w || y < 0 || y >= h) continue;
          if ((int32_t)img[(size_t)y * stride + x] < c) o[bit / 32] |= 1u << (bit % 32);
        }
      }
    }
  }
}

int32_t orc_hamming(const uint32_t* a, const uint32_t* b, int32_t words) {
  int32_t s = 0;
  for (int32_t k = 0; k < words; ++k) s += popcount32(a[k] ^ b[k]);
  return s;
}

int32_t orc_census_texture(const uint32_t* a, int32_t words) {
  int32_t s = 0;
  for (int32_t k = 0; k < words; ++k) s += popcount32(a[k]);
  return s;
}

/* ------------------------------------------------------------------------
 * Shift-sum ambiguity test (Section VI-B, eq. 3): the threshold 0.9 m2 of
 * eq. 2 is replaced by m2/2 + m2/4 + m2/8 + m2/32 computed with shifts.
 * Reading: integer right shifts (each term truncated), and the accept
 * condition of eq. 2, m1 <= threshold.
 * ---------------------------------------------------------------------- */
int32_t orc_shiftsum_threshold(int32_t m2) {
  return (m2 >> 1) + (m2 >> 2) + (m2 >> 3) + (m2 >> 5);
}

int32_t orc_shiftsum_accept(int32_t m1, int32_t m2) {
  return m1 <= orc_shiftsum_threshold(m2) ? 1 : 0;
}

/* The ambiguity test a support search applies: eq. 1-2 with the ratio
 * threshold (orc_ratio_accept), or eq. 3 with the shift-sum. */
int32_t orc_support_accept(const orc_params* p, int32_t m1, int32_t m2) {
  return p->ambiguity ? orc_shiftsum_accept(m1, m2)
                      : orc_ratio_accept(p->support_threshold, m1, m2);
}

/* Exhaustive census search of one support point over d = dmin..dhi: costs
 * are Hamming distances of the support-window census descriptors; m1, d1
 * (smallest d on ties) and m2 as in the gradient search. */
static int census_search(const orc_params* p, const uint32_t* cself, const uint32_t* cother,
                         int32_t words, int32_t u, int32_t v, int32_t w, int32_t dir,
                         int32_t dhi, int64_t* evals, int32_t* d_out) {
  int32_t n = dhi - p->disp_min + 1;
  if (n < 2) return 0;
  int32_t cost[256];
  int32_t m1 = INT_MAX, d1 = -1;
  const uint32_t* a = cself + ((size_t)v * w + u) * words;
  for (int32_t d = p->disp_min; d <= dhi; ++d) {
    int32_t c = orc_hamming(a, cother + ((size_t)v * w + u + dir * d) * words, words);
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
 * Support matching with census descriptors: the lattice, the admissible
 * ranges, the reverse search and the |d2 - d1| check are those of the
 * gradient version (orc_support_match). Reading for the texture test (the
 * paper has none for census): the census popcount of the point's support
 * descriptor (the number of darker window pixels) >= support_texture; with
 * support_texture = 0 the test is off.
 * ---------------------------------------------------------------------- */
void orc_support_match_census(const orc_params* p, const uint32_t* csL,
                              const uint32_t* csR, int32_t words, int32_t w, int32_t h,
                              int16_t* dcan, int64_t* evals) {
  int32_t lw, lh, u0, v0;
  orc_lattice(p, w, h, &lw, &lh, &u0, &v0);
  int32_t s = p->candidate_stepsize;
  for (int32_t l = 0; l < lh; ++l) {
    for (int32_t k = 0; k < lw; ++k) {
      int32_t u = u0 + k * s, v = v0 + l * s;
      int16_t result = -1;
      int32_t d1, d2;
      if (orc_census_texture(csL + ((size_t)v * w + u) * words, words) >= p->support_texture &&
          census_search(p, csL, csR, words, u, v, w, -1, imin(p->disp_max, u - 4), evals,
                        &d1)) {
        int32_t ur = u - d1;
        if (orc_census_texture(csR + ((size_t)v * w + ur) * words, words) >=
                p->support_texture &&
            census_search(p, csR, csL, words, ur, v, w, +1, imin(p->disp_max, w - 5 - ur),
                          evals, &d2) &&
            iabs(d2 - d1) <= p->lr_threshold)
          result = (int16_t)d1;
      }
      dcan[(size_t)l * lw + k] = result;
    }
  }
}

/* ------------------------------------------------------------------------
 * Past-only redundancy (Section VI-C, Fig. 7B: the FPGA filter looks only
 * backwards in the stream, so a run of equal values keeps one value every
 * redun_max_dist + 1 steps instead of vanishing). Reading: a sequential pass
 * along each column from the top (vertical) or each row from the left
 * (horizontal); a point is removed iff one of the previous redun_max_dist
 * positions holds a point that survived this pass with |d' - d| <=
 * redun_threshold.
 * ---------------------------------------------------------------------- */
void orc_filter_redun_past(const orc_params* p, const int16_t* in, int32_t lw, int32_t lh,
                           int32_t vertical, int16_t* out) {
  int32_t r = p->redun_max_dist, t = p->redun_threshold;
  int32_t lines = vertical ? lw : lh, len = vertical ? lh : lw;
  for (int32_t a = 0; a < lines; ++a) {
    for (int32_t b = 0; b < len; ++b) {
      size_t idx = vertical ? (size_t)b * lw + a : (size_t)a * lw + b;
      int32_t d = in[idx];
      int16_t res = (int16_t)d;
      if (d >= 0) {
        for (int32_t j = 1; j <= r && b - j >= 0; ++j) {
          size_t pj = vertical ? (size_t)(b - j) * lw + a : (size_t)a * lw + (b - j);
          int32_t e = out[pj];
          if (e >= 0 && iabs(e - d) <= t) {
            res = -1;
            break;
          }
        }
      }
      out[idx] = res;
    }
  }
}

/* ------------------------------------------------------------------------
 * Support point down-sampling (Section VII-B: the number of support points
 * is reduced to 1/8, 1/14 or 1/32 of those extracted). Reading: the final
 * left list keeps the points whose index in lattice (row-major) order is a
 * multiple of k; the right list and the grid vectors are built from the kept
 * points. Applied in place; returns the new count.
 * ---------------------------------------------------------------------- */
int32_t orc_subsample(int32_t* pts, int32_t n, int32_t k) {
  if (k <= 1) return n;
  int32_t m = 0;
  for (int32_t i = 0; i < n; i += k) {
    memmove(pts + 3 * m, pts + 3 * i, 3 * sizeof(int32_t));
    ++m;
  }
  return m;
}

/* ------------------------------------------------------------------------
 * Dense matching with census descriptors (Section VI-A: dense window W x W,
 * e.g. 5 x 5 = 25 bits; Hamming distance): candidates, admissible partners
 * and the prior are those of orc_dense; the data term is the Hamming
 * distance of the dense census descriptors. Texture (reading, as for support
 * points): census popcount >= match_texture.
 * ---------------------------------------------------------------------- */
int64_t orc_dense_census(const orc_params* p, const uint32_t* cself, const uint32_t* cother,
                         int32_t words, const int16_t* dplane, const uint64_t* grid,
                         int32_t has_list, const int32_t* lut, int32_t w, int32_t h,
                         int32_t right_frame, int16_t* out) {
  int32_t gw, gh, gwords;
  orc_grid_dims(p, w, h, &gw, &gh, &gwords);
  int64_t evals = 0;
  for (int32_t v = 0; v < h; ++v) {
    for (int32_t u = 0; u < w; ++u) {
      int16_t res = -1;
      out[(size_t)v * w + u] = -1;
      if (u < 2 || u > w - 3 || v < 2 || v > h - 3) continue;
      const uint32_t* self = cself + ((size_t)v * w + u) * words;
      if (orc_census_texture(self, words) < p->match_texture) continue;
      int32_t dp = has_list ? dplane[(size_t)v * w + u] : -1;
      int plane = dp >= 0;
      const uint64_t* cell =
          has_list ? grid + ((size_t)(v / p->grid_size) * gw + u / p->grid_size) * gwords : 0;
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
        int32_t E = orc_hamming(self, cother + ((size_t)v * w + uo) * words, words);
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
 * Median post-filter (Section VIII: the most accurate configuration is
 * passed through a median filter for comparison). The paper does not give
 * the window or the handling of invalid pixels; readings: a win x win
 * window (3 or 5) clipped to the image; an invalid pixel stays invalid; a
 * valid one takes the lower median (index (n-1)/2 after sorting) of the
 * valid values in its window.
 * ---------------------------------------------------------------------- */
static int cmp_i16(const void* a, const void* b) {
  int16_t x = *(const int16_t*)a, y = *(const int16_t*)b;
  return (x > y) - (x < y);
}

void orc_median(int32_t win, const int16_t* in, int32_t w, int32_t h, int16_t* out) {
  int32_t r = win / 2;
  int16_t vals[64];
  for (int32_t v = 0; v < h; ++v) {
    for (int32_t u = 0; u < w; ++u) {
      int16_t c = in[(size_t)v * w + u];
      if (c < 0 || win <= 1) {
        out[(size_t)v * w + u] = c;
        continue;
      }
      int32_t n = 0;
      for (int32_t y = v - r; y <= v + r; ++y) {
        if (y < 0 || y >= h) continue;
        for (int32_t x = u - r; x <= u + r; ++x) {
          if (x < 0 || x >= w) continue;
          int16_t e = in[(size_t)y * w + x];
          if (e >= 0) vals[n++] = e;
        }
      }
      qsort(vals, (size_t)n, sizeof(int16_t), cmp_i16);
      out[(size_t)v * w + u] = vals[(n - 1) / 2];
    }
  }
}

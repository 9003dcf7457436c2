/*
 * Plain, single-threaded CPU oracle of the ELAS dense-stereo hot path.
 *
 * TEST INFRASTRUCTURE ONLY. This code is the parity reference for the HIP
 * library. It shares no source, header, table or helper with that library,
 * and nothing in the product path may call it. Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg load it.
 *
 * What it computes follows the ELAS description in Section III-A of
 * Rahnama et al., "Real-Time Dense Stereo Matching with ELAS on FPGA
 * Accelerated Embedded Devices" (arXiv 1802.07210): gradient (Sobel)
 * descriptors, sparse support points chosen by a first/second-minimum
 * ambiguity test (Section VI-B, eq. 1-2), consistency and redundancy filtering
 * of the support points (Section III-A, Fig. 7A), a Delaunay mesh of the
 * support points giving a slanted-plane prior remapped to a per-pixel prior
 * matrix (Section VI-D), grid vectors pooled per region and widened by +-1
 * (Fig. 2), dense SAD matching restricted to the prior's candidates, and a
 * final left/right consistency check. Where the paper is silent, the
 * readings are stated at each function in elas_oracle_*.c.
 *
 * Conventions: u is the column, v the row (growing downwards). Left pixel
 * (u, v) corresponds to right pixel (u - d, v). Disparity maps are int16 with
 * -1 = invalid. All integer arithmetic is exact. Floating point appears in
 * three places only: the ratio test (one FP32 multiply), the prior table
 * (double, rounded to integers) and the plane mean (FP32, fixed order,
 * no contraction; the build uses -ffp-contract=off).
 */
#ifndef ELAS_ORACLE_H
#define ELAS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
  int32_t disp_min;            /* smallest disparity (>= 0) */
  int32_t disp_max;            /* largest disparity; D = max - min + 1 <= 256 */
  float   support_threshold;   /* ratio test: accept iff m1 < thr * m2 (FP32) */
  int32_t support_texture;     /* minimum texture of a 64-byte support descriptor */
  int32_t candidate_stepsize;  /* lattice step s of support candidates */
  int32_t incon_window_size;   /* half window, in lattice units */
  int32_t incon_threshold;     /* |d' - d| <= this counts as consistent */
  int32_t incon_min_support;   /* consistent neighbours needed to keep a point */
  int32_t redun_max_dist;      /* redundancy search distance, lattice units */
  int32_t redun_threshold;     /* |d' - d| <= this counts as redundant */
  int32_t grid_size;           /* grid-vector region size in pixels */
  float   beta;                /* likelihood scale */
  float   gamma;               /* prior floor */
  float   sigma;               /* prior width */
  int32_t sradius;             /* plane candidates: |d - d_plane| <= sradius */
  int32_t match_texture;       /* minimum texture of a 16-byte dense descriptor */
  int32_t lr_threshold;        /* left/right agreement tolerance */
  int32_t full_search;         /* 1: dense candidates = every admissible d */
  /* Section VI variant and optional steps (0/1 defaults give the pipeline
   * above). */
  int32_t descriptor;          /* 0: Sobel descriptors + SAD; 1: census + Hamming */
  int32_t census_support_window; /* support census window W (odd, 3..13) */
  int32_t census_dense_window; /* dense census window W (odd, 3..7) */
  int32_t ambiguity;           /* 0: ratio test (eq. 1-2); 1: shift-sum (eq. 3) */
  int32_t redundancy;          /* 0: two-sided (Fig. 7A); 1: past-only (Fig. 7B) */
  int32_t support_subsample;   /* keep every k-th support point (k >= 1) */
  int32_t median_window;       /* 0 or 1: off; 3 or 5: median post-filter */
  int32_t add_corners;         /* 1: the four image corners join each view's mesh
                                  (nearest point's d); 0: the mesh of the support
                                  points alone, pixels outside their hull get no
                                  plane prior */
} orc_params;

/* ---- stage 1: gradients and descriptors -------------------------------- */
void orc_sobel(const uint8_t* img, int32_t w, int32_t h, int32_t stride,
               int16_t* du, int16_t* dv);
/* 16 bytes per pixel, row-major [h][w][16]; undefined pixels are all-zero. */
void orc_descriptors(const uint8_t* img, int32_t w, int32_t h, int32_t stride,
                     uint8_t* desc);

/* ---- prior table --------------------------------------------------------- */
void orc_prior_lut(const orc_params* p, int32_t* lut /* D entries */);

/* ---- stage 2: support matching on the candidate lattice ------------------ */
/* Lattice geometry: columns u = s*k with 4 <= u <= w-5, rows likewise. */
void orc_lattice(const orc_params* p, int32_t w, int32_t h,
                 int32_t* lw, int32_t* lh, int32_t* u0, int32_t* v0);
void orc_support_match(const orc_params* p, const uint8_t* descL,
                       const uint8_t* descR, int32_t w, int32_t h,
                       int16_t* dcan /* lh*lw */, int64_t* evals);
/* Ratio test exposed for unit tests: accept iff (float)m1 < thr*(float)m2. */
int32_t orc_ratio_accept(float thr, int32_t m1, int32_t m2);

/* ---- stage 3: support filtering ------------------------------------------ */
void orc_filter_incon(const orc_params* p, const int16_t* in, int32_t lw,
                      int32_t lh, int16_t* out);
void orc_filter_redun(const orc_params* p, const int16_t* in, int32_t lw,
                      int32_t lh, int32_t vertical, int16_t* out);

/* ---- support lists --------------------------------------------------------
 * ptsL/ptsR receive (u, v, d) triples; capacity lw*lh triples. Returns counts.
 * corners receive the d of (0,0), (w-1,0), (0,h-1), (w-1,h-1). The left list
 * is down-sampled (support_subsample) before the right list and the corners
 * are built from it; *nL is the kept count. */
void orc_support_lists(const orc_params* p, const int16_t* dcan, int32_t lw,
                       int32_t lh, int32_t w, int32_t h,
                       int32_t* ptsL, int32_t* nL, int32_t* cornersL,
                       int32_t* ptsR, int32_t* nR, int32_t* cornersR);

/* ---- triangulation -------------------------------------------------------
 * pts: n distinct (u, v) pairs. The first four must be the image corners
 * (0,0), (w-1,0), (0,h-1), (w-1,h-1) and every other point must lie strictly
 * inside that rectangle. Writes at most 2n triangles as vertex-index triples
 * (positively oriented) and returns their count, or -1 on bad input. */
int32_t orc_delaunay(const int32_t* pts, int32_t n, int32_t* tris);
/* Delaunay triangulation (same canonical rule) of n distinct points alone, no
 * corners: [ntri][3] vertex indices in positive orientation into tris
 * (capacity 2n). Returns ntri (0 for n < 3 or collinear points), -1 for bad
 * input (duplicates). */
int32_t orc_delaunay_points(const int32_t* pts, int32_t n, int32_t* tris);
/* Exact predicates, exposed for unit tests. */
int64_t orc_orient(const int32_t* a, const int32_t* b, const int32_t* c);
int64_t orc_incircle(const int32_t* a, const int32_t* b, const int32_t* c,
                     const int32_t* d);

/* Canonical triangle records: 9 ints (u,v,d) x 3 with vertices sorted by
 * (v, u), records sorted lexicographically. Planes: 3 floats (a, b, c). */
void orc_canonical_triangles(const int32_t* pts /* (u,v,d) */, const int32_t* tris,
                             int32_t ntri, int32_t* recs);
void orc_plane(const int32_t* rec, float* abc);

/* ---- prior raster: per pixel owner triangle and d_plane -------------------
 * recs/planes in canonical order; owner receives the index of the owning
 * triangle (-1 when none); dplane receives the clamped rounded plane mean. */
void orc_plane_map(const orc_params* p, const int32_t* recs, const float* planes,
                   int32_t ntri, int32_t w, int32_t h, int32_t* owner,
                   int16_t* dplane);

/* ---- grid vectors -------------------------------------------------------- */
void orc_grid_dims(const orc_params* p, int32_t w, int32_t h, int32_t* gw,
                   int32_t* gh, int32_t* words);
void orc_grid(const orc_params* p, const int32_t* pts, int32_t n, int32_t w,
              int32_t h, uint64_t* grid /* gh*gw*words */);

/* ---- dense matching: right_frame = 0 matches the left view against the
 * right one, 1 the reverse. has_list = 0 means no support points (no plane,
 * no grid). Returns the number of candidate evaluations. */
int64_t orc_dense(const orc_params* p, const uint8_t* desc_self,
                  const uint8_t* desc_other, const int16_t* dplane,
                  const uint64_t* grid, int32_t has_list, const int32_t* lut,
                  int32_t w, int32_t h, int32_t right_frame, int16_t* out);

/* ---- final left/right check --------------------------------------------- */
void orc_lrcheck(const orc_params* p, const int16_t* rawL, const int16_t* rawR,
                 int32_t w, int32_t h, int16_t* outL, int16_t* outR);

/* ---- Section VI variant (elas_oracle_variant.c) -------------------------
 * Census descriptors: `words` 32-bit words per pixel, row-major [h][w][words];
 * bit i (word i/32, bit i%32) is the i-th window offset in row-major order,
 * set iff that neighbour is inside the image and darker than the centre. */
void orc_census(const uint8_t* img, int32_t w, int32_t h, int32_t stride, int32_t win,
                uint32_t* out, int32_t words);
int32_t orc_hamming(const uint32_t* a, const uint32_t* b, int32_t words);
int32_t orc_census_texture(const uint32_t* a, int32_t words);
/* eq. 3: m2/2 + m2/4 + m2/8 + m2/32 with truncating shifts; accept iff
 * m1 <= that. orc_support_accept applies the test params->ambiguity names. */
int32_t orc_shiftsum_threshold(int32_t m2);
int32_t orc_shiftsum_accept(int32_t m1, int32_t m2);
int32_t orc_support_accept(const orc_params* p, int32_t m1, int32_t m2);
/* Support matching on census descriptors of the support window (csL/csR
 * computed on the whole image with `words` words per pixel). */
void orc_support_match_census(const orc_params* p, const uint32_t* csL,
                              const uint32_t* csR, int32_t words, int32_t w, int32_t h,
                              int16_t* dcan, int64_t* evals);
/* Past-only redundancy pass along columns (vertical) or rows. */
void orc_filter_redun_past(const orc_params* p, const int16_t* in, int32_t lw, int32_t lh,
                           int32_t vertical, int16_t* out);
/* Keeps every k-th (u, v, d) triple, in place; returns the new count. */
int32_t orc_subsample(int32_t* pts, int32_t n, int32_t k);
/* Dense matching on census descriptors of the dense window. */
int64_t orc_dense_census(const orc_params* p, const uint32_t* cself, const uint32_t* cother,
                         int32_t words, const int16_t* dplane, const uint64_t* grid,
                         int32_t has_list, const int32_t* lut, int32_t w, int32_t h,
                         int32_t right_frame, int16_t* out);
/* Median post-filter of a checked map (win 3 or 5; 0 or 1 copies). */
void orc_median(int32_t win, const int16_t* in, int32_t w, int32_t h, int16_t* out);

/* ---- whole pipeline with every intermediate ------------------------------ */
typedef struct orc_trace {
  int32_t w, h, lw, lh, gw, gh, words, D;
  uint8_t* descL; uint8_t* descR;             /* h*w*16 */
  int16_t* dcan_raw; int16_t* dcan_incon;     /* lh*lw */
  int16_t* dcan_vert; int16_t* dcan_final;
  int32_t nL, nR;
  int32_t* ptsL; int32_t* ptsR;               /* (u,v,d) * n */
  int32_t cornersL[4], cornersR[4];
  int32_t ntriL, ntriR;
  int32_t* recL; int32_t* recR;               /* 9 * ntri, canonical order */
  float* planeL; float* planeR;               /* 3 * ntri */
  int32_t* ownerL; int32_t* ownerR;           /* h*w */
  int16_t* dplaneL; int16_t* dplaneR;         /* h*w */
  uint64_t* gridL; uint64_t* gridR;           /* gh*gw*words */
  int32_t* lut;                               /* D */
  int16_t* rawL; int16_t* rawR;               /* h*w */
  int16_t* outL; int16_t* outR;               /* h*w */
  int64_t support_evals, dense_evals;
  double stage_ms[6]; /* descriptor, support+filter+lists, triangulate+planes+raster, grid,
                         dense, lrcheck (+median) */
  int32_t swords, dwords;                     /* census words per pixel (census mode) */
  uint32_t* csupL; uint32_t* csupR;           /* h*w*swords, support census */
  uint32_t* cdenL; uint32_t* cdenR;           /* h*w*dwords, dense census */
  int16_t* chkL; int16_t* chkR;               /* h*w, checked maps before the median */
  int32_t nL_all;                             /* left list size before down-sampling */
} orc_trace;

/* Runs every stage; allocates the trace arrays (free with orc_trace_free).
 * Returns 0, -1 if the inputs violate the preconditions (9 <= w, h <= 8192,
 * 0 <= disp_min <= disp_max, D <= 256, positive step/grid/beta/gamma/sigma,
 * descriptor/ambiguity/redundancy 0 or 1, census windows odd within their
 * ranges, 1 <= support_subsample <= 64, median_window 0, 1, 3 or 5),
 * or -2 if a triangulation failed its own consistency checks. */
int32_t orc_process(const orc_params* p, const uint8_t* left, const uint8_t* right,
                    int32_t w, int32_t h, int32_t stride, orc_trace* t);
void orc_trace_free(orc_trace* t);

#ifdef __cplusplus
}
#endif
#endif

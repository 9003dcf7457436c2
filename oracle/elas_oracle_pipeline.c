/*
 * Oracle, whole pipeline: the stages of Section III-A in order (with the
 * Section VI variant and the optional steps when the parameters ask for
 * them), keeping every intermediate for stage-by-stage comparison.
 * TEST INFRASTRUCTURE ONLY (see elas_oracle.h).
 */
#define _POSIX_C_SOURCE 199309L
#include "elas_oracle.h"

#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_ms(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

/* Points for triangulation: the four image corners first, then the list
 * (without add_corners: the list alone). */
static int32_t build_mesh(const orc_params* p, const int32_t* list, int32_t n,
                          const int32_t* corners, int32_t w, int32_t h, int32_t** recs,
                          float** planes, int32_t** owner, int16_t* dplane) {
  const int32_t nc = p->add_corners ? 4 : 0;
  int32_t total = n + nc;
  int32_t* uvd = (int32_t*)malloc(sizeof(int32_t) * 3 * total);
  int32_t* uv = (int32_t*)malloc(sizeof(int32_t) * 2 * total);
  const int32_t cu[4] = {0, w - 1, 0, w - 1};
  const int32_t cv[4] = {0, 0, h - 1, h - 1};
  for (int c = 0; c < nc; ++c) {
    uvd[3 * c] = cu[c];
    uvd[3 * c + 1] = cv[c];
    uvd[3 * c + 2] = corners[c];
  }
  memcpy(uvd + 3 * nc, list, sizeof(int32_t) * 3 * n);
  for (int32_t i = 0; i < total; ++i) {
    uv[2 * i] = uvd[3 * i];
    uv[2 * i + 1] = uvd[3 * i + 1];
  }
  int32_t* tris = (int32_t*)malloc(sizeof(int32_t) * 3 * (2 * total + 8));
  int32_t nt = nc ? orc_delaunay(uv, total, tris) : orc_delaunay_points(uv, total, tris);
  if (nt < 0) {
    free(uvd);
    free(uv);
    free(tris);
    return -1;
  }
  *recs = (int32_t*)malloc(sizeof(int32_t) * 9 * (nt > 0 ? nt : 1));
  *planes = (float*)malloc(sizeof(float) * 3 * (nt > 0 ? nt : 1));
  orc_canonical_triangles(uvd, tris, nt, *recs);
  for (int32_t t = 0; t < nt; ++t) orc_plane(*recs + 9 * t, *planes + 3 * t);
  *owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)w * h);
  orc_plane_map(p, *recs, *planes, nt, w, h, *owner, dplane);
  free(uvd);
  free(uv);
  free(tris);
  return nt;
}

int32_t orc_process(const orc_params* p, const uint8_t* left, const uint8_t* right,
                    int32_t w, int32_t h, int32_t stride, orc_trace* t) {
  if (w < 9 || h < 9 || stride < w || p->disp_min < 0 || p->disp_max < p->disp_min ||
      p->disp_max - p->disp_min + 1 > 256 || p->candidate_stepsize <= 0 ||
      p->grid_size <= 0 || !(p->beta > 0) || !(p->gamma > 0) || !(p->sigma > 0) ||
      w > 8192 || h > 8192 || (p->descriptor != 0 && p->descriptor != 1) ||
      (p->ambiguity != 0 && p->ambiguity != 1) || (p->redundancy != 0 && p->redundancy != 1) ||
      p->support_subsample < 1 || p->support_subsample > 64 ||
      (p->median_window != 0 && p->median_window != 1 && p->median_window != 3 &&
       p->median_window != 5) ||
      (p->add_corners != 0 && p->add_corners != 1))
    return -1;
  if (p->descriptor == 1 &&
      (p->census_support_window < 3 || p->census_support_window > 13 ||
       p->census_support_window % 2 == 0 || p->census_dense_window < 3 ||
       p->census_dense_window > 7 || p->census_dense_window % 2 == 0))
    return -1;
  memset(t, 0, sizeof(*t));
  t->w = w;
  t->h = h;
  t->D = p->disp_max - p->disp_min + 1;
  size_t npx = (size_t)w * h;

  double t0 = now_ms();
  const int census = p->descriptor == 1;
  if (census) {
    /* Section VI-A: census descriptors of the support and dense windows */
    int32_t ws = p->census_support_window, wd = p->census_dense_window;
    t->swords = (ws * ws + 31) / 32;
    t->dwords = (wd * wd + 31) / 32;
    t->csupL = (uint32_t*)malloc(npx * t->swords * sizeof(uint32_t));
    t->csupR = (uint32_t*)malloc(npx * t->swords * sizeof(uint32_t));
    t->cdenL = (uint32_t*)malloc(npx * t->dwords * sizeof(uint32_t));
    t->cdenR = (uint32_t*)malloc(npx * t->dwords * sizeof(uint32_t));
    orc_census(left, w, h, stride, ws, t->csupL, t->swords);
    orc_census(right, w, h, stride, ws, t->csupR, t->swords);
    orc_census(left, w, h, stride, wd, t->cdenL, t->dwords);
    orc_census(right, w, h, stride, wd, t->cdenR, t->dwords);
  } else {
    t->descL = (uint8_t*)malloc(npx * 16);
    t->descR = (uint8_t*)malloc(npx * 16);
    orc_descriptors(left, w, h, stride, t->descL);
    orc_descriptors(right, w, h, stride, t->descR);
  }
  double t1 = now_ms();

  int32_t u0, v0;
  orc_lattice(p, w, h, &t->lw, &t->lh, &u0, &v0);
  size_t nl = (size_t)t->lw * t->lh;
  size_t nlc = nl > 0 ? nl : 1;
  t->dcan_raw = (int16_t*)malloc(nlc * sizeof(int16_t));
  t->dcan_incon = (int16_t*)malloc(nlc * sizeof(int16_t));
  t->dcan_vert = (int16_t*)malloc(nlc * sizeof(int16_t));
  t->dcan_final = (int16_t*)malloc(nlc * sizeof(int16_t));
  if (census)
    orc_support_match_census(p, t->csupL, t->csupR, t->swords, w, h, t->dcan_raw,
                             &t->support_evals);
  else
    orc_support_match(p, t->descL, t->descR, w, h, t->dcan_raw, &t->support_evals);
  orc_filter_incon(p, t->dcan_raw, t->lw, t->lh, t->dcan_incon);
  if (p->redundancy == 1) { /* Section VI-C, Fig. 7B */
    orc_filter_redun_past(p, t->dcan_incon, t->lw, t->lh, 1, t->dcan_vert);
    orc_filter_redun_past(p, t->dcan_vert, t->lw, t->lh, 0, t->dcan_final);
  } else {
    orc_filter_redun(p, t->dcan_incon, t->lw, t->lh, 1, t->dcan_vert);
    orc_filter_redun(p, t->dcan_vert, t->lw, t->lh, 0, t->dcan_final);
  }
  t->nL_all = 0;
  for (size_t i = 0; i < nl; ++i) t->nL_all += t->dcan_final[i] >= 0;
  t->ptsL = (int32_t*)malloc(nlc * 3 * sizeof(int32_t));
  t->ptsR = (int32_t*)malloc(nlc * 3 * sizeof(int32_t));
  orc_support_lists(p, t->dcan_final, t->lw, t->lh, w, h, t->ptsL, &t->nL, t->cornersL,
                    t->ptsR, &t->nR, t->cornersR);
  if (!p->add_corners) /* no corners join the meshes */
    for (int c = 0; c < 4; ++c) t->cornersL[c] = t->cornersR[c] = -1;
  double t2 = now_ms();

  t->lut = (int32_t*)malloc(sizeof(int32_t) * t->D);
  orc_prior_lut(p, t->lut);
  t->dplaneL = (int16_t*)malloc(npx * sizeof(int16_t));
  t->dplaneR = (int16_t*)malloc(npx * sizeof(int16_t));
  orc_grid_dims(p, w, h, &t->gw, &t->gh, &t->words);
  size_t gcount = (size_t)t->gw * t->gh * t->words;
  t->gridL = (uint64_t*)calloc(gcount, sizeof(uint64_t));
  t->gridR = (uint64_t*)calloc(gcount, sizeof(uint64_t));
  int has_list = t->nL > 0;
  double t3;
  if (has_list) {
    t->ntriL = build_mesh(p, t->ptsL, t->nL, t->cornersL, w, h, &t->recL, &t->planeL,
                          &t->ownerL, t->dplaneL);
    t->ntriR = build_mesh(p, t->ptsR, t->nR, t->cornersR, w, h, &t->recR, &t->planeR,
                          &t->ownerR, t->dplaneR);
    if (t->ntriL < 0 || t->ntriR < 0) return -2;
    t3 = now_ms();
    orc_grid(p, t->ptsL, t->nL, w, h, t->gridL);
    orc_grid(p, t->ptsR, t->nR, w, h, t->gridR);
  } else {
    t3 = now_ms();
    t->ownerL = (int32_t*)malloc(npx * sizeof(int32_t));
    t->ownerR = (int32_t*)malloc(npx * sizeof(int32_t));
    for (size_t i = 0; i < npx; ++i) {
      t->ownerL[i] = t->ownerR[i] = -1;
      t->dplaneL[i] = t->dplaneR[i] = -1;
    }
  }
  double t4 = now_ms();

  t->rawL = (int16_t*)malloc(npx * sizeof(int16_t));
  t->rawR = (int16_t*)malloc(npx * sizeof(int16_t));
  if (census) {
    t->dense_evals = orc_dense_census(p, t->cdenL, t->cdenR, t->dwords, t->dplaneL, t->gridL,
                                      has_list, t->lut, w, h, 0, t->rawL);
    t->dense_evals += orc_dense_census(p, t->cdenR, t->cdenL, t->dwords, t->dplaneR,
                                       t->gridR, has_list, t->lut, w, h, 1, t->rawR);
  } else {
    t->dense_evals = orc_dense(p, t->descL, t->descR, t->dplaneL, t->gridL, has_list, t->lut,
                               w, h, 0, t->rawL);
    t->dense_evals += orc_dense(p, t->descR, t->descL, t->dplaneR, t->gridR, has_list,
                                t->lut, w, h, 1, t->rawR);
  }
  double t5 = now_ms();
  t->chkL = (int16_t*)malloc(npx * sizeof(int16_t));
  t->chkR = (int16_t*)malloc(npx * sizeof(int16_t));
  t->outL = (int16_t*)malloc(npx * sizeof(int16_t));
  t->outR = (int16_t*)malloc(npx * sizeof(int16_t));
  orc_lrcheck(p, t->rawL, t->rawR, w, h, t->chkL, t->chkR);
  /* Section VIII: optional median post-filter of the checked maps */
  orc_median(p->median_window, t->chkL, w, h, t->outL);
  orc_median(p->median_window, t->chkR, w, h, t->outR);
  double t6 = now_ms();
  t->stage_ms[0] = t1 - t0;
  t->stage_ms[1] = t2 - t1;
  t->stage_ms[2] = t3 - t2;
  t->stage_ms[3] = t4 - t3;
  t->stage_ms[4] = t5 - t4;
  t->stage_ms[5] = t6 - t5;
  return 0;
}

void orc_trace_free(orc_trace* t) {
  void* ptrs[] = {t->descL, t->descR, t->dcan_raw, t->dcan_incon, t->dcan_vert,
                  t->dcan_final, t->ptsL, t->ptsR, t->recL, t->recR, t->planeL,
                  t->planeR, t->ownerL, t->ownerR, t->dplaneL, t->dplaneR, t->gridL,
                  t->gridR, t->lut, t->rawL, t->rawR, t->outL, t->outR,
                  t->csupL, t->csupR, t->cdenL, t->cdenR, t->chkL, t->chkR};
  for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
  memset(t, 0, sizeof(*t));
}

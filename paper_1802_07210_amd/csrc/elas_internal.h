// Internal types shared by the HIP kernels, the host mesh builder and the
// C-ABI layer of elas_mi355x.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace elas {

constexpr int kMaxD = 256;
constexpr int32_t kNoOwner = 0x7FFFFFFF;
constexpr int kMeshLdsBytes = 160 * 1024 - 2048;  // dynamic LDS of one mesh workgroup
// Frames meshed on the device have both sides at most this long: the mesh
// packs a point into a 32-bit key with 12-bit coordinates, and its fp64
// in-circle test is exact only for coordinates below 2^12.
constexpr int kDeviceMeshMaxSide = 4096;

// Image, lattice and grid geometry of one (w, h) for one parameter set.
struct Geometry {
  int32_t w, h;
  int32_t lw, lh;     // support lattice: lw columns, lh rows
  int32_t lu0, lv0;   // first lattice column / row in pixels
  int32_t step;       // lattice step in pixels
  int32_t gw, gh;     // grid-vector regions
  int32_t gwords;     // 32-bit words per region mask (even: 64-bit aligned masks)
};

// Parameters as the kernels consume them (passed by value).
struct KParams {
  int32_t dmin, dmax, D;
  float support_threshold;
  int32_t support_texture;
  int32_t incon_window, incon_threshold, incon_min_support;
  int32_t redun_max_dist, redun_threshold;
  int32_t grid_size, sradius, match_texture, lr_threshold, full_search;
  int32_t lut_bias;   // -lut[0]: makes every energy non-negative for key packing
};

// One triangle as the raster and dense kernels read it: integer vertices in
// positive orientation and the FP32 plane d = a*u + b*v + c.
struct RasterTri {
  int16_t u[3];
  int16_t v[3];
  float a, b, c;
};
static_assert(sizeof(RasterTri) == 24, "RasterTri layout");

// Per-frame mesh summary in device memory, written by the device mesh
// kernel or uploaded by the host mesh step; read by raster and dense.
struct MeshHeader {
  int32_t n[2];          // support points, left and right view
  int32_t ntri[2];       // triangles (2n + 2, or 0 without support points)
  int32_t corners[8];    // d of the four image corners, left then right view
  int64_t support_evals; // support-search evaluations of the frame
  int32_t status[2];     // 0; 1 if a view's flip rounds hit their limit; 2 if its
                         // initial triangulation failed a consistency check
};

// ---- host mesh builder (elas_mesh.cpp) ----------------------------------
// pts: n support points (u, v, d), all strictly inside the image; corners: d
// of the four image corners. Builds the canonical Delaunay mesh of corners +
// points and writes, in canonical order, exactly 2n + 2 raster records to
// tri_out and (if not null) 9-int records and 3-float planes for
// verification. Returns the triangle count (2n + 2) or -1 if an internal
// consistency check fails.
struct MeshScratch;
MeshScratch* mesh_scratch_create();
void mesh_scratch_destroy(MeshScratch*);
int32_t build_mesh(MeshScratch* s, const int32_t* pts, int32_t n, const int32_t* corners,
                   int32_t w, int32_t h, RasterTri* tri_out, int32_t* recs_out,
                   float* planes_out);

// ---- kernel launchers (elas_kernels.hip) ---------------------------------
hipError_t launch_descriptor(const uint8_t* left, const uint8_t* right, int32_t stride,
                             const Geometry& g, uint8_t* descL, uint8_t* descR, hipStream_t s);
hipError_t launch_support(const uint8_t* descL, const uint8_t* descR, const Geometry& g,
                          const KParams& p, int16_t* dcan, int32_t* evals, hipStream_t s);
// Fused consistency + redundancy filters; also clears the grid masks.
size_t filter_lds_bytes(const KParams& p);
hipError_t launch_filter(const int16_t* raw, const Geometry& g, const KParams& p,
                         int16_t* incon, int16_t* vert, int16_t* fin, uint32_t* gridL,
                         uint32_t* gridR, hipStream_t s);
// Per-row support lists into host-mapped memory (hrowL/hrowR: [lh][lw] packed
// u | d << 16; hcnt: left counts, right counts, evaluation counts, lh each)
// and the grid masks.
hipError_t launch_rows(const int16_t* fin, const int32_t* evals, const Geometry& g,
                       const KParams& p, int32_t* hrowL, int32_t* hrowR, int32_t* hcnt,
                       uint32_t* gridL, uint32_t* gridR, hipStream_t s);
// Device mesh of both views (elas_mesh_device.hip), for frames with both
// sides at most kDeviceMeshMaxSide. rowsL/rowsR/cnt as written by k_rows;
// outputs the header, the gathered lists (ptsL/ptsR, (u,v,d) triples),
// canonical records and planes per view, and the combined raster records
// (left view first). gscratch: 2 * mesh_global_scratch_per_view bytes, used
// only when a view does not fit in LDS.
size_t mesh_global_scratch_per_view(const Geometry& g);
hipError_t launch_mesh(const int32_t* rowsL, const int32_t* rowsR, const int32_t* cnt,
                       const Geometry& g, int32_t dmin, MeshHeader* hdr, int32_t* ptsL,
                       int32_t* ptsR, int32_t* recsL, int32_t* recsR, float* planesL,
                       float* planesR, RasterTri* tris, char* gscratch, hipStream_t s);
// Owner maps of both views (every pixel written; kNoOwner where no triangle).
hipError_t launch_raster(const RasterTri* tris, const MeshHeader* hdr, const Geometry& g,
                         int32_t* ownerL, int32_t* ownerR, hipStream_t s);
hipError_t launch_dense(const uint8_t* descL, const uint8_t* descR, const int32_t* ownerL,
                        const int32_t* ownerR, const RasterTri* tris, const MeshHeader* hdr,
                        const uint32_t* gridL, const uint32_t* gridR, const int32_t* lut,
                        const Geometry& g, const KParams& p,
                        int16_t* dplaneL, int16_t* dplaneR, int16_t* rawL, int16_t* rawR,
                        int32_t* dense_counts, hipStream_t s);
// Blocks of the dense launch (one candidate-count entry per block).
int32_t dense_blocks(const Geometry& g);
hipError_t launch_lrcheck(const int16_t* rawL, const int16_t* rawR, const Geometry& g,
                          const KParams& p, int16_t* outL, int16_t* outR, hipStream_t s);

}  // namespace elas

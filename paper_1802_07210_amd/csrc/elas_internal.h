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
// Flip rounds a device mesh view may take before it reports failure; far
// above what any frame needs (17 at 640x480), so it only binds when lowered.
constexpr int kMeshMaxRounds = 32000;

// Image, lattice and grid geometry of one (w, h) for one parameter set.
struct Geometry {
  int32_t w, h;
  int32_t lw, lh;     // support lattice: lw columns, lh rows
  int32_t lu0, lv0;   // first lattice column / row in pixels
  int32_t step;       // lattice step in pixels
  int32_t gw, gh;     // grid-vector regions
  int32_t gwords;     // 32-bit words per region mask (even: 64-bit aligned masks)
  int32_t ftile;      // support-filter tile side in lattice points (8 or 16)
  int32_t srun;       // lattice points per support workgroup (8, 16 or 32; fewer
                      // when the staged columns would not fit in LDS)
  uint64_t rowmul;    // ceil(2^40 / w): row of pixel index px = (px * rowmul) >> 40,
                      // exact while px * w < 2^40 (px < 2^27, w <= 8192)
  uint32_t gdiv;      // ceil(2^31 / grid_size): x / grid_size = umulhi(2x, gdiv)
                      // exactly for 0 <= x < 2^31 / grid_size
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
  // Section VI variant and optional steps
  int32_t descriptor;   // 0: Sobel descriptors + SAD; 1: census + Hamming
  int32_t cs_win;       // support census window (odd, 3..13)
  int32_t cd_win;       // dense census window (odd, 3..7)
  int32_t cs_q;         // 16-byte words per support census descriptor (1 or 2)
  int32_t ambiguity;    // 0: ratio test (eq. 1-2); 1: shift-sum (eq. 3)
  int32_t redundancy;   // 0: two-sided; 1: past-only
  int32_t subsample;    // keep every k-th support point
  int32_t median;       // 0: no median; 3 or 5: median window
  int32_t mesh_max_rounds;  // flip rounds before the device mesh gives up (a test
                            // hook lowers it; the default never binds)
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
  int32_t rounds[2];     // device mesh: flip rounds of each view (0 on the host)
  int32_t flips[2];      // device mesh: edge flips of each view
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
// The canonical Delaunay mesh of the n points alone (no corners; points
// anywhere in the image): at most 2n - 5 records in the same canonical order.
// Returns the triangle count (0 for n < 3 or collinear points) or -1.
int32_t build_mesh_points(MeshScratch* s, const int32_t* pts, int32_t n, int32_t w, int32_t h,
                          RasterTri* tri_out, int32_t* recs_out, float* planes_out);

// ---- one frame as the kernels see it -------------------------------------
// Sizes, parameters and every device array of one stereo pair. Passed by
// value to the single-frame kernels and read from a device table by the
// batched ones.
struct Frame {
  Geometry g;
  KParams p;
  int32_t stride;        // row pitch of the input images
  int32_t raster_rows;   // band height of the raster
  const uint8_t* left;
  const uint8_t* right;
  uint8_t* descL;        // gradient: 16 bytes per pixel; census: one uint64 per pixel
  uint8_t* descR;
  uint4* csupL;          // census mode: support census of the lattice rows [lh][w][cs_q]
  uint4* csupR;
  int16_t* dcan_raw;
  int16_t* dcan_incon;
  int16_t* dcan_vert;
  int16_t* dcan_final;
  int32_t* evals;
  uint32_t* gridL;
  uint32_t* gridR;
  int32_t* grangeL;      // per grid region: smallest and largest set bit of its mask
  int32_t* grangeR;      // (0x7FFF and -1 while empty), [gh][gw][2]
  int32_t* rowsL;        // per-row lists [lh][lw], packed u | d << 16
  int32_t* rowsR;
  int32_t* cnt;          // left counts, right counts, evaluation counts [3][lh]
  MeshHeader* hdr;
  int32_t* ptsL;
  int32_t* ptsR;
  int32_t* recsL;
  int32_t* recsR;
  float* planesL;
  float* planesR;
  RasterTri* tris;
  char* mesh_scratch;
  uint64_t mesh_scratch_per_view;
  int32_t* ownerL;
  int32_t* ownerR;
  int16_t* dplaneL;
  int16_t* dplaneR;
  int16_t* rawL;
  int16_t* rawR;
  const int32_t* lut;
  int32_t* dense_counts;  // candidate evaluations per dense block
  int16_t* outL;
  int16_t* outR;
  int16_t* chkL;         // median mode: checked maps before the median
  int16_t* chkR;
  int32_t* mfail;        // pinned host word the device mesh sets (to its nonzero
                         // status) when a view fails; null: the header only
};

// Every device pointer of a frame, as X(member).
#define ELAS_FRAME_POINTERS(X) X(left) X(right) X(descL) X(descR) X(csupL) X(csupR) \
  X(dcan_raw) X(dcan_incon) X(dcan_vert) X(dcan_final) X(evals) X(gridL) X(gridR) X(grangeL) \
  X(grangeR) X(rowsL) X(rowsR) X(cnt) X(hdr) X(ptsL) X(ptsR) X(recsL) X(recsR) X(planesL) \
  X(planesR) X(tris) X(mesh_scratch) X(ownerL) X(ownerR) X(dplaneL) X(dplaneR) X(rawL) X(rawR) \
  X(lut) X(dense_counts) X(outL) X(outR) X(chkL) X(chkR) X(mfail)

// A frame table in device memory holds each pointer as its byte offset from
// the table's own address, and a batched kernel adds that address (a kernel
// argument, so a global-memory pointer) back: the compiler then emits global
// rather than flat memory instructions for them, at one 64-bit scalar add per
// pointer. Offsets are taken modulo 2^64, so a null pointer comes back null.
inline void frame_to_table(Frame* f, uintptr_t table) {
#define ELAS_TO_OFFSET(m) f->m = reinterpret_cast<decltype(f->m)>((uintptr_t)f->m - table);
  ELAS_FRAME_POINTERS(ELAS_TO_OFFSET)
#undef ELAS_TO_OFFSET
}

__device__ __forceinline__ Frame global_frame(const Frame& t, const char* base) {
  Frame F = t;
#define ELAS_FROM_OFFSET(m) \
  F.m = reinterpret_cast<decltype(F.m)>(const_cast<char*>(base) + (uintptr_t)t.m);
  ELAS_FRAME_POINTERS(ELAS_FROM_OFFSET)
#undef ELAS_FROM_OFFSET
  return F;
}

// Stages of the path, in launch order.
// kStageRedun (past-only redundancy) and kStageMedian have no blocks unless
// the parameters select them.
enum Stage : int32_t {
  kStageDescriptor = 0,
  kStageSupport,
  kStageFilter,
  kStageRedun,
  kStageRows,
  kStageMesh,
  kStageRaster,
  kStageDense,
  kStageCheck,
  kStageMedian,
  kStageCount
};

// Tile variants the autotuner chooses between (identical results).
constexpr int kDescVariants = 3;   // descriptor rows per block: 4, 8, 16
constexpr int kDenseVariants = 3;  // dense rows per workgroup: 1, 2, 4

// Workgroups one frame needs for a stage (descriptor variant dv).
int32_t stage_blocks(int32_t stage, const Geometry& g, const KParams& p, int dv);
// Dynamic LDS bytes of a stage for a frame (0 if none).
size_t stage_lds(int32_t stage, const Geometry& g, const KParams& p);
// Band height of the raster for an image width.
int32_t raster_band_rows(int32_t w);

// One stage of one frame. With start/stop events (hipExtLaunchKernel) the
// events take the kernel's own start and end times.
hipError_t launch_stage(int32_t stage, const Frame& f, int variant, hipStream_t s,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// One stage of nf frames in one launch: frames and starts (nf + 1 prefix of
// the per-frame block counts) in device memory; lds: the largest per-frame
// dynamic LDS. Start/stop events as in launch_stage.
// bpf: the workgroups of every frame when all nf frames have that many (a
// block's frame is then one multiply away), else 0 (the frame is searched in
// starts).
// desc_nt: the descriptor stage writes the Sobel descriptors with
// non-temporal stores and the dense stage reads them (and the prior map)
// with non-temporal loads (separate kernels).
hipError_t launch_stage_batch(int32_t stage, const Frame* frames, const int32_t* starts,
                              int32_t nf, int32_t total_blocks, int32_t bpf, size_t lds,
                              int variant, bool desc_nt, hipStream_t s,
                              hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

// Blocks per frame of a prefix table starts[0..nf] when every frame has the
// same number, else 0.
int32_t uniform_blocks(const int32_t* starts, int32_t nf);

// The mesh stage (elas_mesh_device.hip): two workgroups per frame, for
// frames with both sides at most kDeviceMeshMaxSide.
hipError_t launch_mesh_frame(const Frame& f, hipStream_t s, hipEvent_t start = nullptr,
                             hipEvent_t stop = nullptr);
hipError_t launch_mesh_batch(const Frame* frames, int32_t nf, hipStream_t s,
                             hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Device mesh scratch per view (views that do not fit in LDS).
size_t mesh_global_scratch_per_view(const Geometry& g);
// Blocks of the dense launch for a tile variant (one candidate-count entry
// per block); the count array is sized for the largest, dense_blocks_max.
int32_t dense_blocks(const Geometry& g, int variant);
int32_t dense_blocks_max(const Geometry& g);

}  // namespace elas

// ---- entry points behind the C-ABI (elas_api.hip), for the server ---------
// elas_process / elas_process_batch with the device mesh's failure report
// going to the given pinned, device-mapped words (one per pair) instead of
// the handle's.
struct elas_handle;
struct elas_pair;
namespace elas {
int process_one(elas_handle* h, const uint8_t* left, const uint8_t* right, int32_t w,
                int32_t hp, int32_t stride, hipStream_t stream, int16_t* disp_left,
                int16_t* disp_right, int32_t* report);
int process_batch(elas_handle* h, int32_t n, const elas_pair* pairs, hipStream_t stream,
                  int32_t* const* reports);
// Frees the device buffers h keeps for calls on `stream` (single calls and
// batch pools, every size) after the stream has finished; returns their bytes.
int64_t release_stream_buffers(elas_handle* h, hipStream_t stream);
}  // namespace elas

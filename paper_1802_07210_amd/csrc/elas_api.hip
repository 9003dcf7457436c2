// C-ABI of elas_mi355x: parameter validation, the prior table, per-size
// device buffers, and the stage chain of one stereo pair.
//
// Stage chain of elas_process on the caller's stream:
//   k_descriptor (both views; Sobel or census) -> k_support -> k_filter
//   [-> k_redun, past-only redundancy] -> k_rows -> mesh -> k_raster
//   -> k_dense (both views) -> k_lrcheck [-> k_median].
// The mesh step runs either on the device (k_mesh, the default: the frame
// never returns to the host, so the call only enqueues work) or, with
// mesh_on_host, on the host between the two GPU phases as in the paper's
// CPU/FPGA split (Section IV, Fig. 3): wait for the per-row lists, gather
// them, pick the corner disparities, mesh both views on two host threads,
// upload the raster records.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "elas.h"
#include "elas_internal.h"

using namespace elas;

namespace {

thread_local std::string g_create_error;

// Timed kernels of elas_process, each with a start/stop event pair taken by
// hipExtLaunchKernel from the kernel's own dispatch: descriptor, support,
// filter, past-only redundancy, rows, mesh (host mode: events around the host
// step and its upload), raster, dense, check, median.
constexpr int kTimed = 10;

// One background host thread that builds the right view's mesh while the
// calling thread builds the left one (host mesh mode).
class Worker {
 public:
  Worker() : th_([this] { loop(); }) {}
  ~Worker() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    cv_.notify_all();
    th_.join();
  }
  void submit(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(m_);
      job_ = std::move(f);
      pending_ = true;
    }
    cv_.notify_all();
  }
  void wait() {
    std::unique_lock<std::mutex> lk(m_);
    cv_.wait(lk, [this] { return !pending_; });
  }

 private:
  void loop() {
    std::unique_lock<std::mutex> lk(m_);
    for (;;) {
      cv_.wait(lk, [this] { return stop_ || (pending_ && job_); });
      if (stop_) return;
      std::function<void()> f = std::move(job_);
      job_ = nullptr;
      lk.unlock();
      f();
      lk.lock();
      pending_ = false;
      cv_.notify_all();
    }
  }
  std::mutex m_;
  std::condition_variable cv_;
  std::function<void()> job_;
  bool pending_ = false, stop_ = false;
  std::thread th_;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device and pinned host memory for one image size.
struct Buffers {
  Geometry g{};
  size_t bytes = 0;              // device bytes of dev_block
  int32_t ntmax = 0;             // triangle capacity per view (2 * lattice + 2)
  void* dev_block = nullptr;     // every device array, carved below
  uint8_t *descL = nullptr, *descR = nullptr;
  uint4 *csupL = nullptr, *csupR = nullptr;  // census mode: support census
  int16_t *chkL = nullptr, *chkR = nullptr;  // median mode: checked maps
  size_t desc_bytes = 0, csup_bytes = 0;
  int16_t *dcan_raw = nullptr, *dcan_incon = nullptr, *dcan_vert = nullptr,
          *dcan_final = nullptr;
  int32_t* evals = nullptr;
  uint32_t *gridL = nullptr, *gridR = nullptr;
  int32_t *grangeL = nullptr, *grangeR = nullptr;
  int32_t *ownerL = nullptr, *ownerR = nullptr;
  int16_t *dplaneL = nullptr, *dplaneR = nullptr, *rawL = nullptr, *rawR = nullptr;
  int32_t* lut = nullptr;
  int32_t* dense_counts = nullptr;  // candidate evaluations per dense block
  // per-row lists (device copy for the device mesh)
  int32_t *rowsL = nullptr, *rowsR = nullptr, *cnt = nullptr;
  // mesh outputs
  MeshHeader* hdr = nullptr;
  int32_t *ptsL = nullptr, *ptsR = nullptr, *recsL = nullptr, *recsR = nullptr;
  float *planesL = nullptr, *planesR = nullptr;
  RasterTri* tris = nullptr;
  char* mesh_scratch = nullptr;
  // host-mapped per-row lists (host mesh mode): counts [3][lh], rows [lh][lw]
  void* host_block = nullptr;
  int32_t *hcnt = nullptr, *hrowL = nullptr, *hrowR = nullptr;              // host view
  int32_t *hcnt_dev = nullptr, *hrowL_dev = nullptr, *hrowR_dev = nullptr;  // device view
  // pinned staging of the host mesh's raster records + header
  void* up_host = nullptr;
  size_t up_cap = 0;
};

// Per (handle, stream) state of batched calls: the device frame tables and
// launch prefixes, two pinned staging buffers (each reused only after its
// upload has run), a capture stream and the graphs captured per batch shape.
struct BatchCtx {
  void* dev = nullptr;
  size_t dev_cap = 0;
  void* host[2] = {nullptr, nullptr};
  size_t host_cap[2] = {0, 0};
  hipEvent_t done[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int next = 0;
  hipStream_t capture = nullptr;
  std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
  void* tune_dev = nullptr;
  size_t tune_cap = 0;
};

}  // namespace

struct elas_handle {
  elas_params params{};
  KParams kp{};
  std::vector<int32_t> lut;
  // device buffers per (width, height, stream): calls on different streams
  // use disjoint buffers, so their frames can run concurrently
  std::map<std::tuple<int32_t, int32_t, hipStream_t>, Buffers*> cache;
  Buffers* last = nullptr;
  hipStream_t last_stream = nullptr;
  bool have_result = false;
  bool last_on_host = false;
  std::string err;
  double host_mesh_ms = 0.0, host_wait_ms = 0.0;
  MeshScratch* meshL = nullptr;
  MeshScratch* meshR = nullptr;
  std::vector<int32_t> ptsL, ptsR;     // host mesh mode: gathered lists (u, v, d)
  std::vector<int32_t> recsL, recsR;
  std::vector<float> planesL, planesR;
  MeshHeader hhdr{};
  Worker* worker = nullptr;
  hipEvent_t ev_lists = nullptr;
  hipEvent_t ev_upload = nullptr;
  bool upload_pending = false;
  bool timing = false;
  bool have_timing = false;
  hipEvent_t kev[kTimed][2] = {};
  bool kev_used[kTimed] = {};
  // the last timed batch: start/stop events of each launch and its stage
  bool have_batch_timing = false;
  std::vector<hipEvent_t> bev;
  std::vector<int32_t> bev_stage;
  // batches: per-stream frame tables and graphs, per-(size, stream) buffer
  // pools, tile variants chosen by the autotuner per (w, h, D)
  int32_t batch_flags = ELAS_BATCH_GRAPH | ELAS_BATCH_AUTOTUNE;
  std::map<hipStream_t, BatchCtx*> batch;
  std::map<std::tuple<int32_t, int32_t, hipStream_t>, std::vector<Buffers*>> pool;
  std::map<std::tuple<int32_t, int32_t, int32_t>, std::pair<int, int>> tuned;
  // support run length (lattice points per workgroup) per (w, h, D), when
  // tuned or set; otherwise the geometry's default
  std::map<std::tuple<int32_t, int32_t, int32_t>, int32_t> tuned_srun;
  hipStream_t tune_stream = nullptr;
  // device-mesh failure report: a pinned, device-mapped word that the mesh
  // kernel of a failing frame sets to its status; the next call on the
  // handle (or elas_get_stats) turns it into ELAS_ERR_INTERNAL
  int32_t* fail_host = nullptr;
  int32_t* fail_dev = nullptr;
  // the pairs of the last elas_process_batch call, for stage-by-stage reads:
  // the pair's parameter handle and buffers (host-mesh pairs: that handle's
  // last call), its stream, and whether it was meshed on the host
  struct BatchPair {
    elas_handle* ph;
    Buffers* b;
    hipStream_t stream;
    bool on_host;
  };
  std::vector<BatchPair> last_batch;
  int last_dense_variant = 0;  // dense tile variant of the last single call
  // the buffers of the last elas_process_noalloc call (pointers into the
  // device's scratch array; nothing is owned)
  Buffers noalloc_view;
};

namespace {

int fail(elas_handle* h, int code, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_create_error = msg;
  return code;
}

int fail_hip(elas_handle* h, const char* what, hipError_t e) {
  return fail(h, ELAS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                    \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return fail_hip(h, #expr, e_); \
  } while (0)

// The handle's failure report word (allocated once, when a device exists).
int ensure_fail_word(elas_handle* h) {
  if (h->fail_host) return ELAS_OK;
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, 64, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess)
    return fail(h, ELAS_ERR_OOM, std::string("hipHostMalloc of the report word: ") +
                                     hipGetErrorString(e));
  void* d = nullptr;
  e = hipHostGetDevicePointer(&d, p, 0);
  if (e != hipSuccess) {
    (void)hipHostFree(p);
    return fail_hip(h, "hipHostGetDevicePointer of the report word", e);
  }
  h->fail_host = static_cast<int32_t*>(p);
  h->fail_dev = static_cast<int32_t*>(d);
  __atomic_store_n(h->fail_host, 0, __ATOMIC_RELAXED);
  return ELAS_OK;
}

// Reports (once) a device-mesh failure of an earlier frame on this handle
// whose kernel has finished: ELAS_ERR_INTERNAL, else ELAS_OK.
int take_mesh_failure(elas_handle* h) {
  if (!h->fail_host) return ELAS_OK;
  const int32_t st = __atomic_load_n(h->fail_host, __ATOMIC_ACQUIRE);
  if (st == 0) return ELAS_OK;
  __atomic_store_n(h->fail_host, 0, __ATOMIC_RELAXED);
  return fail(h, ELAS_ERR_INTERNAL,
              std::string("the device mesh of an earlier frame on this handle failed (status ") +
                  std::to_string(st) +
                  (st == 1 ? ", flip rounds exhausted" : ", consistency check") +
                  "); that frame's maps were computed without plane priors");
}

void free_buffers(Buffers* b) {
  if (!b) return;
  if (b->dev_block) (void)hipFree(b->dev_block);
  if (b->host_block) (void)hipHostFree(b->host_block);
  if (b->up_host) (void)hipHostFree(b->up_host);
  delete b;
}

Geometry make_geometry(const elas_params& p, int32_t w, int32_t h) {
  Geometry g{};
  g.w = w;
  g.h = h;
  const int32_t s = p.candidate_stepsize;
  const int32_t kmin = (4 + s - 1) / s;
  const int32_t ku = (w - 5) / s, kv = (h - 5) / s;
  g.step = s;
  g.lu0 = kmin * s;
  g.lv0 = kmin * s;
  g.lw = ku >= kmin ? ku - kmin + 1 : 0;
  g.lh = kv >= kmin ? kv - kmin + 1 : 0;
  g.gw = (w + p.grid_size - 1) / p.grid_size;
  g.gh = (h + p.grid_size - 1) / p.grid_size;
  const int32_t D = p.disp_max - p.disp_min + 1;
  g.gwords = 2 * ((D + 63) / 64);
  // 8 x 8 filter tiles while every tile of the frame can have a CU of its
  // own, else 16 x 16 (fewer halo positions per tile)
  g.ftile = ((g.lw + 7) / 8) * ((g.lh + 7) / 8) <= 256 ? 8 : 16;
  // runs of 8 support points while runs of 16 would leave fewer than two
  // workgroups per CU, else 16 (less staging per point)
  g.srun = g.lh * ((g.lw + 15) / 16) < 512 ? 8 : 16;
  g.gdiv = (uint32_t)(((1ull << 31) + (uint64_t)p.grid_size - 1) / (uint64_t)p.grid_size);
  g.rowmul = ((1ull << 40) + (uint64_t)w - 1) / (uint64_t)w;
  return g;
}

// Offsets of every device array of one buffer set (256-byte aligned).
struct BufLayout {
  Geometry g{};
  size_t nlat = 0, nrows = 0;
  int32_t ntmax = 0;
  size_t descL, descR, csL, csR, raw0, inc, vert, fin, evals, gL, gR, grL, grR, oL, oR, dpL,
      dpR, rL, rR,
      lut, cnt, rowsL, rowsR, rc, hdr, pL, pR, recL, recR, plL, plR, tris, ms, chL, chR;
  size_t desc_bytes = 0, csup_bytes = 0;
  size_t total = 0;
};

BufLayout buffer_layout(const elas_params& p, int32_t w, int32_t hp) {
  BufLayout L;
  L.g = make_geometry(p, w, hp);
  const Geometry& g = L.g;
  const size_t npx = (size_t)w * hp;
  const size_t nlat = std::max<size_t>(1, (size_t)g.lw * g.lh);
  const size_t nrows = std::max<size_t>(1, (size_t)g.lh);
  const size_t ngrid = (size_t)g.gw * g.gh * g.gwords;
  L.nlat = nlat;
  L.nrows = nrows;
  L.ntmax = (int32_t)(2 * nlat + 2);
  const size_t ntmax = (size_t)L.ntmax;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  // descriptors: 16 bytes per pixel, or one uint64 of dense census per pixel
  // plus the support census of the lattice rows
  const bool census = p.descriptor == 1;
  const int32_t sw = p.census_support_window;
  const size_t cs_q = (sw * sw + 31) / 32 <= 4 ? 1 : 2;
  L.desc_bytes = npx * (census ? 8 : 16);
  L.csup_bytes = census ? (size_t)g.lh * w * cs_q * 16 : 0;
  L.descL = take(L.desc_bytes);
  L.descR = take(L.desc_bytes);
  L.csL = take(L.csup_bytes);
  L.csR = take(L.csup_bytes);
  L.raw0 = take(nlat * 2);
  L.inc = take(nlat * 2);
  L.vert = take(nlat * 2);
  L.fin = take(nlat * 2);
  L.evals = take(nlat * 4);
  L.gL = take(ngrid * 4 + 8);
  L.gR = take(ngrid * 4 + 8);
  L.grL = take((size_t)g.gw * g.gh * 8);
  L.grR = take((size_t)g.gw * g.gh * 8);
  L.oL = take(npx * 4);
  L.oR = take(npx * 4);
  L.dpL = take(npx * 2);
  L.dpR = take(npx * 2);
  L.rL = take(npx * 2);
  L.rR = take(npx * 2);
  L.lut = take(kMaxD * 4);
  L.cnt = take((size_t)dense_blocks_max(g) * 4);
  L.rowsL = take(nlat * 4);
  L.rowsR = take(nlat * 4);
  L.rc = take(3 * nrows * 4);
  L.hdr = take(sizeof(MeshHeader));
  L.pL = take(nlat * 12);
  L.pR = take(nlat * 12);
  L.recL = take(ntmax * 36);
  L.recR = take(ntmax * 36);
  L.plL = take(ntmax * 12);
  L.plR = take(ntmax * 12);
  L.tris = take(2 * ntmax * sizeof(RasterTri));
  // frames above the device mesh limit are always meshed on the host
  const bool dev_mesh = w <= kDeviceMeshMaxSide && hp <= kDeviceMeshMaxSide;
  L.ms = take(dev_mesh ? 2 * mesh_global_scratch_per_view(g) : 0);
  const size_t nchk = p.median_window > 1 ? npx * 2 : 0;
  L.chL = take(nchk);
  L.chR = take(nchk);
  L.total = off;
  return L;
}

// Points every device array of b at its offset in a block laid out as Lo.
void carve_buffers(const BufLayout& Lo, const elas_params& p, uint8_t* base, Buffers* b) {
  b->g = Lo.g;
  b->ntmax = Lo.ntmax;
  auto at = [&](size_t o) { return static_cast<void*>(base + o); };
  b->descL = static_cast<uint8_t*>(at(Lo.descL));
  b->descR = static_cast<uint8_t*>(at(Lo.descR));
  b->desc_bytes = Lo.desc_bytes;
  b->csup_bytes = Lo.csup_bytes;
  b->csupL = Lo.csup_bytes ? static_cast<uint4*>(at(Lo.csL)) : nullptr;
  b->csupR = Lo.csup_bytes ? static_cast<uint4*>(at(Lo.csR)) : nullptr;
  b->chkL = p.median_window > 1 ? static_cast<int16_t*>(at(Lo.chL)) : nullptr;
  b->chkR = p.median_window > 1 ? static_cast<int16_t*>(at(Lo.chR)) : nullptr;
  b->dcan_raw = static_cast<int16_t*>(at(Lo.raw0));
  b->dcan_incon = static_cast<int16_t*>(at(Lo.inc));
  b->dcan_vert = static_cast<int16_t*>(at(Lo.vert));
  b->dcan_final = static_cast<int16_t*>(at(Lo.fin));
  b->evals = static_cast<int32_t*>(at(Lo.evals));
  b->gridL = static_cast<uint32_t*>(at(Lo.gL));
  b->gridR = static_cast<uint32_t*>(at(Lo.gR));
  b->grangeL = static_cast<int32_t*>(at(Lo.grL));
  b->grangeR = static_cast<int32_t*>(at(Lo.grR));
  b->ownerL = static_cast<int32_t*>(at(Lo.oL));
  b->ownerR = static_cast<int32_t*>(at(Lo.oR));
  b->dplaneL = static_cast<int16_t*>(at(Lo.dpL));
  b->dplaneR = static_cast<int16_t*>(at(Lo.dpR));
  b->rawL = static_cast<int16_t*>(at(Lo.rL));
  b->rawR = static_cast<int16_t*>(at(Lo.rR));
  b->lut = static_cast<int32_t*>(at(Lo.lut));
  b->dense_counts = static_cast<int32_t*>(at(Lo.cnt));
  b->rowsL = static_cast<int32_t*>(at(Lo.rowsL));
  b->rowsR = static_cast<int32_t*>(at(Lo.rowsR));
  b->cnt = static_cast<int32_t*>(at(Lo.rc));
  b->hdr = static_cast<MeshHeader*>(at(Lo.hdr));
  b->ptsL = static_cast<int32_t*>(at(Lo.pL));
  b->ptsR = static_cast<int32_t*>(at(Lo.pR));
  b->recsL = static_cast<int32_t*>(at(Lo.recL));
  b->recsR = static_cast<int32_t*>(at(Lo.recR));
  b->planesL = static_cast<float*>(at(Lo.plL));
  b->planesR = static_cast<float*>(at(Lo.plR));
  b->tris = static_cast<RasterTri*>(at(Lo.tris));
  b->mesh_scratch = static_cast<char*>(at(Lo.ms));
}

int alloc_buffers(elas_handle* h, int32_t w, int32_t hp, Buffers** out) {
  Buffers* b = new Buffers();
  const BufLayout Lo = buffer_layout(h->params, w, hp);
  const size_t nlat = Lo.nlat, nrows = Lo.nrows;
  hipError_t e = hipMalloc(&b->dev_block, Lo.total);
  if (e != hipSuccess) {
    delete b;
    return fail(h, ELAS_ERR_OOM,
                std::string("hipMalloc of device buffers: ") + hipGetErrorString(e));
  }
  carve_buffers(Lo, h->params, static_cast<uint8_t*>(b->dev_block), b);
  b->bytes = Lo.total;
  // host-mapped per-row lists for the host mesh mode
  const size_t hcount = 3 * nrows + 2 * nlat;
  e = hipHostMalloc(&b->host_block, hcount * sizeof(int32_t), hipHostMallocMapped);
  if (e != hipSuccess) {
    free_buffers(b);
    return fail(h, ELAS_ERR_OOM,
                std::string("hipHostMalloc of list buffers: ") + hipGetErrorString(e));
  }
  void* hdev = nullptr;
  e = hipHostGetDevicePointer(&hdev, b->host_block, 0);
  if (e != hipSuccess) {
    free_buffers(b);
    return fail_hip(h, "hipHostGetDevicePointer of the list buffers", e);
  }
  b->hcnt = static_cast<int32_t*>(b->host_block);
  b->hrowL = b->hcnt + 3 * nrows;
  b->hrowR = b->hrowL + nlat;
  b->hcnt_dev = static_cast<int32_t*>(hdev);
  b->hrowL_dev = b->hcnt_dev + 3 * nrows;
  b->hrowR_dev = b->hrowL_dev + nlat;
  e = hipMemcpy(b->lut, h->lut.data(), h->lut.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_buffers(b);
    return fail_hip(h, "hipMemcpy of the prior table", e);
  }
  *out = b;
  return ELAS_OK;
}

// The buffers of single calls on one stream.
int get_buffers(elas_handle* h, int32_t w, int32_t hp, hipStream_t stream, Buffers** out) {
  const auto key = std::make_tuple(w, hp, stream);
  auto it = h->cache.find(key);
  if (it != h->cache.end()) {
    *out = it->second;
    return ELAS_OK;
  }
  const int rc = alloc_buffers(h, w, hp, out);
  if (rc == ELAS_OK) h->cache[key] = *out;
  return rc;
}

// The slot-th buffer set of a batch for one (size, stream).
int pool_buffers(elas_handle* h, int32_t w, int32_t hp, hipStream_t stream, size_t slot,
                 Buffers** out) {
  std::vector<Buffers*>& v = h->pool[std::make_tuple(w, hp, stream)];
  while (v.size() <= slot) {
    Buffers* b = nullptr;
    const int rc = alloc_buffers(h, w, hp, &b);
    if (rc != ELAS_OK) return rc;
    // a batch has workgroups enough to fill the chip: the larger filter
    // tiles and support runs, which compute and stage less halo per point
    // (runs of 32 measured faster up to D = 192, 16 at D = 256)
    b->g.ftile = 16;
    b->g.srun = h->kp.D <= 192 ? 32 : 16;
    v.push_back(b);
  }
  *out = v[slot];
  return ELAS_OK;
}

// Tile variants (descriptor, dense) for a frame size and disparity count:
// the autotuner's choice, else the defaults.
std::pair<int, int> variants_lookup(const elas_handle* h, int32_t w, int32_t hp, int32_t D,
                                    bool batched = false, bool census = false) {
  std::pair<int, int> v;
  auto it = h->tuned.find(std::make_tuple(w, hp, D));
  if (it != h->tuned.end()) {
    v = it->second;
  } else {
    // untuned: 8 descriptor rows per block and 2 dense rows per block; in
    // batches, whose many blocks fill the chip anyway, 16 descriptor rows (a
    // smaller halo share)
    v = std::make_pair(batched ? 2 : 1, 1);
  }
  (void)census;
  return v;
}

std::pair<int, int> variants_for(const elas_handle* h, int32_t w, int32_t hp) {
  return variants_lookup(h, w, hp, h->kp.D, false, h->kp.descriptor != 0);
}

// The frame's support run length: tuned or set for its (w, h, D), else the
// geometry's default.
void apply_support_run(const elas_handle* h, Frame* f) {
  auto it = h->tuned_srun.find(std::make_tuple(f->g.w, f->g.h, f->p.D));
  if (it != h->tuned_srun.end()) f->g.srun = it->second;
}

Frame make_frame(const elas_handle* h, const Buffers* b, const uint8_t* left,
                 const uint8_t* right, int32_t stride, int16_t* outL, int16_t* outR,
                 bool host_lists) {
  Frame f{};
  f.g = b->g;
  f.p = h->kp;
  f.stride = stride;
  f.raster_rows = raster_band_rows(b->g.w);
  f.left = left;
  f.right = right;
  f.descL = b->descL;
  f.descR = b->descR;
  f.csupL = b->csupL;
  f.csupR = b->csupR;
  f.chkL = b->chkL;
  f.chkR = b->chkR;
  f.dcan_raw = b->dcan_raw;
  f.dcan_incon = b->dcan_incon;
  f.dcan_vert = b->dcan_vert;
  f.dcan_final = b->dcan_final;
  f.evals = b->evals;
  f.gridL = b->gridL;
  f.gridR = b->gridR;
  f.grangeL = b->grangeL;
  f.grangeR = b->grangeR;
  f.rowsL = host_lists ? b->hrowL_dev : b->rowsL;
  f.rowsR = host_lists ? b->hrowR_dev : b->rowsR;
  f.cnt = host_lists ? b->hcnt_dev : b->cnt;
  f.hdr = b->hdr;
  f.ptsL = b->ptsL;
  f.ptsR = b->ptsR;
  f.recsL = b->recsL;
  f.recsR = b->recsR;
  f.planesL = b->planesL;
  f.planesR = b->planesR;
  f.tris = b->tris;
  f.mesh_scratch = b->mesh_scratch;
  f.mesh_scratch_per_view =
      (b->g.w <= kDeviceMeshMaxSide && b->g.h <= kDeviceMeshMaxSide)
          ? mesh_global_scratch_per_view(b->g)
          : 0;
  f.ownerL = b->ownerL;
  f.ownerR = b->ownerR;
  f.dplaneL = b->dplaneL;
  f.dplaneR = b->dplaneR;
  f.rawL = b->rawL;
  f.rawR = b->rawR;
  f.lut = b->lut;
  f.dense_counts = b->dense_counts;
  f.outL = outL;
  f.outR = outR;
  f.mfail = h->fail_dev;
  return f;
}

int ensure_upload(elas_handle* h, Buffers* b, size_t bytes) {
  if (bytes <= b->up_cap) return ELAS_OK;
  const size_t cap = align_up(std::max(bytes, b->up_cap * 3 / 2), 1 << 16);
  if (b->up_host) (void)hipHostFree(b->up_host);
  b->up_host = nullptr;
  b->up_cap = 0;
  const hipError_t e = hipHostMalloc(&b->up_host, cap, hipHostMallocDefault);
  if (e != hipSuccess) return fail(h, ELAS_ERR_OOM, "hipHostMalloc of the mesh staging buffer");
  b->up_cap = cap;
  return ELAS_OK;
}

bool finite_positive(float x) { return std::isfinite(x) && x > 0.0f; }

// Frames that the device mesh does not take: mesh_on_host, a side above the
// device mesh limit, or a mesh of the support points alone (no corners).
bool mesh_host_only(const elas_params& p, int32_t w, int32_t hp) {
  return p.mesh_on_host != 0 || p.add_corners == 0 || w > kDeviceMeshMaxSide ||
         hp > kDeviceMeshMaxSide;
}

// Each image corner takes the d of the nearest list point (squared
// distance; the earlier point in list order on ties).
void corner_disparities(const std::vector<int32_t>& pts, int32_t n, int32_t w, int32_t hp,
                        int32_t* out) {
  const int32_t cu[4] = {0, w - 1, 0, w - 1}, cv[4] = {0, 0, hp - 1, hp - 1};
  for (int c = 0; c < 4; ++c) {
    int64_t best = -1;
    int32_t d = -1;
    for (int32_t i = 0; i < n; ++i) {
      const int64_t du = pts[3 * i] - cu[c], dv = pts[3 * i + 1] - cv[c];
      const int64_t dist = du * du + dv * dv;
      if (best < 0 || dist < best) {
        best = dist;
        d = pts[3 * i + 2];
      }
    }
    out[c] = d;
  }
}

// Host mesh mode: concatenates k_rows' per-row lists (left: lattice order;
// right: (v, u) order) into (u, v, d) triples and derives the corners.
void gather_lists(elas_handle* h, Buffers* b, MeshHeader* hd) {
  const Geometry& g = b->g;
  int64_t evals = 0;
  int32_t nL = 0, nR = 0;
  for (int32_t l = 0; l < g.lh; ++l) {
    nL += b->hcnt[l];
    nR += b->hcnt[g.lh + l];
    evals += b->hcnt[2 * g.lh + l];
  }
  h->ptsL.resize((size_t)3 * std::max(nL, 1));
  h->ptsR.resize((size_t)3 * std::max(nR, 1));
  int32_t iL = 0, iR = 0;
  for (int32_t l = 0; l < g.lh; ++l) {
    const int32_t v = g.lv0 + l * g.step;
    const int32_t* rl = b->hrowL + (size_t)l * g.lw;
    for (int32_t j = 0, n = b->hcnt[l]; j < n; ++j, ++iL) {
      h->ptsL[3 * iL] = rl[j] & 0xFFFF;
      h->ptsL[3 * iL + 1] = v;
      h->ptsL[3 * iL + 2] = rl[j] >> 16;
    }
    const int32_t* rr = b->hrowR + (size_t)l * g.lw;
    for (int32_t j = 0, n = b->hcnt[g.lh + l]; j < n; ++j, ++iR) {
      h->ptsR[3 * iR] = rr[j] & 0xFFFF;
      h->ptsR[3 * iR + 1] = v;
      h->ptsR[3 * iR + 2] = rr[j] >> 16;
    }
  }
  *hd = MeshHeader{};
  hd->n[0] = nL;
  hd->n[1] = nR;
  // with corners: 2n + 2 triangles; without: at most 2n - 5, known once built
  hd->ntri[0] = nL > 0 ? 2 * nL + 2 : 0;
  hd->ntri[1] = nR > 0 ? 2 * nR + 2 : 0;
  hd->support_evals = evals;
  if (h->params.add_corners) {
    corner_disparities(h->ptsL, nL, g.w, g.h, hd->corners);
    corner_disparities(h->ptsR, nR, g.w, g.h, hd->corners + 4);
  } else {
    for (int c = 0; c < 8; ++c) hd->corners[c] = -1;
  }
}

// Host mesh mode, after k_rows: wait, gather, mesh both views, upload the
// raster records and the header.
int host_mesh_step(elas_handle* h, Buffers* b, hipStream_t stream) {
  const Geometry& g = b->g;
  const auto tw0 = std::chrono::steady_clock::now();
  HIP_TRY(hipEventRecord(h->ev_lists, stream));
  HIP_TRY(hipEventSynchronize(h->ev_lists));
  const auto t0 = std::chrono::steady_clock::now();
  h->host_wait_ms = std::chrono::duration<double, std::milli>(t0 - tw0).count();
  MeshHeader hd;
  gather_lists(h, b, &hd);
  // capacities: 2n + 2 triangles per view (exact with corners, a bound without)
  const int32_t capL = hd.ntri[0], capR = hd.ntri[1];
  // the staging buffer of the previous call must have been consumed
  if (h->upload_pending) HIP_TRY(hipEventSynchronize(h->ev_upload));
  h->upload_pending = false;
  const size_t tri_bytes = align_up((size_t)(capL + capR) * sizeof(RasterTri), 256);
  int rc = ensure_upload(h, b, tri_bytes + sizeof(MeshHeader));
  if (rc != ELAS_OK) return rc;
  RasterTri* tris = static_cast<RasterTri*>(b->up_host);
  h->recsL.assign((size_t)capL * 9, 0);
  h->planesL.assign((size_t)capL * 3, 0.f);
  h->recsR.assign((size_t)capR * 9, 0);
  h->planesR.assign((size_t)capR * 3, 0.f);
  const bool corners = h->params.add_corners != 0;
  auto mesh = [&](MeshScratch* s, const std::vector<int32_t>& pts, int32_t n, const int32_t* c,
                  RasterTri* out, std::vector<int32_t>& recs, std::vector<float>& planes) {
    if (n == 0) return 0;
    return corners ? build_mesh(s, pts.data(), n, c, g.w, g.h, out, recs.data(), planes.data())
                   : build_mesh_points(s, pts.data(), n, g.w, g.h, out, recs.data(),
                                       planes.data());
  };
  int32_t gotR = -1;
  h->worker->submit([&] {
    gotR = mesh(h->meshR, h->ptsR, hd.n[1], hd.corners + 4, tris + capL, h->recsR, h->planesR);
  });
  const int32_t gotL = mesh(h->meshL, h->ptsL, hd.n[0], hd.corners, tris, h->recsL, h->planesL);
  h->worker->wait();
  if (gotL < 0 || gotR < 0 || (corners && (gotL != capL || gotR != capR)))
    return fail(h, ELAS_ERR_INTERNAL, "host triangulation failed its consistency checks");
  const int32_t ntL = gotL, ntR = gotR;
  hd.ntri[0] = ntL;
  hd.ntri[1] = ntR;
  if (ntL < capL) {  // the right view's records follow the left's
    std::memmove(tris + ntL, tris + capL, (size_t)ntR * sizeof(RasterTri));
    h->recsL.resize((size_t)ntL * 9);
    h->planesL.resize((size_t)ntL * 3);
  }
  h->recsR.resize((size_t)ntR * 9);
  h->planesR.resize((size_t)ntR * 3);
  uint8_t* hdr_host = static_cast<uint8_t*>(b->up_host) + tri_bytes;
  std::memcpy(hdr_host, &hd, sizeof(hd));
  h->hhdr = hd;
  if (ntL + ntR > 0)
    HIP_TRY(hipMemcpyAsync(b->tris, b->up_host, (size_t)(ntL + ntR) * sizeof(RasterTri),
                           hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(b->hdr, hdr_host, sizeof(MeshHeader), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(h->ev_upload, stream));
  h->upload_pending = true;
  h->host_mesh_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return ELAS_OK;
}

// Header of the last call (device mesh: copied back; host mesh: kept).
int last_header(elas_handle* h, MeshHeader* out) {
  if (h->last_on_host) {
    *out = h->hhdr;
    return ELAS_OK;
  }
  HIP_TRY(hipStreamSynchronize(h->last_stream));
  HIP_TRY(hipMemcpy(out, h->last->hdr, sizeof(MeshHeader), hipMemcpyDeviceToHost));
  return ELAS_OK;
}

}  // namespace

extern "C" {

void elas_params_default(elas_params* p) {
  if (!p) return;
  p->disp_min = 0;
  p->disp_max = 127;
  p->support_threshold = 0.85f;
  p->support_texture = 10;
  p->candidate_stepsize = 5;
  p->incon_window_size = 5;
  p->incon_threshold = 5;
  p->incon_min_support = 5;
  p->redun_max_dist = 5;
  p->redun_threshold = 1;
  p->grid_size = 20;
  p->beta = 0.02f;
  p->gamma = 3.0f;
  p->sigma = 1.0f;
  p->sradius = 2;
  p->match_texture = 1;
  p->lr_threshold = 2;
  p->full_search = 0;
  p->mesh_on_host = 0;
  p->descriptor = 0;
  p->census_support_window = 9;
  p->census_dense_window = 5;
  p->ambiguity = 0;
  p->redundancy = 0;
  p->support_subsample = 1;
  p->median_window = 0;
  p->add_corners = 1;
}

int elas_create(const elas_params* p, elas_handle** out) {
  if (!p || !out) return fail(nullptr, ELAS_ERR_ARG, "null argument");
  *out = nullptr;
  const int32_t D = p->disp_max - p->disp_min + 1;
  if (p->disp_min < 0 || p->disp_max < p->disp_min || D > kMaxD)
    return fail(nullptr, ELAS_ERR_ARG,
                "disparity range must satisfy 0 <= min <= max, max-min < 256");
  if (p->candidate_stepsize < 1 || p->grid_size < 1)
    return fail(nullptr, ELAS_ERR_ARG, "candidate_stepsize and grid_size must be >= 1");
  if (p->incon_window_size < 0 || p->incon_threshold < 0 || p->incon_min_support < 0 ||
      p->redun_max_dist < 0 || p->redun_threshold < 0 || p->sradius < 0 ||
      p->lr_threshold < 0 || p->support_texture < 0 || p->match_texture < 0)
    return fail(nullptr, ELAS_ERR_ARG, "windows and thresholds must be >= 0");
  if (!finite_positive(p->beta) || !finite_positive(p->gamma) || !finite_positive(p->sigma) ||
      !std::isfinite(p->support_threshold))
    return fail(nullptr, ELAS_ERR_ARG, "beta, gamma, sigma must be finite and > 0");
  if (p->full_search != 0 && p->full_search != 1)
    return fail(nullptr, ELAS_ERR_ARG, "full_search must be 0 or 1");
  if (p->mesh_on_host != 0 && p->mesh_on_host != 1)
    return fail(nullptr, ELAS_ERR_ARG, "mesh_on_host must be 0 or 1");
  if (p->add_corners != 0 && p->add_corners != 1)
    return fail(nullptr, ELAS_ERR_ARG, "add_corners must be 0 or 1");
  if (p->incon_window_size > 16 || p->redun_max_dist > 16)
    return fail(nullptr, ELAS_ERR_UNSUPPORTED, "filter windows above 16 lattice steps");
  if ((p->descriptor != 0 && p->descriptor != 1) || (p->ambiguity != 0 && p->ambiguity != 1) ||
      (p->redundancy != 0 && p->redundancy != 1))
    return fail(nullptr, ELAS_ERR_ARG, "descriptor, ambiguity and redundancy must be 0 or 1");
  if (p->descriptor == 1 &&
      (p->census_support_window < 3 || p->census_support_window > 13 ||
       p->census_support_window % 2 == 0 || p->census_dense_window < 3 ||
       p->census_dense_window > 7 || p->census_dense_window % 2 == 0))
    return fail(nullptr, ELAS_ERR_ARG,
                "census windows must be odd: support 3..13, dense 3..7");
  if (p->support_subsample < 1 || p->support_subsample > 64)
    return fail(nullptr, ELAS_ERR_ARG, "support_subsample must be 1..64");
  if (p->median_window != 0 && p->median_window != 1 && p->median_window != 3 &&
      p->median_window != 5)
    return fail(nullptr, ELAS_ERR_ARG, "median_window must be 0, 1, 3 or 5");
  // Prior energy of a candidate at distance k from the plane mean: the ELAS
  // plane prior gamma + exp(-k^2 / (2 sigma^2)) as a negative log, over beta,
  // offset by log(gamma)/beta so that far candidates cost 0; rounded.
  std::vector<int32_t> lut(D);
  const double g = p->gamma, s = p->sigma, b = p->beta;
  for (int32_t k = 0; k < D; ++k) {
    const double x =
        -(std::log(g + std::exp(-(double)k * (double)k / (2.0 * s * s))) - std::log(g)) / b;
    if (!(std::fabs(x) < 4.0e6))
      return fail(nullptr, ELAS_ERR_UNSUPPORTED, "prior energy out of range (beta too small)");
    lut[k] = (int32_t)std::lround(x);
  }
  if (-lut[0] > (1 << 22))
    return fail(nullptr, ELAS_ERR_UNSUPPORTED, "prior energy out of the packed-key range");
  elas_handle* h = new (std::nothrow) elas_handle();
  if (!h) return fail(nullptr, ELAS_ERR_OOM, "out of host memory");
  h->params = *p;
  h->lut = std::move(lut);
  KParams& k = h->kp;
  k.dmin = p->disp_min;
  k.dmax = p->disp_max;
  k.D = D;
  k.support_threshold = p->support_threshold;
  k.support_texture = p->support_texture;
  k.incon_window = p->incon_window_size;
  k.incon_threshold = p->incon_threshold;
  k.incon_min_support = p->incon_min_support;
  k.redun_max_dist = p->redun_max_dist;
  k.redun_threshold = p->redun_threshold;
  k.grid_size = p->grid_size;
  k.sradius = p->sradius;
  k.match_texture = p->match_texture;
  k.lr_threshold = p->lr_threshold;
  k.full_search = p->full_search;
  k.lut_bias = -h->lut[0];
  k.descriptor = p->descriptor;
  k.cs_win = p->census_support_window;
  k.cd_win = p->census_dense_window;
  k.cs_q = (k.cs_win * k.cs_win + 31) / 32 <= 4 ? 1 : 2;
  k.ambiguity = p->ambiguity;
  k.redundancy = p->redundancy;
  k.subsample = p->support_subsample;
  k.median = p->median_window > 1 ? p->median_window : 0;
  k.mesh_max_rounds = kMeshMaxRounds;
  // the failure report word, when a device is present (no device: no call
  // on this handle can reach a kernel anyway)
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    const int rc = ensure_fail_word(h);
    if (rc != ELAS_OK) {
      g_create_error = h->err;
      delete h;
      return rc;
    }
  }
  h->meshL = mesh_scratch_create();
  h->meshR = mesh_scratch_create();
  *out = h;
  return ELAS_OK;
}

int elas_destroy(elas_handle* h) {
  if (!h) return ELAS_OK;
  if (!h->cache.empty() || !h->pool.empty()) (void)hipDeviceSynchronize();
  for (auto& kv : h->cache) free_buffers(kv.second);
  for (auto& kv : h->pool)
    for (Buffers* b : kv.second) free_buffers(b);
  for (auto& kv : h->batch) {
    BatchCtx* c = kv.second;
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    for (int k = 0; k < 2; ++k) {
      if (c->done[k]) (void)hipEventDestroy(c->done[k]);
      if (c->host[k]) (void)hipHostFree(c->host[k]);
    }
    if (c->dev) (void)hipFree(c->dev);
    if (c->tune_dev) (void)hipFree(c->tune_dev);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    delete c;
  }
  if (h->ev_lists) (void)hipEventDestroy(h->ev_lists);
  if (h->ev_upload) (void)hipEventDestroy(h->ev_upload);
  for (auto& pr : h->kev)
    for (hipEvent_t& e : pr)
      if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->bev) (void)hipEventDestroy(e);
  delete h->worker;
  if (h->fail_host) (void)hipHostFree(h->fail_host);
  mesh_scratch_destroy(h->meshL);
  mesh_scratch_destroy(h->meshR);
  delete h;
  return ELAS_OK;
}

const char* elas_last_error(const elas_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

int elas_process(elas_handle* h, const uint8_t* left, const uint8_t* right, int32_t w,
                 int32_t hp, int32_t stride, hipStream_t stream, int16_t* disp_left,
                 int16_t* disp_right) {
  return elas::process_one(h, left, right, w, hp, stride, stream, disp_left, disp_right,
                           nullptr);
}

}  // extern "C"

int elas::process_one(elas_handle* h, const uint8_t* left, const uint8_t* right, int32_t w,
                      int32_t hp, int32_t stride, hipStream_t stream, int16_t* disp_left,
                      int16_t* disp_right, int32_t* report) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (!left || !right || !disp_left || !disp_right)
    return fail(h, ELAS_ERR_ARG, "null image or output pointer");
  if (w < 9 || hp < 9 || w > 8192 || hp > 8192)
    return fail(h, ELAS_ERR_ARG, "image size must be 9..8192 in each dimension");
  if (stride < w) return fail(h, ELAS_ERR_ARG, "stride must be >= width");
  int rc0 = take_mesh_failure(h);
  if (rc0 != ELAS_OK) return rc0;
  rc0 = ensure_fail_word(h);
  if (rc0 != ELAS_OK) return rc0;
  const bool on_host = mesh_host_only(h->params, w, hp);
  if (on_host && !h->ev_lists) {
    HIP_TRY(hipEventCreateWithFlags(&h->ev_lists, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&h->ev_upload, hipEventDisableTiming));
  }
  if (on_host && !h->worker) h->worker = new Worker();
  Buffers* b = nullptr;
  int rc = get_buffers(h, w, hp, stream, &b);
  if (rc != ELAS_OK) return rc;
  h->have_result = false;
  h->have_timing = false;
  h->have_batch_timing = false;
  h->last = b;
  h->last_stream = stream;
  h->last_on_host = on_host;
  h->host_mesh_ms = h->host_wait_ms = 0.0;
  const bool timed = h->timing;
  if (timed && !h->kev[0][0])
    for (auto& pr : h->kev)
      for (hipEvent_t& e : pr) HIP_TRY(hipEventCreate(&e));
  for (bool& u : h->kev_used) u = false;

  Frame F = make_frame(h, b, left, right, stride, disp_left, disp_right, on_host);
  apply_support_run(h, &F);
  if (report) F.mfail = report;
  const std::pair<int, int> var = variants_for(h, w, hp);
  h->last_dense_variant = var.second;
  // one stage; while timing, kernel k records its start/stop events
  auto run = [&](int k, int32_t stage, int variant) -> hipError_t {
    if (!timed) return launch_stage(stage, F, variant, stream);
    if (stage == kStageMesh || stage_blocks(stage, F.g, F.p, variant) > 0) h->kev_used[k] = true;
    return launch_stage(stage, F, variant, stream, h->kev[k][0], h->kev[k][1]);
  };
  HIP_TRY(run(0, kStageDescriptor, var.first));
  HIP_TRY(run(1, kStageSupport, 0));
  HIP_TRY(run(2, kStageFilter, 0));
  HIP_TRY(run(3, kStageRedun, 0));
  HIP_TRY(run(4, kStageRows, 0));
  if (on_host) {
    if (timed) HIP_TRY(hipEventRecord(h->kev[5][0], stream));
    rc = host_mesh_step(h, b, stream);
    if (rc != ELAS_OK) return rc;
    if (timed) {
      HIP_TRY(hipEventRecord(h->kev[5][1], stream));
      h->kev_used[5] = true;
    }
  } else {
    HIP_TRY(run(5, kStageMesh, 0));
  }
  HIP_TRY(run(6, kStageRaster, 0));
  HIP_TRY(run(7, kStageDense, var.second));
  HIP_TRY(run(8, kStageCheck, 0));
  HIP_TRY(run(9, kStageMedian, 0));
  h->have_timing = timed;
  h->have_result = true;
  return ELAS_OK;
}

// ---- the entry point that allocates nothing ---------------------------------
// Every device buffer of one frame lives in this file-scope array, one copy
// per GPU, held until the process ends. In host code its name is only a
// stand-in: host code uses the address hipGetSymbolAddress returns for the
// current device, looked up once per device.
constexpr size_t kNoAllocBytes = (size_t)160 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on device dev (the current device).
int scratch_for_device(elas_handle* h, int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(h, ELAS_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(h, "hipGetSymbolAddress of the scratch array", e);
    if (!p) return fail(h, ELAS_ERR_HIP, "hipGetSymbolAddress returned no address");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<uint8_t*>(g_scratch_ptr[dev]);
  return ELAS_OK;
}

// The prior table, written into device memory from a kernel argument (no
// copy node, so a captured call stays a chain of kernels).
struct LutArg {
  int32_t v[kMaxD];
};

__global__ __launch_bounds__(kMaxD) void k_write_lut(LutArg a, int32_t* dst, int n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = a.v[i];
}

}  // namespace

extern "C" {

int elas_process_noalloc(elas_handle* h, const uint8_t* left, const uint8_t* right, int32_t w,
                         int32_t hp, int32_t stride, hipStream_t stream, int16_t* disp_left,
                         int16_t* disp_right) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (!left || !right || !disp_left || !disp_right)
    return fail(h, ELAS_ERR_ARG, "null image or output pointer");
  if (w < 9 || hp < 9 || w > 8192 || hp > 8192)
    return fail(h, ELAS_ERR_ARG, "image size must be 9..8192 in each dimension");
  if (stride < w) return fail(h, ELAS_ERR_ARG, "stride must be >= width");
  if (mesh_host_only(h->params, w, hp))
    return fail(h, ELAS_ERR_UNSUPPORTED,
                "the no-allocation path meshes on the device only (no mesh_on_host, corners "
                "added, sides up to 4096)");
  if (!h->fail_host) return fail(h, ELAS_ERR_UNSUPPORTED, "handle created without a device");
  const BufLayout Lo = buffer_layout(h->params, w, hp);
  if (Lo.total > kNoAllocBytes)
    return fail(h, ELAS_ERR_ARG,
                "frame needs " + std::to_string(Lo.total) + " bytes of scratch, the limit is " +
                    std::to_string(kNoAllocBytes));
  int rc = take_mesh_failure(h);
  if (rc != ELAS_OK) return rc;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (stream) {
    hipDevice_t sdev = 0;
    HIP_TRY(hipStreamGetDevice(stream, &sdev));
    if (sdev != dev) return fail(h, ELAS_ERR_ARG, "the stream belongs to another device");
  }
  uint8_t* base = nullptr;
  rc = scratch_for_device(h, dev, &base);
  if (rc != ELAS_OK) return rc;
  Buffers& b = h->noalloc_view;
  b = Buffers{};
  carve_buffers(Lo, h->params, base, &b);
  h->have_result = false;
  h->have_timing = false;
  h->have_batch_timing = false;
  LutArg la{};
  for (int32_t i = 0; i < h->kp.D; ++i) la.v[i] = h->lut[i];
  hipLaunchKernelGGL(k_write_lut, dim3(1), dim3(kMaxD), 0, stream, la, b.lut, h->kp.D);
  HIP_TRY(hipGetLastError());
  Frame F = make_frame(h, &b, left, right, stride, disp_left, disp_right, false);
  apply_support_run(h, &F);
  const std::pair<int, int> var = variants_for(h, w, hp);
  h->last_dense_variant = var.second;
  for (int32_t st = 0; st < kStageCount; ++st) {
    const int v = st == kStageDescriptor ? var.first : (st == kStageDense ? var.second : 0);
    HIP_TRY(launch_stage(st, F, v, stream));
  }
  h->last = &b;
  h->last_stream = stream;
  h->last_on_host = false;
  h->have_result = true;
  return ELAS_OK;
}

}  // extern "C"

namespace {

// One launch of a batch: a stage (and tile variant) over a table of frames.
struct LaunchRec {
  int32_t stage, variant, nf, total;
  int32_t bpf;   // blocks of every frame when uniform, else 0
  bool desc_nt;  // descriptor and dense stages: descriptors by non-temporal stores and loads
  size_t table_off, starts_off, lds;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int batch_ctx(elas_handle* h, hipStream_t stream, BatchCtx** out) {
  auto it = h->batch.find(stream);
  if (it != h->batch.end()) {
    *out = it->second;
    return ELAS_OK;
  }
  BatchCtx* c = new BatchCtx();
  for (int k = 0; k < 2; ++k)
    HIP_TRY(hipEventCreateWithFlags(&c->done[k], hipEventDisableTiming));
  HIP_TRY(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  h->batch[stream] = c;
  *out = c;
  return ELAS_OK;
}

// A batch whose Sobel descriptors (32 bytes per pixel for the two views)
// reach this size writes them with non-temporal stores, and the dense stage
// (their last reader) reads them, and the prior map, with non-temporal
// loads: beyond about three quarters of the 256 MB last-level (Infinity)
// cache, the dirty lines that ordinary stores leave are written back while
// the support and dense stages read, and lines the dense stage leaves cached
// slow the next batch's non-temporal writes to the same (reused) buffers
// (measured at 640x480 D=128: 24 and 32 pairs per call, and 1280x720 with
// 8, faster both ways; 8 pairs at 640x480, 79 MB, faster with ordinary
// stores and loads; 16 pairs, 157 MB, even).
constexpr uint64_t kDescNtBytes = 192ull << 20;

// Frame tables and block prefixes of every launch, in one blob.
void plan_batch(const std::vector<Frame>& frames, const std::vector<std::pair<int, int>>& var,
                std::vector<LaunchRec>* recs, std::vector<uint8_t>* blob) {
  recs->clear();
  blob->clear();
  uint64_t desc_bytes = 0;
  for (const Frame& f : frames)
    if (f.p.descriptor == 0) desc_bytes += 32ull * (uint64_t)f.g.w * (uint64_t)f.g.h;
  const bool desc_nt = desc_bytes >= kDescNtBytes;
  auto put = [&](const void* p, size_t bytes) {
    const size_t off = blob->size();
    blob->resize(align256(off + bytes));
    std::memcpy(blob->data() + off, p, bytes);
    return off;
  };
  const size_t main_table = put(frames.data(), frames.size() * sizeof(Frame));
  for (int32_t st = 0; st < kStageCount; ++st) {
    const bool tiled = st == kStageDescriptor || st == kStageDense;
    const int nvar = st == kStageDescriptor ? kDescVariants : (st == kStageDense ? kDenseVariants : 1);
    for (int v = 0; v < nvar; ++v) {
      std::vector<Frame> sub;
      std::vector<int32_t> starts(1, 0);
      size_t lds = 0;
      for (size_t i = 0; i < frames.size(); ++i) {
        const int fv = st == kStageDescriptor ? var[i].first : var[i].second;
        if (tiled && fv != v) continue;
        const int dv = tiled ? v : 0;
        sub.push_back(frames[i]);
        starts.push_back(starts.back() + stage_blocks(st, frames[i].g, frames[i].p, dv));
        lds = std::max(lds, stage_lds(st, frames[i].g, frames[i].p));
      }
      if (sub.empty()) continue;
      LaunchRec r{};
      r.stage = st;
      r.variant = v;
      r.nf = (int32_t)sub.size();
      r.total = starts.back();
      r.bpf = uniform_blocks(starts.data(), r.nf);
      r.desc_nt = (st == kStageDescriptor || st == kStageDense) && desc_nt;
      r.lds = lds;
      r.table_off = tiled ? put(sub.data(), sub.size() * sizeof(Frame)) : main_table;
      r.starts_off = put(starts.data(), starts.size() * sizeof(int32_t));
      recs->push_back(r);
    }
  }
}

// ev: null, or a start and a stop event per launch (hipExtLaunchKernel).
hipError_t enqueue_batch(const std::vector<LaunchRec>& recs, uint8_t* dev, hipStream_t s,
                         const hipEvent_t* ev = nullptr) {
  for (size_t i = 0; i < recs.size(); ++i) {
    const LaunchRec& r = recs[i];
    const hipError_t e = launch_stage_batch(
        r.stage, reinterpret_cast<const Frame*>(dev + r.table_off),
        reinterpret_cast<const int32_t*>(dev + r.starts_off), r.nf, r.total, r.bpf, r.lds,
        r.variant, r.desc_nt, s,
        ev ? ev[2 * i] : nullptr, ev ? ev[2 * i + 1] : nullptr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Times the descriptor and dense tile variants on this batch's frames of one
// (w, h, D) and keeps the fastest of each (the stages recompute identical
// outputs, so the batch's results are unaffected).
int autotune(elas_handle* h, BatchCtx* c, const std::vector<Frame>& frames,
             hipStream_t stream, std::pair<int, int>* best, int32_t* best_srun) {
  HIP_TRY(hipStreamSynchronize(stream));
  const size_t need = align256(frames.size() * sizeof(Frame)) + align256((frames.size() + 1) * 4);
  if (need > c->tune_cap) {
    if (c->tune_dev) HIP_TRY(hipFree(c->tune_dev));
    c->tune_dev = nullptr;
    c->tune_cap = 0;
    HIP_TRY(hipMalloc(&c->tune_dev, need));
    c->tune_cap = need;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // descriptor rows (variant 0..2), dense rows (0..2), support run length
  // (16 or 32 lattice points per workgroup, set in the frames' geometry)
  int choice[3] = {0, 1, 0};
  static const int32_t kRuns[2] = {16, 32};
  const int32_t stages[3] = {kStageDescriptor, kStageDense, kStageSupport};
  std::vector<Frame> fr(frames);
  for (int k = 0; k < 3; ++k) {
    float best_ms = 1e30f;
    const int nvar = k == 0 ? kDescVariants : (k == 1 ? kDenseVariants : 2);
    for (int v = 0; v < nvar; ++v) {
      if (k == 2)
        for (Frame& f : fr) f.g.srun = kRuns[v];
      const int lv = k == 2 ? 0 : v;  // the launch's tile variant
      std::vector<int32_t> starts(1, 0);
      for (const Frame& f : fr)
        starts.push_back(starts.back() + stage_blocks(stages[k], f.g, f.p, lv));
      uint8_t* dev = static_cast<uint8_t*>(c->tune_dev);
      const size_t soff = align256(fr.size() * sizeof(Frame));
      std::vector<Frame> table(fr);  // pointers as offsets from the table's address
      for (Frame& f : table) frame_to_table(&f, reinterpret_cast<uintptr_t>(dev));
      HIP_TRY(hipMemcpy(dev, table.data(), table.size() * sizeof(Frame), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(dev + soff, starts.data(), starts.size() * 4, hipMemcpyHostToDevice));
      size_t lds = 0;
      for (const Frame& f : fr) lds = std::max(lds, stage_lds(stages[k], f.g, f.p));
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIP_TRY(hipEventRecord(e0, stream));
        HIP_TRY(launch_stage_batch(stages[k], reinterpret_cast<const Frame*>(dev),
                                   reinterpret_cast<const int32_t*>(dev + soff),
                                   (int32_t)fr.size(), starts.back(),
                                   uniform_blocks(starts.data(), (int32_t)fr.size()), lds, lv,
                                   false, stream));
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms_min = std::min(ms_min, ms);
      }
      if (ms_min < best_ms) {
        best_ms = ms_min;
        choice[k] = v;
      }
    }
  }
  HIP_TRY(hipEventDestroy(e0));
  HIP_TRY(hipEventDestroy(e1));
  *best = std::make_pair(choice[0], choice[1]);
  *best_srun = kRuns[choice[2]];
  return ELAS_OK;
}

}  // namespace

extern "C" {

int elas_set_batch_flags(elas_handle* h, int32_t flags) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (flags & ~(ELAS_BATCH_GRAPH | ELAS_BATCH_AUTOTUNE))
    return fail(h, ELAS_ERR_ARG, "unknown batch flags");
  h->batch_flags = flags;
  return ELAS_OK;
}

int elas_process_batch(elas_handle* h, int32_t n, const elas_pair* pairs, hipStream_t stream) {
  return elas::process_batch(h, n, pairs, stream, nullptr);
}

}  // extern "C"

int elas::process_batch(elas_handle* h, int32_t n, const elas_pair* pairs, hipStream_t stream,
                        int32_t* const* reports) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (n < 0 || (n > 0 && !pairs)) return fail(h, ELAS_ERR_ARG, "bad pair array");
  for (int32_t i = 0; i < n; ++i) {
    const elas_pair& q = pairs[i];
    if (!q.left || !q.right || !q.disp_left || !q.disp_right)
      return fail(h, ELAS_ERR_ARG, "null image or output pointer in pair " + std::to_string(i));
    if (q.w < 9 || q.h < 9 || q.w > 8192 || q.h > 8192 || q.stride < q.w)
      return fail(h, ELAS_ERR_ARG, "bad size or stride in pair " + std::to_string(i));
  }
  int rc0 = take_mesh_failure(h);
  if (rc0 != ELAS_OK) return rc0;
  rc0 = ensure_fail_word(h);
  if (rc0 != ELAS_OK) return rc0;
  // pairs the device mesh cannot take go through single calls (host mesh)
  h->last_batch.assign(n, elas_handle::BatchPair{nullptr, nullptr, stream, false});
  std::vector<int32_t> dev_idx;
  for (int32_t i = 0; i < n; ++i) {
    const elas_pair& q = pairs[i];
    elas_handle* ph = q.params ? q.params : h;
    if (mesh_host_only(ph->params, q.w, q.h)) {
      const int rc = process_one(ph, q.left, q.right, q.w, q.h, q.stride, stream, q.disp_left,
                                 q.disp_right, reports ? reports[i] : h->fail_dev);
      if (rc != ELAS_OK) return fail(h, rc, std::string("pair ") + std::to_string(i) + ": " +
                                                elas_last_error(ph));
      h->last_batch[i] = elas_handle::BatchPair{ph, ph->last, stream, ph->last_on_host};
    } else {
      dev_idx.push_back(i);
    }
  }
  if (dev_idx.empty()) return ELAS_OK;
  std::vector<Frame> frames;
  std::vector<std::pair<int, int>> var;
  std::map<std::tuple<elas_handle*, int32_t, int32_t>, size_t> slots;
  for (int32_t i : dev_idx) {
    const elas_pair& q = pairs[i];
    elas_handle* ph = q.params ? q.params : h;
    size_t& slot = slots[std::make_tuple(ph, q.w, q.h)];
    Buffers* b = nullptr;
    int rc = pool_buffers(ph, q.w, q.h, stream, slot++, &b);
    if (rc != ELAS_OK) return fail(h, rc, elas_last_error(ph));
    frames.push_back(make_frame(ph, b, q.left, q.right, q.stride, q.disp_left, q.disp_right,
                                false));
    apply_support_run(h, &frames.back());
    // a failing device mesh reports on the calling handle (or the pair's word)
    frames.back().mfail = reports ? reports[i] : h->fail_dev;
    h->last_batch[i] = elas_handle::BatchPair{ph, b, stream, false};
    var.push_back(variants_lookup(h, q.w, q.h, ph->kp.D, true, ph->kp.descriptor != 0));
  }
  BatchCtx* c = nullptr;
  int rc = batch_ctx(h, stream, &c);
  if (rc != ELAS_OK) return rc;
  std::vector<LaunchRec> recs;
  std::vector<uint8_t> blob;
  plan_batch(frames, var, &recs, &blob);
  if (blob.size() > c->dev_cap) {  // grow the device tables; captured graphs refer to them
    HIP_TRY(hipDeviceSynchronize());
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    if (c->dev) HIP_TRY(hipFree(c->dev));
    c->dev = nullptr;
    c->dev_cap = 0;
    const size_t cap = align256(blob.size() * 2);
    HIP_TRY(hipMalloc(&c->dev, cap));
    c->dev_cap = cap;
  }
  const int k = c->next;
  c->next ^= 1;
  if (c->pending[k]) HIP_TRY(hipEventSynchronize(c->done[k]));
  c->pending[k] = false;
  if (blob.size() > c->host_cap[k]) {
    if (c->host[k]) HIP_TRY(hipHostFree(c->host[k]));
    c->host[k] = nullptr;
    c->host_cap[k] = 0;
    const size_t cap = align256(blob.size() * 2);
    HIP_TRY(hipHostMalloc(&c->host[k], cap, hipHostMallocDefault));
    c->host_cap[k] = cap;
  }
  // each frame table holds its pointers as offsets from its own device
  // address (several launches share the main table: converted once)
  std::vector<size_t> converted;
  for (const LaunchRec& r : recs) {
    if (std::find(converted.begin(), converted.end(), r.table_off) != converted.end()) continue;
    converted.push_back(r.table_off);
    const uintptr_t table = reinterpret_cast<uintptr_t>(c->dev) + r.table_off;
    for (int32_t i = 0; i < r.nf; ++i) {
      Frame f;
      uint8_t* at = blob.data() + r.table_off + (size_t)i * sizeof(Frame);
      std::memcpy(&f, at, sizeof(Frame));
      frame_to_table(&f, table);
      std::memcpy(at, &f, sizeof(Frame));
    }
  }
  std::memcpy(c->host[k], blob.data(), blob.size());
  HIP_TRY(hipMemcpyAsync(c->dev, c->host[k], blob.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(c->done[k], stream));
  c->pending[k] = true;
  uint8_t* dev = static_cast<uint8_t*>(c->dev);
  h->have_batch_timing = false;
  if (h->timing) {
    // timed: launched directly (not from a graph), each launch with its own
    // events; stages without workgroups launch nothing and are left out
    std::vector<LaunchRec> run;
    for (const LaunchRec& r : recs)
      if (r.total > 0 || r.stage == kStageMesh) run.push_back(r);
    while (h->bev.size() < 2 * run.size()) {
      hipEvent_t e = nullptr;
      HIP_TRY(hipEventCreate(&e));
      h->bev.push_back(e);
    }
    h->bev_stage.clear();
    for (const LaunchRec& r : run) h->bev_stage.push_back(r.stage);
    HIP_TRY(enqueue_batch(run, dev, stream, h->bev.data()));
    h->have_batch_timing = !run.empty();
  } else if (h->batch_flags & ELAS_BATCH_GRAPH) {
    std::vector<int64_t> sig;
    sig.push_back((int64_t)(uintptr_t)dev);
    for (const LaunchRec& r : recs) {
      sig.push_back(r.stage);
      sig.push_back(r.variant);
      sig.push_back(r.nf);
      sig.push_back(r.total);
      sig.push_back(r.bpf);
      sig.push_back(r.desc_nt ? 1 : 0);
      sig.push_back((int64_t)r.lds);
      sig.push_back((int64_t)r.table_off);
      sig.push_back((int64_t)r.starts_off);
    }
    auto it = c->graphs.find(sig);
    if (it == c->graphs.end()) {
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
      const hipError_t le = enqueue_batch(recs, dev, c->capture);
      const hipError_t ce = hipStreamEndCapture(c->capture, &graph);
      if (le != hipSuccess) return fail_hip(h, "batch launch during capture", le);
      if (ce != hipSuccess) return fail_hip(h, "hipStreamEndCapture", ce);
      hipGraphExec_t exec = nullptr;
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return fail_hip(h, "hipGraphInstantiate", ie);
      it = c->graphs.emplace(sig, exec).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, stream));
  } else {
    HIP_TRY(enqueue_batch(recs, dev, stream));
  }
  if (h->batch_flags & ELAS_BATCH_AUTOTUNE) {
    std::map<std::tuple<int32_t, int32_t, int32_t>, std::vector<Frame>> groups;
    for (const Frame& f : frames) {
      const auto key = std::make_tuple(f.g.w, f.g.h, f.p.D);
      if (!h->tuned.count(key)) groups[key].push_back(f);
    }
    for (auto& kv : groups) {
      std::pair<int, int> best;
      int32_t srun = 16;
      rc = autotune(h, c, kv.second, stream, &best, &srun);
      if (rc != ELAS_OK) return rc;
      h->tuned[kv.first] = best;
      h->tuned_srun[kv.first] = srun;
    }
  }
  return ELAS_OK;
}

int64_t elas::release_stream_buffers(elas_handle* h, hipStream_t stream) {
  (void)hipStreamSynchronize(stream);
  int64_t freed = 0;
  bool last_freed = false;
  auto drop = [&](Buffers* b) {
    freed += (int64_t)b->bytes;
    if (b == h->last) last_freed = true;
    for (auto& q : h->last_batch)
      if (q.b == b) q.b = nullptr;
    free_buffers(b);
  };
  for (auto it = h->cache.begin(); it != h->cache.end();) {
    if (std::get<2>(it->first) == stream) {
      drop(it->second);
      it = h->cache.erase(it);
    } else {
      ++it;
    }
  }
  for (auto it = h->pool.begin(); it != h->pool.end();) {
    if (std::get<2>(it->first) == stream) {
      for (Buffers* b : it->second) drop(b);
      it = h->pool.erase(it);
    } else {
      ++it;
    }
  }
  if (last_freed) {
    h->last = nullptr;
    h->have_result = false;
    h->have_timing = false;
  }
  return freed;
}

extern "C" {

int elas_device_bytes(elas_handle* h, int64_t* bytes) {
  if (!h || !bytes) return fail(h, ELAS_ERR_ARG, "null argument");
  int64_t n = 0;
  for (auto& kv : h->cache) n += (int64_t)kv.second->bytes;
  for (auto& kv : h->pool)
    for (Buffers* b : kv.second) n += (int64_t)b->bytes;
  for (auto& kv : h->batch) n += (int64_t)(kv.second->dev_cap + kv.second->tune_cap);
  *bytes = n;
  return ELAS_OK;
}

int elas_frame_bytes(elas_handle* h, int32_t w, int32_t hp, int64_t* bytes) {
  if (!h || !bytes) return fail(h, ELAS_ERR_ARG, "null argument");
  if (w < 9 || hp < 9 || w > 8192 || hp > 8192)
    return fail(h, ELAS_ERR_ARG, "image size must be 9..8192 in each dimension");
  *bytes = (int64_t)buffer_layout(h->params, w, hp).total;
  return ELAS_OK;
}

int elas_set_tile_variants(elas_handle* h, int32_t w, int32_t hp, int32_t desc_rows,
                           int32_t dense_rows, int32_t support_run) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  static const int32_t drows[3] = {4, 8, 16}, nrows[3] = {1, 2, 4};
  int dv = -1, nv = -1;
  for (int k = 0; k < 3; ++k) {
    if (drows[k] == desc_rows) dv = k;
    if (nrows[k] == dense_rows) nv = k;
  }
  if (dv < 0 || nv < 0 || w < 9 || hp < 9 ||
      (support_run != 8 && support_run != 16 && support_run != 32))
    return fail(h, ELAS_ERR_ARG,
                "descriptor rows must be 4, 8 or 16, dense rows 1, 2 or 4, support run 8, 16 "
                "or 32");
  const auto key = std::make_tuple(w, hp, h->kp.D);
  h->tuned[key] = std::make_pair(dv, nv);
  h->tuned_srun[key] = support_run;
  return ELAS_OK;
}

int elas_get_tuned_variants(elas_handle* h, int32_t w, int32_t hp, int32_t* desc_rows,
                            int32_t* dense_batch, int32_t* support_run) {
  if (!h || !desc_rows || !dense_batch || !support_run)
    return fail(h, ELAS_ERR_ARG, "null argument");
  const auto key = std::make_tuple(w, hp, h->kp.D);
  auto it = h->tuned.find(key);
  if (it == h->tuned.end()) return fail(h, ELAS_ERR_ARG, "no tuned variants for this size");
  static const int32_t rows[3] = {4, 8, 16}, batch[3] = {1, 2, 4};  // descriptor / dense rows
  *desc_rows = rows[it->second.first];
  *dense_batch = batch[it->second.second];
  auto is = h->tuned_srun.find(key);
  *support_run = is != h->tuned_srun.end() ? is->second : 16;
  return ELAS_OK;
}

}  // extern "C"

extern "C" {

int elas_set_mesh_round_limit(elas_handle* h, int32_t rounds) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (rounds < 1) return fail(h, ELAS_ERR_ARG, "round limit must be >= 1");
  h->kp.mesh_max_rounds = std::min(rounds, kMeshMaxRounds);
  return ELAS_OK;
}

int elas_set_timing(elas_handle* h, int32_t enable) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  h->timing = enable != 0;
  return ELAS_OK;
}

int elas_get_timing(elas_handle* h, elas_timing* out) {
  if (!h || !out) return fail(h, ELAS_ERR_ARG, "null argument");
  if (h->have_batch_timing) {  // the last timed call was a batch: launch times per stage
    const size_t nl = h->bev_stage.size();
    HIP_TRY(hipEventSynchronize(h->bev[2 * nl - 1]));
    float st[kStageCount] = {};
    for (size_t i = 0; i < nl; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->bev[2 * i], h->bev[2 * i + 1]));
      st[h->bev_stage[i]] += ms;
    }
    float span = 0.f;
    HIP_TRY(hipEventElapsedTime(&span, h->bev[0], h->bev[2 * nl - 1]));
    *out = elas_timing{};
    out->descriptor_ms = st[kStageDescriptor];
    out->support_ms = st[kStageSupport];
    out->filter_ms = st[kStageFilter] + st[kStageRedun];
    out->rows_ms = st[kStageRows];
    out->mesh_ms = st[kStageMesh];
    out->raster_ms = st[kStageRaster];
    out->dense_ms = st[kStageDense];
    out->lrcheck_ms = st[kStageCheck] + st[kStageMedian];
    out->device_span_ms = span;
    return ELAS_OK;
  }
  if (!h->have_result || !h->have_timing)
    return fail(h, ELAS_ERR_ARG, "no completed call with timing enabled");
  int last = 0;
  for (int k = 0; k < kTimed; ++k)
    if (h->kev_used[k]) last = k;
  HIP_TRY(hipEventSynchronize(h->kev[last][1]));
  float ms[kTimed] = {};
  for (int k = 0; k < kTimed; ++k)
    if (h->kev_used[k]) HIP_TRY(hipEventElapsedTime(&ms[k], h->kev[k][0], h->kev[k][1]));
  float span = 0.f;
  HIP_TRY(hipEventElapsedTime(&span, h->kev[0][0], h->kev[last][1]));
  out->descriptor_ms = ms[0];
  out->support_ms = ms[1];
  out->filter_ms = ms[2] + ms[3];
  out->rows_ms = ms[4];
  out->mesh_ms = ms[5];
  out->raster_ms = ms[6];
  out->dense_ms = ms[7];
  out->lrcheck_ms = ms[8] + ms[9];
  out->device_span_ms = span;
  out->host_wait_ms = h->host_wait_ms;
  out->host_mesh_ms = h->host_mesh_ms;
  return ELAS_OK;
}

int elas_get_stats(elas_handle* h, elas_stats* out) {
  if (!h || !out) return fail(h, ELAS_ERR_ARG, "null argument");
  if (!h->have_result) return fail(h, ELAS_ERR_ARG, "no completed call");
  MeshHeader hd;
  int rc = last_header(h, &hd);
  if (rc != ELAS_OK) return rc;
  HIP_TRY(hipStreamSynchronize(h->last_stream));
  std::vector<int32_t> counts(dense_blocks(h->last->g, h->last_dense_variant));
  HIP_TRY(hipMemcpy(counts.data(), h->last->dense_counts, counts.size() * sizeof(int32_t),
                    hipMemcpyDeviceToHost));
  int64_t cnt = 0;
  for (int32_t c : counts) cnt += c;
  rc = take_mesh_failure(h);
  if (hd.status[0] || hd.status[1])
    return fail(h, ELAS_ERR_INTERNAL,
                std::string("the device mesh of the last frame failed (status ") +
                    std::to_string(std::max(hd.status[0], hd.status[1])) + ")");
  if (rc != ELAS_OK) return rc;
  out->support_evals = hd.support_evals;
  out->dense_evals = cnt;
  out->n_support_left = hd.n[0];
  out->n_support_right = hd.n[1];
  out->n_tri_left = hd.ntri[0];
  out->n_tri_right = hd.ntri[1];
  out->host_mesh_ms = h->host_mesh_ms;
  for (int k = 0; k < 2; ++k) {
    out->mesh_rounds[k] = hd.rounds[k];
    out->mesh_flips[k] = hd.flips[k];
  }
  return ELAS_OK;
}

}  // extern "C"

namespace {

// One intermediate of a frame computed with ph's parameters in buffers b on
// `stream` (errors are reported on h). For a host-meshed frame the lists,
// triangles and planes are ph's host copies of its last call.
int read_intermediate(elas_handle* h, elas_handle* ph, Buffers* b, hipStream_t stream,
                      bool hm, int32_t which, void* dst, int64_t bytes, int64_t* needed) {
  const Geometry& g = b->g;
  MeshHeader hd;
  if (hm) {
    hd = ph->hhdr;
  } else {
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(&hd, b->hdr, sizeof(MeshHeader), hipMemcpyDeviceToHost));
  }
  const int64_t npx = (int64_t)g.w * g.h, nlat = (int64_t)g.lw * g.lh;
  const void* dsrc = nullptr;
  const void* hsrc = nullptr;
  int64_t size = 0;
  switch (which) {
    case ELAS_I_DESC_LEFT:
      if (ph->params.descriptor) return fail(h, ELAS_ERR_ARG, "census mode has no gradient descriptors");
      dsrc = b->descL; size = npx * 16; break;
    case ELAS_I_DESC_RIGHT:
      if (ph->params.descriptor) return fail(h, ELAS_ERR_ARG, "census mode has no gradient descriptors");
      dsrc = b->descR; size = npx * 16; break;
    case ELAS_I_CENSUS_DENSE_LEFT:
    case ELAS_I_CENSUS_DENSE_RIGHT:
      if (!ph->params.descriptor) return fail(h, ELAS_ERR_ARG, "not in census mode");
      dsrc = which == ELAS_I_CENSUS_DENSE_LEFT ? b->descL : b->descR;
      size = npx * 8;
      break;
    case ELAS_I_CENSUS_SUPPORT_LEFT:
    case ELAS_I_CENSUS_SUPPORT_RIGHT:
      if (!ph->params.descriptor) return fail(h, ELAS_ERR_ARG, "not in census mode");
      dsrc = which == ELAS_I_CENSUS_SUPPORT_LEFT ? (const void*)b->csupL : (const void*)b->csupR;
      size = (int64_t)b->csup_bytes;
      break;
    case ELAS_I_CHECKED_LEFT:
    case ELAS_I_CHECKED_RIGHT:
      if (ph->params.median_window <= 1) return fail(h, ELAS_ERR_ARG, "no median filter set");
      dsrc = which == ELAS_I_CHECKED_LEFT ? b->chkL : b->chkR;
      size = npx * 2;
      break;
    case ELAS_I_DCAN_RAW: dsrc = b->dcan_raw; size = nlat * 2; break;
    case ELAS_I_DCAN_INCON: dsrc = b->dcan_incon; size = nlat * 2; break;
    case ELAS_I_DCAN_VERT: dsrc = b->dcan_vert; size = nlat * 2; break;
    case ELAS_I_DCAN_FINAL: dsrc = b->dcan_final; size = nlat * 2; break;
    case ELAS_I_SUPPORT_LEFT:
      size = (int64_t)hd.n[0] * 12;
      if (hm) hsrc = ph->ptsL.data(); else dsrc = b->ptsL;
      break;
    case ELAS_I_SUPPORT_RIGHT:
      size = (int64_t)hd.n[1] * 12;
      if (hm) hsrc = ph->ptsR.data(); else dsrc = b->ptsR;
      break;
    case ELAS_I_CORNERS: hsrc = hd.corners; size = 32; break;
    case ELAS_I_TRI_LEFT:
      size = (int64_t)hd.ntri[0] * 36;
      if (hm) hsrc = ph->recsL.data(); else dsrc = b->recsL;
      break;
    case ELAS_I_TRI_RIGHT:
      size = (int64_t)hd.ntri[1] * 36;
      if (hm) hsrc = ph->recsR.data(); else dsrc = b->recsR;
      break;
    case ELAS_I_PLANE_LEFT:
      size = (int64_t)hd.ntri[0] * 12;
      if (hm) hsrc = ph->planesL.data(); else dsrc = b->planesL;
      break;
    case ELAS_I_PLANE_RIGHT:
      size = (int64_t)hd.ntri[1] * 12;
      if (hm) hsrc = ph->planesR.data(); else dsrc = b->planesR;
      break;
    case ELAS_I_OWNER_LEFT: dsrc = b->ownerL; size = npx * 4; break;
    case ELAS_I_OWNER_RIGHT: dsrc = b->ownerR; size = npx * 4; break;
    case ELAS_I_DPLANE_LEFT: dsrc = b->dplaneL; size = npx * 2; break;
    case ELAS_I_DPLANE_RIGHT: dsrc = b->dplaneR; size = npx * 2; break;
    case ELAS_I_GRID_LEFT: dsrc = b->gridL; size = (int64_t)g.gw * g.gh * g.gwords * 4; break;
    case ELAS_I_GRID_RIGHT: dsrc = b->gridR; size = (int64_t)g.gw * g.gh * g.gwords * 4; break;
    case ELAS_I_RAW_LEFT: dsrc = b->rawL; size = npx * 2; break;
    case ELAS_I_RAW_RIGHT: dsrc = b->rawR; size = npx * 2; break;
    case ELAS_I_LUT: hsrc = ph->lut.data(); size = (int64_t)ph->lut.size() * 4; break;
    default: return fail(h, ELAS_ERR_ARG, "unknown intermediate");
  }
  if (needed) *needed = size;
  if (!dst) return ELAS_OK;
  if (bytes < size) return fail(h, ELAS_ERR_ARG, "destination too small");
  if (size == 0) return ELAS_OK;
  if (hsrc) {
    std::memcpy(dst, hsrc, (size_t)size);
    return ELAS_OK;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(dst, dsrc, (size_t)size, hipMemcpyDeviceToHost));
  return ELAS_OK;
}

}  // namespace

extern "C" {

int elas_get_intermediate(elas_handle* h, int32_t which, void* dst, int64_t bytes,
                          int64_t* needed) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (!h->have_result) return fail(h, ELAS_ERR_ARG, "no completed call");
  return read_intermediate(h, h, h->last, h->last_stream, h->last_on_host, which, dst, bytes,
                           needed);
}

int elas_get_batch_intermediate(elas_handle* h, int32_t pair, int32_t which, void* dst,
                                int64_t bytes, int64_t* needed) {
  if (!h) return fail(nullptr, ELAS_ERR_ARG, "null handle");
  if (pair < 0 || pair >= (int32_t)h->last_batch.size())
    return fail(h, ELAS_ERR_ARG, "no such pair in the last batch");
  const elas_handle::BatchPair& q = h->last_batch[pair];
  // the buffers must still be the parameter handle's (not released since)
  bool held = q.b && q.b == q.ph->last && q.on_host;
  for (auto& kv : q.ph->pool)
    for (Buffers* b : kv.second) held |= b == q.b;
  if (!held) return fail(h, ELAS_ERR_ARG, "the pair's buffers are no longer held");
  return read_intermediate(h, q.ph, q.b, q.stream, q.on_host, which, dst, bytes, needed);
}


int elas_triangulate(const int32_t* pts, int32_t n, const int32_t* corners, int32_t w,
                     int32_t h, int32_t* recs_out, float* planes_out) {
  if (!pts || !recs_out || !planes_out || n < 1 || w < 3 || h < 3 || w > 8192 || h > 8192)
    return fail(nullptr, ELAS_ERR_ARG, "bad triangulation arguments");
  for (int32_t i = 0; i < n; ++i) {
    const int32_t u = pts[3 * i], v = pts[3 * i + 1];
    const bool ok = corners ? (u > 0 && u < w - 1 && v > 0 && v < h - 1)
                            : (u >= 0 && u <= w - 1 && v >= 0 && v <= h - 1);
    if (!ok) return fail(nullptr, ELAS_ERR_ARG, "support point outside the image (interior)");
  }
  MeshScratch* s = mesh_scratch_create();
  std::vector<RasterTri> tris((size_t)2 * n + 2);
  const int32_t nt = corners
                         ? build_mesh(s, pts, n, corners, w, h, tris.data(), recs_out, planes_out)
                         : build_mesh_points(s, pts, n, w, h, tris.data(), recs_out, planes_out);
  mesh_scratch_destroy(s);
  if (nt < 0 || (corners && nt != 2 * n + 2))
    return fail(nullptr, ELAS_ERR_ARG, "triangulation rejected its input");
  return nt;
}

}  // extern "C"

/*
 * elas_mi355x: the data-parallel hot path of ELAS dense stereo on AMD
 * Instinct MI355X (gfx950).
 *
 * Problem statement (Rahnama et al., arXiv 1802.07210, Sections I and III-A):
 * a rectified 8-bit grey stereo pair goes in, dense left and right disparity
 * maps come out. The path: gradient (Sobel) descriptors; sparse support
 * points matched across the full disparity range and kept by a
 * first/second-minimum ambiguity test (Section VI-B, eq. 1-2) plus a
 * reverse check; consistency and redundancy filtering (Section III-A,
 * Fig. 7A); a Delaunay mesh of the support points turned into an image-sized
 * matrix of slanted-plane priors and one-hot grid vectors (Section VI-D,
 * Fig. 2); per-pixel SAD matching over the candidates the prior allows; a
 * final left/right consistency check. The paper's post-processing is not
 * part of the path (Section III-A excludes it).
 *
 * Conventions: u is the column, v the row. Left pixel (u, v) corresponds to
 * right pixel (u - d, v). Output maps are int16, row stride w, value -1 for
 * invalid pixels, otherwise a disparity in [disp_min, disp_max].
 *
 * Error behaviour: every entry point returns ELAS_OK (0) or a negative
 * ELAS_ERR_* code; no C++ exception crosses this interface. After a failure
 * elas_last_error() describes it. Work that fails on the device after a
 * call has returned (the device mesh exhausting its flip rounds or failing a
 * consistency check; its frame is then matched without plane priors, so its
 * maps differ from the reference pipeline) is reported as ELAS_ERR_INTERNAL:
 * the failing kernel sets a pinned report word of the calling handle, and the
 * first later call on that handle (elas_process, elas_process_batch,
 * elas_process_noalloc, elas_get_stats) returns the error, once, without
 * doing its own work. elas_get_stats synchronises first, so it always
 * reports a failure of the last call. A server fails the tickets of the
 * affected pairs instead.
 *
 * Threading: a handle is not thread-safe. Calls on one handle must be
 * ordered (one host thread, and either one stream or streams the caller
 * synchronises). Different handles are independent.
 */
#ifndef ELAS_MI355X_H
#define ELAS_MI355X_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define ELAS_API __attribute__((visibility("default")))
#else
#define ELAS_API
#endif

#define ELAS_OK 0
#define ELAS_ERR_ARG (-1)          /* bad argument or parameter */
#define ELAS_ERR_OOM (-2)          /* device or pinned host allocation failed */
#define ELAS_ERR_HIP (-3)          /* a HIP runtime call failed; see elas_last_error */
#define ELAS_ERR_UNSUPPORTED (-4)  /* parameters outside what the kernels support */
#define ELAS_ERR_INTERNAL (-5)     /* an internal consistency check failed */

/* Matching parameters. Defaults (elas_params_default) are the values the
 * workloads use; fields the paper does not fix are the readings stated in
 * each comment. */
typedef struct elas_params {
  int32_t disp_min;            /* smallest disparity, >= 0 (0) */
  int32_t disp_max;            /* largest disparity; D = max-min+1 in 1..256 (127) */
  float   support_threshold;   /* ambiguity test, eq. 1-2: keep iff m1 < t*m2 in FP32 (0.85) */
  int32_t support_texture;     /* min texture of a 512-bit support descriptor (10) */
  int32_t candidate_stepsize;  /* support candidate lattice step in pixels (5) */
  int32_t incon_window_size;   /* consistency window half-size, lattice steps (5) */
  int32_t incon_threshold;     /* |d'-d| <= this is consistent (5) */
  int32_t incon_min_support;   /* consistent neighbours needed (5) */
  int32_t redun_max_dist;      /* redundancy search distance, lattice steps (5) */
  int32_t redun_threshold;     /* |d'-d| <= this is redundant (1) */
  int32_t grid_size;           /* grid-vector region size in pixels, Fig. 2 (20) */
  float   beta;                /* likelihood scale of the SAD energy (0.02) */
  float   gamma;               /* floor of the plane prior (3) */
  float   sigma;               /* width of the plane prior (1) */
  int32_t sradius;             /* plane candidates |d - d_plane| <= sradius (2) */
  int32_t match_texture;       /* min texture of a 128-bit dense descriptor (1) */
  int32_t lr_threshold;        /* left/right agreement tolerance (2) */
  int32_t full_search;         /* 1: dense candidates = every admissible d (0) */
  int32_t mesh_on_host;        /* 1: triangulate on the host between the two GPU
                                  phases, as the paper's CPU/FPGA split does
                                  (Section IV); 0: on the device (0) */
  /* The embedded variant (Section VI) and the optional steps. */
  int32_t descriptor;          /* 0: Sobel descriptors + SAD; 1: census descriptors
                                  + Hamming distance, Section VI-A (0). Census bit i
                                  = i-th window offset in row-major order, set iff
                                  that neighbour is inside the image and darker than
                                  the centre; texture = number of set bits */
  int32_t census_support_window; /* support census window, odd 3..13 (9) */
  int32_t census_dense_window; /* dense census window, odd 3..7 (5) */
  int32_t ambiguity;           /* 0: eq. 1-2 ratio test; 1: eq. 3 shift-sum, keep iff
                                  m1 <= m2/2 + m2/4 + m2/8 + m2/32 (truncating) (0) */
  int32_t redundancy;          /* 0: two-sided redundancy (Fig. 7A); 1: past-only
                                  (Section VI-C, Fig. 7B): down each lattice column,
                                  then along each row, a point goes iff a point that
                                  survived the pass lies within redun_max_dist
                                  earlier positions with |d'-d| <= redun_threshold (0) */
  int32_t support_subsample;   /* 1..64: keep the support points whose index in
                                  lattice order is a multiple of k, before the right
                                  list, corners and grid vectors (Section VII-B) (1) */
  int32_t median_window;       /* 0 or 1: none; 3 or 5: median of the checked maps
                                  (Section VIII): invalid pixels stay invalid, valid
                                  ones take the lower median of the valid values in
                                  the window clipped to the image (0) */
  int32_t add_corners;         /* 1: the four image corners join each view's mesh,
                                  each with the d of its nearest support point, so
                                  every pixel has a plane prior (1); 0: the mesh of
                                  the support points alone (Section III-A
                                  triangulates the support points only): pixels
                                  outside their convex hull get no plane prior and
                                  take their candidates from the grid vectors
                                  alone. 0 meshes on the host */
} elas_params;

typedef struct elas_handle elas_handle;

/* Counters of the most recent elas_process call on a handle. */
typedef struct elas_stats {
  int64_t support_evals;       /* 512-bit SAD evaluations, both search directions */
  int64_t dense_evals;         /* candidate evaluations summed over both dense maps */
  int32_t n_support_left;      /* support points, left view (corners excluded) */
  int32_t n_support_right;     /* support points, right view */
  int32_t n_tri_left;          /* triangles of the left-view mesh */
  int32_t n_tri_right;
  double  host_mesh_ms;        /* host time spent triangulating (both views) */
  int32_t mesh_rounds[2];      /* device mesh: synchronous flip rounds, left and right
                                  view (0 when meshed on the host) */
  int32_t mesh_flips[2];       /* device mesh: edge flips, left and right view */
} elas_stats;

/* Per-kernel device times of the most recent elas_process call (only while
 * timing is enabled with elas_set_timing): each kernel is launched with
 * hipExtLaunchKernel start/stop events, which take the kernel's own start and
 * end, so the figures exclude launch gaps and match a profiler's kernel
 * durations. */
typedef struct elas_timing {
  float descriptor_ms;         /* k_descriptor (Sobel or census), both views */
  float support_ms;            /* k_support (both search directions) */
  float filter_ms;             /* k_filter (consistency, two-sided redundancy) plus
                                  k_redun when past-only redundancy is set */
  float rows_ms;               /* k_rows: support lists and grid vectors */
  float mesh_ms;               /* device mesh kernel, or (mesh_on_host) the host
                                  step and the upload of its records */
  float raster_ms;             /* k_raster */
  float dense_ms;              /* k_dense, both views */
  float lrcheck_ms;            /* k_check, plus k_median when a median is set */
  float device_span_ms;        /* first kernel start to last kernel end, gaps and
                                  host step included */
  double host_wait_ms;         /* calling thread blocked until the lists were ready */
  double host_mesh_ms;         /* host triangulation and record building */
} elas_timing;

/* Fills *p with the default parameters: the matching parameters of the
 * original algorithm (Section III-A) at the values given beside each field,
 * the Sobel descriptor and eq. 1-2 ratio test of the plain path, and none of
 * the Section VI changes. A NULL p is ignored. */
ELAS_API void elas_params_default(elas_params* p);

/* Validates *p and creates a handle (Section III-A: the matching parameters;
 * the prior table of the plane prior). Computes the prior table and, when a
 * device is present, allocates the handle's pinned failure report word;
 * device memory is allocated by the first elas_process per image size.
 * Returns ELAS_ERR_ARG for invalid values (null pointers, D outside 1..256,
 * negative windows or thresholds, step or grid size < 1, non-positive or
 * non-finite beta/gamma/sigma) and ELAS_ERR_UNSUPPORTED when the prior
 * energies exceed the kernels' packed-key range (|lut[0]| > 2^22) or a
 * filter window exceeds 16 lattice steps (incon_window_size, redun_max_dist). */
ELAS_API int elas_create(const elas_params* p, elas_handle** out);

/* Frees the handle and everything it owns (the per-size buffers of the
 * path of Section III-A). Waits for its pending work. NULL is accepted.
 * Returns ELAS_OK; HIP errors while waiting or freeing are ignored and the
 * handle is freed regardless. */
ELAS_API int elas_destroy(elas_handle* h);

/* Computes both disparity maps of one pair.
 *   left, right      device pointers, uint8, h_px rows of `stride` bytes
 *                    (the first w bytes of each row are used); caller-owned.
 *   w, h_px          image size, 9..8192 each.
 *   stride           row pitch of left and right in bytes, >= w.
 *   stream           HIP stream the work is ordered on (0 = null stream).
 *   disp_left/right  device pointers, int16, w*h_px elements, row stride w;
 *                    caller-owned.
 * The path of Section III-A, Fig. 1: descriptors, support matching and its
 * filters, the mesh and its plane prior, dense matching, the left/right
 * check (with the Section VI options the parameters select).
 * Stream-ordered: outputs are valid once `stream` reaches the end of the
 * enqueued work; with the default device mesh the call only enqueues work.
 * With mesh_on_host the call blocks the calling thread until the support
 * stage has finished, triangulates on the host, then enqueues the rest (the
 * CPU/accelerator split of the paper, Section IV); frames wider or taller
 * than 4096 pixels, and every frame with add_corners = 0, are triangulated
 * this way. Inputs must stay valid
 * until the stream passes the work. Device buffers are kept per (image size,
 * stream): they are allocated on the first call for that pair (which
 * synchronises the device) and reused by later calls on the same stream, so
 * frames issued on different streams run concurrently on the device. A
 * handle is used by one host thread at a time. */
ELAS_API int elas_process(elas_handle* h, const uint8_t* left, const uint8_t* right,
                          int32_t w, int32_t h_px, int32_t stride, hipStream_t stream,
                          int16_t* disp_left, int16_t* disp_right);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): elas_process without any
 * allocation. Same arguments, results and stream ordering as elas_process
 * (bit-identical maps). Every device buffer of the frame lives in one
 * library-owned device array of 160 MiB per GPU (held until the process
 * ends), so the frame's footprint, elas_frame_bytes, must be at most
 * 167772160 bytes (every workload shape fits: 1280x720 at D = 192 needs
 * about 62 MiB): ELAS_ERR_ARG otherwise. The call makes no hipMalloc, hipFree
 * or other allocating call, no memset and no copy: the prior table is
 * written by a kernel from its argument, so the call enqueues kernels only.
 * The stream must belong to the current device (ELAS_ERR_ARG otherwise).
 * Device mesh only: ELAS_ERR_UNSUPPORTED with mesh_on_host, add_corners = 0
 * or a side above 4096, or for a handle created without a device. All calls on one GPU share
 * that GPU's array, which keeps the last call's contents (elas_get_stats and
 * elas_get_intermediate read them): calls that overlap on one GPU (other
 * streams, other handles, other host threads) race; order them. Timing is
 * not recorded. */
ELAS_API int elas_process_noalloc(elas_handle* h, const uint8_t* left, const uint8_t* right,
                                  int32_t w, int32_t h_px, int32_t stride, hipStream_t stream,
                                  int16_t* disp_left, int16_t* disp_right);

/* One stereo pair of a batch (all pointers device memory, caller-owned). */
typedef struct elas_pair {
  const uint8_t* left;          /* uint8, h rows of `stride` bytes */
  const uint8_t* right;
  int32_t w, h, stride;         /* as for elas_process */
  int16_t* disp_left;           /* int16 [h][w] outputs */
  int16_t* disp_right;
  elas_handle* params;          /* NULL: the batch handle's parameters; otherwise
                                   this handle's (e.g. another disparity range) */
} elas_pair;

/* Flags of elas_process_batch (both set by default). The batch is the
 * device's form of the paper's pipelining (Section V-B: many inputs in the
 * accelerator at once); capture and tuning only change how it is launched.
 * elas_set_batch_flags returns ELAS_ERR_ARG for a null handle or unknown
 * bits. */
enum elas_batch_flags {
  ELAS_BATCH_GRAPH = 1,         /* capture each batch shape's launches in a HIP graph
                                   once and replay it */
  ELAS_BATCH_AUTOTUNE = 2       /* on the first batch with a new (w, h, D), time the
                                   descriptor (4/8/16 rows per block), dense (1/2/4
                                   rows per block) and support (16/32 lattice points per
                                   block) variants on its frames and keep the fastest;
                                   results are identical for all */
};
ELAS_API int elas_set_batch_flags(elas_handle* h, int32_t flags);

/* Several frames in flight at once, as the paper's dual system keeps two
 * frames in its pipeline (Section VII-D), taken further: computes n pairs of
 * possibly different sizes and disparity ranges with one
 * launch per stage (and tile variant) for the whole batch: every stage's
 * kernel covers the workgroups of all frames, a workgroup finds its frame in
 * a device table (uploaded by the call from pinned memory), and the two mesh
 * workgroups of every frame run side by side. Equivalent, pair by pair, to
 * elas_process with the pair's parameters; bit-identical outputs. Buffers
 * come from per-(size, stream) pools in the pair's parameter handle, so
 * batches on different streams run concurrently; a batch reuses them only
 * after the stream has passed the previous batch. Pairs the device mesh
 * cannot take (a side above 4096, mesh_on_host, or add_corners = 0) are processed by
 * elas_process on the same stream first. Stream-ordered; the call returns
 * after enqueueing, except for the autotuning pass (synchronous, once per new
 * size). The handle is used by one host thread at a time.
 * Errors: ELAS_ERR_ARG (null handle, n < 0, a null pointer or bad size in a
 * pair, with the pair's index in elas_last_error), ELAS_ERR_OOM, ELAS_ERR_HIP. */
ELAS_API int elas_process_batch(elas_handle* h, int32_t n, const elas_pair* pairs,
                                hipStream_t stream);

/* Tile variants the autotuner chose for (w, h) at this handle's disparity
 * count: descriptor rows per block, dense rows per block (the rows a
 * workgroup stages in LDS, the device's counterpart of the line buffers of
 * Section V-A) and support run length (lattice points per support workgroup,
 * whose reachable descriptor columns it stages in LDS: 16 or 32 when tuned).
 * ELAS_ERR_ARG for null pointers or if none has been chosen yet. */
ELAS_API int elas_get_tuned_variants(elas_handle* h, int32_t w, int32_t h_px,
                                     int32_t* desc_rows, int32_t* dense_rows,
                                     int32_t* support_run);

/* Fixes the tile variants of (w, h) at this handle's disparity count, as the
 * autotuner would (descriptor rows per block 4, 8 or 16; dense rows per
 * block 1, 2 or 4: the LDS row tiles of Section V-A's line buffers; support
 * run length 8, 16 or 32 lattice points per workgroup); used by single and
 * batched calls, and the autotuner then leaves that size alone. Results do
 * not depend on the variants. ELAS_ERR_ARG for other values or a side below
 * 9. */
ELAS_API int elas_set_tile_variants(elas_handle* h, int32_t w, int32_t h_px, int32_t desc_rows,
                                    int32_t dense_rows, int32_t support_run);

/* Device bytes of the buffers one pair of size (w, h_px) needs with h's
 * parameters (descriptors, lattice, grid, mesh, maps: every intermediate of
 * Section III-A stays resident in HBM, where Section V-A streams through line
 * buffers); what a server admits against its memory budget. No HIP call.
 * ELAS_ERR_ARG for null pointers or sizes outside 9..8192. */
ELAS_API int elas_frame_bytes(elas_handle* h, int32_t w, int32_t h_px, int64_t* bytes);

/* Device bytes the handle holds now (the Section V-A memory of every frame
 * in flight): the buffer sets of every (size, stream) of single and batched
 * calls, and the batch tables. No HIP call. ELAS_ERR_ARG for null pointers. */
ELAS_API int elas_device_bytes(elas_handle* h, int64_t* bytes);

/* ---- serving: continuous batching of pairs from many cameras ----------
 * The paper's throughput setting (Section VII-D: frames streamed through
 * the pipelined accelerators, two frames in flight in the dual system), for
 * many cameras at once. A server owns a worker thread and max_inflight
 * streams. elas_server_submit
 * queues a pair (device images and outputs, caller-owned until the ticket
 * completes) and returns a ticket at once. Whenever a stream is free and
 * pairs wait, the worker launches the longest-waiting ones (up to max_batch,
 * and only while the buffer sets they need fit memory_budget: a stream keeps
 * one set of elas_frame_bytes per pair of a size in its largest batch; when
 * the oldest pair does not fit, idle streams' sets are freed first) as one
 * elas_process_batch call; pairs that arrive while
 * others run are admitted as streams and memory free up, and overlap on the
 * device with the batches already running. With plain = 1 the server runs
 * one pair at a time through elas_process (the unbatched baseline). Results
 * are identical to elas_process of the same pair. Latency = submission to
 * the worker observing the batch's completion (host clock). The handle h and
 * every pair's parameter handle belong to the worker while the server
 * exists; nothing else may use them. */
typedef struct elas_server elas_server;
typedef struct elas_server_config {
  int32_t max_batch;            /* pairs per launch, 1..1024 (32) */
  int32_t max_inflight;         /* batches on the device at once, 1..16 (3) */
  int64_t memory_budget;        /* device bytes the server's pairs may keep resident:
                                   buffer sets per (stream, size), (32 GiB) */
  int32_t plain;                /* 1: one pair at a time via elas_process (0) */
} elas_server_config;
typedef struct elas_server_stats {
  int64_t submitted, completed;
  int64_t batches, batched_pairs;  /* launches and the pairs they carried */
  int64_t peak_bytes_in_flight;    /* footprint of the pairs on the device at once */
  int64_t queued;                  /* waiting now */
  int64_t bytes_in_flight;         /* admitted now */
  int64_t resident_bytes;          /* buffer sets held for the server's pairs now */
  int64_t peak_resident_bytes;     /* and at most; never above memory_budget */
} elas_server_stats;
/* Fills *c with the defaults given beside each field. */
ELAS_API void elas_server_config_default(elas_server_config* c);
/* ELAS_ERR_ARG for out-of-range settings, ELAS_ERR_HIP if streams fail. */
ELAS_API int elas_server_create(elas_handle* h, const elas_server_config* cfg,
                                elas_server** out);
/* ELAS_ERR_ARG for a bad pair or one larger than the whole budget. The
 * pair's images must be complete when it is submitted (the caller has
 * synchronised with whatever wrote them); otherwise use elas_server_submit_on. */
ELAS_API int elas_server_submit(elas_server* s, const elas_pair* pair, int64_t* ticket);
/* As elas_server_submit, ordered after the work already enqueued on
 * `producer` (the stream that wrote the images or last used the outputs): an
 * event recorded there at submission is waited for on the device before the
 * pair's batch runs. producer = NULL is the null stream. */
ELAS_API int elas_server_submit_on(elas_server* s, const elas_pair* pair, hipStream_t producer,
                                   int64_t* ticket);
/* Blocks until the ticket completes; *latency_ms (optional) receives its
 * latency. Returns the pair's status (a ticket is reported once):
 * ELAS_ERR_INTERNAL if its device mesh failed (see the top of this header). */
ELAS_API int elas_server_wait(elas_server* s, int64_t ticket, double* latency_ms);
/* Non-blocking: *done = 1 and the status and latency once complete. */
ELAS_API int elas_server_poll(elas_server* s, int64_t ticket, int32_t* done,
                              double* latency_ms);
/* Counters since creation (ELAS_ERR_ARG for null pointers). */
ELAS_API int elas_server_get_stats(elas_server* s, elas_server_stats* out);
/* The server's last failure; owned by the server, valid until its next call. */
ELAS_API const char* elas_server_last_error(const elas_server* s);
/* Finishes every queued and running pair, then frees the server. */
ELAS_API int elas_server_destroy(elas_server* s);

/* Copies the counters of the last elas_process call (synchronises with its
 * stream first): the work of Section III-A's stages (support and dense SAD
 * evaluations, support points, triangles) that Section VII-B's per-frame
 * times scale with. ELAS_ERR_ARG before any completed call; ELAS_ERR_INTERNAL
 * if a device mesh failed since the last call. */
ELAS_API int elas_get_stats(elas_handle* h, elas_stats* out);

/* Test hook: caps the flip rounds of the device mesh that builds Section
 * III-A's Delaunay triangulation (1..32000, larger values clamp; the default
 * 32000 never binds, a frame needs a few tens; ELAS_ERR_ARG below 1). A view that is not legal
 * within the cap gives up, its frame is matched without plane priors, and the
 * failure is reported as described at the top of this header. Lets tests
 * force the failure path while every kernel still exits normally. */
ELAS_API int elas_set_mesh_round_limit(elas_handle* h, int32_t rounds);

/* Turns per-stage event timing on (1) or off (0) for later calls: the
 * stage breakdown of a frame's time that Section VII-B reports per
 * accelerator. Timing adds one event record per stage boundary to the
 * stream. ELAS_ERR_ARG for a null handle. */
ELAS_API int elas_set_timing(elas_handle* h, int32_t enable);

/* Stage times of the last call made with timing on (synchronises with its
 * stream), split by the stages of Section III-A as Section VII-B splits a
 * frame's time. ELAS_ERR_ARG if no such call has completed. After an
 * elas_process_batch call each figure is the summed duration of that stage's
 * launches for the whole batch (a timed batch is launched directly, not from
 * a graph), device_span_ms runs from the first launch's start to the last
 * one's end, and the host fields are 0. */
ELAS_API int elas_get_timing(elas_handle* h, elas_timing* out);

/* Describes the last failure on h (or of elas_create when h is NULL): the
 * library's error reporting, which no passage of the paper defines. The
 * string belongs to the library and stays valid until the next call. */
ELAS_API const char* elas_last_error(const elas_handle* h);

/* Intermediate results of the last elas_process call, for stage-by-stage
 * verification: one array per step of Section III-A (Fig. 1 (b)-(h)), and of
 * the Section VI variants. Layouts (row-major; w, h image size; lw, lh lattice size;
 * gw, gh grid size; n list length; ntri triangle count):
 *   DESC_*     uint8   [h][w][16]   16-byte descriptor, all-zero if undefined
 *   DCAN_*     int16   [lh][lw]     support disparity per lattice point or -1
 *                                   (RAW: matched, INCON: after consistency,
 *                                   VERT/FINAL: after vertical/horizontal
 *                                   redundancy)
 *   SUPPORT_*  int32   [n][3]       (u, v, d); left in lattice order, right
 *                                   sorted by (v, u)
 *   CORNERS    int32   [8]          d of (0,0),(w-1,0),(0,h-1),(w-1,h-1),
 *                                   left view then right view (-1 if no list)
 *   TRI_*      int32   [ntri][9]    (u,v,d) x 3, vertices sorted by (v,u),
 *                                   triangles sorted by their vertex triples
 *   PLANE_*    float   [ntri][3]    (a, b, c) of d = a*u + b*v + c
 *   OWNER_*    int32   [h][w]       owning triangle index or 0x7FFFFFFF
 *   DPLANE_*   int16   [h][w]       plane prior disparity or -1
 *   GRID_*     uint64  [gh][gw][ceil(D/64)]  bit d-disp_min set if allowed
 *   RAW_*      int16   [h][w]       dense maps before the final check
 *   LUT        int32   [D]          prior energy by |d - d_plane|
 * `bytes` is the capacity of dst_host; *needed (if not NULL) receives the
 * size of the intermediate. Returns ELAS_ERR_ARG if the capacity is too
 * small or no call has completed. Synchronises with the last call's stream. */
enum elas_intermediate {
  ELAS_I_DESC_LEFT = 0, ELAS_I_DESC_RIGHT = 1,
  ELAS_I_DCAN_RAW = 2, ELAS_I_DCAN_INCON = 3, ELAS_I_DCAN_VERT = 4, ELAS_I_DCAN_FINAL = 5,
  ELAS_I_SUPPORT_LEFT = 6, ELAS_I_SUPPORT_RIGHT = 7, ELAS_I_CORNERS = 8,
  ELAS_I_TRI_LEFT = 9, ELAS_I_TRI_RIGHT = 10,
  ELAS_I_PLANE_LEFT = 11, ELAS_I_PLANE_RIGHT = 12,
  ELAS_I_OWNER_LEFT = 13, ELAS_I_OWNER_RIGHT = 14,
  ELAS_I_DPLANE_LEFT = 15, ELAS_I_DPLANE_RIGHT = 16,
  ELAS_I_GRID_LEFT = 17, ELAS_I_GRID_RIGHT = 18,
  ELAS_I_RAW_LEFT = 19, ELAS_I_RAW_RIGHT = 20,
  ELAS_I_LUT = 21,
  /* census mode: dense census, one uint64 per pixel [h][w]; support census of
   * the lattice rows [lh][w][4 * q] uint32 words, q = 1 for windows up to 11,
   * 2 for 13 (zero-padded) */
  ELAS_I_CENSUS_DENSE_LEFT = 22, ELAS_I_CENSUS_DENSE_RIGHT = 23,
  ELAS_I_CENSUS_SUPPORT_LEFT = 24, ELAS_I_CENSUS_SUPPORT_RIGHT = 25,
  /* median mode: the checked maps before the median [h][w] int16 */
  ELAS_I_CHECKED_LEFT = 26, ELAS_I_CHECKED_RIGHT = 27,
  ELAS_I_COUNT = 28
};
ELAS_API int elas_get_intermediate(elas_handle* h, int32_t which, void* dst_host,
                                   int64_t bytes, int64_t* needed);

/* As elas_get_intermediate, for pair `pair` (0-based) of the last
 * elas_process_batch call made on h: the stages computed by the batched
 * kernels, for stage-by-stage verification of a batch. A pair meshed on the
 * host was computed by elas_process on its parameter handle, and reads come
 * from that handle's last call. Valid until the next call that uses the
 * pair's buffers (a later batch on the same stream, or a call on its
 * parameter handle); synchronises with the batch's stream. ELAS_ERR_ARG for a
 * pair outside the last batch. */
ELAS_API int elas_get_batch_intermediate(elas_handle* h, int32_t pair, int32_t which,
                                         void* dst_host, int64_t bytes, int64_t* needed);

/* The mesh step on its own, on the host (Section III-A: Delaunay
 * triangulation of the support points and one slanted plane per triangle;
 * Section IV leaves this sequential step on the CPU). Makes no HIP call.
 *   pts      n support points as (u, v, d) int32 triples, distinct; with
 *            corners each strictly inside the image (0 < u < w-1,
 *            0 < v < h-1), without them anywhere in it.
 *   corners  d of the image corners (0,0), (w-1,0), (0,h-1), (w-1,h-1); NULL:
 *            the mesh of the points alone (add_corners = 0).
 *   recs_out capacity (2n+2)*9 int32: canonical triangles, layout of TRI_*.
 *   planes_out capacity (2n+2)*3 float: planes, layout of PLANE_*.
 * The mesh is the Delaunay triangulation of corners + points (or of the
 * points alone) in which every set of four or more co-circular points is
 * split as a fan from its (v, u)-smallest point. Returns the triangle count
 * (2n+2 with corners; 2n-2-h without, h = points on the hull, 0 for fewer
 * than three or collinear points), ELAS_ERR_ARG for bad input (n < 1, null
 * pointers, points outside, duplicates), or ELAS_ERR_INTERNAL. */
ELAS_API int elas_triangulate(const int32_t* pts, int32_t n, const int32_t* corners, int32_t w,
                              int32_t h, int32_t* recs_out, float* planes_out);

#ifdef __cplusplus
}
#endif
#endif /* ELAS_MI355X_H */

/* splatsort: per-frame tile-and-depth sort of 3D Gaussian Splatting on
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Operation (arXiv 2511.16298, Background, "Duplication with Tiles" and
 * "Sorting"; Design, "Sorting Optimizations in Context of 3DGS"): projected
 * Gaussians go in; out come all (tile, Gaussian) pairs whose 16x16-pixel tile
 * meets the Gaussian's axis-aligned bounding box, as 64-bit keys
 * (tile id << 32 | raw FP32 depth bits) with 32-bit Gaussian-index values,
 * ordered by tile, then depth, then index, and each tile's [start, end)
 * range into that list.
 *
 * Conventions shared by every call:
 *  - Pointers named d_* or documented "device" point to device memory on the
 *    current HIP device; the caller owns them; the library never frees or
 *    retains them past the call (except the arena given to a server).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls validate their arguments synchronously and return an error before
 *    enqueuing anything; then they enqueue asynchronously on `stream` and
 *    return SS_OK.  Outputs are valid once the stream has reached that point.
 *  - Errors found on the device (capacity, overflow, invalid input) are
 *    written to a device status word; when it is not SS_OK the contents of
 *    keys, values and ranges are unspecified.
 *  - No call blocks on the GPU unless documented.  No exceptions cross the
 *    ABI.  Calls that share a workspace must not overlap in time.
 *  - The sort passes wait on earlier workgroups of their own launch
 *    (decoupled look-back), and the GPU's XCDs dispatch their share of each
 *    grid independently.  Two sorting calls whose kernels run at the same time
 *    on one GPU (different streams) can therefore wait on each other in a
 *    cycle, which the bounded wait ends with SS_ERR_TIMEOUT: issue a GPU's
 *    sorting calls on one stream, or order them with events.  Kernels without
 *    such waits (other work, the server's sizing counts) may overlap freely.
 */
#ifndef SPLATSORT_H
#define SPLATSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SS_ABI_VERSION 1

typedef enum ss_status {
  SS_OK = 0,
  SS_ERR_INVALID_ARGUMENT = 1, /* a NULL pointer, a size out of range, bad alignment */
  SS_ERR_UNSUPPORTED = 2,      /* an option value this build does not implement */
  SS_ERR_CAPACITY = 3,         /* device: the frame has more pairs than pair_capacity */
  SS_ERR_OVERFLOW = 4,         /* device: the frame has 2^32 pairs or more */
  SS_ERR_INVALID_INPUT = 5,    /* device: a Gaussian that touches a tile has a depth
                                  that is not positive and finite */
  SS_ERR_WORKSPACE = 6,        /* the workspace is smaller than required */
  SS_ERR_HIP = 7,              /* a HIP runtime call failed */
  SS_ERR_BUDGET = 8,           /* server: the request can never fit the arena */
  SS_ERR_TIMEOUT = 9           /* device: a bounded inter-workgroup wait gave up */
} ss_status;

/* One projected Gaussian, the packed output group the duplication step reads
 * (Design, "Output Data Grouping": 2D mean, depth and radius together).
 * 16 bytes, 16-byte aligned; one 128-bit load per Gaussian. */
typedef struct ss_gaussian2d {
  int32_t mean_x;  /* signed 1/16-pixel fixed point; off-image allowed */
  int32_t mean_y;
  float depth;     /* view depth; must be positive and finite if the
                      Gaussian touches a tile; its raw bits form the key */
  uint32_t radius; /* pixels; 0 = culled */
} ss_gaussian2d;

/* Tile overlap rule: with cx = mean_x / 16 px, tile column tx is touched iff
 * the open interval (cx - radius, cx + radius) meets [16 tx, 16 tx + 16);
 * rows likewise.  Partial edge tiles count.  Tile id = ty * tiles_x + tx. */
typedef struct ss_frame {
  uint32_t width;          /* pixels, 1 .. SS_MAX_IMAGE_PX */
  uint32_t height;         /* pixels, 1 .. SS_MAX_IMAGE_PX */
  uint32_t tile_px;        /* must be 16 */
  uint32_t num_gaussians;  /* N, 0 .. 2^31 - 1 */
  const ss_gaussian2d* gaussians; /* device [N]; may be NULL when N == 0 */
} ss_frame;

#define SS_MAX_IMAGE_PX 1048560u        /* 65535 tiles of 16 px per axis */
#define SS_MAX_PAIR_CAPACITY 1073741823u /* 2^30 - 1 pairs per sort */

typedef struct ss_frame_out {
  uint32_t pair_capacity;  /* entries of keys/values, 0 .. SS_MAX_PAIR_CAPACITY */
  uint64_t* keys;          /* device [pair_capacity]: sorted keys */
  uint32_t* values;        /* device [pair_capacity]: Gaussian indices */
  uint32_t* tile_ranges;   /* device [2 T]: start, end of tile t at [2t], [2t+1];
                              the ranges partition [0, M) in tile order; an
                              empty tile gets [p, p), p = pairs of lower tiles */
  uint32_t* tiles_touched; /* device [N] or NULL: pairs per Gaussian */
  uint32_t* offsets;       /* device [N] or NULL: exclusive prefix sum of tiles_touched */
  uint32_t* num_pairs;     /* device scalar M (min(M, 2^32-1)) or NULL */
  uint32_t* status;        /* device scalar ss_status or NULL */
} ss_frame_out;

/* Radix digit width and instrumentation.  Zero-initialise, then set
 * struct_size = sizeof(ss_options).  A NULL options pointer means defaults. */
typedef struct ss_timer ss_timer;
typedef struct ss_options {
  uint32_t struct_size;
  uint32_t radix_bits;     /* 0 = default (8); supported: 4, 6, 8 */
  uint32_t items_per_thread; /* 0 = default (16; 8 for the depth-first tile
                                passes of a pair capacity below 2^23);
                                supported: 8, 12, 16 */
  uint32_t flags;          /* SS_FLAG_* (0 = none) */
  ss_timer* timer;         /* optional: record HIP events around every kernel */
  uint32_t workgroup_size; /* sort-pass threads: 0 = default (512 where
                              supported, else 256); 512 needs radix_bits 8
                              and items 8 or 16.  A pass tile holds
                              workgroup_size * items_per_thread pairs. */
  uint32_t algorithm;      /* SS_ALGO_*; all give bit-identical frame results */
  /* Fields below are read only when struct_size covers them. */
  uint32_t spin_limit;     /* depth-first path: polls a workgroup makes in a
                              wait on other workgroups (decoupled look-back,
                              published digit bases) before it gives up with
                              SS_ERR_TIMEOUT; 0 = 2^20, far above any
                              legitimate wait */
  uint32_t fault;          /* SS_FAULT_* (0 = none): test hook */
} ss_options;

/* Test hook: the workgroups that publish the digit bases of the first pass
 * over the pairs publish nothing, so every tile's bounded wait for its bases
 * ends in SS_ERR_TIMEOUT (after spin_limit polls), while every kernel still
 * runs to its end.  Depth-first path.  For tests of the timeout path. */
#define SS_FAULT_NONE 0u
#define SS_FAULT_WITHHOLD_BASES 1u

/* SS_ALGO_DIRECT: duplicate in index order, then ceil((ceil(log2 T) + 32) /
 * radix_bits) passes over all M pairs.  SS_ALGO_DEPTH_FIRST: sort the N
 * Gaussians by depth first (four 8-bit passes over N), duplicate in depth
 * order, then sort the pairs by tile id alone (ceil(log2 T) bits in
 * P = ceil(ceil(log2 T) / radix_bits) passes; with 8-bit digits in
 * 512-thread passes the bits are split evenly, ceil(ceil(log2 T) / P) per
 * pass); a Gaussian adds at most one pair per tile, so the stable tile sort
 * leaves each tile in (depth, index) order.  radix_bits, items and
 * workgroup_size apply to the passes over the pairs.  AUTO = DEPTH_FIRST,
 * except that SS_FLAG_UNSORTED implies DIRECT. */
#define SS_ALGO_AUTO 0u
#define SS_ALGO_DEPTH_FIRST 1u
#define SS_ALGO_DIRECT 2u
/* SS_ALGO_BITONIC: the paper's own sort (Background, "Sorting"; Design,
 * "Sorting Optimizations in Context of 3DGS"): duplicate in index order, then
 * a bitonic network over the pairs padded to a power of two, comparing
 * (key, value); partner steps below 4,096 elements run fused in LDS, longer
 * ones three at a time.  Frames only (not batches); in ss_sort_pairs it
 * orders by (key bits [0, key_bits), value), which equals the stable order
 * when the values of equal keys increase in input order.  Workspace grows to
 * the padded size. */
#define SS_ALGO_BITONIC 3u
/* SS_ALGO_TILE_FIRST (frames only): duplicate in index order, sort the pairs
 * stably by tile id alone (as depth-first does), then sort each tile's run
 * stably by depth, one workgroup per tile: in LDS up to 8,192 pairs, longer
 * runs in chunks through the workspace.  The depth sort of the Gaussians is
 * not needed.  Same output as the other algorithms. */
#define SS_ALGO_TILE_FIRST 4u

/* Stop after duplication: keys/values receive the duplicated pairs in
 * duplication order (Gaussian by Gaussian, tiles row-major); no sort and no
 * ranges.  For stage-by-stage verification. */
#define SS_FLAG_UNSORTED 1u
/* The paper's key normalisation (Design, "Sorting Optimizations in Context of
 * 3DGS": the 64-bit key replaced by one 32-bit float holding 20 bits of tile
 * number and the depth brought below 2^10), with SS_ALGO_BITONIC in
 * ss_sort_frame only: the network orders the pairs by (k, value) with
 * k = FP32(tile * 2^10 + min(depth, 1024 - 2^-14)) rounded toward zero, so k
 * stays inside [tile * 2^10, (tile + 1) * 2^10) and the tiles stay in order;
 * depths closer than one unit in the last place of k (2^(e - 23), e the
 * binary exponent of k: 1/8 for tile 1000, 1 for tile 8000) are not
 * separated and keep index order.  This is lossy: the order inside a tile is
 * the exact order only up to that quantum.  Output keys are the exact 64-bit
 * keys (tile << 32 | depth bits) in that order; ranges as usual.  Needs
 * T <= 2^20 (else SS_ERR_UNSUPPORTED); any other algorithm, ss_sort_pairs,
 * batches or SS_FLAG_UNSORTED with it are SS_ERR_UNSUPPORTED. */
#define SS_FLAG_KEY32_LOSSY 2u
/* Depth-first path (frames and batches): the first pass of the Gaussian depth
 * sort drops the Gaussians that touch no tile, when they are more than 1/16
 * of all, and the later passes and the duplication step handle only the rest.
 * Same output.  Pays off for frames where many Gaussians fall outside the
 * image, such as one GPU's band of a frame split by tile rows (every GPU
 * sees all Gaussians); on frames with few culled Gaussians the extra decision
 * costs a few microseconds.  No effect on the other algorithms. */
#define SS_FLAG_DROP_CULLED 4u
/* Depth-first path (frames and batches), 512-thread passes: the sort passes
 * over the pairs run as persistent kernels, one grid of at most as many
 * workgroups as the GPU holds at once, each taking tickets in order from an
 * atomic counter (the base-publishing workgroups first, then the tiles)
 * until none are left.  A ticket is only ever taken by a running workgroup,
 * so every wait is on a workgroup that runs.  Same output.  Ignored with
 * 256-thread passes. */
#define SS_FLAG_PERSISTENT 8u

/* Library identification. */
uint32_t ss_abi_version(void);
const char* ss_status_string(ss_status s);

/* Tile grid of a frame: T = tiles_x * tiles_y, and the sorted key width
 * b = ceil(log2 T) + 32 (32 when T == 1).  Host only, no GPU work. */
ss_status ss_frame_geometry(const ss_frame* frame, uint32_t* tiles_x, uint32_t* tiles_y,
                            uint32_t* key_bits);

/* Bytes of workspace that ss_sort_frame needs for this frame shape and
 * capacity (depends on N, T, pair_capacity and the options only).  The
 * workspace must be 256-byte aligned device memory. */
ss_status ss_workspace_bytes(const ss_frame* frame, uint32_t pair_capacity,
                             const ss_options* options, size_t* bytes);

/* Counting and scan only: per-Gaussian tile counts, their exclusive prefix sum and
 * the total M, so a caller can size the pair buffers (one 4-byte read back).
 * Any of d_tiles_touched, d_offsets may be NULL; d_num_pairs and d_status
 * are required.  Uses the same workspace as ss_sort_frame with capacity 0. */
ss_status ss_count_pairs(const ss_frame* frame, uint32_t* d_tiles_touched, uint32_t* d_offsets,
                         uint32_t* d_num_pairs, uint32_t* d_status,
                         void* workspace, size_t workspace_bytes, void* stream);

/* The whole path for one frame: count, scan, duplicate, sort, and identify
 * the tile ranges (Background, "Duplication with Tiles" and "Sorting"; the
 * Evaluation's stage table lists the same steps).  By default (depth-first)
 * the Gaussians are sorted by depth, their pairs written in depth order and
 * then sorted stably by tile id alone; frames of at most 256 tiles and
 * 16,384 Gaussians (without tiles_touched / offsets outputs) take a
 * two-kernel path; SS_ALGO_DIRECT counts, scans and duplicates in index
 * order and sorts key bits [0, b).  Every path gives the same output. */
ss_status ss_sort_frame(const ss_frame* frame, const ss_frame_out* out,
                        void* workspace, size_t workspace_bytes, void* stream,
                        const ss_options* options);

/* ss_sort_frame without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a library-owned array
 * of SS_NOALLOC_SCRATCH_BYTES in device memory, one per GPU, held until the
 * process ends; the call allocates nothing (device or host).  Frames whose
 * ss_workspace_bytes exceeds it return SS_ERR_WORKSPACE before anything is
 * enqueued (the full-HD frame of 10^6 Gaussians fits).  Depth-first path
 * only: other algorithms, SS_FLAG_UNSORTED and SS_FLAG_KEY32_LOSSY are
 * SS_ERR_UNSUPPORTED.  The array serves the GPU that `stream` belongs to;
 * every call on that GPU shares it, so calls that overlap on one GPU race
 * (order them on one stream).  Outputs, errors and results are those of
 * ss_sort_frame. */
#define SS_NOALLOC_SCRATCH_BYTES (128u << 20)
ss_status ss_sort_frame_noalloc(const ss_frame* frame, const ss_frame_out* out, void* stream,
                                const ss_options* options);

/* Many frames in one segmented sort (up to SS_MAX_BATCH_FRAMES).  Frame f's
 * tiles are renumbered tile_base[f] + t, tile_base the exclusive prefix sum
 * of the frames' tile counts; keys hold global tile ids, values frame-local
 * Gaussian indices.  Frame f's pairs are one contiguous segment, equal to
 * what ss_sort_frame gives for frame f alone (with its keys' tile part
 * offset by tile_base[f]).  Always the depth-first algorithm. */
#define SS_MAX_BATCH_FRAMES 256u
typedef struct ss_batch_out {
  uint32_t pair_capacity;   /* entries of keys/values for all frames together */
  uint64_t* keys;           /* device [pair_capacity] */
  uint32_t* values;         /* device [pair_capacity] */
  uint32_t* tile_ranges;    /* device [2 * sum of T]: global pair indices */
  uint32_t* frame_pairs;    /* device [n_frames]: pairs of each frame, or NULL */
  uint32_t* frame_pair_base;/* device [n_frames]: first pair of each frame, or NULL */
  uint32_t* num_pairs;      /* device scalar: all pairs, or NULL */
  uint32_t* status;         /* device scalar ss_status, or NULL */
} ss_batch_out;

ss_status ss_batch_workspace_bytes(const ss_frame* frames, uint32_t n_frames, uint32_t pair_capacity,
                                   const ss_options* options, size_t* bytes);
ss_status ss_sort_batch(const ss_frame* frames, uint32_t n_frames, const ss_batch_out* out,
                        void* workspace, size_t workspace_bytes, void* stream,
                        const ss_options* options);

/* Batched sizing (counting and scan for many frames): the pair count of every
 * frame, written to d_frame_pairs[n_frames] (saturated at 2^32 - 1), their
 * sum to *d_num_pairs, and SS_OK / SS_ERR_OVERFLOW / SS_ERR_INVALID_INPUT to
 * *d_status.  Nothing else is written. */
ss_status ss_batch_count_workspace_bytes(const ss_frame* frames, uint32_t n_frames, size_t* bytes);
ss_status ss_batch_count_pairs(const ss_frame* frames, uint32_t n_frames, uint32_t* d_frame_pairs,
                               uint32_t* d_num_pairs, uint32_t* d_status, void* workspace,
                               size_t workspace_bytes, void* stream);

/* A plan: one batch shape (frame sizes, record and output pointers, the
 * workspace) with the batched pipeline captured once into a HIP graph and
 * replayed by ss_plan_launch.  Inputs may change between launches; their
 * addresses and the frame shapes may not.  With autotune != 0, creation
 * times every compiled pass configuration (radix width 4/6/8, items per
 * thread, workgroup size) on the given data and keeps the fastest; the
 * results are identical whichever is chosen.  Creation synchronises the
 * stream; the workspace must hold ss_plan_workspace_bytes.  Graph capture
 * runs on a stream the plan owns.  With tune_cache (a file path), the choice
 * is looked up first under (device architecture, HIP runtime version, ABI
 * version, and the ceil(log2) of the frame count, Gaussians, pair capacity,
 * total and largest frame's tiles); a hit skips the timing (ss_plan_config
 * then reports no candidate times), a miss times the candidates and records
 * the winner in the file (one text line per key, replaced in place; written
 * through a temporary file and a rename).  A file that cannot be read or
 * written only costs the timing. */
typedef struct ss_plan ss_plan;
typedef struct ss_plan_desc {
  uint32_t struct_size;      /* sizeof(ss_plan_desc) */
  uint32_t n_frames;
  const ss_frame* frames;    /* host array [n_frames]; gaussians are device pointers */
  ss_batch_out out;
  void* workspace;
  size_t workspace_bytes;
  uint32_t autotune;         /* 0: use options; 1: time the candidates, keep the fastest */
  uint32_t tune_repeats;     /* launches timed per candidate (0 = 5) */
  ss_options options;        /* starting / fixed configuration (timer ignored) */
  const char* tune_cache;    /* autotune cache file, or NULL; read only when
                                struct_size covers it */
} ss_plan_desc;

ss_status ss_plan_workspace_bytes(const ss_frame* frames, uint32_t n_frames, uint32_t pair_capacity,
                                  size_t* bytes);
ss_status ss_plan_create(ss_plan** plan, const ss_plan_desc* desc, void* stream);
ss_status ss_plan_launch(ss_plan* plan, void* stream);
/* The configuration in use (after autotuning) and the tuned time per launch
 * of each candidate tried (ms, in the order they were tried; up to n). */
ss_status ss_plan_config(const ss_plan* plan, ss_options* chosen, double* candidate_ms, uint32_t* n);
void ss_plan_destroy(ss_plan* plan);

/* Serving.  Frame-sort requests arrive over time (ss_server_submit from any
 * host thread).  A scheduler thread owned by the server sizes the waiting
 * requests with one batched count, admits the longest FIFO prefix whose
 * round (workspace + outputs) fits the caller's arena now, and launches it
 * as one segmented sort (ss_sort_batch).  Up to n_streams rounds are in
 * flight at once, queued back to back on one stream the server owns (never
 * side by side, see the conventions above); the sizing counts run on a second
 * stream, so a round runs while the next is being sized and launched
 * (continuous batching).  A request that could not fit even an empty arena completes
 * with SS_ERR_BUDGET; others wait for space.  Outputs stay in the arena until
 * ss_server_release; workspace is freed when the round completes.  With
 * max_batch_frames = 1 and n_streams = 1 the server is a one-request-at-a-
 * time plain path.  The records of a request must stay valid and unchanged
 * until it completes.  Results are bit-identical to ss_sort_frame on the
 * frame alone (after removing the round offsets below). */
typedef struct ss_server ss_server;
typedef struct ss_server_desc {
  uint32_t struct_size;       /* sizeof(ss_server_desc) */
  uint32_t max_batch_frames;  /* frames per round, 1 .. SS_MAX_BATCH_FRAMES */
  uint32_t n_streams;         /* rounds in flight at once, 1 .. 8 */
  uint32_t reserved;          /* 0 */
  ss_options options;         /* pass configuration of every round (timer ignored) */
} ss_server_desc;

typedef struct ss_result {
  ss_status status;
  uint32_t num_pairs;           /* M of this frame */
  const uint64_t* keys;         /* device [M], in the arena; tile part = tile_base + t */
  const uint32_t* values;       /* device [M]: Gaussian indices of the frame */
  const uint32_t* tile_ranges;  /* device [2 T]: pair indices of the round; subtract pair_base */
  uint32_t tile_base;           /* first global tile id of the frame in its round */
  uint32_t pair_base;           /* first pair of the frame in its round */
  uint32_t round_frames;        /* frames sorted together with this one */
  uint32_t reserved;
  double submit_us, start_us, done_us;  /* host steady clock: submitted, launched, seen complete */
} ss_result;

typedef struct ss_server_counters {
  uint64_t rounds, admitted, completed, rejected, pending, arena_used;
  double mean_round_frames;
} ss_server_counters;

ss_status ss_server_create(ss_server** server, void* d_arena, size_t arena_bytes, const ss_server_desc* desc);
ss_status ss_server_submit(ss_server* server, const ss_frame* frame, uint64_t* ticket);
/* Blocks until the request has completed; out stays valid until release. */
ss_status ss_server_wait(ss_server* server, uint64_t ticket, ss_result* out);
ss_status ss_server_release(ss_server* server, uint64_t ticket);
ss_status ss_server_stats(ss_server* server, ss_server_counters* out);
/* Drains every submitted request, then stops the scheduler. */
void ss_server_destroy(ss_server* server);

/* The sort alone on caller data (the paper's random key-value sort benchmark,
 * Evaluation, "Datasets"): stable sort of n pairs by key bits [0, key_bits);
 * keys must be < 2^key_bits.  keys_in/values_in are not modified; they may
 * not alias the outputs.  Workspace: ss_sort_pairs_workspace_bytes. */
ss_status ss_sort_pairs_workspace_bytes(uint32_t n, uint32_t key_bits, const ss_options* options,
                                        size_t* bytes);
ss_status ss_sort_pairs(const uint64_t* keys_in, const uint32_t* values_in, uint32_t n,
                        uint32_t key_bits, uint64_t* keys_out, uint32_t* values_out,
                        void* workspace, size_t workspace_bytes, void* stream,
                        const ss_options* options);

/* Measurement helpers. */
/* A plain streaming copy of `bytes` (multiple of 16, 16-byte aligned) used to
 * calibrate memory-traffic counters and to report achievable bandwidth. */
ss_status ss_copy_bytes(void* d_dst, const void* d_src, size_t bytes, void* stream,
                        const ss_options* options);

/* ---------------------------------------------------------------------------
 * Rendering (the step after the sort; paper: Background, "Rendering", and
 * Design, "Efficient Tile-Based Rendering").  Every pixel of a 16x16 tile
 * composites the tile's sorted Gaussians front to back by alpha blending, with
 * the compositing rule of 3D Gaussian Splatting that the paper builds on:
 * pixel (x, y) is sampled at (x + 1/2, y + 1/2) in the frame of the means
 * (mean_x / 16, mean_y / 16); d = mean - sample; q = a dx^2 + 2 b dx dy +
 * c dy^2 with the conic (a, b, c) = inverse 2D covariance; alpha = opacity *
 * exp(-q / 2); colour += rgb * alpha * T, T *= 1 - alpha from T = 1; the pixel
 * gets colour + T * background.  Unless SS_RENDER_EXACT is set, the
 * rasteriser's thresholds apply: q < 0 is skipped, alpha is capped at 0.99,
 * alpha < 1/255 is skipped, and a pixel stops before a Gaussian that would
 * take T below 1e-4.  FP32 arithmetic.
 * ------------------------------------------------------------------------- */
#define SS_RENDER_EXACT 1u

typedef struct ss_render_desc {
  uint32_t struct_size;         /* sizeof(ss_render_desc) */
  uint32_t flags;               /* SS_RENDER_* */
  const float* conic_opacity;   /* device [N][4]: a, b, c, opacity in [0, 1] (16-B aligned) */
  const float* rgb;             /* device [N][4]: r, g, b, unused (16-B aligned) */
  const uint32_t* values;       /* device: the frame's sorted Gaussian indices */
  const uint32_t* tile_ranges;  /* device [2T]: the frame's tile ranges */
  const uint32_t* status;       /* device status of the sort, or NULL; when it
                                   does not read SS_OK nothing is written */
  float background[3];
  float* out_color;             /* device [3][H][W] planar, row-major */
  float* out_T;                 /* device [H][W] final transmittance, or NULL */
  uint32_t* out_contrib;        /* device [H][W] Gaussians composited, or NULL */
  uint32_t* out_tile_evals;     /* device [T] (pixel, Gaussian) evaluations per
                                   tile (the arithmetic done), or NULL */
  ss_timer* timer;              /* optional (kind SS_KERNEL_RENDER) */
} ss_render_desc;

/* Renders one sorted frame: `frame` gives the image size and the records
 * (the means), `desc` the render inputs and outputs; values and ranges are
 * those of an ss_sort_frame call on the same frame (one workgroup wave per
 * tile; nothing else is read or written).  Errors: SS_ERR_INVALID_ARGUMENT for
 * a NULL or misaligned pointer or an unknown flag. */
ss_status ss_render_frame(const ss_frame* frame, const ss_render_desc* desc, void* stream);

/* ---------------------------------------------------------------------------
 * Preprocessing (the step before the sort; paper: Background,
 * "Preprocessing", and Design, "Variable Packing" with its input and output
 * group tables: mean and opacity, 3D covariance and spherical-harmonic
 * coefficients in; 2D mean, depth and radius together, conic and opacity,
 * colour out), with the projection rule of 3D Gaussian Splatting that the
 * paper builds on.  For Gaussian g with world mean p:
 *   t = R p + T (camera frame); culled when t.z <= near_plane;
 *   pixel = (fx t.x / t.z + cx, fy t.y / t.z + cy);
 *   2D covariance = J R S R^T J^T + 0.3 I, where S is the 3D covariance and
 *   J the Jacobian of the projection at t with t.x / t.z and t.y / t.z first
 *   clamped to +-1.3 tan_fov; culled when its determinant is 0;
 *   conic = its inverse (a, b, c) = (C11, -C01, C00) / det;
 *   radius = ceil(3 sqrt(mid + sqrt(max(0.1, mid^2 - det)))), mid = half the
 *   trace (3 standard deviations along the major axis);
 *   colour = max(0, 1/2 + sum over SH degrees l <= sh_degree of coefficient
 *   x real spherical harmonic Y_lm (with the Condon-Shortley phase) of the
 *   unit direction from cam_pos to p), per channel.
 * Record: mean_x/y = 16 x pixel rounded half to even (clamped to +-2^30),
 * depth = t.z (also for culled Gaussians), radius; culled Gaussians get
 * mean 0, radius 0, zero conic and colour.  FP32 arithmetic.
 * ------------------------------------------------------------------------- */
typedef struct ss_camera {
  float view[12];            /* [R | T] world to camera, row-major 3 x 4 */
  float fx, fy, cx, cy;      /* focal lengths and principal point, pixels */
  float tan_fovx, tan_fovy;  /* tangents of the half field of view (> 0) */
  float cam_pos[3];          /* camera centre in world coordinates */
  float near_plane;
  uint32_t sh_degree;        /* 0 .. 3 */
} ss_camera;

typedef struct ss_preprocess_desc {
  uint32_t struct_size;          /* sizeof(ss_preprocess_desc) */
  uint32_t num_gaussians;        /* N, 0 .. 2^31 - 1 */
  const float* mean3d_opacity;   /* device [N][4]: x, y, z, opacity (16-B aligned) */
  const float* cov3d;            /* device [N][8]: xx, xy, xz, yy, yz, zz, unused x2
                                    (16-B aligned) */
  const float* sh;               /* device [N][48]: 16 coefficients x RGB in
                                    (l, m = -l..l) order (16-B aligned); only the
                                    first (sh_degree + 1)^2 triples are used */
  ss_gaussian2d* out_records;    /* device [N]: the sort's input records */
  float* out_conic_opacity;      /* device [N][4]: a, b, c, opacity (render input) */
  float* out_rgb;                /* device [N][4]: r, g, b, 0 (render input) */
  ss_timer* timer;               /* optional (kind SS_KERNEL_PREPROCESS) */
} ss_preprocess_desc;

/* Projects N Gaussians (one thread each; every output element is written).
 * Inputs must be finite.  The buffers are the caller's; nothing is allocated.
 * Errors: SS_ERR_INVALID_ARGUMENT for a NULL or misaligned pointer, a size
 * mismatch (struct_size), N >= 2^31, sh_degree > 3, non-positive tan_fov or a
 * non-finite camera value; SS_ERR_HIP if the launch fails. */
ss_status ss_preprocess(const ss_camera* camera, const ss_preprocess_desc* desc, void* stream);

typedef enum ss_kernel_kind {
  SS_KERNEL_CLEAR = 0,      /* zeroes counters and look-back state */
  SS_KERNEL_COUNT_DUP = 1,  /* direct: count, scan and duplicate fused; depth-first: count and keys */
  SS_KERNEL_SORT_PASS = 2,  /* one digit pass of the sort over the pairs */
  SS_KERNEL_RANGES = 3,     /* tile ranges */
  SS_KERNEL_COPY = 4,       /* ss_copy_bytes */
  SS_KERNEL_HIST = 5,       /* digit histograms of caller keys (ss_sort_pairs) */
  SS_KERNEL_DIGIT_BASES = 6, /* pair totals of ss_batch_count_pairs (sort passes derive
                               their digit bases from the histograms) */
  SS_KERNEL_DEPTH_PASS = 7, /* depth-first: one pass of the Gaussian depth sort */
  SS_KERNEL_EXPAND = 8,     /* depth-first: pairs in depth order */
  SS_KERNEL_RENDER = 9,     /* ss_render_frame */
  SS_KERNEL_PREPROCESS = 10, /* ss_preprocess */
  SS_KERNEL_TILE_SORT = 11, /* tile-first: each tile's run sorted by depth */
  SS_KERNEL_KINDS = 12
} ss_kernel_kind;

/* Event pool for per-kernel timing.  Create once (host), pass in
 * ss_options.timer, synchronise the stream, then read the summed time and
 * launch count per kernel kind.  The sort passes of one call are timed as
 * one group (no events between them); their launch count is the number of
 * passes.  max_launches bounds the number of event pairs.  Reset before
 * reuse.  Not thread-safe. */
ss_status ss_timer_create(ss_timer** timer, uint32_t max_launches);
ss_status ss_timer_reset(ss_timer* timer);
ss_status ss_timer_read(ss_timer* timer, uint32_t kind, double* total_ms, uint32_t* launches);
void ss_timer_destroy(ss_timer* timer);

#ifdef __cplusplus
}
#endif

#endif /* SPLATSORT_H */

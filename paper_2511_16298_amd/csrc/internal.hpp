// Internal launch interface between the host ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "splatsort.h"

namespace ss {

// Gaussians per workgroup of the fused count / scan / duplicate kernel.
constexpr uint32_t kCountTile = 1024;
// Histogram copies: workgroups spread their global atomics over this many
// copies to cut same-address contention; passes sum the copies.
constexpr uint32_t kHistCopies = 8;

struct CountDupArgs {
  const ss_gaussian2d* gaussians;
  uint32_t n;
  uint32_t tiles_x, tiles_y;
  uint32_t capacity;        // pairs that may be written; 0 with dup = false
  uint32_t npasses;         // sort passes whose digit histograms are gathered
  uint32_t* tiles_touched;  // optional [n]
  uint32_t* offsets;        // optional [n]
  uint64_t* keys;           // [capacity] unsorted pairs
  uint32_t* values;
  uint64_t* lookback;       // zeroed [nblocks]
  uint32_t* hist;           // zeroed [kHistCopies][npasses][bins]
  uint32_t* num_pairs;
  uint32_t* status;
  uint32_t nblocks;
};

// One frame of a (possibly one-frame) batch, as the depth-first kernels see it.
struct FrameInfo {
  uint32_t gauss_base;   // first global Gaussian index of the frame
  uint32_t n;            // Gaussians of the frame
  uint32_t tiles_x, tiles_y;
  uint32_t tile_base;    // first global tile id of the frame
  uint32_t pad;
  const ss_gaussian2d* gaussians;
};
static_assert(sizeof(FrameInfo) == 32, "frame table entry");

// A (tile, depth, index) pair held in one 64-bit item: tile << tile_shift |
// depth field << idx_bits | frame-local index.  The depth field is the depth
// bits minus (b_min << 24), b_min the smallest top byte of a depth that has
// pairs, when every such depth then fits (trimmed); otherwise it is the
// Gaussian's position in depth order, and the unpacking pass reads the depth
// bits there (depth_sorted).  Both sides decide the same way from the two
// words the depth sort's first pass stores from its top-byte histogram:
// depth_top[0] = largest, depth_top[1] = smallest top byte of such a depth.
struct PackedPairs {
  uint32_t tile_shift;          // 64 - tile bits
  uint32_t idx_bits;            // index field width
  const uint32_t* depth_top;    // [2]
  const uint32_t* depth_sorted; // raw depth bits in depth order (the fallback's lookup)
};

__device__ __forceinline__ bool packed_depth_trimmed(uint32_t top_max, uint32_t top_min, const PackedPairs& p,
                                                     uint32_t* ebase) {
  *ebase = top_min << 24;
  const uint32_t dbits = p.tile_shift - p.idx_bits;
  const uint64_t span = top_max >= top_min ? static_cast<uint64_t>(top_max - top_min + 1) : 1ull;
  return dbits >= 32 || (span << 24) <= (1ull << dbits);
}

struct PassArgs {
  const void* kin;            // uint64_t or uint32_t keys
  const uint32_t* vin;
  void* kout;
  uint32_t* vout;
  const uint32_t* num_pairs;  // device M; NULL means n_fixed
  uint32_t n_fixed;
  uint32_t* status;           // device status word or NULL
  uint32_t shift;             // first key bit of this digit
  // Where the digit bases come from.  32-bit-key passes (the Gaussian depth
  // sort, one small grid) sum the kHistCopies histogram copies themselves,
  // copy c at hist + c * hist_stride.  64-bit-key passes read `bases`
  // ([bins] exclusive prefixes of the digit totals, bit 31 set once
  // published, zeroed before the first pass); in the first pass of a chain
  // (publish_passes > 0) an extra workgroup 0 computes them from `hist` for
  // this and the next publish_passes - 1 passes (pass q at + q * bins of both).
  uint32_t* bases;
  const uint32_t* hist;
  uint32_t hist_stride;
  uint32_t publish_passes;
  uint32_t* lookback;         // zeroed [nblocks][bins]
  // The Gaussian depth sort's handling of culled Gaussians (key 0xFFFFFFFF,
  // digit 255 of every pass; no other key has a top byte of 255, since depths
  // are positive).  First pass (culled != NULL: the last pass's digit-255
  // histogram word of copy 0, copies hist_stride apart): C = their sum; when
  // C > n / 16 the pass drops the culled, writing the n - C others densely
  // from position 0, and tile 0 stores what it keeps (n - C, or n) in *kept.
  // Later passes (n_total != 0): their items are *num_pairs (the kept count)
  // and the totals of digit 255 (histograms of all n_total keys) shrink by
  // the n_total - *num_pairs dropped ones.
  const uint32_t* culled;
  uint32_t* kept;
  uint32_t n_total;
  // 32-bit keys: an optional second 32-bit value per item (NULL: none), moved
  // with the first; the depth sort carries the Gaussians' packed rectangles
  const uint32_t* pin;
  uint32_t* pout;
  // The depth sort's first pass: when not NULL, its workgroup 0 stores here,
  // after its tile, the largest and smallest top byte among the depth keys
  // of Gaussians with pairs (from hist_top, copy c at + c * hist_stride, of
  // the keys' top byte; bin 255 holds the culled ones).
  uint32_t* depth_top_out;
  const uint32_t* hist_top;
  // Packed pairs (64-bit items without values, see PackedPairs): the layout
  // and, for the pass that unpacks them, where the depth bits come from.
  PackedPairs packed;
  // Tile ranges written by the last tile pass (NULL: not this pass).  Its
  // look-back words are 64-bit (lookback64, zeroed [nblocks][bins]): count,
  // and 1 + the largest tile part below this pass's digit among the counted
  // pairs, so that the first pair of a digit run knows its predecessor's
  // tile; each digit's first pair overall is left to k_ranges_fix.
  uint32_t* ranges;
  uint32_t low_bits;          // tile bits below this pass's digit
  uint64_t* lookback64;
  // Segmented 64-bit passes (a batch whose pairs are frame-major, after the
  // segmented depth sort): no workgroup's tile straddles two frames, a frame's
  // workgroups look back only among themselves, digit bases are per frame.
  // The chain's first pass starts with seg_frames publishing workgroups, one
  // per frame.  hist: [copy][frame][pass][bins] (hist_stride between copies),
  // bases: [frame][pass][bins] (bases_frame_stride between frames).
  const uint32_t* seg_wgs;    // [frames + 1] first tile workgroup of each frame; NULL: not segmented
  const uint32_t* seg_base;   // [frames + 1] first pair of each frame (the last: all pairs)
  uint32_t seg_frames;
  uint32_t bases_frame_stride;
  const FrameInfo* table;     // kPassUnpack, segmented: tile_base of each frame
  // Segmented depth sort (32-bit keys, a batch): the Gaussians of every
  // frame, [gauss_base, gauss_base + n) of the table, are sorted apart, in
  // tiles of their own with a look-back chain of their own, from the
  // frame's histograms (hist + frame * 4 * 256) and with digit bases from
  // the frame's first Gaussian; the workgroups past the frames' tiles exit.
  bool depth_seg;
  uint32_t n_frames;
  // Bounded waits: polls before SS_ERR_TIMEOUT (kSpinLimit when 0).  fault:
  // SS_FAULT_* test hook (SS_FAULT_WITHHOLD_BASES: the chain's publishing
  // workgroups publish nothing, so every tile's wait for its bases times out).
  uint32_t spin_limit;
  uint32_t fault;
  // Persistent pass (64-bit keys): a grid of at most the resident workgroups,
  // each taking tickets (publishing workgroups first, then tiles in order)
  // from this zeroed counter until none are left.
  uint32_t* tickets;
};

struct HistArgs {
  const uint64_t* keys;
  uint32_t n;
  uint32_t npasses;
  uint32_t* hist;             // zeroed [kHistCopies][npasses][bins]
};


// Frames carried by value in one launch's arguments.
constexpr uint32_t kArgFrames = 32;
constexpr uint32_t kMaxFrames = 256;

struct TableChunk {
  uint32_t first;        // table index of f[0]
  uint32_t count;        // valid entries of f
  FrameInfo f[kArgFrames];
};

// Depth-first kernels (see depthfirst.hip).
struct CountKeysArgs {
  const FrameInfo* table;   // [n_frames] in device memory
  uint32_t n_frames;
  uint32_t n;               // Gaussians of all frames
  uint64_t* rect;           // out [n]: x0 | y0 << 16 | w << 32 | h << 48 (tiles)
  uint32_t* rect32;         // or, when every frame has at most 256 tiles per axis (then
                            // rect is not written): x0 | y0 << 8 | (w - 1) << 16 | (h - 1) << 24
  uint32_t* key;            // out [n]: depth bits, or 0xFFFFFFFF when culled
  uint32_t* val;            // out [n]: global Gaussian index
  uint32_t* tiles_touched;  // optional [n]
  uint32_t* hist;           // zeroed [kHistCopies][4][256] depth digit histograms
  uint32_t* frame_hist;     // or NULL; else also zeroed [kHistCopies][n_frames][4][256]: the
                            // same per frame (the segmented depth sort)
  unsigned long long* totals;  // zeroed [1 + n_frames]: pairs per frame at [1 + f]
                               // (only workgroups that span several frames add here)
  unsigned long long* block_total;  // [nblocks] pairs of a one-frame workgroup, else 0
  uint32_t* block_frame;    // [nblocks] that workgroup's frame
  uint32_t* bad;            // zeroed flag: a touching Gaussian has a bad depth
};

// Pair totals: per frame (sum of the count workgroups' totals), all frames,
// and from them num_pairs and the status word.
struct PairTotalsArgs {
  const unsigned long long* totals;       // [1 + n_frames], from multi-frame count workgroups
  const unsigned long long* block_total;  // [count_blocks]
  const uint32_t* block_frame;            // [count_blocks]
  uint32_t count_blocks;
  const uint32_t* bad;
  uint32_t n_frames;
  uint32_t capacity;
  uint32_t* num_pairs;
  uint32_t* status;            // set only while it still reads SS_OK
  uint32_t* frame_pairs;       // optional
  uint32_t* frame_pair_base;   // optional
  // segmented tile passes: [n_frames + 1] first pair and first tile
  // workgroup of each frame (workgroups of seg_tile pairs), or NULL
  uint32_t* seg_base;
  uint32_t* seg_wgs;
  uint32_t seg_tile;
};

struct ExpandArgs {
  const FrameInfo* table;
  uint32_t n_frames;
  uint32_t n;               // Gaussians (bound of the indices)
  const uint32_t* n_sorted; // device count of the depth-sorted (live) Gaussians, or NULL (then n)
  const uint32_t* key;      // sorted depth keys
  const uint32_t* val;      // sorted global indices
  const uint64_t* rect;     // by global index
  const uint32_t* rect32;   // or packed rectangles in depth order (sorted with the keys; a
                            // culled Gaussian's is ignored: its key is 0xFFFFFFFF)
  const uint32_t* rect32_idx; // or packed rectangles by global index (gathered; the same
                              // layout, a culled one's likewise ignored)
  bool small_rects;         // every frame has at most 256 tiles per axis
  uint32_t capacity;
  uint64_t* keys;           // out pairs: global tile << 32 | depth bits (or packed items)
  uint32_t* values;         // out: frame-local Gaussian index (unused when packed)
  bool packed;              // write packed 64-bit items (layout `pk`) instead
  PackedPairs pk;
  // segmented (frame-major Gaussians): items carry frame-local tiles and the
  // tile-digit histograms are per frame ([copy][frame][npasses][bins])
  bool seg;
  uint32_t npasses;         // tile-digit passes that follow
  uint32_t radix_bits;      // their digit width (<= 8)
  uint32_t* hist;           // zeroed [kHistCopies][npasses][1 << radix_bits] (segmented:
                            // [kHistCopies][n_frames][npasses][1 << radix_bits])
  uint64_t* lookback;       // zeroed [nblocks]
  uint32_t* status;
  uint32_t nblocks;
  uint32_t spin_limit;      // look-back polls before SS_ERR_TIMEOUT (0: kSpinLimit)
  // Gaussians in index order (tile-first): no depth sort ran, so every
  // workgroup takes the live depth keys' top-byte range from the count
  // kernel's top-byte histogram (copies top_hist_stride apart), and
  // workgroup 0 stores it at depth_top_out for the tile passes
  const uint32_t* top_hist;
  uint32_t top_hist_stride;
  uint32_t* depth_top_out;
  PairTotalsArgs totals;    // finished by workgroup 0
  // single frames with packed rectangles: every workgroup's pair count,
  // written by k_expand_totals beforehand; each workgroup then sums those
  // before it instead of looking back (NULL: look-back)
  const unsigned long long* wg_totals;
  // with wg_totals: the depth histograms' culled words (digit 255 of the top
  // byte, kHistCopies of them culled_stride apart); the depth-sorted
  // Gaussians from n minus their sum on are the culled ones
  const uint32_t* culled;
  uint32_t culled_stride;
};

hipError_t launch_put_table(const TableChunk& c, FrameInfo* table, hipStream_t s);
hipError_t launch_count_keys(const CountKeysArgs& a, hipStream_t s);
hipError_t launch_pair_totals(const PairTotalsArgs& a, hipStream_t s);
hipError_t launch_expand(const ExpandArgs& a, hipStream_t s);
// Each expand workgroup's pair count into a.wg_totals (single frame, packed rectangles).
hipError_t launch_expand_totals(const ExpandArgs& a, unsigned long long* wg_totals, hipStream_t s);
constexpr uint32_t kCountKeysTile = 2048;   // Gaussians per count workgroup
constexpr uint32_t kExpandTile = 2048;      // Gaussians per expand workgroup

// Zeroes `bytes` (a multiple of 16) at p and, if not NULL, the word `extra`;
// with a non-NULL chunk also stores its frames into `table`.
hipError_t launch_clear(void* p, size_t bytes, uint32_t* extra, const TableChunk* chunk, FrameInfo* table,
                        hipStream_t s);
hipError_t launch_count_dup(const CountDupArgs& a, int radix_bits, bool dup, hipStream_t s);
hipError_t launch_ranges(const uint64_t* keys, const uint32_t* num_pairs, const uint32_t* status,
                         uint32_t capacity, uint32_t num_tiles, uint32_t* ranges, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_hist(const HistArgs& a, int radix_bits, hipStream_t s);
// mode: kPassKV (key + value), kPassItems (packed items in and out),
// kPassUnpack (packed items in; keys + values out, tile ranges when
// a.ranges != NULL).
constexpr int kPassKV = 0, kPassItems = 1, kPassUnpack = 2;
hipError_t launch_pass(const PassArgs& a, int key_bytes, int radix_bits, int items, int threads, uint32_t nblocks,
                       hipStream_t s, int mode = kPassKV);
// Whether a packed pass of this shape is compiled.
bool packed_pass_supported(int radix_bits, int items, int threads);
// After a last pass with fused ranges: each digit's first pair (its
// predecessor is in another digit run) and the tail past the last pair.
hipError_t launch_ranges_fix(const uint64_t* keys, const uint32_t* num_pairs, const uint32_t* status,
                             const uint32_t* bases, uint32_t bins, uint32_t num_tiles, uint32_t* ranges,
                             hipStream_t s);
// The same per frame of a segmented batch (one workgroup per frame):
// bases [frame][...] frame_stride apart, seg_base [frames + 1].
hipError_t launch_ranges_fix_seg(const uint64_t* keys, const uint32_t* status, const uint32_t* bases, uint32_t bins,
                                 uint32_t frame_stride, const uint32_t* seg_base, const FrameInfo* table,
                                 uint32_t n_frames, uint32_t* ranges, hipStream_t s);
// The compiled digit width (>= bits) that a pass of this shape can use when
// its digit has only `bits` significant bits, or 0 (use radix_bits).
int narrow_pass_bits(int bits, int key_bytes, int radix_bits, int items, int threads);

// Tile-first ordering (see tilesort.hip): every tile's run of pairs, in
// Gaussian index order, sorted stably by depth, one workgroup per tile.
constexpr uint32_t kTileSortCap = 8192;   // pairs of a run sorted in LDS
struct TileSortArgs {
  uint64_t* keys;           // [M] tile << 32 | depth bits, runs by tile
  uint32_t* values;         // [M] Gaussian index
  const uint32_t* ranges;   // [2 num_tiles] each tile's run
  uint32_t num_tiles;
  uint64_t* alt;            // [M] scratch for runs longer than kTileSortCap
  const uint32_t* status;   // or NULL
};
hipError_t launch_tile_sort(const TileSortArgs& a, hipStream_t s);

// Small frames in two kernels (see tiny.hip): at most kTinyMaxTiles tiles
// and kTinyMaxGaussians Gaussians, one frame.
constexpr uint32_t kTinyGaussians = 512;       // Gaussians per bucketing workgroup
constexpr uint32_t kTinyMaxGaussians = 16384;
constexpr uint32_t kTinyMaxBlocks = kTinyMaxGaussians / kTinyGaussians;
constexpr uint32_t kTinyMaxTiles = 256;
struct TinyArgs {
  const ss_gaussian2d* gaussians;
  uint32_t n;
  uint32_t tiles_x, tiles_y;
  uint32_t nblocks;         // ceil(n / kTinyGaussians)
  uint64_t* region;         // [nblocks][region_cap] pairs grouped by tile per workgroup
  uint32_t region_cap;      // min(kTinyGaussians * tiles, capacity): a workgroup's most pairs
  uint32_t* rows;           // [nblocks][2 tiles + 1]: per-tile counts, their exclusive
                            // prefix, a bad-depth flag
  uint32_t capacity;
  uint64_t* keys;
  uint32_t* values;
  uint32_t* ranges;
  uint32_t* num_pairs;
  uint32_t* status;
};
// bucket = true: kernel 1 (skipped for no Gaussians); false: kernel 2.
hipError_t launch_tiny(const TinyArgs& a, hipStream_t s, bool bucket);

// Render (see render.hip).
struct RenderArgs {
  const ss_gaussian2d* gaussians;
  const float* conic_opacity;   // [N][4]
  const float* rgb;             // [N][4]
  const uint32_t* values;
  const uint32_t* ranges;       // [2T]
  const uint32_t* status;       // or NULL
  uint32_t width, height, tiles_x, tiles_y;
  float bg[3];
  float* color;                 // [3][H][W]
  float* T;                     // [H][W] or NULL
  uint32_t* contrib;            // [H][W] or NULL
  uint32_t* tile_evals;         // [T] or NULL
};
hipError_t launch_render(const RenderArgs& a, bool exact, hipStream_t s);

// Preprocess: one thread per Gaussian (see preprocess.hip).
struct PreprocessArgs {
  ss_camera cam;
  uint32_t n;
  const float* mean3d_opacity;  // [N][4]
  const float* cov3d;           // [N][8]
  const float* sh;              // [N][48]
  ss_gaussian2d* records;       // [N]
  float* conic_opacity;         // [N][4]
  float* rgb;                   // [N][4]
};
hipError_t launch_preprocess(const PreprocessArgs& a, hipStream_t s);

// The paper's bitonic network (see bitonic.hip), over a power-of-two padded
// buffer sorted in place by (key, value).
struct BitonicArgs {
  void* keys;                   // [2^log_n] padded buffer: uint64_t, or uint32_t when key32
  uint32_t* vals;
  uint32_t log_n;
  const uint32_t* num_pairs;    // device count of valid entries, or NULL (then n_fixed)
  uint32_t n_fixed;
  const uint32_t* status;       // or NULL
  uint64_t* out_keys;           // the last kernel writes the valid entries here
  uint32_t* out_vals;
  uint32_t out_capacity;
  bool key32;                   // the paper's normalised 32-bit float key (source keys are frame keys)
  const ss_gaussian2d* gaussians; // key32: the frame's records, to rebuild the exact output keys
};
uint32_t bitonic_log_size(uint64_t n);          // smallest l >= 1 with 2^l >= n
uint32_t bitonic_launches(uint32_t log_n);
// Pads (and, with src_k, first loads src[0, n) with keys masked by key_mask,
// or normalised to 32 bits when key32), then sorts and writes the first n
// entries to out_*.
hipError_t launch_bitonic(const BitonicArgs& a, const uint64_t* src_k, const uint32_t* src_v, uint64_t key_mask,
                          hipStream_t s);

// Sort-pass configurations (radix width, items per thread, workgroup size)
// compiled into the library.
bool pass_config_supported(int radix_bits, int items, int threads);

}  // namespace ss

// Host side of the C ABI declared in splatsort.h: argument validation,
// workspace layout and the launch sequences of the hot path.
#include <stdint.h>

#include <cmath>
#include <cstddef>
#include <new>
#include <vector>

#include "internal.hpp"
#include "splatsort.h"

namespace ss {
namespace {

constexpr uint32_t kDefaultRadix = 8;
constexpr uint32_t kDefaultItems = 16;
constexpr uint32_t kDefaultThreads = 512;
constexpr size_t kAlign = 256;
// tile passes: at most ceil(32 / 4)
constexpr uint32_t kMaxTilePasses = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// Counter words at the start of the workspace.

// the normalised 32-bit key holds 20 bits of tile number
constexpr uint64_t kKey32MaxTiles = uint64_t{1} << 20;

struct Options {
  uint32_t radix_bits = kDefaultRadix;
  uint32_t items = kDefaultItems;
  uint32_t threads = kDefaultThreads;
  uint32_t flags = 0;
  uint32_t algorithm = SS_ALGO_AUTO;
  ss_timer* timer = nullptr;
  bool items_default = true;  // items_per_thread left at 0 (the frame size may choose)
  uint32_t spin_limit = 0;    // 0: the kernels' default
  uint32_t fault = SS_FAULT_NONE;
};

ss_status parse_options(const ss_options* o, Options* out) {
  *out = Options{};
  if (o == nullptr) return SS_OK;
  // callers built before spin_limit and fault existed pass the shorter struct
  if (o->struct_size < offsetof(ss_options, spin_limit)) return SS_ERR_INVALID_ARGUMENT;
  if ((o->flags & ~(SS_FLAG_UNSORTED | SS_FLAG_KEY32_LOSSY | SS_FLAG_DROP_CULLED | SS_FLAG_PERSISTENT)) != 0)
    return SS_ERR_UNSUPPORTED;
  if (o->struct_size >= sizeof(ss_options)) {
    if (o->fault > SS_FAULT_WITHHOLD_BASES) return SS_ERR_UNSUPPORTED;
    out->spin_limit = o->spin_limit;
    out->fault = o->fault;
  }
  if (o->algorithm > SS_ALGO_TILE_FIRST) return SS_ERR_UNSUPPORTED;
  // the normalised 32-bit key belongs to the bitonic network and needs the sort
  if ((o->flags & SS_FLAG_KEY32_LOSSY) != 0 &&
      (o->algorithm != SS_ALGO_BITONIC || (o->flags & SS_FLAG_UNSORTED) != 0))
    return SS_ERR_UNSUPPORTED;
  out->flags = o->flags;
  out->algorithm = o->algorithm;
  if (o->radix_bits != 0) out->radix_bits = o->radix_bits;
  if (o->items_per_thread != 0) {
    out->items = o->items_per_thread;
    out->items_default = false;
  }
  // default workgroup: 512 where that configuration exists, else 256
  out->threads = pass_config_supported(static_cast<int>(out->radix_bits), static_cast<int>(out->items), 512)
                     ? 512u : 256u;
  if (o->workgroup_size != 0) out->threads = o->workgroup_size;
  if (!pass_config_supported(static_cast<int>(out->radix_bits), static_cast<int>(out->items),
                             static_cast<int>(out->threads)))
    return SS_ERR_UNSUPPORTED;
  out->timer = o->timer;
  return SS_OK;
}

uint32_t ceil_log2(uint64_t t) {
  uint32_t b = 0;
  while ((uint64_t{1} << b) < t) ++b;
  return b;
}

struct Geometry {
  uint32_t tiles_x = 0, tiles_y = 0, num_tiles = 0, key_bits = 0;
};

ss_status frame_geometry(const ss_frame* f, Geometry* g) {
  if (f == nullptr) return SS_ERR_INVALID_ARGUMENT;
  if (f->tile_px != 16) return SS_ERR_INVALID_ARGUMENT;
  if (f->width < 1 || f->height < 1 || f->width > SS_MAX_IMAGE_PX || f->height > SS_MAX_IMAGE_PX)
    return SS_ERR_INVALID_ARGUMENT;
  if (f->num_gaussians > 0x7FFFFFFFu) return SS_ERR_INVALID_ARGUMENT;
  if (f->num_gaussians > 0 && (f->gaussians == nullptr || !aligned(f->gaussians, 16)))
    return SS_ERR_INVALID_ARGUMENT;
  g->tiles_x = (f->width + 15) / 16;
  g->tiles_y = (f->height + 15) / 16;
  const uint64_t t = static_cast<uint64_t>(g->tiles_x) * g->tiles_y;  // < 2^32 by the size limit
  g->num_tiles = static_cast<uint32_t>(t);
  g->key_bits = 32 + ceil_log2(t);
  return SS_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---------------------------------------------------------------------------
// Direct path: count/scan/duplicate in index order, then P passes over the
// full key.  Workspace: [scalars | bases | scan look-back |
// histograms | pass look-back] zeroed per call, then the alternate buffers.
// ---------------------------------------------------------------------------
struct Layout {
  uint32_t npasses = 0, bins = 0, count_blocks = 0, pass_blocks = 0, tile = 0, log_pad = 0;
  size_t scan_lb = 0, hist = 0, pass_lb = 0, scalars = 0, bases = 0, clear_end = 0;
  size_t alt_keys = 0, alt_vals = 0, total = 0;
};

Layout make_layout(uint32_t n_gauss, uint32_t capacity, uint32_t key_bits, const Options& o) {
  Layout L;
  L.bins = 1u << o.radix_bits;
  const bool bitonic = o.algorithm == SS_ALGO_BITONIC;
  // the bitonic network sorts in place in the (power-of-two padded) alternate buffers
  L.npasses = bitonic ? 0u : (key_bits + o.radix_bits - 1) / o.radix_bits;
  L.log_pad = bitonic ? bitonic_log_size(capacity > 2 ? capacity : 2) : 0u;
  const size_t alt = bitonic ? (size_t{1} << L.log_pad) : capacity;
  L.count_blocks = n_gauss == 0 ? 1u : (n_gauss + kCountTile - 1) / kCountTile;
  L.tile = o.threads * o.items;
  L.pass_blocks = (capacity + L.tile - 1) / L.tile;
  size_t off = 0;
  L.scalars = off;   off = align_up(off + 4 * sizeof(uint32_t));
  L.bases = off;     off = align_up(off + static_cast<size_t>(L.npasses) * L.bins * sizeof(uint32_t));
  L.scan_lb = off;   off = align_up(off + static_cast<size_t>(L.count_blocks) * sizeof(uint64_t));
  L.hist = off;      off = align_up(off + static_cast<size_t>(kHistCopies) * L.npasses * L.bins * sizeof(uint32_t));
  L.pass_lb = off;   off = align_up(off + static_cast<size_t>(L.npasses) * L.pass_blocks * L.bins * sizeof(uint32_t));
  L.clear_end = off;
  L.alt_keys = off;  off = align_up(off + alt * sizeof(uint64_t));
  L.alt_vals = off;  off = align_up(off + alt * sizeof(uint32_t));
  L.total = off;
  return L;
}

// ---------------------------------------------------------------------------
// Depth-first path (one frame or a batch).  Zeroed part: scalars,
// bad flag, totals, count-only scan look-back, expand look-back, histograms
// and look-back words of the depth and tile passes; then the frame table,
// tile digit bases, rectangles, the Gaussian sort buffers and the alternate
// pair buffers.
// ---------------------------------------------------------------------------
struct PassCfg {
  uint32_t items = 16, threads = 512;
  uint32_t tile() const { return items * threads; }
};

// Depth-sort passes run over N Gaussians (8-byte items).  Their time is
// set by per-workgroup latency (look-back round trips) more than by
// bandwidth, so fewer, larger workgroups win; below 2^21 Gaussians a
// half-size tile keeps more CUs busy, and 1,024 threads of 4 items each
// (sixteen waves) rank it sooner than 512 of 8.
PassCfg depth_cfg(uint32_t n) {
  if (n < (1u << 21)) return PassCfg{4, 1024};
  return PassCfg{16, 512};
}

struct DfLayout {
  uint32_t n = 0, n_frames = 0, capacity = 0, total_tiles = 0, tile_bits = 0, tpasses = 0, tbins = 256, trb = 8;
  // packed pairs through the tile passes (PackedPairs): tile << (64 - tile
  // bits) | depth field << idx_bits | index
  bool packed = false;
  uint32_t idx_bits = 0;
  // Segmented batch (several frames): the depth sort orders every frame's
  // Gaussians apart, inside the frame's own index range, so each frame's
  // pairs come out contiguous and the tile passes sort every frame on its
  // own, on frame-local tile ids (tile_bits then counts the largest frame's
  // tiles).
  bool seg = false;
  PassCfg dcfg, tcfg;
  uint32_t dblocks = 0, tblocks = 0, eblocks = 0, count_blocks = 0, ck_blocks = 0;
  size_t block_total = 0, block_frame = 0;
  size_t scalars = 0, bad = 0, totals = 0, scan_lb = 0, expand_lb = 0, hist_d = 0, hist_f = 0, hist_t = 0,
         lb_d = 0, lb_t = 0, clear_end = 0, table = 0, bases_t = 0, rect = 0, key = 0, val = 0,
         key_alt = 0, val_alt = 0, alt_keys = 0, alt_vals = 0, seg_base = 0, seg_wgs = 0, tickets = 0, wg_totals = 0,
         total = 0;
};

// Pairs travel through the tile passes as one 64-bit item when the tile id,
// the largest frame-local index and a depth field fit: the depth field needs
// 27 bits for depths spanning up to 16 binades (23 mantissa bits plus the
// exponent above the smallest one), and at least the bits of a position in
// depth order (the fallback when the depths span more).
bool use_packed(uint32_t tile_bits, uint32_t tpasses, uint32_t idx_bits, uint32_t n, const PassCfg& tcfg,
                uint32_t trb) {
  if (tpasses == 0 || tile_bits > 32) return false;
  if (!packed_pass_supported(static_cast<int>(trb), static_cast<int>(tcfg.items), static_cast<int>(tcfg.threads)))
    return false;
  const uint32_t depth_field = 64 - tile_bits - idx_bits;
  return idx_bits < 32 && depth_field >= 27 && ceil_log2(n) <= depth_field;
}

// Tile passes for `bits` tile bits.  With 8-bit digits in 512-thread passes,
// several passes split the bits evenly (13 bits: 7 + 6 instead of 8 + 5): the
// widest pass has fewer digits, so its runs of one digit, and its writes, are
// longer.
void plan_tile_passes(DfLayout& L, uint32_t bits, const Options& o) {
  L.tile_bits = bits;
  L.tpasses = (bits + o.radix_bits - 1) / o.radix_bits;
  L.trb = o.radix_bits;
  if (L.tpasses >= 2 && o.radix_bits == 8 && o.threads == 512 && (o.items == 8 || o.items == 16))
    L.trb = (bits + L.tpasses - 1) / L.tpasses;
  L.tbins = 1u << L.trb;
}

DfLayout make_df_layout(uint32_t n, uint32_t n_frames, uint32_t capacity, uint64_t total_tiles, const Options& o,
                        uint32_t max_frame_n, uint64_t max_frame_tiles) {
  DfLayout L;
  L.n = n;
  L.n_frames = n_frames;
  L.capacity = capacity;
  L.total_tiles = static_cast<uint32_t>(total_tiles);
  plan_tile_passes(L, ceil_log2(total_tiles), o);
  L.dcfg = depth_cfg(n);
  L.tcfg = PassCfg{o.items, o.threads};
  // default shape, fewer than 2^23 pairs: 4,096-pair tiles (twice the
  // workgroups, so more of them load while others rank; measured faster up
  // to the full-HD frame, slower from the 27.6M-pair frame on)
  if (o.items_default && o.threads == 512 && o.items == 16 && capacity < (1u << 23)) L.tcfg.items = 8;
  L.dblocks = (n + L.dcfg.tile() - 1) / L.dcfg.tile();
  L.idx_bits = ceil_log2(max_frame_n);
  L.packed = use_packed(L.tile_bits, L.tpasses, L.idx_bits, n, L.tcfg, L.trb);
  // Segmented batch: frame-local tiles (at most 2^16 per frame, as the
  // expansion's 16-bit tile field holds) in packed pairs, without dropping
  // culled Gaussians (the segmented depth sort places frame f at its first Gaussian)
  if (n_frames > 1 && (o.flags & SS_FLAG_DROP_CULLED) == 0) {
    const uint32_t lbits = ceil_log2(max_frame_tiles);
    if (lbits >= 1 && lbits <= 16) {
      const DfLayout whole = L;
      plan_tile_passes(L, lbits, o);
      if (use_packed(L.tile_bits, L.tpasses, L.idx_bits, n, L.tcfg, L.trb)) {
        L.seg = true;
        L.packed = true;
      } else {
        L = whole;
      }
    }
  }
  // a segmented pass has up to one partial workgroup per frame (the depth
  // sort's too: it sorts every frame's Gaussians apart)
  if (L.seg) L.dblocks += n_frames;
  L.tblocks = (capacity + L.tcfg.tile() - 1) / L.tcfg.tile() + (L.seg ? n_frames : 0u);
  const uint32_t hframes = L.seg ? n_frames : 1u;  // tile histograms and bases per frame
  L.eblocks = n == 0 ? 1u : (n + kExpandTile - 1) / kExpandTile;  // workgroup 0 also finishes the totals
  L.count_blocks = n == 0 ? 1u : (n + kCountTile - 1) / kCountTile;
  size_t off = 0;
  L.scalars = off;   off = align_up(off + 8 * sizeof(uint32_t));  // status, M, offsets' M and status, live,
                                                                     // depth top byte max / min
  L.bad = off;       off = align_up(off + sizeof(uint32_t));
  L.totals = off;    off = align_up(off + (1 + static_cast<size_t>(n_frames)) * sizeof(uint64_t));
  L.ck_blocks = (n + kCountKeysTile - 1) / kCountKeysTile;
  L.block_total = off; off = align_up(off + static_cast<size_t>(L.ck_blocks) * sizeof(uint64_t));
  L.block_frame = off; off = align_up(off + static_cast<size_t>(L.ck_blocks) * sizeof(uint32_t));
  L.scan_lb = off;   off = align_up(off + static_cast<size_t>(L.count_blocks) * sizeof(uint64_t));
  L.expand_lb = off; off = align_up(off + static_cast<size_t>(L.eblocks) * sizeof(uint64_t));
  L.hist_d = off;    off = align_up(off + static_cast<size_t>(kHistCopies) * 4 * 256 * sizeof(uint32_t));
  // segmented: the depth-digit histograms per frame too
  L.hist_f = off;    off = align_up(off + (L.seg ? static_cast<size_t>(kHistCopies) * n_frames * 4 * 256 : 0u) *
                                            sizeof(uint32_t));
  L.hist_t = off;    off = align_up(off + static_cast<size_t>(kHistCopies) * hframes * L.tpasses * L.tbins *
                                            sizeof(uint32_t));
  // four depth passes
  L.lb_d = off;      off = align_up(off + static_cast<size_t>(4) * L.dblocks * 256 * sizeof(uint32_t));
  // packed: the last tile pass's look-back words are 64-bit (one more slice)
  L.lb_t = off;      off = align_up(off + static_cast<size_t>(L.tpasses + (L.packed ? 1 : 0)) * L.tblocks * L.tbins *
                                            sizeof(uint32_t));
  L.bases_t = off;   off = align_up(off + static_cast<size_t>(hframes) * L.tpasses * L.tbins * sizeof(uint32_t));
  L.tickets = off;   off = align_up(off + kMaxTilePasses * sizeof(uint32_t));  // persistent tile passes
  L.clear_end = off;
  // written whole by the expansion's totals
  L.seg_base = off;  off = align_up(off + (L.seg ? n_frames + 1u : 0u) * sizeof(uint32_t));
  L.seg_wgs = off;   off = align_up(off + (L.seg ? n_frames + 1u : 0u) * sizeof(uint32_t));
  L.wg_totals = off; off = align_up(off + static_cast<size_t>(L.eblocks) * sizeof(uint64_t));  // expand's
  L.table = off;     off = align_up(off + static_cast<size_t>(n_frames) * sizeof(FrameInfo));
  L.rect = off;      off = align_up(off + static_cast<size_t>(n) * sizeof(uint64_t));
  L.key = off;       off = align_up(off + static_cast<size_t>(n) * sizeof(uint32_t));
  L.val = off;       off = align_up(off + static_cast<size_t>(n) * sizeof(uint32_t));
  L.key_alt = off;   off = align_up(off + static_cast<size_t>(n) * sizeof(uint32_t));
  L.val_alt = off;   off = align_up(off + static_cast<size_t>(n) * sizeof(uint32_t));
  L.alt_keys = off;  off = align_up(off + static_cast<size_t>(capacity) * sizeof(uint64_t));
  L.alt_vals = off;  off = align_up(off + static_cast<size_t>(capacity) * sizeof(uint32_t));
  L.total = off;
  return L;
}

}  // namespace
}  // namespace ss

struct ss_timer {
  std::vector<hipEvent_t> events;  // two per record
  std::vector<uint32_t> kinds;
  std::vector<uint32_t> launches;  // kernels covered by each record
  uint32_t used = 0;
};

namespace ss {
namespace {

// Runs launches, bracketed by timer events when a timer is attached.
class Launcher {
 public:
  Launcher(hipStream_t s, ss_timer* t) : s_(s), t_(t) {}
  template <typename F>
  ss_status run(uint32_t kind, F&& launch) {
    return run_group(kind, 1, [&] { return launch() == hipSuccess ? SS_OK : SS_ERR_HIP; });
  }
  // Several consecutive launches of one kind under a single pair of events
  // (no event between them, so their own durations are not inflated).
  template <typename F>
  ss_status run_group(uint32_t kind, uint32_t count, F&& launches) {
    int slot = -1;
    if (t_ != nullptr && t_->used < t_->kinds.size()) {
      slot = static_cast<int>(t_->used++);
      t_->kinds[slot] = kind;
      t_->launches[slot] = count;
      if (hipEventRecord(t_->events[2 * slot], s_) != hipSuccess) return SS_ERR_HIP;
    }
    const ss_status st = launches();
    if (st != SS_OK) return st;
    if (slot >= 0 && hipEventRecord(t_->events[2 * slot + 1], s_) != hipSuccess) return SS_ERR_HIP;
    return SS_OK;
  }

 private:
  hipStream_t s_;
  ss_timer* t_;
};

#define SS_TRY(x)                     \
  do {                                \
    const ss_status st_ = (x);        \
    if (st_ != SS_OK) return st_;     \
  } while (0)

// A chain of P digit passes.  Pass p reads src[p], writes dst[p], sorts on
// bits [shift0 + RB p, shift0 + RB (p + 1)).
struct PassChain {
  uint32_t npasses;
  uint32_t key_bytes;
  uint32_t shift0;
  uint32_t radix_bits;
  PassCfg cfg;
  uint32_t nblocks;
  const void* const* ksrc;
  const uint32_t* const* vsrc;
  void* const* kdst;
  uint32_t* const* vdst;
  const uint32_t* num_pairs;  // device M or NULL (then n_fixed)
  uint32_t n_fixed;
  uint32_t* status;
  uint32_t* bases;            // 64-bit keys: [npasses][bins] published digit bases (zeroed), or NULL
  const uint32_t* hist;       // pass p's totals at hist + p * bins, copies hist_stride apart
  uint32_t hist_stride;
  uint32_t* lookback;         // [npasses][nblocks][bins]
  uint32_t last_bits;         // significant bits of the last pass's digit when fewer
                              // than radix_bits (keys known to be below 2^(shift0 +
                              // radix_bits (npasses - 1) + last_bits)), else 0
  // the Gaussian depth sort: the culled count's histogram words (the first
  // pass may drop the culled), and where it stores the count it keeps
  const uint32_t* culled;
  uint32_t* kept;
  // 32-bit keys: a second value moved with the first (pass p reads psrc[p],
  // writes pdst[p]), or NULL
  const uint32_t* const* psrc;
  uint32_t* const* pdst;
  // packed pairs (64-bit items): NULL for key + value passes.  The last pass
  // unpacks into kdst/vdst and writes the tile ranges, with 64-bit look-back
  // words at lookback64.
  const PackedPairs* packed;
  uint32_t* ranges;
  uint64_t* lookback64;
  // the depth sort: its first pass stores the top-byte range of the depth
  // keys with pairs (for packed pairs) at depth_top_out, from hist_top
  uint32_t* depth_top_out;
  const uint32_t* hist_top;
  // the segmented depth sort (32-bit keys): every frame's Gaussians apart
  bool depth_seg;
  const FrameInfo* table;     // the segmented depth sort and unpacking pass
  uint32_t n_frames;
  // segmented 64-bit passes (PassArgs): per-frame workgroups, pairs, and
  // histograms and bases frame_stride apart
  const uint32_t* seg_wgs;
  const uint32_t* seg_base;
  uint32_t frame_stride;
  // waits, test hook, persistent 64-bit passes (pass p's zeroed counter at
  // tickets + p; NULL: one workgroup per tile)
  uint32_t spin_limit;
  uint32_t fault;
  uint32_t* tickets;
};

ss_status run_chain(Launcher& L, uint32_t kind, const PassChain& c, hipStream_t s) {
  if (c.npasses == 0) return SS_OK;
  const uint32_t bins = 1u << c.radix_bits;
  return L.run_group(kind, c.npasses, [&]() -> ss_status {
    for (uint32_t p = 0; p < c.npasses; ++p) {
      PassArgs a{};
      a.kin = c.ksrc[p];
      a.vin = c.vsrc[p];
      a.kout = c.kdst[p];
      a.vout = c.vdst[p];
      a.num_pairs = c.num_pairs;
      a.n_fixed = c.n_fixed;
      a.status = c.status;
      a.shift = c.shift0 + p * c.radix_bits;
      a.bases = c.bases ? c.bases + static_cast<size_t>(p) * bins : nullptr;
      a.hist = c.hist ? c.hist + static_cast<size_t>(p) * bins : nullptr;
      a.hist_stride = c.hist_stride;
      a.publish_passes = c.bases != nullptr && p == 0 ? c.npasses : 0u;
      if (c.kept != nullptr) {
        if (p == 0) {
          a.culled = c.culled;
          a.kept = c.kept;
        } else {
          a.num_pairs = c.kept;
          a.n_total = c.n_fixed;
        }
      }
      if (c.psrc != nullptr) {
        a.pin = c.psrc[p];
        a.pout = c.pdst[p];
      }
      if (p == 0 && c.depth_top_out != nullptr) {
        a.depth_top_out = c.depth_top_out;
        a.hist_top = c.hist_top;
      }
      a.spin_limit = c.spin_limit;
      a.fault = c.fault;
      a.tickets = c.tickets ? c.tickets + p : nullptr;
      a.depth_seg = c.depth_seg;
      a.table = c.table;
      a.n_frames = c.n_frames;
      if (c.seg_wgs != nullptr) {
        a.seg_wgs = c.seg_wgs;
        a.seg_base = c.seg_base;
        a.seg_frames = c.n_frames;
        a.bases_frame_stride = c.frame_stride;
      }
      int mode = kPassKV;
      if (c.packed != nullptr) {
        a.packed = *c.packed;
        mode = p + 1 == c.npasses ? kPassUnpack : kPassItems;
        if (mode == kPassUnpack) {
          a.ranges = c.ranges;
          a.low_bits = a.shift - c.packed->tile_shift;
          a.lookback64 = c.lookback64;
        }
      }
      a.lookback = c.lookback + static_cast<size_t>(p) * c.nblocks * bins;
      // the last pass ranks only its significant digit bits where a narrower
      // pass exists (its digits above them are empty; the histogram, base and
      // look-back layouts stay those of radix_bits)
      int rb = static_cast<int>(c.radix_bits);
      if (p + 1 == c.npasses && c.last_bits != 0 && c.last_bits < c.radix_bits) {
        const int narrow = narrow_pass_bits(static_cast<int>(c.last_bits), static_cast<int>(c.key_bytes),
                                            static_cast<int>(c.radix_bits), static_cast<int>(c.cfg.items),
                                            static_cast<int>(c.cfg.threads));
        if (narrow != 0) rb = narrow;
      }
      if (launch_pass(a, static_cast<int>(c.key_bytes), rb, static_cast<int>(c.cfg.items),
                      static_cast<int>(c.cfg.threads), c.nblocks, s, mode) != hipSuccess)
        return SS_ERR_HIP;
    }
    return SS_OK;
  });
}

// ----------------------------- direct path ---------------------------------
ss_status run_direct(Launcher& L, const ss_frame* frame, const Geometry& g, const ss_frame_out* out,
                     const Options& o, void* ws, hipStream_t s) {
  const uint32_t cap = out->pair_capacity;
  const Layout lay = make_layout(frame->num_gaussians, cap, g.key_bits, o);
  uint32_t* scal = at<uint32_t>(ws, lay.scalars);
  uint32_t* d_status = out->status ? out->status : scal + 0;
  uint32_t* d_num_pairs = out->num_pairs ? out->num_pairs : scal + 1;
  const bool unsorted = (o.flags & SS_FLAG_UNSORTED) != 0;
  const bool bitonic = o.algorithm == SS_ALGO_BITONIC && !unsorted;
  const bool key32 = (o.flags & SS_FLAG_KEY32_LOSSY) != 0;
  const uint32_t P = unsorted ? 0 : lay.npasses;
  // dup writes buf[0]; pass p reads buf[p % 2] and writes buf[(p + 1) % 2];
  // the data ends in buf[P % 2], which must be the caller's output.  The
  // bitonic network instead sorts the padded alternate buffer in place and
  // its last kernel writes the output.
  uint64_t* bk[2];
  uint32_t* bv[2];
  bk[P % 2] = out->keys;
  bv[P % 2] = out->values;
  bk[(P + 1) % 2] = at<uint64_t>(ws, lay.alt_keys);
  bv[(P + 1) % 2] = at<uint32_t>(ws, lay.alt_vals);
  if (bitonic && !key32) {
    bk[0] = at<uint64_t>(ws, lay.alt_keys);
    bv[0] = at<uint32_t>(ws, lay.alt_vals);
  }
  // key32: the pairs are duplicated into the caller's output, normalised from
  // there into the padded buffer, and written back with their exact keys
  if (key32) {
    bk[0] = out->keys;
    bv[0] = out->values;
  }

  SS_TRY(L.run(SS_KERNEL_CLEAR, [&] { return launch_clear(ws, lay.clear_end, d_status, nullptr, nullptr, s); }));
  CountDupArgs a{};
  a.gaussians = frame->gaussians;
  a.n = frame->num_gaussians;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  a.capacity = cap;
  a.npasses = lay.npasses;
  a.tiles_touched = out->tiles_touched;
  a.offsets = out->offsets;
  a.keys = bk[0];
  a.values = bv[0];
  a.lookback = at<uint64_t>(ws, lay.scan_lb);
  a.hist = at<uint32_t>(ws, lay.hist);
  a.num_pairs = d_num_pairs;
  a.status = d_status;
  a.nblocks = lay.count_blocks;
  SS_TRY(L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_count_dup(a, static_cast<int>(o.radix_bits), true, s); }));
  if (unsorted) return SS_OK;
  if (bitonic) {
    BitonicArgs b{at<void>(ws, lay.alt_keys), at<uint32_t>(ws, lay.alt_vals), lay.log_pad, d_num_pairs, 0,
                  d_status, out->keys, out->values, cap, key32, frame->gaussians};
    SS_TRY(L.run_group(SS_KERNEL_SORT_PASS, bitonic_launches(lay.log_pad), [&] {
      return launch_bitonic(b, key32 ? out->keys : nullptr, key32 ? out->values : nullptr, ~0ull, s) == hipSuccess
                 ? SS_OK : SS_ERR_HIP;
    }));
    return L.run(SS_KERNEL_RANGES, [&] {
      return launch_ranges(out->keys, d_num_pairs, d_status, cap, g.num_tiles, out->tile_ranges, s);
    });
  }
  uint32_t* bases = at<uint32_t>(ws, lay.bases);
  std::vector<const void*> ks(P);
  std::vector<const uint32_t*> vs(P);
  std::vector<void*> kd(P);
  std::vector<uint32_t*> vd(P);
  for (uint32_t p = 0; p < P; ++p) {
    ks[p] = bk[p % 2];
    vs[p] = bv[p % 2];
    kd[p] = bk[(p + 1) % 2];
    vd[p] = bv[(p + 1) % 2];
  }
  PassChain c{P, 8, 0, o.radix_bits, PassCfg{o.items, o.threads}, lay.pass_blocks, ks.data(), vs.data(),
              kd.data(), vd.data(), d_num_pairs, 0, d_status, bases, a.hist, lay.npasses * lay.bins,
              at<uint32_t>(ws, lay.pass_lb), g.key_bits - o.radix_bits * (P - 1)};
  SS_TRY(run_chain(L, SS_KERNEL_SORT_PASS, c, s));
  return L.run(SS_KERNEL_RANGES, [&] {
    return launch_ranges(out->keys, d_num_pairs, d_status, cap, g.num_tiles, out->tile_ranges, s);
  });
}

// Zeroes the workspace head and stores the frame table: the first kArgFrames
// frames ride along with the clear kernel, the rest in further launches.
ss_status clear_and_upload(Launcher& L, void* ws, size_t clear_bytes, uint32_t* d_status, const FrameInfo* host_table,
                           uint32_t n_frames, FrameInfo* table, hipStream_t s) {
  for (uint32_t first = 0; first == 0 || first < n_frames; first += kArgFrames) {
    TableChunk c{};
    c.first = first;
    c.count = n_frames - first < kArgFrames ? n_frames - first : kArgFrames;
    for (uint32_t i = 0; i < c.count; ++i) c.f[i] = host_table[first + i];
    if (first == 0)
      SS_TRY(L.run(SS_KERNEL_CLEAR, [&] { return launch_clear(ws, clear_bytes, d_status, &c, table, s); }));
    else
      SS_TRY(L.run(SS_KERNEL_CLEAR, [&] { return launch_put_table(c, table, s); }));
  }
  return SS_OK;
}

// --------------------------- depth-first path ------------------------------
struct DfIO {
  const FrameInfo* host_table;  // [n_frames], gaussians pointers are device pointers
  const ss_frame* frames;       // for the optional index-order offsets (one frame)
  uint64_t* keys;
  uint32_t* values;
  uint32_t* ranges;
  uint32_t* tiles_touched;      // single frame only, may be NULL
  uint32_t* offsets;            // single frame only, may be NULL
  uint32_t* num_pairs;          // may be NULL
  uint32_t* status;             // may be NULL
  uint32_t* frame_pairs;        // batch only, may be NULL
  uint32_t* frame_pair_base;    // batch only, may be NULL
};

// Tile-first: every tile's run (index order, after the tile passes) sorted
// stably by depth; runs too long for LDS use the alternate pair buffer.
ss_status sort_tile_runs(Launcher& L, const DfLayout& lay, const DfIO& io, void* ws, uint32_t* d_status,
                         hipStream_t s) {
  TileSortArgs t{io.keys, io.values, io.ranges, lay.total_tiles, at<uint64_t>(ws, lay.alt_keys), d_status};
  return L.run(SS_KERNEL_TILE_SORT, [&] { return launch_tile_sort(t, s); });
}

ss_status run_depth_first(Launcher& L, const DfLayout& lay, const Options& o, const DfIO& io, void* ws,
                          hipStream_t s) {
  uint32_t* scal = at<uint32_t>(ws, lay.scalars);
  uint32_t* d_status = io.status ? io.status : scal + 0;
  uint32_t* d_num_pairs = io.num_pairs ? io.num_pairs : scal + 1;
  FrameInfo* table = at<FrameInfo>(ws, lay.table);

  SS_TRY(clear_and_upload(L, ws, lay.clear_end, d_status, io.host_table, lay.n_frames, table, s));
  if (io.offsets != nullptr) {
    // the index-order scan exists only for this optional output
    CountDupArgs a{};
    a.gaussians = io.frames->gaussians;
    a.n = io.frames->num_gaussians;
    a.tiles_x = io.host_table[0].tiles_x;
    a.tiles_y = io.host_table[0].tiles_y;
    a.offsets = io.offsets;
    a.lookback = at<uint64_t>(ws, lay.scan_lb);
    a.num_pairs = scal + 2;
    a.status = scal + 3;
    a.nblocks = lay.count_blocks;
    SS_TRY(L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_count_dup(a, 8, false, s); }));
  }

  uint32_t* key = at<uint32_t>(ws, lay.key);
  uint32_t* val = at<uint32_t>(ws, lay.val);
  uint32_t* key_alt = at<uint32_t>(ws, lay.key_alt);
  uint32_t* val_alt = at<uint32_t>(ws, lay.val_alt);
  // Frames of at most 256 tiles per axis pack a rectangle into 32 bits, which
  // the depth sort carries beside the indices: expand then reads the
  // rectangles in sequence instead of gathering a cache line per Gaussian.
  // The two packed buffers share the 64-bit rectangles' space.  Up to 2^23
  // Gaussians the depth passes absorb the extra 8 B per Gaussian almost for
  // free (they wait on the look-back more than on memory).  Beyond that they
  // are bandwidth-bound, and carrying pays only where the gather is worse: a
  // single frame's gather is random over all its rectangles (21.8M
  // Gaussians: 2.95 -> 2.82 ms packed), a batch's stays inside one frame at
  // a time, mostly in cache (64 frames, 38.8M Gaussians: 4.73 against
  // 4.83 ms packed).
  bool small_rects = true;
  for (uint32_t f = 0; f < lay.n_frames; ++f)
    small_rects = small_rects && io.host_table[f].tiles_x <= 256 && io.host_table[f].tiles_y <= 256;
  const bool pack = small_rects && (lay.n <= (1u << 23) || lay.n_frames == 1);
  // not carried but small: packed all the same, by index, so that expand
  // gathers 4 B per Gaussian and a frame's rectangles stay in cache longer
  const bool gather32 = small_rects && !pack && o.algorithm != SS_ALGO_TILE_FIRST;
  uint32_t* rect32 = pack || gather32 ? at<uint32_t>(ws, lay.rect) : nullptr;
  uint32_t* rect32_alt = pack ? rect32 + lay.n : nullptr;
  CountKeysArgs ck{};
  ck.table = table;
  ck.n_frames = lay.n_frames;
  ck.n = lay.n;
  ck.rect = at<uint64_t>(ws, lay.rect);
  ck.rect32 = rect32;
  ck.key = key;
  ck.val = val;
  ck.tiles_touched = io.tiles_touched;
  ck.hist = at<uint32_t>(ws, lay.hist_d);
  ck.frame_hist = lay.seg ? at<uint32_t>(ws, lay.hist_f) : nullptr;
  ck.totals = at<unsigned long long>(ws, lay.totals);
  ck.block_total = at<unsigned long long>(ws, lay.block_total);
  ck.block_frame = at<uint32_t>(ws, lay.block_frame);
  ck.bad = at<uint32_t>(ws, lay.bad);
  // Tile-first (frames): no depth sort; the pairs are written in index
  // order, partitioned stably by tile, and each tile's run is sorted by
  // depth at the end.
  const bool tile_first = o.algorithm == SS_ALGO_TILE_FIRST;
  // with SS_FLAG_DROP_CULLED: Gaussians the depth sort keeps, stored by its first pass
  uint32_t* live = (o.flags & SS_FLAG_DROP_CULLED) != 0 && !tile_first ? scal + 4 : nullptr;
  SS_TRY(L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_count_keys(ck, s); }));

  // stable sort of the Gaussians by depth: key -> alt -> key -> alt -> key;
  // culled ones (no pairs) sort last, or, with SS_FLAG_DROP_CULLED and when
  // they are many, the first pass drops them and the others sort the rest.
  // Segmented (batches): each frame's Gaussians apart, from its own
  // histograms, so that they end frame-major, in depth order, culled last,
  // at the frame's first Gaussian.
  if (!tile_first) {
    const void* ks[4] = {key, key_alt, key, key_alt};
    const uint32_t* vs[4] = {val, val_alt, val, val_alt};
    void* kd[4] = {key_alt, key, key_alt, key};
    uint32_t* vd[4] = {val_alt, val, val_alt, val};
    const uint32_t* ps[4] = {rect32, rect32_alt, rect32, rect32_alt};
    uint32_t* pd[4] = {rect32_alt, rect32, rect32_alt, rect32};
    PassChain c{4, 4, 0, 8, lay.dcfg, lay.dblocks, ks, vs, kd, vd, nullptr, lay.n, d_status,
                nullptr, ck.hist, 4 * 256, at<uint32_t>(ws, lay.lb_d), 0,
                live ? ck.hist + 3 * 256 + 255 : nullptr, live,  // digit 255 of the top byte: culled only
                pack ? ps : nullptr, pack ? pd : nullptr};
    if (lay.packed) {
      c.depth_top_out = scal + 5;
      c.hist_top = ck.hist + 3 * 256;
    }
    if (lay.seg) {
      c.hist = ck.frame_hist;
      c.hist_stride = lay.n_frames * 4 * 256;
      c.depth_seg = true;
      c.table = table;
      c.n_frames = lay.n_frames;
    }
    c.spin_limit = o.spin_limit;
    SS_TRY(run_chain(L, SS_KERNEL_DEPTH_PASS, c, s));
  }
  // the Gaussians in (frame-major when segmented) depth order; tile-first:
  // in index order, as the count kernel wrote them
  const uint32_t* skey = key;
  const uint32_t* sval = val;
  const uint32_t* srect32 = pack ? rect32 : nullptr;

  // expand into pairs, then sort them by tile id alone
  const uint32_t P = lay.tpasses;
  uint64_t* bk[2];
  uint32_t* bv[2];
  bk[P % 2] = io.keys;
  bv[P % 2] = io.values;
  bk[(P + 1) % 2] = at<uint64_t>(ws, lay.alt_keys);
  bv[(P + 1) % 2] = at<uint32_t>(ws, lay.alt_vals);
  // Packed pairs: items ping-pong between the workspace and the output key
  // array, so that the last pass reads the workspace and unpacks into the
  // output: pass p reads the workspace when P - 1 - p is even.
  PackedPairs pk{};
  uint64_t* items_in[kMaxTilePasses + 1];
  if (lay.packed) {
    pk.tile_shift = 64 - lay.tile_bits;
    pk.idx_bits = lay.idx_bits;
    pk.depth_top = scal + 5;
    pk.depth_sorted = skey;
    for (uint32_t p = 0; p < P; ++p) items_in[p] = (P - 1 - p) % 2 == 0 ? at<uint64_t>(ws, lay.alt_keys) : io.keys;
    bk[0] = items_in[0];
  }
  ExpandArgs e{};
  e.table = table;
  e.n_frames = lay.n_frames;
  e.n = lay.n;
  e.n_sorted = live;
  e.key = skey;
  e.val = sval;
  e.rect = ck.rect;
  e.rect32 = srect32;
  e.rect32_idx = gather32 ? rect32 : nullptr;
  e.small_rects = small_rects;
  e.capacity = lay.capacity;
  e.keys = bk[0];
  e.values = bv[0];
  e.npasses = P;
  e.radix_bits = lay.trb;
  e.hist = at<uint32_t>(ws, lay.hist_t);
  e.lookback = at<uint64_t>(ws, lay.expand_lb);
  e.status = d_status;
  e.nblocks = lay.eblocks;
  e.spin_limit = o.spin_limit;
  if (tile_first && lay.packed) {
    e.top_hist = ck.hist + 3 * 256;
    e.top_hist_stride = 4 * 256;
    e.depth_top_out = scal + 5;
  }
  e.packed = lay.packed;
  e.pk = pk;
  e.seg = lay.seg;
  e.totals = PairTotalsArgs{ck.totals, ck.block_total, ck.block_frame, lay.ck_blocks, ck.bad, lay.n_frames,
                            lay.capacity, d_num_pairs, d_status, io.frame_pairs, io.frame_pair_base};
  uint32_t* seg_base = lay.seg ? at<uint32_t>(ws, lay.seg_base) : nullptr;
  uint32_t* seg_wgs = lay.seg ? at<uint32_t>(ws, lay.seg_wgs) : nullptr;
  e.totals.seg_base = seg_base;
  e.totals.seg_wgs = seg_wgs;
  e.totals.seg_tile = lay.tcfg.tile();
  // a single frame whose rectangles travel with the depth sort: each expand
  // workgroup's pair count is counted first, so expand needs no look-back
  const bool wg_totals = pack && !lay.seg && !tile_first;
  unsigned long long* d_wg_totals = at<unsigned long long>(ws, lay.wg_totals);
  e.wg_totals = wg_totals ? d_wg_totals : nullptr;
  e.culled = ck.hist + 3 * 256 + 255;  // digit 255 of the top byte: culled only
  e.culled_stride = 4 * 256;
  SS_TRY(L.run_group(SS_KERNEL_EXPAND, wg_totals ? 2u : 1u, [&]() -> ss_status {
    if (wg_totals && launch_expand_totals(e, d_wg_totals, s) != hipSuccess) return SS_ERR_HIP;
    return launch_expand(e, s) == hipSuccess ? SS_OK : SS_ERR_HIP;
  }));
  if (P > 0) {
    uint32_t* bases_t = at<uint32_t>(ws, lay.bases_t);
    // fixed arrays: the frame path allocates nothing on the host either
    const void* ks[kMaxTilePasses];
    const uint32_t* vs[kMaxTilePasses];
    void* kd[kMaxTilePasses];
    uint32_t* vd[kMaxTilePasses];
    for (uint32_t p = 0; p < P; ++p) {
      ks[p] = bk[p % 2];
      vs[p] = bv[p % 2];
      kd[p] = bk[(p + 1) % 2];
      vd[p] = bv[(p + 1) % 2];
      if (lay.packed) {
        ks[p] = items_in[p];
        vs[p] = nullptr;
        kd[p] = p + 1 < P ? static_cast<void*>(items_in[p + 1]) : static_cast<void*>(io.keys);
        vd[p] = p + 1 < P ? nullptr : io.values;
      }
    }
    uint32_t* lb_t = at<uint32_t>(ws, lay.lb_t);
    PassChain c{P, 8, lay.packed ? pk.tile_shift : 32u, lay.trb, lay.tcfg, lay.tblocks, ks, vs,
                kd, vd, d_num_pairs, 0, d_status, bases_t, e.hist,
                (lay.seg ? lay.n_frames : 1u) * P * lay.tbins, lb_t, lay.tile_bits - lay.trb * (P - 1)};
    if (lay.packed) {
      c.packed = &pk;
      c.ranges = io.ranges;
      // after the 32-bit words of passes 0 .. P-2 (a multiple of 64 bytes)
      c.lookback64 = reinterpret_cast<uint64_t*>(lb_t + static_cast<size_t>(P - 1) * lay.tblocks * lay.tbins);
    }
    if (lay.seg) {
      c.table = table;
      c.n_frames = lay.n_frames;
      c.seg_wgs = seg_wgs;
      c.seg_base = seg_base;
      c.frame_stride = P * lay.tbins;
    }
    c.spin_limit = o.spin_limit;
    c.fault = o.fault;
    if ((o.flags & SS_FLAG_PERSISTENT) != 0 && lay.tcfg.threads == 512) c.tickets = at<uint32_t>(ws, lay.tickets);
    SS_TRY(run_chain(L, SS_KERNEL_SORT_PASS, c, s));
    if (lay.packed) {
      // the digits of the last pass: those of its (possibly narrower)
      // instantiation, whose bases are all published (when it is also the
      // first pass, it publishes only those)
      uint32_t last_rb = lay.trb;
      const uint32_t last_bits = lay.tile_bits - lay.trb * (P - 1);
      const int narrow = narrow_pass_bits(static_cast<int>(last_bits), 8, static_cast<int>(lay.trb),
                                          static_cast<int>(lay.tcfg.items), static_cast<int>(lay.tcfg.threads));
      if (last_bits < lay.trb && narrow != 0) last_rb = static_cast<uint32_t>(narrow);
      if (lay.seg)
        return L.run(SS_KERNEL_RANGES, [&] {
          return launch_ranges_fix_seg(io.keys, d_status, bases_t + static_cast<size_t>(P - 1) * lay.tbins,
                                       1u << last_rb, P * lay.tbins, seg_base, table, lay.n_frames, io.ranges, s);
        });
      SS_TRY(L.run(SS_KERNEL_RANGES, [&] {
        return launch_ranges_fix(io.keys, d_num_pairs, d_status, bases_t + static_cast<size_t>(P - 1) * lay.tbins,
                                 1u << last_rb, lay.total_tiles, io.ranges, s);
      }));
      return tile_first ? sort_tile_runs(L, lay, io, ws, d_status, s) : SS_OK;
    }
  }
  SS_TRY(L.run(SS_KERNEL_RANGES, [&] {
    return launch_ranges(io.keys, d_num_pairs, d_status, lay.capacity, lay.total_tiles, io.ranges, s);
  }));
  return tile_first ? sort_tile_runs(L, lay, io, ws, d_status, s) : SS_OK;
}

// ----------------------------- small frames --------------------------------
// At most 256 tiles and 16,384 Gaussians, one frame, without the optional
// per-Gaussian outputs: two kernels (tiny.hip).  Workspace: per-tile count
// rows of the bucketing workgroups, then their pair regions.
struct TinyLayout {
  uint32_t nblocks = 0, region_cap = 0;
  size_t rows = 0, region = 0, total = 0;
};

bool tiny_shape(uint32_t n, uint32_t num_tiles, const Options& o) {
  return (o.algorithm == SS_ALGO_AUTO || o.algorithm == SS_ALGO_DEPTH_FIRST) &&
         (o.flags & (SS_FLAG_UNSORTED | SS_FLAG_KEY32_LOSSY)) == 0 && num_tiles <= kTinyMaxTiles &&
         n <= kTinyMaxGaussians;
}

TinyLayout make_tiny_layout(uint32_t n, uint32_t num_tiles, uint32_t capacity) {
  TinyLayout L;
  L.nblocks = (n + kTinyGaussians - 1) / kTinyGaussians;
  const uint64_t most = static_cast<uint64_t>(kTinyGaussians) * num_tiles;
  L.region_cap = static_cast<uint32_t>(most < capacity ? most : capacity);
  size_t off = 0;
  L.rows = off;    off = align_up(off + static_cast<size_t>(L.nblocks) * (2 * num_tiles + 1) * sizeof(uint32_t));
  L.region = off;  off = align_up(off + static_cast<size_t>(L.nblocks) * L.region_cap * sizeof(uint64_t));
  L.total = off;
  return L;
}

ss_status run_tiny(Launcher& L, const ss_frame* frame, const Geometry& g, const ss_frame_out* out, void* ws,
                   hipStream_t s) {
  const TinyLayout lay = make_tiny_layout(frame->num_gaussians, g.num_tiles, out->pair_capacity);
  TinyArgs a{};
  a.gaussians = frame->gaussians;
  a.n = frame->num_gaussians;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  a.nblocks = lay.nblocks;
  a.region = at<uint64_t>(ws, lay.region);
  a.region_cap = lay.region_cap;
  a.rows = at<uint32_t>(ws, lay.rows);
  a.capacity = out->pair_capacity;
  a.keys = out->keys;
  a.values = out->values;
  a.ranges = out->tile_ranges;
  a.num_pairs = out->num_pairs;  // both set by the caller
  a.status = out->status;
  SS_TRY(L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_tiny(a, s, true); }));
  return L.run(SS_KERNEL_SORT_PASS, [&] { return launch_tiny(a, s, false); });
}

// Duplication in index order: the direct radix path, the bitonic network and
// the unsorted stage.
bool use_direct(const Options& o) {
  return o.algorithm == SS_ALGO_DIRECT || o.algorithm == SS_ALGO_BITONIC || (o.flags & SS_FLAG_UNSORTED) != 0;
}

FrameInfo frame_info(const ss_frame* f, const Geometry& g, uint32_t gauss_base, uint32_t tile_base) {
  FrameInfo fi{};
  fi.gauss_base = gauss_base;
  fi.n = f->num_gaussians;
  fi.tiles_x = g.tiles_x;
  fi.tiles_y = g.tiles_y;
  fi.tile_base = tile_base;
  fi.gaussians = f->gaussians;
  return fi;
}

struct BatchShape {
  std::vector<FrameInfo> table;
  uint64_t n = 0, tiles = 0;
  uint32_t max_n = 0;   // Gaussians of the largest frame
  uint64_t max_tiles = 0;  // tiles of the frame with the most
};

ss_status batch_shape(const ss_frame* frames, uint32_t n_frames, BatchShape* b) {
  if (frames == nullptr || n_frames == 0 || n_frames > kMaxFrames) return SS_ERR_INVALID_ARGUMENT;
  b->table.resize(n_frames);
  b->n = 0;
  b->tiles = 0;
  for (uint32_t f = 0; f < n_frames; ++f) {
    Geometry g;
    SS_TRY(frame_geometry(&frames[f], &g));
    b->table[f] = frame_info(&frames[f], g, static_cast<uint32_t>(b->n), static_cast<uint32_t>(b->tiles));
    b->n += frames[f].num_gaussians;
    b->tiles += g.num_tiles;
    if (frames[f].num_gaussians > b->max_n) b->max_n = frames[f].num_gaussians;
    if (g.num_tiles > b->max_tiles) b->max_tiles = g.num_tiles;
    if (b->n > 0x7FFFFFFFull || b->tiles > 0xFFFFFFFFull) return SS_ERR_INVALID_ARGUMENT;
  }
  return SS_OK;
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" {

uint32_t ss_abi_version(void) { return SS_ABI_VERSION; }

ss_status ss_render_frame(const ss_frame* frame, const ss_render_desc* desc, void* stream) {
  using namespace ss;
  Geometry g;
  SS_TRY(frame_geometry(frame, &g));
  if (desc == nullptr || desc->struct_size < sizeof(ss_render_desc)) return SS_ERR_INVALID_ARGUMENT;
  if ((desc->flags & ~SS_RENDER_EXACT) != 0) return SS_ERR_INVALID_ARGUMENT;
  if (desc->out_color == nullptr || desc->tile_ranges == nullptr) return SS_ERR_INVALID_ARGUMENT;
  if (frame->num_gaussians > 0 &&
      (desc->conic_opacity == nullptr || desc->rgb == nullptr || desc->values == nullptr))
    return SS_ERR_INVALID_ARGUMENT;
  if (!aligned(desc->conic_opacity, 16) || !aligned(desc->rgb, 16) || !aligned(desc->out_color, 4) ||
      !aligned(desc->tile_ranges, 4) || !aligned(desc->values, 4))
    return SS_ERR_INVALID_ARGUMENT;
  RenderArgs a{};
  a.gaussians = frame->gaussians;
  a.conic_opacity = desc->conic_opacity;
  a.rgb = desc->rgb;
  a.values = desc->values;
  a.ranges = desc->tile_ranges;
  a.status = desc->status;
  a.width = frame->width;
  a.height = frame->height;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  for (int c = 0; c < 3; ++c) a.bg[c] = desc->background[c];
  a.color = desc->out_color;
  a.T = desc->out_T;
  a.contrib = desc->out_contrib;
  a.tile_evals = desc->out_tile_evals;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, desc->timer);
  return L.run(SS_KERNEL_RENDER,
               [&] { return launch_render(a, (desc->flags & SS_RENDER_EXACT) != 0, s); });
}

ss_status ss_preprocess(const ss_camera* camera, const ss_preprocess_desc* desc, void* stream) {
  using namespace ss;
  if (camera == nullptr || desc == nullptr || desc->struct_size < sizeof(ss_preprocess_desc))
    return SS_ERR_INVALID_ARGUMENT;
  const ss_camera& c = *camera;
  if (c.sh_degree > 3 || !(c.tan_fovx > 0.0f) || !(c.tan_fovy > 0.0f)) return SS_ERR_INVALID_ARGUMENT;
  const float scalars[] = {c.fx, c.fy, c.cx, c.cy, c.tan_fovx, c.tan_fovy, c.near_plane,
                           c.cam_pos[0], c.cam_pos[1], c.cam_pos[2]};
  for (float v : scalars)
    if (!std::isfinite(v)) return SS_ERR_INVALID_ARGUMENT;
  for (float v : c.view)
    if (!std::isfinite(v)) return SS_ERR_INVALID_ARGUMENT;
  const uint32_t n = desc->num_gaussians;
  if (n > 0x7fffffffu) return SS_ERR_INVALID_ARGUMENT;
  if (n > 0) {
    const void* ptrs[] = {desc->mean3d_opacity, desc->cov3d, desc->sh, desc->out_records,
                          desc->out_conic_opacity, desc->out_rgb};
    for (const void* q : ptrs)
      if (q == nullptr || !aligned(q, 16)) return SS_ERR_INVALID_ARGUMENT;
  }
  PreprocessArgs a{};
  a.cam = c;
  a.n = n;
  a.mean3d_opacity = desc->mean3d_opacity;
  a.cov3d = desc->cov3d;
  a.sh = desc->sh;
  a.records = desc->out_records;
  a.conic_opacity = desc->out_conic_opacity;
  a.rgb = desc->out_rgb;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, desc->timer);
  return L.run(SS_KERNEL_PREPROCESS, [&] { return launch_preprocess(a, s); });
}

const char* ss_status_string(ss_status s) {
  switch (s) {
    case SS_OK: return "ok";
    case SS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SS_ERR_UNSUPPORTED: return "unsupported option";
    case SS_ERR_CAPACITY: return "more pairs than pair_capacity";
    case SS_ERR_OVERFLOW: return "2^32 or more pairs";
    case SS_ERR_INVALID_INPUT: return "depth not positive and finite";
    case SS_ERR_WORKSPACE: return "workspace too small or misaligned";
    case SS_ERR_HIP: return "HIP runtime error";
    case SS_ERR_BUDGET: return "request exceeds the memory budget";
    case SS_ERR_TIMEOUT: return "device wait timed out";
  }
  return "unknown status";
}

ss_status ss_frame_geometry(const ss_frame* frame, uint32_t* tiles_x, uint32_t* tiles_y,
                            uint32_t* key_bits) {
  Geometry g;
  SS_TRY(frame_geometry(frame, &g));
  if (tiles_x) *tiles_x = g.tiles_x;
  if (tiles_y) *tiles_y = g.tiles_y;
  if (key_bits) *key_bits = g.key_bits;
  return SS_OK;
}

ss_status ss_workspace_bytes(const ss_frame* frame, uint32_t pair_capacity, const ss_options* options,
                             size_t* bytes) {
  if (bytes == nullptr) return SS_ERR_INVALID_ARGUMENT;
  Geometry g;
  SS_TRY(frame_geometry(frame, &g));
  Options o;
  SS_TRY(parse_options(options, &o));
  if (pair_capacity > SS_MAX_PAIR_CAPACITY) return SS_ERR_INVALID_ARGUMENT;
  size_t sort = use_direct(o) ? make_layout(frame->num_gaussians, pair_capacity, g.key_bits, o).total
                              : make_df_layout(frame->num_gaussians, 1, pair_capacity, g.num_tiles, o,
                                               frame->num_gaussians, g.num_tiles).total;
  // small frames take the two-kernel path unless per-Gaussian outputs are
  // asked for, so both layouts must fit (the extra 8 words hold the status
  // when the caller gives none)
  if (tiny_shape(frame->num_gaussians, g.num_tiles, o)) {
    const size_t tiny = make_tiny_layout(frame->num_gaussians, g.num_tiles, pair_capacity).total + 256;
    sort = sort > tiny ? sort : tiny;
  }
  // ss_count_pairs runs in any workspace sized here (its own layout can be
  // the larger one, e.g. for N = 0)
  const size_t count = make_layout(frame->num_gaussians, 0, g.key_bits, Options{}).total;
  *bytes = sort > count ? sort : count;
  return SS_OK;
}

ss_status ss_count_pairs(const ss_frame* frame, uint32_t* d_tiles_touched, uint32_t* d_offsets,
                         uint32_t* d_num_pairs, uint32_t* d_status, void* workspace,
                         size_t workspace_bytes, void* stream) {
  Geometry g;
  SS_TRY(frame_geometry(frame, &g));
  if (d_num_pairs == nullptr || d_status == nullptr) return SS_ERR_INVALID_ARGUMENT;
  Options o;
  const Layout lay = make_layout(frame->num_gaussians, 0, g.key_bits, o);
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < lay.total)
    return SS_ERR_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, nullptr);
  SS_TRY(L.run(SS_KERNEL_CLEAR, [&] { return launch_clear(workspace, lay.clear_end, d_status, nullptr, nullptr, s); }));
  CountDupArgs a{};
  a.gaussians = frame->gaussians;
  a.n = frame->num_gaussians;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  a.tiles_touched = d_tiles_touched;
  a.offsets = d_offsets;
  a.lookback = at<uint64_t>(workspace, lay.scan_lb);
  a.hist = at<uint32_t>(workspace, lay.hist);
  a.num_pairs = d_num_pairs;
  a.status = d_status;
  a.nblocks = lay.count_blocks;
  return L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_count_dup(a, static_cast<int>(o.radix_bits), false, s); });
}

ss_status ss_sort_frame(const ss_frame* frame, const ss_frame_out* out, void* workspace,
                        size_t workspace_bytes, void* stream, const ss_options* options) {
  Geometry g;
  SS_TRY(frame_geometry(frame, &g));
  Options o;
  SS_TRY(parse_options(options, &o));
  if (out == nullptr || out->tile_ranges == nullptr) return SS_ERR_INVALID_ARGUMENT;
  if ((o.flags & SS_FLAG_KEY32_LOSSY) != 0 && g.num_tiles > kKey32MaxTiles) return SS_ERR_UNSUPPORTED;
  const uint32_t cap = out->pair_capacity;
  if (cap > SS_MAX_PAIR_CAPACITY) return SS_ERR_INVALID_ARGUMENT;
  if (cap > 0 && (out->keys == nullptr || out->values == nullptr)) return SS_ERR_INVALID_ARGUMENT;
  if (!aligned(out->keys, 8) || !aligned(out->values, 4) || !aligned(out->tile_ranges, 4))
    return SS_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  SS_TRY(ss_workspace_bytes(frame, cap, options, &need));
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < need) return SS_ERR_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, o.timer);
  if (use_direct(o)) return run_direct(L, frame, g, out, o, workspace, s);
  if (tiny_shape(frame->num_gaussians, g.num_tiles, o) && out->tiles_touched == nullptr && out->offsets == nullptr) {
    // status and pair count: the caller's words, else the workspace's last 256 bytes
    ss_frame_out o2 = *out;
    if (o2.status == nullptr) o2.status = at<uint32_t>(workspace, need - 256);
    if (o2.num_pairs == nullptr) o2.num_pairs = at<uint32_t>(workspace, need - 256) + 1;
    return run_tiny(L, frame, g, &o2, workspace, s);
  }
  const FrameInfo fi = frame_info(frame, g, 0, 0);
  const DfLayout lay = make_df_layout(frame->num_gaussians, 1, cap, g.num_tiles, o, frame->num_gaussians, g.num_tiles);
  DfIO io{&fi, frame, out->keys, out->values, out->tile_ranges, out->tiles_touched, out->offsets,
          out->num_pairs, out->status, nullptr, nullptr};
  return run_depth_first(L, lay, o, io, workspace, s);
}

ss_status ss_batch_workspace_bytes(const ss_frame* frames, uint32_t n_frames, uint32_t pair_capacity,
                                   const ss_options* options, size_t* bytes) {
  if (bytes == nullptr || pair_capacity > SS_MAX_PAIR_CAPACITY) return SS_ERR_INVALID_ARGUMENT;
  BatchShape b;
  SS_TRY(batch_shape(frames, n_frames, &b));
  Options o;
  SS_TRY(parse_options(options, &o));
  if (use_direct(o) || o.algorithm == SS_ALGO_TILE_FIRST) return SS_ERR_UNSUPPORTED;
  *bytes = make_df_layout(static_cast<uint32_t>(b.n), n_frames, pair_capacity, b.tiles, o, b.max_n, b.max_tiles).total;
  return SS_OK;
}

ss_status ss_sort_batch(const ss_frame* frames, uint32_t n_frames, const ss_batch_out* out, void* workspace,
                        size_t workspace_bytes, void* stream, const ss_options* options) {
  BatchShape b;
  SS_TRY(batch_shape(frames, n_frames, &b));
  Options o;
  SS_TRY(parse_options(options, &o));
  if (use_direct(o) || o.algorithm == SS_ALGO_TILE_FIRST) return SS_ERR_UNSUPPORTED;
  if (out == nullptr || out->tile_ranges == nullptr) return SS_ERR_INVALID_ARGUMENT;
  const uint32_t cap = out->pair_capacity;
  if (cap > SS_MAX_PAIR_CAPACITY) return SS_ERR_INVALID_ARGUMENT;
  if (cap > 0 && (out->keys == nullptr || out->values == nullptr)) return SS_ERR_INVALID_ARGUMENT;
  if (!aligned(out->keys, 8) || !aligned(out->values, 4) || !aligned(out->tile_ranges, 4))
    return SS_ERR_INVALID_ARGUMENT;
  const DfLayout lay = make_df_layout(static_cast<uint32_t>(b.n), n_frames, cap, b.tiles, o, b.max_n, b.max_tiles);
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < lay.total) return SS_ERR_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, o.timer);
  DfIO io{b.table.data(), frames, out->keys, out->values, out->tile_ranges, nullptr, nullptr,
          out->num_pairs, out->status, out->frame_pairs, out->frame_pair_base};
  return run_depth_first(L, lay, o, io, workspace, s);
}

// Batched sizing: per-frame pair counts only.
struct CountLayout {
  uint32_t ck_blocks = 0;
  size_t scalars = 0, bad = 0, totals = 0, block_total = 0, block_frame = 0, clear_end = 0,
         table = 0, total = 0;
};

static CountLayout make_count_layout(uint64_t n, uint32_t n_frames) {
  CountLayout L;
  L.ck_blocks = static_cast<uint32_t>((n + kCountKeysTile - 1) / kCountKeysTile);
  size_t off = 0;
  L.scalars = off;     off = align_up(off + 4 * sizeof(uint32_t));
  L.bad = off;         off = align_up(off + sizeof(uint32_t));
  L.totals = off;      off = align_up(off + (1 + static_cast<size_t>(n_frames)) * sizeof(uint64_t));
  L.clear_end = off;
  L.block_total = off; off = align_up(off + static_cast<size_t>(L.ck_blocks) * sizeof(uint64_t));
  L.block_frame = off; off = align_up(off + static_cast<size_t>(L.ck_blocks) * sizeof(uint32_t));
  L.table = off;       off = align_up(off + static_cast<size_t>(n_frames) * sizeof(FrameInfo));
  L.total = off;
  return L;
}

ss_status ss_batch_count_workspace_bytes(const ss_frame* frames, uint32_t n_frames, size_t* bytes) {
  if (bytes == nullptr) return SS_ERR_INVALID_ARGUMENT;
  BatchShape b;
  SS_TRY(batch_shape(frames, n_frames, &b));
  *bytes = make_count_layout(b.n, n_frames).total;
  return SS_OK;
}

ss_status ss_batch_count_pairs(const ss_frame* frames, uint32_t n_frames, uint32_t* d_frame_pairs,
                               uint32_t* d_num_pairs, uint32_t* d_status, void* workspace, size_t workspace_bytes,
                               void* stream) {
  BatchShape b;
  SS_TRY(batch_shape(frames, n_frames, &b));
  if (d_frame_pairs == nullptr || d_num_pairs == nullptr || d_status == nullptr) return SS_ERR_INVALID_ARGUMENT;
  const CountLayout lay = make_count_layout(b.n, n_frames);
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < lay.total) return SS_ERR_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, nullptr);
  FrameInfo* table = at<FrameInfo>(workspace, lay.table);
  SS_TRY(clear_and_upload(L, workspace, lay.clear_end, d_status, b.table.data(), n_frames, table, s));
  CountKeysArgs ck{};
  ck.table = table;
  ck.n_frames = n_frames;
  ck.n = static_cast<uint32_t>(b.n);
  ck.totals = at<unsigned long long>(workspace, lay.totals);
  ck.block_total = at<unsigned long long>(workspace, lay.block_total);
  ck.block_frame = at<uint32_t>(workspace, lay.block_frame);
  ck.bad = at<uint32_t>(workspace, lay.bad);
  SS_TRY(L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_count_keys(ck, s); }));
  PairTotalsArgs pt{ck.totals, ck.block_total, ck.block_frame, lay.ck_blocks, ck.bad, n_frames,
                    0xFFFFFFFFu, d_num_pairs, d_status, d_frame_pairs, nullptr};
  return L.run(SS_KERNEL_DIGIT_BASES, [&] { return launch_pair_totals(pt, s); });
}

ss_status ss_sort_pairs_workspace_bytes(uint32_t n, uint32_t key_bits, const ss_options* options,
                                        size_t* bytes) {
  if (bytes == nullptr || key_bits < 1 || key_bits > 64 || n > SS_MAX_PAIR_CAPACITY)
    return SS_ERR_INVALID_ARGUMENT;
  Options o;
  SS_TRY(parse_options(options, &o));
  *bytes = make_layout(0, n, key_bits, o).total;
  return SS_OK;
}

ss_status ss_sort_pairs(const uint64_t* keys_in, const uint32_t* values_in, uint32_t n, uint32_t key_bits,
                        uint64_t* keys_out, uint32_t* values_out, void* workspace, size_t workspace_bytes,
                        void* stream, const ss_options* options) {
  if (key_bits < 1 || key_bits > 64 || n > SS_MAX_PAIR_CAPACITY) return SS_ERR_INVALID_ARGUMENT;
  if (n > 0 && (keys_in == nullptr || values_in == nullptr || keys_out == nullptr || values_out == nullptr))
    return SS_ERR_INVALID_ARGUMENT;
  if (!aligned(keys_in, 8) || !aligned(keys_out, 8) || !aligned(values_in, 4) || !aligned(values_out, 4))
    return SS_ERR_INVALID_ARGUMENT;
  if (n > 0 && (static_cast<const void*>(keys_in) == keys_out || static_cast<const void*>(values_in) == values_out))
    return SS_ERR_INVALID_ARGUMENT;
  Options o;
  SS_TRY(parse_options(options, &o));
  if ((o.flags & SS_FLAG_KEY32_LOSSY) != 0) return SS_ERR_UNSUPPORTED;  // needs frame keys
  const Layout lay = make_layout(0, n, key_bits, o);
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < lay.total)
    return SS_ERR_WORKSPACE;
  if (n == 0) return SS_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, o.timer);
  if (o.algorithm == SS_ALGO_BITONIC) {
    // order by (key bits [0, key_bits), value): the stable order when the
    // values of equal keys increase in input order (e.g. input positions)
    const uint64_t mask = key_bits == 64 ? ~0ull : (1ull << key_bits) - 1;
    BitonicArgs b{at<uint64_t>(workspace, lay.alt_keys), at<uint32_t>(workspace, lay.alt_vals), lay.log_pad,
                  nullptr, n, nullptr, keys_out, values_out, n};
    return L.run_group(SS_KERNEL_SORT_PASS, bitonic_launches(lay.log_pad), [&] {
      return launch_bitonic(b, keys_in, values_in, mask, s) == hipSuccess ? SS_OK : SS_ERR_HIP;
    });
  }
  SS_TRY(L.run(SS_KERNEL_CLEAR, [&] { return launch_clear(workspace, lay.clear_end, nullptr, nullptr, nullptr, s); }));
  HistArgs h{keys_in, n, lay.npasses, at<uint32_t>(workspace, lay.hist)};
  SS_TRY(L.run(SS_KERNEL_HIST, [&] { return launch_hist(h, static_cast<int>(o.radix_bits), s); }));
  uint32_t* bases = at<uint32_t>(workspace, lay.bases);
  uint64_t* alt_k = at<uint64_t>(workspace, lay.alt_keys);
  uint32_t* alt_v = at<uint32_t>(workspace, lay.alt_vals);
  const uint32_t P = lay.npasses;
  std::vector<const void*> ks(P);
  std::vector<const uint32_t*> vs(P);
  std::vector<void*> kd(P);
  std::vector<uint32_t*> vd(P);
  for (uint32_t p = 0; p < P; ++p) {
    const bool to_out = ((P - 1 - p) % 2) == 0;
    kd[p] = to_out ? static_cast<void*>(keys_out) : static_cast<void*>(alt_k);
    vd[p] = to_out ? values_out : alt_v;
    ks[p] = p == 0 ? static_cast<const void*>(keys_in) : kd[p - 1];
    vs[p] = p == 0 ? values_in : vd[p - 1];
  }
  PassChain c{P, 8, 0, o.radix_bits, PassCfg{o.items, o.threads}, lay.pass_blocks, ks.data(), vs.data(),
              kd.data(), vd.data(), nullptr, n, nullptr, bases, h.hist, lay.npasses * lay.bins,
              at<uint32_t>(workspace, lay.pass_lb)};
  return run_chain(L, SS_KERNEL_SORT_PASS, c, s);
}

ss_status ss_copy_bytes(void* d_dst, const void* d_src, size_t bytes, void* stream, const ss_options* options) {
  if ((bytes % 16) != 0 || (bytes > 0 && (d_dst == nullptr || d_src == nullptr)) || !aligned(d_dst, 16) ||
      !aligned(d_src, 16))
    return SS_ERR_INVALID_ARGUMENT;
  Options o;
  SS_TRY(parse_options(options, &o));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, o.timer);
  return L.run(SS_KERNEL_COPY, [&] { return launch_copy(d_dst, d_src, bytes, s); });
}

ss_status ss_timer_create(ss_timer** timer, uint32_t max_launches) {
  if (timer == nullptr || max_launches == 0) return SS_ERR_INVALID_ARGUMENT;
  ss_timer* t = new (std::nothrow) ss_timer;
  if (t == nullptr) return SS_ERR_HIP;
  t->events.resize(2 * static_cast<size_t>(max_launches));
  t->kinds.resize(max_launches);
  t->launches.resize(max_launches);
  for (size_t i = 0; i < t->events.size(); ++i) {
    if (hipEventCreate(&t->events[i]) != hipSuccess) {
      for (size_t j = 0; j < i; ++j) (void)hipEventDestroy(t->events[j]);
      delete t;
      return SS_ERR_HIP;
    }
  }
  *timer = t;
  return SS_OK;
}

ss_status ss_timer_reset(ss_timer* timer) {
  if (timer == nullptr) return SS_ERR_INVALID_ARGUMENT;
  timer->used = 0;
  return SS_OK;
}

ss_status ss_timer_read(ss_timer* timer, uint32_t kind, double* total_ms, uint32_t* launches) {
  if (timer == nullptr || total_ms == nullptr || launches == nullptr) return SS_ERR_INVALID_ARGUMENT;
  double sum = 0.0;
  uint32_t cnt = 0;
  for (uint32_t i = 0; i < timer->used; ++i) {
    if (timer->kinds[i] != kind) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, timer->events[2 * i], timer->events[2 * i + 1]) != hipSuccess) return SS_ERR_HIP;
    sum += ms;
    cnt += timer->launches[i];
  }
  *total_ms = sum;
  *launches = cnt;
  return SS_OK;
}

void ss_timer_destroy(ss_timer* timer) {
  if (timer == nullptr) return;
  for (hipEvent_t e : timer->events) (void)hipEventDestroy(e);
  delete timer;
}

}  // extern "C"

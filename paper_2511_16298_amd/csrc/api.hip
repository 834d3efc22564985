// Host side of the C ABI declared in splatsort.h: argument validation,
// workspace layout and the launch sequence of the hot path.
#include <stdint.h>

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

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Counter words at the start of the workspace.
constexpr uint32_t kCounterTicket = 0;   // count / duplicate workgroup tickets
constexpr uint32_t kCounterPass = 16;    // + p: tickets of sort pass p (p < 48)

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

struct Options {
  uint32_t radix_bits = kDefaultRadix;
  uint32_t items = kDefaultItems;
  uint32_t threads = kDefaultThreads;
  uint32_t flags = 0;
  ss_timer* timer = nullptr;
};

ss_status parse_options(const ss_options* o, Options* out) {
  *out = Options{};
  if (o == nullptr) return SS_OK;
  if (o->struct_size < sizeof(ss_options)) return SS_ERR_INVALID_ARGUMENT;
  if ((o->flags & ~SS_FLAG_UNSORTED) != 0) return SS_ERR_UNSUPPORTED;
  out->flags = o->flags;
  if (o->radix_bits != 0) out->radix_bits = o->radix_bits;
  if (o->items_per_thread != 0) out->items = o->items_per_thread;
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
  const uint32_t tile_bits = t <= 1 ? 0u : 32u - static_cast<uint32_t>(__builtin_clz(g->num_tiles - 1));
  g->key_bits = 32 + tile_bits;
  return SS_OK;
}

// Workspace: [counters | scan look-back | histograms | pass look-back | scalars]
// is zeroed at the start of every call; the alternate pair buffers follow.
struct Layout {
  uint32_t npasses = 0, bins = 0, count_blocks = 0, pass_blocks = 0, tile = 0;
  size_t counters = 0, scan_lb = 0, hist = 0, pass_lb = 0, scalars = 0, bases = 0, clear_end = 0;
  size_t alt_keys = 0, alt_vals = 0, total = 0;
};

Layout make_layout(uint32_t n_gauss, uint32_t capacity, uint32_t key_bits, const Options& o) {
  Layout L;
  L.bins = 1u << o.radix_bits;
  L.npasses = (key_bits + o.radix_bits - 1) / o.radix_bits;
  L.count_blocks = n_gauss == 0 ? 1u : (n_gauss + kCountTile - 1) / kCountTile;
  L.tile = o.threads * o.items;
  L.pass_blocks = (capacity + L.tile - 1) / L.tile;
  size_t off = 0;
  L.counters = off;  off = align_up(off + 64 * sizeof(uint32_t));
  L.scalars = off;   off = align_up(off + 4 * sizeof(uint32_t));
  L.bases = off;     off = align_up(off + static_cast<size_t>(L.npasses) * L.bins * sizeof(uint32_t));
  L.scan_lb = off;   off = align_up(off + static_cast<size_t>(L.count_blocks) * sizeof(uint64_t));
  L.hist = off;      off = align_up(off + static_cast<size_t>(kHistCopies) * L.npasses * L.bins * sizeof(uint32_t));
  L.pass_lb = off;   off = align_up(off + static_cast<size_t>(L.npasses) * L.pass_blocks * L.bins * sizeof(uint32_t));
  L.clear_end = off;
  L.alt_keys = off;  off = align_up(off + static_cast<size_t>(capacity) * sizeof(uint64_t));
  L.alt_vals = off;  off = align_up(off + static_cast<size_t>(capacity) * sizeof(uint32_t));
  L.total = off;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
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

// Runs one launch, bracketed by timer events when a timer is attached.
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

// Sort passes p = 0 .. P-1 over key bits [p * RB, (p + 1) * RB).  Pass p
// reads src[p] and writes dst[p]; the caller arranges the buffers so the last
// pass lands in the output.
ss_status run_passes(Launcher& L, const Layout& lay, const Options& o, void* ws,
                     const uint64_t* const* ksrc, const uint32_t* const* vsrc, uint64_t* const* kdst,
                     uint32_t* const* vdst, const uint32_t* d_num_pairs, uint32_t n_fixed,
                     uint32_t* d_status, hipStream_t s) {
  uint32_t* counters = at<uint32_t>(ws, lay.counters);
  uint32_t* plb = at<uint32_t>(ws, lay.pass_lb);
  return L.run_group(SS_KERNEL_SORT_PASS, lay.npasses, [&]() -> ss_status {
  for (uint32_t p = 0; p < lay.npasses; ++p) {
    PassArgs a{};
    a.kin = ksrc[p];
    a.vin = vsrc[p];
    a.kout = kdst[p];
    a.vout = vdst[p];
    a.num_pairs = d_num_pairs;
    a.n_fixed = n_fixed;
    a.status = d_status;
    a.shift = p * o.radix_bits;
    a.bases = at<uint32_t>(ws, lay.bases) + static_cast<size_t>(p) * lay.bins;
    a.ticket = counters + kCounterPass + p;
    a.lookback = plb + static_cast<size_t>(p) * lay.pass_blocks * lay.bins;
    if (launch_pass(a, 8, static_cast<int>(o.radix_bits), static_cast<int>(o.items), static_cast<int>(o.threads),
                    lay.pass_blocks, s) != hipSuccess)
      return SS_ERR_HIP;
  }
  return SS_OK;
  });
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" {

uint32_t ss_abi_version(void) { return SS_ABI_VERSION; }

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
  *bytes = make_layout(frame->num_gaussians, pair_capacity, g.key_bits, o).total;
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
  SS_TRY(L.run(SS_KERNEL_CLEAR, [&] {
    return launch_clear(workspace, lay.clear_end, d_status, s);
  }));
  CountDupArgs a{};
  a.gaussians = frame->gaussians;
  a.n = frame->num_gaussians;
  a.tiles_x = g.tiles_x;
  a.tiles_y = g.tiles_y;
  a.capacity = 0;
  a.npasses = 0;
  a.tiles_touched = d_tiles_touched;
  a.offsets = d_offsets;
  a.ticket = at<uint32_t>(workspace, lay.counters) + kCounterTicket;
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
  const uint32_t cap = out->pair_capacity;
  if (cap > SS_MAX_PAIR_CAPACITY) return SS_ERR_INVALID_ARGUMENT;
  if (cap > 0 && (out->keys == nullptr || out->values == nullptr)) return SS_ERR_INVALID_ARGUMENT;
  if (!aligned(out->keys, 8) || !aligned(out->values, 4) || !aligned(out->tile_ranges, 4))
    return SS_ERR_INVALID_ARGUMENT;
  const Layout lay = make_layout(frame->num_gaussians, cap, g.key_bits, o);
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < lay.total)
    return SS_ERR_WORKSPACE;

  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, o.timer);
  uint32_t* scal = at<uint32_t>(workspace, lay.scalars);
  uint32_t* d_status = out->status ? out->status : scal + 0;
  uint32_t* d_num_pairs = out->num_pairs ? out->num_pairs : scal + 1;

  // dup writes buf[0]; pass p reads buf[p % 2] and writes buf[(p + 1) % 2];
  // the data ends in buf[P % 2], which must be the caller's output.
  uint64_t* alt_k = at<uint64_t>(workspace, lay.alt_keys);
  uint32_t* alt_v = at<uint32_t>(workspace, lay.alt_vals);
  const bool unsorted = (o.flags & SS_FLAG_UNSORTED) != 0;
  const uint32_t P = unsorted ? 0 : lay.npasses;
  uint64_t* bk[2];
  uint32_t* bv[2];
  bk[P % 2] = out->keys;
  bv[P % 2] = out->values;
  bk[(P + 1) % 2] = alt_k;
  bv[(P + 1) % 2] = alt_v;

  SS_TRY(L.run(SS_KERNEL_CLEAR, [&] {
    return launch_clear(workspace, lay.clear_end, d_status, s);
  }));

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
  a.ticket = at<uint32_t>(workspace, lay.counters) + kCounterTicket;
  a.lookback = at<uint64_t>(workspace, lay.scan_lb);
  a.hist = at<uint32_t>(workspace, lay.hist);
  a.num_pairs = d_num_pairs;
  a.status = d_status;
  a.nblocks = lay.count_blocks;
  SS_TRY(L.run(SS_KERNEL_COUNT_DUP, [&] { return launch_count_dup(a, static_cast<int>(o.radix_bits), true, s); }));
  if (unsorted) return SS_OK;
  SS_TRY(L.run(SS_KERNEL_DIGIT_BASES, [&] {
    return launch_digit_bases(a.hist, lay.npasses, at<uint32_t>(workspace, lay.bases),
                              static_cast<int>(o.radix_bits), s);
  }));

  std::vector<const uint64_t*> ks(lay.npasses);
  std::vector<const uint32_t*> vs(lay.npasses);
  std::vector<uint64_t*> kd(lay.npasses);
  std::vector<uint32_t*> vd(lay.npasses);
  for (uint32_t p = 0; p < lay.npasses; ++p) {
    ks[p] = bk[p % 2];
    vs[p] = bv[p % 2];
    kd[p] = bk[(p + 1) % 2];
    vd[p] = bv[(p + 1) % 2];
  }
  SS_TRY(run_passes(L, lay, o, workspace, ks.data(), vs.data(), kd.data(), vd.data(), d_num_pairs, 0,
                    d_status, s));

  return L.run(SS_KERNEL_RANGES, [&] {
    return launch_ranges(out->keys, d_num_pairs, d_status, cap, g.num_tiles, out->tile_ranges, s);
  });
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
  const Layout lay = make_layout(0, n, key_bits, o);
  if (workspace == nullptr || !aligned(workspace, kAlign) || workspace_bytes < lay.total)
    return SS_ERR_WORKSPACE;
  if (n == 0) return SS_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Launcher L(s, o.timer);
  SS_TRY(L.run(SS_KERNEL_CLEAR, [&] { return launch_clear(workspace, lay.clear_end, nullptr, s); }));
  HistArgs h{keys_in, n, lay.npasses, at<uint32_t>(workspace, lay.hist)};
  SS_TRY(L.run(SS_KERNEL_HIST, [&] { return launch_hist(h, static_cast<int>(o.radix_bits), s); }));
  SS_TRY(L.run(SS_KERNEL_HIST, [&] {
    return launch_digit_bases(h.hist, lay.npasses, at<uint32_t>(workspace, lay.bases),
                              static_cast<int>(o.radix_bits), s);
  }));
  uint64_t* alt_k = at<uint64_t>(workspace, lay.alt_keys);
  uint32_t* alt_v = at<uint32_t>(workspace, lay.alt_vals);
  const uint32_t P = lay.npasses;
  std::vector<const uint64_t*> ks(P);
  std::vector<const uint32_t*> vs(P);
  std::vector<uint64_t*> kd(P);
  std::vector<uint32_t*> vd(P);
  for (uint32_t p = 0; p < P; ++p) {
    const bool to_out = ((P - 1 - p) % 2) == 0;
    kd[p] = to_out ? keys_out : alt_k;
    vd[p] = to_out ? values_out : alt_v;
    ks[p] = p == 0 ? keys_in : kd[p - 1];
    vs[p] = p == 0 ? values_in : vd[p - 1];
  }
  return run_passes(L, lay, o, workspace, ks.data(), vs.data(), kd.data(), vd.data(), nullptr, n, nullptr, s);
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

// Depth-first form of the tile-and-depth sort, for one frame or a batch of
// frames.  The result is identical to sorting all (tile, Gaussian) pairs by
// (tile, depth, index) (paper: Background, "Duplication with Tiles" and
// "Sorting"), reached with fewer passes over the pairs:
//   1. count:  per Gaussian, its tile rectangle and pair count; its depth key
//              (culled Gaussians get 0xFFFFFFFF and sort last);
//   2. sort the N Gaussians stably by depth (four 8-bit passes over N);
//   3. expand: walk the Gaussians in depth order and write their pairs, tile
//              by tile in row-major order, with global tile ids;
//   4. sort the pairs stably by tile id alone (ceil(log2 T) bits, two 8-bit
//              passes for 8,160 tiles; none for one tile).
// After step 3 the pairs of any one tile already appear in (depth, index)
// order, because a Gaussian contributes at most one pair per tile; a stable
// sort by tile keeps that order.  A batch renumbers frame f's tiles
// tile_base[f] + t and keeps frame-local Gaussian indices as values.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

constexpr uint32_t kCountKeysThreads = 512;
constexpr uint32_t kCountKeysItems = kCountKeysTile / kCountKeysThreads;
constexpr unsigned long long kCulledOne = 1ull << 48;  // culled count, above the pair count
constexpr uint32_t kExpandThreads = 512;
constexpr uint32_t kExpandPer = kExpandTile / kExpandThreads;  // Gaussians per thread
constexpr uint32_t kChunk = 4096;                             // pairs per expansion round
constexpr uint32_t kChunkPer = kChunk / kExpandThreads;
constexpr uint64_t kSat = 1ull << 40;

__device__ __forceinline__ uint32_t clamp_tile(int64_t v, uint32_t n) {
  return v < 0 ? 0u : (v > static_cast<int64_t>(n) ? n : static_cast<uint32_t>(v));
}

// Largest f with table[f].gauss_base <= g (frames are in order).
__device__ __forceinline__ uint32_t frame_of(const FrameInfo* tab, uint32_t n_frames, uint32_t g) {
  uint32_t lo = 0, hi = n_frames;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tab[mid].gauss_base <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One 16-byte record read through a global-memory pointer (four adjacent
// words, which the compiler merges into one load).
__device__ __forceinline__ int4 load_record(const ss_gaussian2d* p) {
  typedef const int __attribute__((address_space(1))) GlobalWord;
  const GlobalWord* q = (const GlobalWord*)p;
  return make_int4(q[0], q[1], q[2], q[3]);
}

__global__ void k_put_table(TableChunk c, FrameInfo* __restrict__ table) {
  if (threadIdx.x < c.count) table[c.first + threadIdx.x] = c.f[threadIdx.x];
}

// Step 1.  2048 Gaussians per workgroup of 512 threads, loaded striped
// (coalesced 16-byte loads).  No scan here: only totals (all pairs and per
// frame) by atomics, and the four depth-digit histograms of the Gaussian sort.
__global__ __launch_bounds__(kCountKeysThreads) void k_count_keys(CountKeysArgs a) {
  __shared__ FrameInfo s_tab[kMaxFrames];
  __shared__ uint32_t s_hist[4 * 256];
  __shared__ unsigned long long s_fm[kMaxFrames];
  __shared__ unsigned long long s_tmp[kCountKeysThreads / kWave];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < a.n_frames; i += kCountKeysThreads) {
    s_tab[i] = a.table[i];
    s_fm[i] = 0;
  }
  for (uint32_t i = tid; i < 4 * 256; i += kCountKeysThreads) s_hist[i] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kCountKeysTile;
  const uint32_t last = min(base + kCountKeysTile, a.n) - 1;
  const bool one_frame = a.n_frames == 1 || frame_of(s_tab, a.n_frames, base) == frame_of(s_tab, a.n_frames, last);

  // all records first, unconditionally (slots past n reread the last
  // record) and through a global-memory pointer: the table's pointers would
  // otherwise be read as generic ones, split around the radius test, and
  // each item would wait for its own loads
  int4 rec[kCountKeysItems];
  uint32_t fr[kCountKeysItems];
#pragma unroll
  for (uint32_t j = 0; j < kCountKeysItems; ++j) {
    const uint32_t g = min(base + j * kCountKeysThreads + tid, a.n - 1);
    fr[j] = a.n_frames == 1 ? 0u : frame_of(s_tab, a.n_frames, g);
    rec[j] = load_record(s_tab[fr[j]].gaussians + (g - s_tab[fr[j]].gauss_base));
  }
  bool bad = false;
  uint64_t tsum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kCountKeysItems; ++j) {
    const uint32_t g = base + j * kCountKeysThreads + tid;
    if (g >= a.n) continue;
    const uint32_t f = fr[j];
    const FrameInfo& F = s_tab[f];
    const int4 r = rec[j];
    const uint32_t radius = static_cast<uint32_t>(r.w);
    const uint32_t dbits = static_cast<uint32_t>(r.z);
    uint32_t cnt = 0;
    uint64_t rect = 0;
    if (radius != 0) {
      const int64_t R = static_cast<int64_t>(radius) << 4;
      const int64_t X = r.x, Y = r.y;
      const uint32_t x0 = clamp_tile((X - R) >> 8, F.tiles_x);
      const uint32_t x1 = clamp_tile((X + R + 255) >> 8, F.tiles_x);
      const uint32_t y0 = clamp_tile((Y - R) >> 8, F.tiles_y);
      const uint32_t y1 = clamp_tile((Y + R + 255) >> 8, F.tiles_y);
      if (x1 > x0 && y1 > y0) {
        cnt = (x1 - x0) * (y1 - y0);
        rect = static_cast<uint64_t>(x0) | (static_cast<uint64_t>(y0) << 16) |
               (static_cast<uint64_t>(x1 - x0) << 32) | (static_cast<uint64_t>(y1 - y0) << 48);
      }
    }
    if (cnt != 0 && dbits - 1u >= 0x7F7FFFFFu) bad = true;
    const uint32_t key = cnt != 0 ? dbits : 0xFFFFFFFFu;
    if (a.key != nullptr) {  // NULL: counts only (batched sizing)
      if (a.rect32 != nullptr) {
        // at most 256 tiles per axis: x0, y0 < 256 and 1 <= w, h <= 256
        const uint32_t w = static_cast<uint32_t>(rect >> 32) & 0xFFFFu, h = static_cast<uint32_t>(rect >> 48);
        a.rect32[g] = cnt == 0 ? 0u
                               : (static_cast<uint32_t>(rect) & 0xFFu) | ((static_cast<uint32_t>(rect >> 16) & 0xFFu) << 8) |
                                     ((w - 1u) << 16) | ((h - 1u) << 24);
      } else {
        a.rect[g] = rect;
      }
      a.key[g] = key;
      a.val[g] = g;
      // culled keys (0xFFFFFFFF) all hit digit 255: counted per thread and
      // added once per workgroup below instead of contending in LDS
      if (cnt != 0) {
#pragma unroll
        for (uint32_t p = 0; p < 4; ++p) atomicAdd(&s_hist[p * 256 + ((key >> (8 * p)) & 255u)], 1u);
      } else {
        tsum += kCulledOne;
      }
      // per-frame histograms: a workgroup inside one frame flushes its LDS
      // copy below; one that spans frames (at most one per frame boundary
      // for frames of a workgroup or more) adds each Gaussian here
      if (a.frame_hist != nullptr && !one_frame) {
        uint32_t* fh = a.frame_hist + (static_cast<size_t>(blockIdx.x % kHistCopies) * a.n_frames + f) * 4 * 256;
#pragma unroll
        for (uint32_t p = 0; p < 4; ++p) atomicAdd(&fh[p * 256 + ((key >> (8 * p)) & 255u)], 1u);
      }
    }
    if (a.tiles_touched) a.tiles_touched[g] = cnt;
    if (!one_frame && cnt) atomicAdd(&s_fm[f], static_cast<unsigned long long>(cnt));
    tsum += cnt;
  }
  const bool any_bad = __syncthreads_or(bad);
  // one scan sums the pairs (below 2^43: 2,048 Gaussians of at most 2^32
  // tiles) and, from bit 48, the culled Gaussians (at most 2,048)
  unsigned long long both;
  block_exclusive_scan<unsigned long long, kCountKeysThreads>(tsum, s_tmp, both);
  const unsigned long long btotal = both & (kCulledOne - 1);
  const uint32_t culled = static_cast<uint32_t>(both >> 48);
  if (tid == 0) {
    a.block_total[blockIdx.x] = one_frame ? btotal : 0ull;
    a.block_frame[blockIdx.x] = frame_of(s_tab, a.n_frames, base);
    if (any_bad) atomicOr(a.bad, 1u);
  }
  if (!one_frame)
    for (uint32_t f = tid; f < a.n_frames; f += kCountKeysThreads)
      if (s_fm[f]) atomicAdd(&a.totals[1 + f], s_fm[f]);
  if (a.key == nullptr) return;
  if (tid == 0 && culled != 0)
    for (uint32_t p = 0; p < 4; ++p) s_hist[p * 256 + 255] += culled;
  __syncthreads();
  uint32_t* gh = a.hist + static_cast<size_t>(blockIdx.x % kHistCopies) * 4 * 256;
  uint32_t* fh = nullptr;
  if (a.frame_hist != nullptr && one_frame)
    fh = a.frame_hist + (static_cast<size_t>(blockIdx.x % kHistCopies) * a.n_frames +
                         frame_of(s_tab, a.n_frames, base)) * 4 * 256;
  for (uint32_t i = tid; i < 4 * 256; i += kCountKeysThreads) {
    const uint32_t v = s_hist[i];
    if (v) {
      atomicAdd(&gh[i], v);
      if (fh != nullptr) atomicAdd(&fh[i], v);
    }
  }
}

// Pair totals after the count kernel: per frame, the sum of the one-frame
// count workgroups' totals plus what multi-frame workgroups added directly;
// then all pairs, num_pairs, the status (bad depth, over 2^32 pairs, over
// capacity) and the per-frame pair counts and first pairs.  One workgroup of
// THREADS >= 256 threads; s_fm holds kMaxFrames values.
template <int THREADS>
__device__ __forceinline__ void finish_totals(const PairTotalsArgs& a, unsigned long long* s_fm,
                                              unsigned long long* s_tmp64, uint32_t* s_tmp) {
  const uint32_t d = threadIdx.x;
  for (uint32_t f = d; f < a.n_frames; f += THREADS) s_fm[f] = a.totals[1 + f];
  __syncthreads();
  for (uint32_t b = d; b < a.count_blocks; b += THREADS) {
    const unsigned long long t = a.block_total[b];
    if (t) atomicAdd(&s_fm[a.block_frame[b]], t);
  }
  __syncthreads();
  const unsigned long long fm = d < a.n_frames ? s_fm[d] : 0ull;
  unsigned long long m;
  block_exclusive_scan<unsigned long long, THREADS>(fm, s_tmp64, m);
  if (d == 0) {
    uint32_t st = SS_OK;
    if (*a.bad) st = SS_ERR_INVALID_INPUT;
    else if (m > 0xFFFFFFFFull) st = SS_ERR_OVERFLOW;
    else if (m > a.capacity) st = SS_ERR_CAPACITY;
    *a.num_pairs = m > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(m);
    if (*a.status == SS_OK) *a.status = st;
  }
  if (a.frame_pairs == nullptr && a.seg_base == nullptr) return;
  const uint32_t f32 = fm > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(fm);
  uint32_t all;
  const uint32_t ex = block_exclusive_scan<uint32_t, THREADS>(f32, s_tmp, all);
  if (d < a.n_frames) {
    if (a.frame_pairs) a.frame_pairs[d] = f32;
    if (a.frame_pair_base) a.frame_pair_base[d] = ex;
  }
  if (a.seg_base == nullptr) return;
  // segmented tile passes (meaningful only while the status stays SS_OK,
  // i.e. all pairs fit in 32 bits): each frame's first pair and first
  // workgroup
  const uint32_t wgs = static_cast<uint32_t>((static_cast<uint64_t>(f32) + a.seg_tile - 1) / a.seg_tile);
  uint32_t wall;
  const uint32_t wex = block_exclusive_scan<uint32_t, THREADS>(wgs, s_tmp, wall);
  if (d < a.n_frames) {
    a.seg_base[d] = ex;
    a.seg_wgs[d] = wex;
  }
  if (d == 0) {
    a.seg_base[a.n_frames] = all;
    a.seg_wgs[a.n_frames] = wall;
  }
}

// The totals alone (batched sizing: counts without the sort).
__global__ __launch_bounds__(256) void k_pair_totals(PairTotalsArgs a) {
  __shared__ unsigned long long s_fm[kMaxFrames];
  __shared__ unsigned long long s_tmp64[4];
  __shared__ uint32_t s_tmp[4];
  finish_totals<256>(a, s_fm, s_tmp64, s_tmp);
}

template <typename T, int THREADS>
__device__ __forceinline__ T block_reduce_sum(T v, T* s_tmp) {
  T total;
  block_exclusive_scan<T, THREADS>(v, s_tmp, total);
  return total;
}

// Inclusive max-scan over the workgroup (one value per thread).
template <int THREADS>
__device__ __forceinline__ uint32_t block_inclusive_max(uint32_t v, uint32_t* s_tmp) {
  constexpr int kWaves = THREADS / kWave;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  v = wave_inclusive_max(v);
  if (lane == kWave - 1) s_tmp[wave] = v;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w)
    if (static_cast<uint32_t>(w) < wave) before = max(before, s_tmp[w]);
  __syncthreads();
  return max(before, v);
}

// The pair count of each expand workgroup's Gaussians, counted as k_expand
// counts them (packed rectangles in depth order, culled ones without pairs),
// so that expand needs no look-back: all totals exist before it starts.
__global__ __launch_bounds__(kExpandThreads) void k_expand_totals(ExpandArgs a, unsigned long long* wg_totals) {
  __shared__ unsigned long long s_tmp64[kExpandThreads / kWave];
  const uint32_t tid = threadIdx.x;
  const uint32_t base = blockIdx.x * kExpandTile;
  const uint32_t n_sorted = a.n_sorted ? *a.n_sorted : a.n;
  // the culled Gaussians sort last: positions from n minus their count on
  // have no pairs (the count, digit 255 of the top depth byte, is summed by
  // the first lanes of every wave while the rectangles load)
  const uint32_t lane = tid % kWave;
  const uint32_t c = lane < kHistCopies ? a.culled[static_cast<size_t>(lane) * a.culled_stride] : 0u;
  uint32_t r[kExpandPer];
#pragma unroll
  for (uint32_t j = 0; j < kExpandPer; ++j) {
    const uint32_t pos = base + j * kExpandThreads + tid;
    r[j] = pos < n_sorted ? a.rect32[pos] : 0u;
  }
  const uint32_t live = a.n - static_cast<uint32_t>(__builtin_amdgcn_readlane(wave_inclusive_scan<uint32_t>(c), kWave - 1));
  unsigned long long v = 0;
#pragma unroll
  for (uint32_t j = 0; j < kExpandPer; ++j) {
    const uint32_t pos = base + j * kExpandThreads + tid;
    if (pos < n_sorted && pos < live) v += (((r[j] >> 16) & 0xFFu) + 1u) * (((r[j] >> 24) & 0xFFu) + 1u);
  }
  const unsigned long long total = block_reduce_sum<unsigned long long, kExpandThreads>(v, s_tmp64);
  if (tid == 0) wg_totals[blockIdx.x] = total;
}

// Step 3.  2048 Gaussians (in depth order) per workgroup of 512 threads.
// Counts come from the rectangles; a workgroup scan plus a decoupled
// look-back whose window is the whole workgroup (512 earlier workgroups per
// round trip) gives the first pair of the workgroup.  The pairs are then
// written in rounds of 4096: an owner map marks, for every Gaussian starting
// inside the round, its first slot; a max-scan spreads the owners over the
// round; thread t writes slots t, t + 512, ... (coalesced).
// LDS: about 51 KB of fixed arrays (three workgroups per CU), plus the frame
// table and the tile-digit histograms sized by the launch (launch_expand).
// Workgroup 0 finishes the pair totals in the owner map's space, before its
// first expansion round.
//
// Segmented (a.seg: the Gaussians are frame-major, so frame f holds
// positions [gauss_base[f], gauss_base[f] + n_f)): pairs carry frame-local
// tiles and the histograms are per frame.  LDS holds those of the frames of
// the workgroup's first and last Gaussian; pairs of a frame between them
// (frames smaller than a workgroup) count straight into global memory.
//
// SMALL (a.small_rects) and SEG (a.seg) are template parameters so that each
// instantiation carries only its own row division and histogram target.
template <bool SMALL, bool SEG>
__global__ __launch_bounds__(kExpandThreads) void k_expand(ExpandArgs a) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  FrameInfo* s_tab = reinterpret_cast<FrameInfo*>(s_dyn);  // [n_frames]
  // [1 or 2 frames][npasses << radix_bits]
  uint32_t* s_hist = reinterpret_cast<uint32_t*>(s_dyn + a.n_frames * sizeof(FrameInfo));
  __shared__ uint32_t s_off[kExpandTile];
  // per Gaussian, read as one 16-byte word per pair: x = global tile of
  // (x0, y0) (segmented: frame-local | frame << 16), y = w | tiles_x << 16,
  // z = depth bits, w = frame-local index; packed items instead hold in
  // (z, w) the low and high words of their bits below the tile field
  // (depth field << idx_bits | index)
  __shared__ uint4 s_info[kExpandTile];
  __shared__ __align__(16) uint16_t s_map[kChunk];
  __shared__ uint32_t s_incl[kExpandThreads];
  __shared__ unsigned long long s_tmp64[kExpandThreads / kWave];
  __shared__ uint32_t s_tmp[kExpandThreads / kWave];
  __shared__ uint32_t s_first, s_retry, s_timeout;
  __shared__ unsigned long long s_prefix;
  static_assert(kChunk * sizeof(uint16_t) >= kMaxFrames * sizeof(unsigned long long), "totals in the map");
  unsigned long long* s_fm = reinterpret_cast<unsigned long long*>(s_map);

  // No status test on entry: workgroup 0 sets the status from the totals
  // while the others run, and every workgroup must publish its look-back
  // word.  Writes stay below capacity whatever the status becomes.
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_timeout = 0;
  for (uint32_t i = tid; i < a.n_frames; i += kExpandThreads) s_tab[i] = a.table[i];
  const uint32_t rb = a.radix_bits;
  const uint32_t bins = 1u << rb;
  const uint32_t hframe = a.npasses * bins;  // one frame's histograms
  const uint32_t hwords = SEG ? 2 * hframe : hframe;
  for (uint32_t i = tid; i < hwords; i += kExpandThreads) s_hist[i] = 0;
  __syncthreads();
  const uint32_t ticket = blockIdx.x;   // look-back order (see common.hpp)
  const uint32_t base = ticket * kExpandTile;
  // segmented: the frames whose histograms live in LDS
  uint32_t f_lo = 0, f_hi = 0;
  if (SEG && a.n != 0) {
    f_lo = frame_of(s_tab, a.n_frames, min(base, a.n - 1));
    f_hi = frame_of(s_tab, a.n_frames, min(base + kExpandTile, a.n) - 1);
  }
  const uint32_t n_sorted = a.n_sorted ? *a.n_sorted : a.n;  // Gaussians the depth sort kept
  uint32_t top_max = 0, top_min = 0;
  if (a.packed) {
    if (a.top_hist != nullptr) {
      // the top-byte range of the live depth keys, from the histogram
      // (bins below 128: positive depths; bin 255 holds the culled)
      if (tid == 0) {
        s_first = 0;      // max, reusing the look-back's words before the look-back
        s_retry = 0xFFu;  // min
      }
      __syncthreads();
      if (tid < 128) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t k = 0; k < kHistCopies; ++k) c += a.top_hist[static_cast<size_t>(k) * a.top_hist_stride + tid];
        if (c != 0) {
          atomicMax(&s_first, tid);
          atomicMin(&s_retry, tid);
        }
      }
      __syncthreads();
      top_max = s_first;
      top_min = s_retry <= s_first ? s_retry : 0u;
      __syncthreads();
      if (blockIdx.x == 0 && tid == 0 && a.depth_top_out != nullptr) {
        a.depth_top_out[0] = top_max;
        a.depth_top_out[1] = top_min;
      }
    } else {
      top_max = a.pk.depth_top[0];
      top_min = a.pk.depth_top[1];
    }
  }
  uint32_t ebase = 0;
  const bool trimmed = a.packed && packed_depth_trimmed(top_max, top_min, a.pk, &ebase);

  // ---- Gaussians of this workgroup: striped loads, per-Gaussian info ----
#pragma unroll
  for (uint32_t j = 0; j < kExpandPer; ++j) {
    const uint32_t i = j * kExpandThreads + tid;
    const uint32_t pos = base + i;
    uint32_t cnt = 0;
    const uint32_t g = pos < n_sorted ? a.val[pos] : 0xFFFFFFFFu;
    if (g < a.n) {  // a sorted index is always < n; the test only keeps reads in bounds
      const uint32_t f = a.n_frames == 1 ? 0u : frame_of(s_tab, a.n_frames, g);
      const uint32_t dep = a.key[pos];
      uint32_t w, h, x0, y0;
      if (a.rect32 != nullptr || a.rect32_idx != nullptr) {
        // packed, in depth order: read in sequence instead of gathered by
        // index; else gathered, 4 B instead of 8
        const uint32_t r = a.rect32 != nullptr ? a.rect32[pos] : a.rect32_idx[g];
        const bool live = dep != 0xFFFFFFFFu;
        x0 = r & 0xFFu;
        y0 = (r >> 8) & 0xFFu;
        w = live ? ((r >> 16) & 0xFFu) + 1u : 0u;
        h = ((r >> 24) & 0xFFu) + 1u;
      } else {
        const uint64_t r = a.rect[g];
        w = static_cast<uint32_t>(r >> 32) & 0xFFFFu;
        h = static_cast<uint32_t>(r >> 48);
        x0 = static_cast<uint32_t>(r) & 0xFFFFu;
        y0 = static_cast<uint32_t>(r >> 16) & 0xFFFFu;
      }
      const uint32_t tx = s_tab[f].tiles_x;
      cnt = w * h;
      // packed items carry the depth field: trimmed depth bits, or the
      // position in depth order (the unpacking pass looks the bits up)
      const uint32_t local = g - s_tab[f].gauss_base;
      uint64_t low = (static_cast<uint64_t>(trimmed ? dep - ebase : pos) << a.pk.idx_bits) | local;
      if (!a.packed) low = (static_cast<uint64_t>(local) << 32) | dep;
      s_info[i] = make_uint4(SEG ? (y0 * tx + x0) | (f << 16) : s_tab[f].tile_base + y0 * tx + x0,
                             w | (tx << 16), static_cast<uint32_t>(low), static_cast<uint32_t>(low >> 32));
    }
    s_off[i] = cnt;
  }
  __syncthreads();
  // ---- workgroup scan (blocked: thread t owns 4t .. 4t+3) ----
  uint32_t c[kExpandPer];
  unsigned long long tsum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kExpandPer; ++k) {
    c[k] = s_off[kExpandPer * tid + k];
    tsum += c[k];
  }
  unsigned long long btotal;
  const unsigned long long texcl = block_exclusive_scan<unsigned long long, kExpandThreads>(tsum, s_tmp64, btotal);
  {
    unsigned long long run = texcl;
#pragma unroll
    for (uint32_t k = 0; k < kExpandPer; ++k) {
      s_off[kExpandPer * tid + k] = run > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(run);
      run += c[k];
    }
  }

  // ---- pairs of earlier workgroups: their totals, or a decoupled look-back
  // whose window is the whole workgroup ----
  const unsigned long long mine = btotal > kSat ? kSat : btotal;
  unsigned long long excl = 0;
  if (a.wg_totals != nullptr) {
    unsigned long long v = 0;
    for (uint32_t k = tid; k < ticket; k += kExpandThreads) v += a.wg_totals[k];
    excl = block_reduce_sum<unsigned long long, kExpandThreads>(v, s_tmp64);
    if (excl > kSat) excl = kSat;
  } else if (ticket == 0) {
    if (tid == 0) st_agent(&a.lookback[0], kLbInc64 | mine);
  } else {
    if (tid == 0) st_agent(&a.lookback[ticket], kLbAgg64 | mine);
    int64_t top = static_cast<int64_t>(ticket) - 1;
    uint32_t spins = 0;
    while (true) {
      const int64_t idx = top - static_cast<int64_t>(tid);
      const uint64_t w = idx >= 0 ? ld_agent(&a.lookback[idx]) : kLbInc64;
      const uint32_t state = static_cast<uint32_t>(w >> 62);
      if (tid == 0) {
        s_first = 0xFFFFFFFFu;
        s_retry = 0;
      }
      __syncthreads();
      if (state == 2) atomicMin(&s_first, tid);
      __syncthreads();
      const uint32_t first = s_first;
      if (state == 0 && tid < first) s_retry = 1;
      __syncthreads();
      if (s_retry) {
        if (++spins > spin_limit_of(a.spin_limit)) {
          if (tid == 0) s_timeout = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        __syncthreads();
        continue;
      }
      const unsigned long long v = tid <= first ? (w & kLbMask64) : 0ull;
      const unsigned long long sum = block_reduce_sum<unsigned long long, kExpandThreads>(v, s_tmp64);
      excl += sum;
      if (excl > kSat) excl = kSat;
      if (first != 0xFFFFFFFFu) break;
      top -= kExpandThreads;
    }
    if (tid == 0) {
      const unsigned long long inc = excl + btotal;
      st_agent(&a.lookback[ticket], kLbInc64 | (inc > kSat ? kSat : inc));
    }
  }
  if (tid == 0) s_prefix = excl;
  __syncthreads();
  if (ticket == 0) finish_totals<kExpandThreads>(a.totals, s_fm, s_tmp64, s_tmp);
  if (s_timeout) {
    if (tid == 0) st_agent(const_cast<uint32_t*>(a.status), static_cast<uint32_t>(SS_ERR_TIMEOUT));
    return;
  }
  const unsigned long long prefix = s_prefix;
  uint32_t total = 0;
  if (prefix < a.capacity) {
    const unsigned long long room = a.capacity - prefix;
    total = static_cast<uint32_t>(btotal < room ? btotal : room);
  }
  uint64_t* __restrict__ keys = a.keys + prefix;
  uint32_t* __restrict__ vals = a.values + prefix;

  // ---- expansion in rounds of kChunk pairs ----
  for (uint32_t cb = 0; cb < total; cb += kChunk) {
#pragma unroll
    for (uint32_t k = 0; k < kChunkPer; ++k) s_map[k * kExpandThreads + tid] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kExpandPer; ++k) {
      const uint32_t i = kExpandPer * tid + k;
      const uint32_t o = s_off[i];
      if (c[k] != 0 && o < cb + kChunk && o + c[k] > cb)
        s_map[(o > cb ? o : cb) - cb] = static_cast<uint16_t>(i + 1);
    }
    __syncthreads();
    // inclusive max-scan of the markers: per thread over its 8 slots, then
    // across threads; slots before a thread's first marker take the maximum
    // of all earlier threads
    uint32_t m[kChunkPer];
    uint32_t run = 0;
#pragma unroll
    for (uint32_t k = 0; k < kChunkPer; ++k) {
      run = max(run, static_cast<uint32_t>(s_map[kChunkPer * tid + k]));
      m[k] = run;
    }
    s_incl[tid] = block_inclusive_max<kExpandThreads>(run, s_tmp);
    __syncthreads();
    const uint32_t prev = tid == 0 ? 0u : s_incl[tid - 1];
#pragma unroll
    for (uint32_t k = 0; k < kChunkPer; ++k) s_map[kChunkPer * tid + k] = static_cast<uint16_t>(max(m[k], prev));
    __syncthreads();
    // one loop per (packed items, two tile passes), so that neither test is
    // taken per pair
    auto write_round = [&](auto packed_tag, auto two_tag) {
      constexpr bool kPacked = decltype(packed_tag)::value, kTwo = decltype(two_tag)::value;
#pragma unroll
      for (uint32_t k = 0; k < kChunkPer; ++k) {
        const uint32_t q = cb + k * kExpandThreads + tid;
        if (q < total) {
          const uint32_t i = static_cast<uint32_t>(s_map[q - cb]) - 1u;
          if (i >= kExpandTile) continue;  // every slot has an owner; kept for safety
          const uint32_t kk = q - s_off[i];
          const uint4 gi = s_info[i];
          const uint32_t org = gi.x, wt = gi.y;
          const uint32_t w = wt & 0xFFFFu;
          // row of pair kk in the w-wide rectangle.  Rectangles of at most
          // 256 x 256 tiles (kk < 2^16): floor((kk + 1/2) / w) in fp32 is exact,
          // its true value lying at least 1/512 from an integer while the
          // rounding errors stay below 256 * 2^-21.
          const uint32_t dy = SMALL ? static_cast<uint32_t>((static_cast<float>(kk) + 0.5f) *
                                                                    __builtin_amdgcn_rcpf(static_cast<float>(w)))
                                            : kk / w;
          // every factor is below 2^24 (w, dy, tiles_x < 2^16): 24-bit products
          const uint32_t dx = kk - __umul24(dy, w);
          const uint32_t tile = (SEG ? org & 0xFFFFu : org) + __umul24(dy, wt >> 16) + dx;
          if (kPacked) {
            // the tile field lies in the high word (tile_shift >= 32)
            keys[q] = (static_cast<uint64_t>((tile << (a.pk.tile_shift - 32)) | gi.w) << 32) | gi.z;
          } else {
            keys[q] = (static_cast<uint64_t>(tile) << 32) | gi.z;
            vals[q] = gi.w;
          }
          uint32_t* h = s_hist;
          if (SEG) {
            const uint32_t f = org >> 16;
            h = f == f_lo ? s_hist
                : f == f_hi ? s_hist + hframe
                            : a.hist + (static_cast<size_t>(ticket % kHistCopies) * a.n_frames + f) * hframe;
          }
          if (kTwo) {  // the usual count (up to 16 tile bits), without loop control
            atomicAdd(&h[tile & (bins - 1)], 1u);
            atomicAdd(&h[bins + ((tile >> rb) & (bins - 1))], 1u);
          } else {
            for (uint32_t p = 0; p < a.npasses; ++p) atomicAdd(&h[p * bins + ((tile >> (rb * p)) & (bins - 1))], 1u);
          }
        }
      }
    };
    if (a.packed) {
      if (a.npasses == 2) write_round(std::true_type{}, std::true_type{});
      else write_round(std::true_type{}, std::false_type{});
    } else {
      if (a.npasses == 2) write_round(std::false_type{}, std::true_type{});
      else write_round(std::false_type{}, std::false_type{});
    }
    __syncthreads();
  }
  // histogram copy ticket % kHistCopies: [npasses][bins], or, segmented,
  // [frame][npasses][bins]
  const size_t copy = static_cast<size_t>(ticket % kHistCopies) * (SEG ? a.n_frames : 1u) * hframe;
  for (uint32_t i = tid; i < hwords; i += kExpandThreads) {
    const uint32_t v = s_hist[i];
    const uint32_t f = i < hframe ? f_lo : f_hi;
    if (v) atomicAdd(&a.hist[copy + (SEG ? static_cast<size_t>(f) * hframe : 0u) + i % hframe], v);
  }
}

}  // namespace

hipError_t launch_put_table(const TableChunk& c, FrameInfo* table, hipStream_t s) {
  hipLaunchKernelGGL(k_put_table, dim3(1), dim3(kArgFrames), 0, s, c, table);
  return hipGetLastError();
}

hipError_t launch_count_keys(const CountKeysArgs& a, hipStream_t s) {
  const uint32_t blocks = (a.n + kCountKeysTile - 1) / kCountKeysTile;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_keys, dim3(blocks), dim3(kCountKeysThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pair_totals(const PairTotalsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_totals, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_expand_totals(const ExpandArgs& a, unsigned long long* wg_totals, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_totals, dim3(a.nblocks), dim3(kExpandThreads), 0, s, a, wg_totals);
  return hipGetLastError();
}

hipError_t launch_expand(const ExpandArgs& a, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  const size_t dyn = a.n_frames * sizeof(FrameInfo) + (static_cast<size_t>(a.npasses) << a.radix_bits) * 4 *
                                                         (a.seg ? 2u : 1u);
  if (a.small_rects) {
    if (a.seg) hipLaunchKernelGGL((k_expand<true, true>), dim3(a.nblocks), dim3(kExpandThreads), dyn, s, a);
    else hipLaunchKernelGGL((k_expand<true, false>), dim3(a.nblocks), dim3(kExpandThreads), dyn, s, a);
  } else {
    if (a.seg) hipLaunchKernelGGL((k_expand<false, true>), dim3(a.nblocks), dim3(kExpandThreads), dyn, s, a);
    else hipLaunchKernelGGL((k_expand<false, false>), dim3(a.nblocks), dim3(kExpandThreads), dyn, s, a);
  }
  return hipGetLastError();
}

}  // namespace ss

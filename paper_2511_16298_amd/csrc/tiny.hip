// Small frames (at most 256 tiles and 16,384 Gaussians) in two kernels, for
// latency: the same result as the other paths -- all (tile, Gaussian) pairs
// ordered by (tile, depth, index) and the tile ranges (paper: Background,
// "Duplication with Tiles" and "Sorting") -- reached by bucketing instead of
// global radix passes:
//   1. k_tiny_bucket, one workgroup per 512 consecutive Gaussians: tile
//      rectangles, the workgroup's pairs written to its own region grouped
//      by tile, and its per-tile counts;
//   2. k_tiny_tiles, one workgroup per tile: the tile's runs gathered from
//      every region, sorted by (depth, index) inside LDS, written at the
//      tile's start; the range, the pair count and the status.
// A frame's launches of global passes each cost more than the work they do
// on a frame this small; here each kernel is one round of loads, LDS work
// and stores.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

constexpr uint32_t kTinyThreads = kTinyGaussians;   // one Gaussian per thread
constexpr uint32_t kTinyWaves = kTinyThreads / kWave;
constexpr uint32_t kSortThreads = 1024;
constexpr uint32_t kSortItems = kTinyMaxGaussians / kSortThreads;   // 16
constexpr uint32_t kSortWaves = kSortThreads / kWave;

__device__ __forceinline__ uint32_t tclamp(int64_t v, uint32_t n) {
  return v < 0 ? 0u : (v > static_cast<int64_t>(n) ? n : static_cast<uint32_t>(v));
}

// ---------------------------------------------------------------------------
// Kernel 1.  One Gaussian per thread: its rectangle, then its pairs counted
// per tile (LDS atomics), the workgroup's per-tile prefix, and each pair
// written to region[lstart[tile] + the next slot of that tile] (LDS atomics
// again: the order inside a tile's run is not fixed, kernel 2 sorts by depth
// and index).  Item: depth bits << 32 | Gaussian index.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTinyThreads) void k_tiny_bucket(TinyArgs a) {
  __shared__ uint32_t s_cnt[kTinyMaxTiles];      // per-tile pairs of this workgroup
  __shared__ uint32_t s_cursor[kTinyMaxTiles];   // next free slot of each tile's run
  __shared__ uint32_t s_tmp[kTinyWaves];

  const uint32_t tid = threadIdx.x;
  const uint32_t T = a.tiles_x * a.tiles_y;
  for (uint32_t i = tid; i < kTinyMaxTiles; i += kTinyThreads) s_cnt[i] = 0;
  __syncthreads();
  const uint32_t g = blockIdx.x * kTinyGaussians + tid;
  uint32_t x0 = 0, y0 = 0, w = 0, h = 0, dbits = 0;
  bool bad = false;
  if (g < a.n) {
    const int4 r = reinterpret_cast<const int4*>(a.gaussians)[g];
    const uint32_t radius = static_cast<uint32_t>(r.w);
    dbits = static_cast<uint32_t>(r.z);
    if (radius != 0) {
      const int64_t R = static_cast<int64_t>(radius) << 4;
      x0 = tclamp((static_cast<int64_t>(r.x) - R) >> 8, a.tiles_x);
      const uint32_t x1 = tclamp((static_cast<int64_t>(r.x) + R + 255) >> 8, a.tiles_x);
      y0 = tclamp((static_cast<int64_t>(r.y) - R) >> 8, a.tiles_y);
      const uint32_t y1 = tclamp((static_cast<int64_t>(r.y) + R + 255) >> 8, a.tiles_y);
      if (x1 > x0 && y1 > y0) {
        w = x1 - x0;
        h = y1 - y0;
      }
    }
    if (w != 0 && dbits - 1u >= 0x7F7FFFFFu) bad = true;
    for (uint32_t yy = 0; yy < h; ++yy)
      for (uint32_t xx = 0; xx < w; ++xx) atomicAdd(&s_cnt[(y0 + yy) * a.tiles_x + x0 + xx], 1u);
  }
  const bool any_bad = __syncthreads_or(bad);
  // for kernel 2: per-tile counts, their exclusive prefix (where each tile's
  // run starts in the region) and the bad flag
  uint32_t* row = a.rows + static_cast<size_t>(blockIdx.x) * (2 * T + 1);
  const uint32_t tc = tid < T ? s_cnt[tid] : 0u;
  uint32_t all;
  const uint32_t ls = block_exclusive_scan<uint32_t, kTinyThreads>(tc, s_tmp, all);
  if (tid < kTinyMaxTiles) s_cursor[tid] = ls;
  if (tid < T) {
    row[tid] = tc;
    row[T + tid] = ls;
  }
  if (tid == 0) row[2 * T] = any_bad ? 1u : 0u;
  __syncthreads();
  uint64_t* region = a.region + static_cast<size_t>(blockIdx.x) * a.region_cap;
  const uint64_t item = (static_cast<uint64_t>(dbits) << 32) | g;
  for (uint32_t yy = 0; yy < h; ++yy) {
    for (uint32_t xx = 0; xx < w; ++xx) {
      const uint32_t at = atomicAdd(&s_cursor[(y0 + yy) * a.tiles_x + x0 + xx], 1u);
      // a region holds the frame's pair capacity: more pairs than that is a
      // capacity error that kernel 2 reports, and nothing lands past the end
      if (at < a.region_cap) region[at] = item;
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel 2.  Workgroup t: the tile's start is the sum of every workgroup's
// counts of lower tiles; its runs are gathered and ordered by (depth, index):
// by counting when they fit one item per thread, else by 8-bit LSD passes
// (index bits, then depth bits) with wave-ballot ranking in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortThreads) void k_tiny_tiles(TinyArgs a) {
  __shared__ __align__(16) uint64_t s_buf[kTinyMaxGaussians + 2];
  __shared__ uint32_t s_wcnt[kSortWaves * 256];   // LSD passes: per-wave digit counts
  __shared__ uint32_t s_dstart[256];
  __shared__ uint32_t s_roff[kTinyMaxBlocks];      // this tile's run in each region
  __shared__ uint32_t s_run[kTinyMaxBlocks + 1];   // where each region's run lands in s_buf
  __shared__ unsigned long long s_tmp64[kSortWaves];
  __shared__ uint32_t s_tmp[kSortWaves];
  __shared__ uint32_t s_start, s_n, s_m, s_bad;

  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const uint32_t T = a.tiles_x * a.tiles_y;
  const uint32_t t = blockIdx.x;
  const uint32_t nb = a.nblocks;
  const uint32_t stride = 2 * T + 1;
  // tile totals over the workgroups (independent loads), their prefix (this
  // tile's start), all pairs, any bad depth; this tile's run in each region
  uint32_t tot = 0, badf = 0, rlen = 0, roff = 0;
  if (tid < T) {
    uint32_t v[kTinyMaxBlocks];   // every load issued before the first use
#pragma unroll
    for (uint32_t b = 0; b < kTinyMaxBlocks; ++b) v[b] = b < nb ? a.rows[b * stride + tid] : 0u;
#pragma unroll
    for (uint32_t b = 0; b < kTinyMaxBlocks; ++b) tot += v[b];
  }
  if (tid < nb) {
    badf = a.rows[tid * stride + 2 * T];
    rlen = a.rows[tid * stride + t];
    roff = a.rows[tid * stride + T + t];
  }
  // one scan for three prefixes: tile totals (bits 0-23: at most 2^22 pairs),
  // this tile's run lengths by region (bits 24-43) and bad flags (from 44)
  unsigned long long all;
  const unsigned long long ex = block_exclusive_scan<unsigned long long, kSortThreads>(
      (static_cast<unsigned long long>(badf) << 44) | (static_cast<unsigned long long>(rlen) << 24) | tot, s_tmp64,
      all);
  if (tid == t) {
    s_start = static_cast<uint32_t>(ex & 0xFFFFFFull);
    s_n = tot;
  }
  if (tid == 0) {
    s_m = static_cast<uint32_t>(all & 0xFFFFFFull);
    s_bad = static_cast<uint32_t>(all >> 44);
  }
  // where each region's run lands in s_buf
  if (tid < nb) {
    s_roff[tid] = roff;
    s_run[tid] = static_cast<uint32_t>((ex >> 24) & 0xFFFFFull);
  }
  if (tid == 0) s_run[nb] = static_cast<uint32_t>((all >> 24) & 0xFFFFFull);
  __syncthreads();
  const uint32_t m = s_m, start = s_start, n = s_n;
  uint32_t st = SS_OK;
  if (s_bad) st = SS_ERR_INVALID_INPUT;
  else if (m > a.capacity) st = SS_ERR_CAPACITY;
  if (t == 0 && tid == 0) {
    *a.num_pairs = m;
    *a.status = st;
  }
  if (st != SS_OK) return;
  if (tid == 0) {
    a.ranges[2 * t] = start;
    a.ranges[2 * t + 1] = start + n;
  }
  if (n == 0) return;
  // gather the runs (each contiguous in its region) into s_buf in region
  // order: item q of the tile comes from the region b whose run holds it
  for (uint32_t q = tid; q < n; q += kSortThreads) {
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_run[mid] <= q) lo = mid;
      else hi = mid;
    }
    s_buf[q] = a.region[static_cast<size_t>(lo) * a.region_cap + s_roff[lo] + (q - s_run[lo])];
  }
  __syncthreads();
  uint64_t* keys = a.keys + start;
  uint32_t* vals = a.values + start;
  const uint64_t tile_hi = static_cast<uint64_t>(t) << 32;

  if (n <= kSortThreads) {
    // rank by counting: items (depth bits << 32 | index) are distinct, so an
    // item's place is the number of smaller ones; the run is padded to an
    // even count with all-ones items (above every valid one), read two at a time
    const uint32_t n2 = (n + 1) & ~1u;
    if (n2 > n && tid == 0) s_buf[n] = ~0ull;
    __syncthreads();
    if (tid < n) {
      const uint64_t me = s_buf[tid];
      uint32_t r = 0;
#pragma unroll 4
      for (uint32_t j = 0; j < n2; j += 2) {
        const ulonglong2 q = *reinterpret_cast<const ulonglong2*>(s_buf + j);
        r += (q.x < me) + (q.y < me);
      }
      keys[r] = tile_hi | static_cast<uint32_t>(me >> 32);
      vals[r] = static_cast<uint32_t>(me);
    }
    return;
  }

  // stable 8-bit LSD passes over the index (bits 0-13: fewer than 2^14
  // Gaussians) and then the depth bits (32-63), items wave-striped in
  // registers (wave w holds [w * 64 * 16, (w + 1) * 64 * 16))
  uint64_t it[kSortItems];
#pragma unroll
  for (uint32_t j = 0; j < kSortItems; ++j) {
    const uint32_t q = wave * (kWave * kSortItems) + j * kWave + lane;
    it[j] = q < n ? s_buf[q] : 0ull;
  }
  constexpr uint32_t kShifts[6] = {0, 8, 32, 40, 48, 56};
  for (uint32_t sp = 0; sp < 6; ++sp) {
    const uint32_t shift = kShifts[sp];
    for (uint32_t i = tid; i < kSortWaves * 256; i += kSortThreads) s_wcnt[i] = 0;
    __syncthreads();
    uint32_t* wc = s_wcnt + wave * 256;
    uint32_t dg[kSortItems], pos[kSortItems];
#pragma unroll
    for (uint32_t j = 0; j < kSortItems; ++j) {
      const uint32_t q = wave * (kWave * kSortItems) + j * kWave + lane;
      const bool valid = q < n;
      dg[j] = valid ? static_cast<uint32_t>(it[j] >> shift) & 255u : 256u;
      const uint64_t peers = match_digit<8>(dg[j], ballot(valid));
      uint32_t r = 0;
      if (valid) {
        const uint32_t old = wc[dg[j]];
        const uint32_t below = popc_below(peers);
        r = old + below;
        __builtin_amdgcn_wave_barrier();
        if (below == 0) wc[dg[j]] = old + static_cast<uint32_t>(__popcll(peers));
      }
      __builtin_amdgcn_wave_barrier();
      pos[j] = r;
    }
    __syncthreads();
    uint32_t dcnt = 0;
    if (tid < 256) {
      for (uint32_t w = 0; w < kSortWaves; ++w) {
        const uint32_t x = s_wcnt[w * 256 + tid];
        s_wcnt[w * 256 + tid] = dcnt;
        dcnt += x;
      }
    }
    uint32_t dall;
    const uint32_t dex = block_exclusive_scan<uint32_t, kSortThreads>(dcnt, s_tmp, dall);
    if (tid < 256) s_dstart[tid] = dex;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kSortItems; ++j)
      if (dg[j] < 256) s_buf[s_dstart[dg[j]] + wc[dg[j]] + pos[j]] = it[j];
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kSortItems; ++j) {
      const uint32_t q = wave * (kWave * kSortItems) + j * kWave + lane;
      it[j] = q < n ? s_buf[q] : 0ull;
    }
    __syncthreads();
  }
#pragma unroll
  for (uint32_t j = 0; j < kSortItems; ++j) {
    const uint32_t q = wave * (kWave * kSortItems) + j * kWave + lane;
    if (q < n) {
      keys[q] = tile_hi | static_cast<uint32_t>(it[j] >> 32);
      vals[q] = static_cast<uint32_t>(it[j]);
    }
  }
}

}  // namespace

hipError_t launch_tiny(const TinyArgs& a, hipStream_t s, bool bucket) {
  if (bucket) {
    if (a.nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tiny_bucket, dim3(a.nblocks), dim3(kTinyThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_tiny_tiles, dim3(a.tiles_x * a.tiles_y), dim3(kSortThreads), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace ss

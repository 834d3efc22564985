// Frame kernels of the tile-and-depth sort: scratch clear, the fused
// count / scan / duplicate step (paper: Background, "Duplication with Tiles";
// evaluation table columns "Scan" and "Duplicate with tiles"), the digit
// histogram of caller keys, tile-range identification (Design, "Sorting
// Optimizations in Context of 3DGS": only the tile part of the key is used)
// and a streaming copy used to calibrate traffic counters.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

constexpr int kCountThreads = 256;
constexpr int kCountItems = kCountTile / kCountThreads;  // Gaussians per thread
static_assert(kCountTile == 1024, "the duplicate search below walks 10 bits");

// Saturation point of look-back counts: any total at or above it is already
// far beyond the 2^32 - 1 pair limit, and 64 saturated values still sum
// without wrapping.
constexpr uint64_t kCountSat = 1ull << 40;

__device__ __forceinline__ uint32_t clamp_tile(int64_t v, uint32_t n) {
  return v < 0 ? 0u : (v > static_cast<int64_t>(n) ? n : static_cast<uint32_t>(v));
}

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
  const uint64_t s = a + b;
  return s > kCountSat ? kCountSat : s;
}

__global__ void k_clear(uint4* __restrict__ p, size_t n16, uint32_t* __restrict__ extra, TableChunk c,
                        FrameInfo* __restrict__ table) {
  if (extra != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *extra = 0;
  if (blockIdx.x == 0 && threadIdx.x < c.count) table[c.first + threadIdx.x] = c.f[threadIdx.x];
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n16) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

// Workgroup b takes the 1024 consecutive Gaussians of tile b (look-back order
// as described in common.hpp).
//  count: overlap rectangle of each Gaussian's open bounding box with the tile
//      grid, in 1/16-px integers: x0 = floor((X - 16 r) / 256),
//      x1 = ceil((X + 16 r) / 256), clamped to [0, tiles_x]; radius 0 culls.
//  scan: workgroup scan of the counts, then a decoupled look-back over earlier
//      workgroups' aggregates gives the global exclusive offset.
//  duplicate: the workgroup's pairs are spread evenly over its threads: thread t
//      writes local pairs t, t + 256, ...; each finds its Gaussian by a
//      10-step search of the local offsets in LDS, so a Gaussian covering a
//      thousand tiles costs no more than a thousand small ones.  Keys are
//      (ty * tiles_x + tx) << 32 | depth bits; tiles of one Gaussian in
//      row-major order.  The digit histograms of every sort pass are
//      gathered on the way (depth digits once per Gaussian weighted by its
//      count, tile digits per pair).
template <int RB, bool DUP>
__global__ __launch_bounds__(kCountThreads) void k_count_dup(CountDupArgs a) {
  constexpr int BINS = 1 << RB;
  constexpr int MAXP = (64 + RB - 1) / RB;
  __shared__ uint4 s_rect[kCountTile];   // x0, y0, width, depth bits
  __shared__ uint32_t s_loc[kCountTile]; // counts, then local exclusive offsets
  __shared__ uint32_t s_hist[DUP ? MAXP * BINS : 1];
  __shared__ uint64_t s_tmp[kCountThreads / kWave];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_bad;

  const int tid = threadIdx.x;
  const uint32_t npasses = a.npasses;
  const uint32_t depth_passes = 32 / RB < npasses ? 32 / RB : npasses;
  if (DUP)
    for (uint32_t i = tid; i < npasses * BINS; i += kCountThreads) s_hist[i] = 0;
  __syncthreads();
  const uint32_t ticket = blockIdx.x;
  const uint64_t gbase = static_cast<uint64_t>(ticket) * kCountTile;

  // ---- count (striped, coalesced 16-byte loads) ----
  bool bad = false;
#pragma unroll
  for (int j = 0; j < kCountItems; ++j) {
    const uint32_t li = j * kCountThreads + tid;
    const uint64_t gi = gbase + li;
    uint32_t cnt = 0;
    uint4 rect = make_uint4(0, 0, 1, 0);
    if (gi < a.n) {
      const int4 g = reinterpret_cast<const int4*>(a.gaussians)[gi];
      const uint32_t radius = static_cast<uint32_t>(g.w);
      const uint32_t dbits = static_cast<uint32_t>(g.z);
      if (radius != 0) {
        const int64_t R = static_cast<int64_t>(radius) << 4;
        const int64_t X = g.x, Y = g.y;
        const uint32_t x0 = clamp_tile((X - R) >> 8, a.tiles_x);
        const uint32_t x1 = clamp_tile((X + R + 255) >> 8, a.tiles_x);
        const uint32_t y0 = clamp_tile((Y - R) >> 8, a.tiles_y);
        const uint32_t y1 = clamp_tile((Y + R + 255) >> 8, a.tiles_y);
        if (x1 > x0 && y1 > y0) {
          cnt = (x1 - x0) * (y1 - y0);
          rect = make_uint4(x0, y0, x1 - x0, dbits);
        }
      }
      // positive finite <=> bits in [1, 0x7F7FFFFF]
      if (cnt != 0 && dbits - 1u >= 0x7F7FFFFFu) bad = true;
      if (a.tiles_touched) a.tiles_touched[gi] = cnt;
      if (DUP && cnt != 0)
        for (uint32_t p = 0; p < depth_passes; ++p)
          atomicAdd(&s_hist[p * BINS + ((dbits >> (p * RB)) & (BINS - 1))], cnt);
    }
    s_rect[li] = rect;
    s_loc[li] = cnt;
  }
  const bool any_bad = __syncthreads_or(bad);

  // ---- scan: workgroup scan (blocked: thread t owns Gaussians 4t .. 4t+3) ----
  uint32_t c[kCountItems];
  uint64_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kCountItems; ++k) {
    c[k] = s_loc[kCountItems * tid + k];
    tsum += c[k];
  }
  uint64_t btotal;
  const uint64_t texcl = block_exclusive_scan<uint64_t, kCountThreads>(tsum, s_tmp, btotal);
  {
    uint64_t run = texcl;
#pragma unroll
    for (int k = 0; k < kCountItems; ++k) {
      s_loc[kCountItems * tid + k] = run > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(run);
      run += c[k];
    }
  }

  // ---- scan: decoupled look-back over earlier workgroups (wave 0) ----
  if (tid < kWave) {
    const uint32_t lane = tid;
    const uint64_t mine = (btotal > kCountSat ? kCountSat : btotal) | (any_bad ? kLbBad64 : 0);
    uint64_t excl = 0;
    bool excl_bad = false;
    if (ticket == 0) {
      if (lane == 0) st_agent(&a.lookback[0], kLbInc64 | mine);
    } else {
      if (lane == 0) st_agent(&a.lookback[ticket], kLbAgg64 | mine);
      int64_t top = static_cast<int64_t>(ticket) - 1;  // window: top, top-1, ..., top-63
      uint32_t spins = 0;
      while (true) {
        const int64_t idx = top - lane;
        const uint64_t w = idx >= 0 ? ld_agent(&a.lookback[idx]) : kLbInc64;
        const uint32_t state = static_cast<uint32_t>(w >> 62);
        const uint64_t inc_mask = ballot(state == 2);
        const uint64_t empty_mask = ballot(state == 0);
        const uint64_t upto = inc_mask ? (((inc_mask & (~inc_mask + 1)) << 1) - 1) : ~0ull;
        if (empty_mask & upto) {
          if (++spins > kSpinLimit) {
            if (lane == 0) st_agent(a.status, static_cast<uint32_t>(SS_ERR_TIMEOUT));
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        const bool in = (upto >> lane) & 1ull;
        uint64_t v = in ? (w & kLbMask64) : 0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
        excl = sat_add(excl, v);
        excl_bad |= ballot(in && (w & kLbBad64)) != 0;
        if (inc_mask) break;
        top -= kWave;
      }
      if (lane == 0)
        st_agent(&a.lookback[ticket], kLbInc64 | sat_add(excl, btotal) |
                                          ((excl_bad || any_bad) ? kLbBad64 : 0));
    }
    if (lane == 0) {
      s_prefix = excl;
      s_bad = (excl_bad || any_bad) ? 1u : 0u;
    }
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;

  if (tid == 0 && ticket == a.nblocks - 1) {
    const uint64_t total = sat_add(prefix, btotal);
    uint32_t st = SS_OK;
    if (s_bad) st = SS_ERR_INVALID_INPUT;
    else if (total > 0xFFFFFFFFull) st = SS_ERR_OVERFLOW;
    else if (DUP && total > a.capacity) st = SS_ERR_CAPACITY;
    *a.num_pairs = total > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(total);
    // a timeout raised by any workgroup wins over the computed status
    if (ld_agent(a.status) != SS_ERR_TIMEOUT) *a.status = st;
  }

  if (a.offsets) {
    uint64_t run = prefix + texcl;
#pragma unroll
    for (int k = 0; k < kCountItems; ++k) {
      const uint64_t gi = gbase + kCountItems * tid + k;
      if (gi < a.n) a.offsets[gi] = static_cast<uint32_t>(run);
      run += c[k];
    }
  }
  if (!DUP) return;

  // ---- duplicate, spread evenly over the workgroup ----
  uint32_t q_end = 0;
  if (prefix < a.capacity) {
    const uint64_t room = a.capacity - prefix;
    q_end = static_cast<uint32_t>(btotal < room ? btotal : room);
  }
  uint64_t* __restrict__ keys = a.keys + prefix;
  uint32_t* __restrict__ vals = a.values + prefix;
  for (uint32_t q = tid; q < q_end; q += kCountThreads) {
    uint32_t lo = 0;
#pragma unroll
    for (uint32_t step = kCountTile / 2; step; step >>= 1)
      if (s_loc[lo + step] <= q) lo += step;
    const uint4 r = s_rect[lo];
    const uint32_t k = q - s_loc[lo];
    const uint32_t dy = k / r.z;
    const uint32_t dx = k - dy * r.z;
    const uint32_t tile = (r.y + dy) * a.tiles_x + (r.x + dx);
    const uint64_t key = (static_cast<uint64_t>(tile) << 32) | r.w;
    keys[q] = key;
    vals[q] = static_cast<uint32_t>(gbase) + lo;
    for (uint32_t p = depth_passes; p < npasses; ++p)
      atomicAdd(&s_hist[p * BINS + static_cast<uint32_t>((key >> (p * RB)) & (BINS - 1))], 1u);
  }
  __syncthreads();
  uint32_t* gh = a.hist + static_cast<size_t>(ticket % kHistCopies) * npasses * BINS;
  for (uint32_t i = tid; i < npasses * BINS; i += kCountThreads) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(&gh[i], v);
  }
}

// Digit histograms of caller-supplied keys (sort-only entry point).
template <int RB>
__global__ __launch_bounds__(256) void k_hist(HistArgs a) {
  constexpr int BINS = 1 << RB;
  constexpr int MAXP = (64 + RB - 1) / RB;
  constexpr uint32_t kPerBlock = 256 * 16;
  __shared__ uint32_t s_hist[MAXP * BINS];
  const uint32_t npasses = a.npasses;
  for (uint32_t i = threadIdx.x; i < npasses * BINS; i += 256) s_hist[i] = 0;
  __syncthreads();
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kPerBlock;
  for (uint32_t j = 0; j < 16; ++j) {
    const uint64_t i = base + j * 256 + threadIdx.x;
    if (i < a.n) {
      const uint64_t key = a.keys[i];
      for (uint32_t p = 0; p < npasses; ++p)
        atomicAdd(&s_hist[p * BINS + static_cast<uint32_t>((key >> (p * RB)) & (BINS - 1))], 1u);
    }
  }
  __syncthreads();
  uint32_t* gh = a.hist + static_cast<size_t>(blockIdx.x % kHistCopies) * npasses * BINS;
  for (uint32_t i = threadIdx.x; i < npasses * BINS; i += 256) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(&gh[i], v);
  }
}

// Exclusive prefix over digits of the global digit totals of every pass
// (the histogram copies summed).  One workgroup of 256 threads per pass.
// Tile ranges: thread i compares the tile of pair i - 1 with the tile of pair i
// (tile -1 before the first pair, tile T after the last).  At a change from
// a to b it closes a at i, gives every tile strictly between a and b the
// empty range [i, i), and opens b at i.  Every range word is written by
// exactly one thread.
__global__ __launch_bounds__(256) void k_ranges(const uint64_t* __restrict__ keys,
                                                const uint32_t* __restrict__ num_pairs,
                                                const uint32_t* __restrict__ status,
                                                uint32_t num_tiles, uint32_t* __restrict__ ranges) {
  if (status && *status != SS_OK) return;
  const uint32_t m = *num_pairs;
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > m) return;
  const int64_t T = num_tiles;
  int64_t prev = i == 0 ? -1 : static_cast<int64_t>(keys[i - 1] >> 32);
  int64_t cur = i == m ? T : static_cast<int64_t>(keys[i] >> 32);
  // sorted keys never exceed T - 1; clamping only keeps writes in bounds
  prev = prev < T ? prev : T - 1;
  cur = cur < T ? cur : T;
  if (cur <= prev) return;
  const uint32_t pos = static_cast<uint32_t>(i);
  if (prev >= 0) ranges[2 * prev + 1] = pos;
  for (int64_t t = prev + 1; t < cur; ++t) {
    ranges[2 * t] = pos;
    ranges[2 * t + 1] = pos;
  }
  if (cur < static_cast<int64_t>(num_tiles)) ranges[2 * cur] = pos;
}

template <int RB>
hipError_t count_dup_rb(const CountDupArgs& a, bool dup, hipStream_t s) {
  const dim3 grid(a.nblocks), block(kCountThreads);
  if (dup)
    hipLaunchKernelGGL((k_count_dup<RB, true>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_count_dup<RB, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int RB>
hipError_t hist_rb(const HistArgs& a, hipStream_t s) {
  const uint32_t blocks = (a.n + 4095) / 4096;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_hist<RB>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

uint32_t stream_grid(size_t n16) {
  size_t g = (n16 + 255) / 256;
  if (g > 4096) g = 4096;
  if (g == 0) g = 1;
  return static_cast<uint32_t>(g);
}

}  // namespace

hipError_t launch_clear(void* p, size_t bytes, uint32_t* extra, const TableChunk* chunk, FrameInfo* table,
                        hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0 && extra == nullptr && (chunk == nullptr || chunk->count == 0)) return hipSuccess;
  TableChunk c{};
  if (chunk != nullptr) c = *chunk;
  hipLaunchKernelGGL(k_clear, dim3(stream_grid(n16)), dim3(256), 0, s, static_cast<uint4*>(p), n16, extra, c,
                     table);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(stream_grid(n16) * 4), dim3(256), 0, s, static_cast<uint4*>(dst),
                     static_cast<const uint4*>(src), n16);
  return hipGetLastError();
}

hipError_t launch_count_dup(const CountDupArgs& a, int radix_bits, bool dup, hipStream_t s) {
  switch (radix_bits) {
    case 4: return count_dup_rb<4>(a, dup, s);
    case 6: return count_dup_rb<6>(a, dup, s);
    case 8: return count_dup_rb<8>(a, dup, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hist(const HistArgs& a, int radix_bits, hipStream_t s) {
  switch (radix_bits) {
    case 4: return hist_rb<4>(a, s);
    case 6: return hist_rb<6>(a, s);
    case 8: return hist_rb<8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ranges(const uint64_t* keys, const uint32_t* num_pairs, const uint32_t* status,
                         uint32_t capacity, uint32_t num_tiles, uint32_t* ranges, hipStream_t s) {
  const uint64_t threads = static_cast<uint64_t>(capacity) + 1;
  const uint32_t blocks = static_cast<uint32_t>((threads + 255) / 256);
  hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(256), 0, s, keys, num_pairs, status, num_tiles, ranges);
  return hipGetLastError();
}

}  // namespace ss

// Tile-first form of the tile-and-depth sort (SS_ALGO_TILE_FIRST): the pairs
// are duplicated in Gaussian index order and partitioned stably by tile id,
// so each tile's run is in index order; this kernel then sorts every run
// stably by depth, which gives the (tile, depth, index) order of the full
// 64-bit key sort (paper: Background, "Duplication with Tiles" and
// "Sorting").  One workgroup per tile.  Runs of at most kTileSortCap pairs
// are sorted in LDS; longer runs go through the workspace's alternate pair
// buffer, one chunk of kTileSortCap pairs at a time, by the same workgroup.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

constexpr uint32_t kThreads = 512;
constexpr uint32_t kWaves = kThreads / kWave;
constexpr uint32_t kItems = kTileSortCap / kThreads;   // 16

// An item: depth bits << 32 | Gaussian index.  Digit p: byte p of the depth.
__device__ __forceinline__ uint32_t item_digit(uint64_t it, uint32_t p) {
  return static_cast<uint32_t>(it >> (32 + 8 * p)) & 255u;
}

struct RankSmem {
  uint32_t wcnt[kWaves * 256];   // per-wave digit counts, then the waves' offsets
  uint32_t dstart[256];          // the chunk's first slot of each digit
  uint32_t tmp[kWaves];
};

// Stable ranking of one chunk held wave-contiguously (wave w holds chunk
// items [w * 64 * J, (w + 1) * 64 * J), lane l of slot j item
// w * 64 * J + j * 64 + l) by digit p: returns in pos[j] each valid item's
// slot in digit order, and in *count the chunk's per-digit counts
// (dstart holds their exclusive prefix).  J = slots per thread.
__device__ __forceinline__ void rank_chunk(const uint64_t (&it)[kItems], uint32_t p, uint32_t n, uint32_t J,
                                           RankSmem& sm, uint32_t (&dg)[kItems], uint32_t (&pos)[kItems],
                                           uint32_t* count) {
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (uint32_t i = tid; i < kWaves * 256; i += kThreads) sm.wcnt[i] = 0;
  __syncthreads();
  uint32_t* wc = sm.wcnt + wave * 256;
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j) {
    if (j >= J) break;  // uniform over the workgroup
    const uint32_t q = wave * (kWave * J) + j * kWave + lane;
    const bool valid = q < n;
    dg[j] = valid ? item_digit(it[j], p) : 256u;
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
#pragma unroll
    for (uint32_t w = 0; w < kWaves; ++w) {
      const uint32_t x = sm.wcnt[w * 256 + tid];
      sm.wcnt[w * 256 + tid] = dcnt;
      dcnt += x;
    }
  }
  uint32_t dall;
  const uint32_t dex = block_exclusive_scan<uint32_t, kThreads>(dcnt, sm.tmp, dall);
  if (tid < 256) {
    sm.dstart[tid] = dex;
    if (count) count[tid] = dcnt;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j) {
    if (j >= J) break;
    if (dg[j] < 256) pos[j] += sm.dstart[dg[j]] + wc[dg[j]];
  }
}

struct TileSmem {
  uint64_t buf[kTileSortCap];
  RankSmem rank;
  uint32_t base[256], cnt[256], and_bits, or_bits;
};

// Tile t's run, sorted by the whole workgroup.
__device__ __forceinline__ void sort_run(const TileSortArgs& a, uint32_t t, TileSmem& ts) {
  uint64_t* s_buf = ts.buf;
  RankSmem& sm = ts.rank;
  uint32_t* s_base = ts.base;
  uint32_t* s_cnt = ts.cnt;
  uint32_t& s_and = ts.and_bits;
  uint32_t& s_or = ts.or_bits;
  const uint32_t start = a.ranges[2 * t], end = a.ranges[2 * t + 1];
  const uint32_t n = end > start ? end - start : 0u;
  if (n <= 1) return;
  const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  uint64_t* keys = a.keys + start;
  uint32_t* vals = a.values + start;
  const uint64_t tile_hi = static_cast<uint64_t>(t) << 32;

  // the depth bytes that vary inside the run (a digit shared by every pair
  // leaves a stable pass unchanged, so its pass is skipped)
  if (tid == 0) {
    s_and = ~0u;
    s_or = 0u;
  }
  __syncthreads();
  {
    uint32_t an = ~0u, orr = 0u;
    for (uint32_t q = tid; q < n; q += kThreads) {
      const uint32_t d = static_cast<uint32_t>(keys[q]);
      an &= d;
      orr |= d;
    }
    atomicAnd(&s_and, an);
    atomicOr(&s_or, orr);
  }
  __syncthreads();
  const uint32_t vary = s_and ^ s_or;
  if (vary == 0) return;  // equal depths: the run is already in index order
  // byte p of the depth takes a pass when it varies
  auto varies = [vary](uint32_t p) { return ((vary >> (8 * p)) & 255u) != 0; };

  uint64_t it[kItems];
  uint32_t dg[kItems], pos[kItems];
  if (n <= kTileSortCap) {
    // ---- the whole run in LDS ----
    const uint32_t J = (n + kThreads - 1) / kThreads;
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j) {
      if (j >= J) break;
      const uint32_t q = wave * (kWave * J) + j * kWave + lane;
      it[j] = q < n ? (static_cast<uint64_t>(static_cast<uint32_t>(keys[q])) << 32) | vals[q] : 0ull;
    }
    for (uint32_t p = 0; p < 4; ++p) {
      if (!varies(p)) continue;
      rank_chunk(it, p, n, J, sm, dg, pos, nullptr);
#pragma unroll
      for (uint32_t j = 0; j < kItems; ++j) {
        if (j >= J) break;
        if (dg[j] < 256) s_buf[pos[j]] = it[j];
      }
      __syncthreads();
#pragma unroll
      for (uint32_t j = 0; j < kItems; ++j) {
        if (j >= J) break;
        const uint32_t q = wave * (kWave * J) + j * kWave + lane;
        it[j] = q < n ? s_buf[q] : 0ull;
      }
      __syncthreads();
    }
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j) {
      if (j >= J) break;
      const uint32_t q = wave * (kWave * J) + j * kWave + lane;
      if (q < n) {
        keys[q] = tile_hi | static_cast<uint32_t>(it[j] >> 32);
        vals[q] = static_cast<uint32_t>(it[j]);
      }
    }
    return;
  }

  // ---- a run longer than LDS holds: stable passes through global memory,
  // items (depth << 32 | index) ping-ponging between the alternate buffer
  // and the key array, chunk by chunk in order ----
  uint64_t* alt = a.alt + start;
  uint32_t k = 0;   // passes done
  for (uint32_t p = 0; p < 4; ++p) {
    if (!varies(p)) continue;
    // items of this pass: the original pairs (k = 0), else the last pass's output
    const uint64_t* src = (k % 2 == 1) ? alt : keys;
    uint64_t* dst = (k % 2 == 0) ? alt : keys;
    // digit totals of the whole run, then their exclusive prefix
    for (uint32_t i = tid; i < 256; i += kThreads) s_cnt[i] = 0;
    __syncthreads();
    // (device-scope loads: the previous pass's items were written by other
    // threads of this workgroup, and the CU's L1 may hold older lines)
    for (uint32_t q = tid; q < n; q += kThreads) {
      const uint64_t x = k == 0 ? (static_cast<uint64_t>(static_cast<uint32_t>(keys[q])) << 32)
                                : ld_agent(&src[q]);
      atomicAdd(&s_cnt[item_digit(x, p)], 1u);
    }
    __syncthreads();
    {
      const uint32_t c = tid < 256 ? s_cnt[tid] : 0u;
      uint32_t all;
      const uint32_t ex = block_exclusive_scan<uint32_t, kThreads>(c, sm.tmp, all);
      if (tid < 256) s_base[tid] = ex;
      __syncthreads();
    }
    for (uint32_t c0 = 0; c0 < n; c0 += kTileSortCap) {
      const uint32_t cn = n - c0 < kTileSortCap ? n - c0 : kTileSortCap;
      const uint32_t J = (cn + kThreads - 1) / kThreads;
#pragma unroll
      for (uint32_t j = 0; j < kItems; ++j) {
        if (j >= J) break;
        const uint32_t q = wave * (kWave * J) + j * kWave + lane;
        const uint32_t g = c0 + q;
        it[j] = 0;
        if (q < cn)
          it[j] = k == 0 ? (static_cast<uint64_t>(static_cast<uint32_t>(keys[g])) << 32) | vals[g]
                         : ld_agent(&src[g]);
      }
      rank_chunk(it, p, cn, J, sm, dg, pos, s_cnt);
      // slot pos in digit order -> run position s_base[d] + (pos - dstart[d])
#pragma unroll
      for (uint32_t j = 0; j < kItems; ++j) {
        if (j >= J) break;
        if (dg[j] < 256) dst[s_base[dg[j]] + pos[j] - sm.dstart[dg[j]]] = it[j];
      }
      __syncthreads();
      if (tid < 256) s_base[tid] += s_cnt[tid];
      __syncthreads();
    }
    // the pass's output is complete (in L2) before the next pass reads it
    __threadfence();
    __syncthreads();
    ++k;
  }
  // items -> (tile << 32 | depth bits, index); with an odd number of passes
  // they are in the alternate buffer
  const uint64_t* fin = (k % 2 == 1) ? alt : keys;
  for (uint32_t q = tid; q < n; q += kThreads) {
    const uint64_t x = ld_agent(&fin[q]);
    keys[q] = tile_hi | static_cast<uint32_t>(x >> 32);
    vals[q] = static_cast<uint32_t>(x);
  }
}

// Workgroup b sorts tile b.
__global__ __launch_bounds__(kThreads) void k_tile_sort(TileSortArgs a) {
  __shared__ __align__(16) TileSmem ts;
  if (a.status && *a.status != SS_OK) return;
  sort_run(a, blockIdx.x, ts);
}

// More tiles than one dispatch should hold (a dispatch has fewer than 2^32
// work-items): workgroup b sorts tiles b, b + grid, ... (the runs are
// independent).  A separate kernel: the loop costs the one-tile kernel
// registers.
constexpr uint32_t kMaxGrid = 1u << 20;
__global__ __launch_bounds__(kThreads) void k_tile_sort_strided(TileSortArgs a) {
  __shared__ __align__(16) TileSmem ts;
  if (a.status && *a.status != SS_OK) return;
  for (uint32_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
    sort_run(a, t, ts);
    __syncthreads();  // the next run reuses the LDS
  }
}

}  // namespace

hipError_t launch_tile_sort(const TileSortArgs& a, hipStream_t s) {
  if (a.num_tiles == 0) return hipSuccess;
  if (a.num_tiles <= kMaxGrid)
    hipLaunchKernelGGL(k_tile_sort, dim3(a.num_tiles), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_tile_sort_strided, dim3(kMaxGrid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace ss

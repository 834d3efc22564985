// The paper's own sort, re-expressed for MI355X (paper: Background,
// "Sorting"; Design, "Sorting Optimizations in Context of 3DGS" -- a bitonic
// network whose compare-and-swap partners are kept close by a layout
// transformation, with the last steps of a stage fused into one kernel).
//
// The 2D-texture layout transformation only serves a texture cache; on
// MI355X the same goal -- partners close, every step's reads contiguous --
// falls out of two kernels:
//   * a local kernel runs every step whose partner distance is below a
//     4,096-element chunk inside LDS (all of stages 1..12, and steps 12..1 of
//     every later stage: the paper's stage fusion taken to the whole chunk);
//   * a global kernel fuses up to three consecutive longer-distance steps of
//     a stage: each thread holds the 8 elements that those steps compare among
//     themselves (the paper fuses two steps over the 4 values of a texel),
//     and consecutive threads touch consecutive addresses.
// The network sorts a power-of-two padded array.  Elements compare as
// (key, value) pairs, so for the frame's pairs -- unique (tile, Gaussian) --
// the result is the stable order of the radix paths, bit for bit.
//
// The paper's key normalisation (Design, "Sorting Optimizations in Context
// of 3DGS": the 64-bit key becomes one 32-bit float, 20 bits of tile number
// and the depth brought below 2^10) is the 32-bit-key instantiation: key =
// tile * 2^10 + min(depth, largest float below 2^10), rounded toward zero in
// FP32 so that no key reaches the next tile's; positive floats order like
// their bit patterns, so the network compares the bits.  Depths closer than
// one unit in the last place of the sum share a key and fall back to index
// order.  The last kernel rebuilds the exact 64-bit key of each pair from its
// tile and its Gaussian's depth.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

constexpr uint32_t kChunkLog = 12;
constexpr uint32_t kChunk = 1u << kChunkLog;
constexpr uint32_t kLocalThreads = 256;
constexpr uint32_t kLocalItems = kChunk / kLocalThreads;
constexpr uint32_t kGlobalThreads = 256;
constexpr uint32_t kMaxFuse = 3;

// largest FP32 value below 2^10 (0x447FFFFF)
constexpr float kDepthCap = 1023.99993896484375f;

template <typename K>
__device__ __forceinline__ bool greater(K ka, uint32_t va, K kb, uint32_t vb) {
  return ka > kb || (ka == kb && va > vb);
}

// Order (a, b) ascending (or descending) in place.
template <typename K>
__device__ __forceinline__ void cmp_swap(K& ka, uint32_t& va, K& kb, uint32_t& vb, bool asc) {
  if (greater(ka, va, kb, vb) == asc) {
    const K tk = ka;
    ka = kb;
    kb = tk;
    const uint32_t tv = va;
    va = vb;
    vb = tv;
  }
}

// The normalised 32-bit key of a frame key (tile << 32 | depth bits): FP32
// tile * 1024 (exact below 2^20 tiles) plus the capped depth, rounded toward
// zero: the rounded-to-nearest sum, stepped down one unit when it exceeds the
// exact sum (whose error the two-sum identity gives exactly).
__device__ __forceinline__ uint32_t lossy_key32(uint64_t key) {
  const float t = static_cast<float>(static_cast<uint32_t>(key >> 32)) * 1024.0f;
  const float d = fminf(__uint_as_float(static_cast<uint32_t>(key)), kDepthCap);
  const float sum = t + d;
  const float bv = sum - t;
  const float err = (t - (sum - bv)) + (d - bv);
  const uint32_t bits = __float_as_uint(sum);
  return err < 0.0f ? bits - 1 : bits;
}

template <typename K>
__device__ __forceinline__ K* key_buf(const BitonicArgs& a) {
  return static_cast<K*>(a.keys);
}
template <typename K>
__device__ __forceinline__ K key_max() {
  return static_cast<K>(~K{0});
}

__device__ __forceinline__ uint32_t valid_count(const BitonicArgs& a) {
  return a.num_pairs ? *a.num_pairs : a.n_fixed;
}

// Fill the padded buffer: entries [0, n) from the source (when given; 64-bit
// keys masked to key_mask, 32-bit keys normalised), [n, 2^log_n) with the
// largest pair.
template <typename K>
__global__ __launch_bounds__(256) void k_bitonic_load(BitonicArgs a, const uint64_t* __restrict__ src_k,
                                                      const uint32_t* __restrict__ src_v, uint64_t key_mask) {
  if (a.status && *a.status != SS_OK) return;
  const uint32_t n = valid_count(a);
  const uint64_t size = 1ull << a.log_n;
  K* keys = key_buf<K>(a);
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < size;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (i < n) {
      if (src_k) {
        if constexpr (sizeof(K) == 8) keys[i] = src_k[i] & key_mask;
        else keys[i] = lossy_key32(src_k[i]);
        a.vals[i] = src_v[i];
      }
    } else {
      keys[i] = key_max<K>();
      a.vals[i] = ~0u;
    }
  }
}

// Stages s0..s1 inside one chunk of the array; for each stage the steps whose
// partner distance is below the chunk.  Chunks shorter than kChunk happen
// only when the whole array is shorter.  With `final` the chunk is written to
// the caller's output (entries below the valid count) instead of back; 32-bit
// keys leave as the exact 64-bit key (tile from the normalised key, depth bits
// from the Gaussian's record).
template <typename K>
__global__ __launch_bounds__(kLocalThreads) void k_bitonic_local(BitonicArgs a, uint32_t s0, uint32_t s1,
                                                                 bool final_pass) {
  __shared__ K sk[kChunk];
  __shared__ uint32_t sv[kChunk];
  K* keys = key_buf<K>(a);
  if (a.status && *a.status != SS_OK) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t clog = a.log_n < kChunkLog ? a.log_n : kChunkLog;
  const uint32_t csize = 1u << clog;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) << clog;
#pragma unroll
  for (uint32_t m = 0; m < kLocalItems; ++m) {
    const uint32_t i = m * kLocalThreads + tid;
    if (i < csize) {
      sk[i] = keys[base + i];
      sv[i] = a.vals[base + i];
    }
  }
  __syncthreads();
  const uint32_t pairs = csize / 2;
  for (uint32_t s = s0; s <= s1; ++s) {
    const uint32_t jtop = s < clog ? s : clog;
    for (uint32_t j = jtop; j >= 1; --j) {
      const uint32_t b = j - 1;
      for (uint32_t q = tid; q < pairs; q += kLocalThreads) {
        const uint32_t lo = ((q >> b) << (b + 1)) | (q & ((1u << b) - 1));
        const uint32_t hi = lo | (1u << b);
        const bool asc = (((base + lo) >> s) & 1) == 0;
        K k0 = sk[lo], k1 = sk[hi];
        uint32_t v0 = sv[lo], v1 = sv[hi];
        cmp_swap(k0, v0, k1, v1, asc);
        sk[lo] = k0;
        sk[hi] = k1;
        sv[lo] = v0;
        sv[hi] = v1;
      }
      __syncthreads();
    }
  }
  if (final_pass) {
    const uint32_t n = valid_count(a);
#pragma unroll
    for (uint32_t m = 0; m < kLocalItems; ++m) {
      const uint32_t i = m * kLocalThreads + tid;
      if (i < csize && base + i < n && base + i < a.out_capacity) {
        if constexpr (sizeof(K) == 8) {
          a.out_keys[base + i] = sk[i];
        } else {
          // floor(key) lies in [tile * 1024, tile * 1024 + 1023]
          const uint32_t tile = static_cast<uint32_t>(__uint_as_float(sk[i])) >> 10;
          a.out_keys[base + i] = (static_cast<uint64_t>(tile) << 32) |
                                 __float_as_uint(a.gaussians[sv[i]].depth);
        }
        a.out_vals[base + i] = sv[i];
      }
    }
  } else {
#pragma unroll
    for (uint32_t m = 0; m < kLocalItems; ++m) {
      const uint32_t i = m * kLocalThreads + tid;
      if (i < csize) {
        keys[base + i] = sk[i];
        a.vals[base + i] = sv[i];
      }
    }
  }
}

// Steps j_hi, j_hi - 1, ..., j_hi - t + 1 of stage s (partner distances of
// at least one chunk).  Thread g owns the 2^t elements i0 + m 2^(j_hi - t),
// m < 2^t, where i0 is g with t zero bits inserted at bit j_hi - t.
template <typename K, uint32_t T>
__global__ __launch_bounds__(kGlobalThreads) void k_bitonic_global(BitonicArgs a, uint32_t s, uint32_t j_hi) {
  constexpr uint32_t E = 1u << T;
  if (a.status && *a.status != SS_OK) return;
  K* keys = key_buf<K>(a);
  const uint64_t g = static_cast<uint64_t>(blockIdx.x) * kGlobalThreads + threadIdx.x;
  if (g >= (1ull << (a.log_n - T))) return;
  const uint32_t blo = j_hi - T;
  const uint64_t i0 = ((g >> blo) << (blo + T)) | (g & ((1ull << blo) - 1));
  const bool asc = ((i0 >> s) & 1) == 0;
  K k[E];
  uint32_t v[E];
#pragma unroll
  for (uint32_t m = 0; m < E; ++m) {
    k[m] = keys[i0 + (static_cast<uint64_t>(m) << blo)];
    v[m] = a.vals[i0 + (static_cast<uint64_t>(m) << blo)];
  }
#pragma unroll
  for (int bit = static_cast<int>(T) - 1; bit >= 0; --bit) {
#pragma unroll
    for (uint32_t m = 0; m < E; ++m)
      if ((m & (1u << bit)) == 0) cmp_swap(k[m], v[m], k[m | (1u << bit)], v[m | (1u << bit)], asc);
  }
#pragma unroll
  for (uint32_t m = 0; m < E; ++m) {
    keys[i0 + (static_cast<uint64_t>(m) << blo)] = k[m];
    a.vals[i0 + (static_cast<uint64_t>(m) << blo)] = v[m];
  }
}

uint32_t grid_for(uint64_t threads, uint32_t block) {
  const uint64_t g = (threads + block - 1) / block;
  return static_cast<uint32_t>(g < 1 ? 1 : g);
}

}  // namespace

uint32_t bitonic_log_size(uint64_t n) {
  uint32_t l = 1;
  while ((1ull << l) < n) ++l;
  return l;
}

uint32_t bitonic_launches(uint32_t log_n) {
  const uint32_t clog = log_n < kChunkLog ? log_n : kChunkLog;
  uint32_t n = 2;  // load + first local
  for (uint32_t st = clog + 1; st <= log_n; ++st) n += (st - clog + kMaxFuse - 1) / kMaxFuse + 1;
  return n;
}

namespace {

template <typename K>
hipError_t launch_network(const BitonicArgs& a, const uint64_t* src_k, const uint32_t* src_v, uint64_t key_mask,
                          hipStream_t s) {
  const uint64_t size = 1ull << a.log_n;
  const uint32_t load_grid = grid_for(size, 256) < 4096 ? grid_for(size, 256) : 4096;
  hipLaunchKernelGGL(k_bitonic_load<K>, dim3(load_grid), dim3(256), 0, s, a, src_k, src_v, key_mask);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  const uint32_t clog = a.log_n < kChunkLog ? a.log_n : kChunkLog;
  const uint32_t chunks = static_cast<uint32_t>(size >> clog);
  hipLaunchKernelGGL(k_bitonic_local<K>, dim3(chunks), dim3(kLocalThreads), 0, s, a, 1u, clog, a.log_n == clog);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  for (uint32_t st = clog + 1; st <= a.log_n; ++st) {
    uint32_t j = st;
    while (j > clog) {
      const uint32_t t = j - clog < kMaxFuse ? j - clog : kMaxFuse;
      const uint32_t grid = grid_for(size >> t, kGlobalThreads);
      if (t == 3) hipLaunchKernelGGL((k_bitonic_global<K, 3>), dim3(grid), dim3(kGlobalThreads), 0, s, a, st, j);
      else if (t == 2) hipLaunchKernelGGL((k_bitonic_global<K, 2>), dim3(grid), dim3(kGlobalThreads), 0, s, a, st, j);
      else hipLaunchKernelGGL((k_bitonic_global<K, 1>), dim3(grid), dim3(kGlobalThreads), 0, s, a, st, j);
      if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
      j -= t;
    }
    hipLaunchKernelGGL(k_bitonic_local<K>, dim3(chunks), dim3(kLocalThreads), 0, s, a, st, st, st == a.log_n);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_bitonic(const BitonicArgs& a, const uint64_t* src_k, const uint32_t* src_v, uint64_t key_mask,
                          hipStream_t s) {
  return a.key32 ? launch_network<uint32_t>(a, src_k, src_v, key_mask, s)
                 : launch_network<uint64_t>(a, src_k, src_v, key_mask, s);
}

}  // namespace ss

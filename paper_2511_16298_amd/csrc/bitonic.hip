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

__device__ __forceinline__ bool greater(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
  return ka > kb || (ka == kb && va > vb);
}

// Order (a, b) ascending (or descending) in place.
__device__ __forceinline__ void cmp_swap(uint64_t& ka, uint32_t& va, uint64_t& kb, uint32_t& vb, bool asc) {
  if (greater(ka, va, kb, vb) == asc) {
    const uint64_t tk = ka;
    ka = kb;
    kb = tk;
    const uint32_t tv = va;
    va = vb;
    vb = tv;
  }
}

__device__ __forceinline__ uint32_t valid_count(const BitonicArgs& a) {
  return a.num_pairs ? *a.num_pairs : a.n_fixed;
}

// Fill the padded buffer: entries [0, n) from the source (when given, with the
// key masked to key_mask), [n, 2^log_n) with the largest pair.
__global__ __launch_bounds__(256) void k_bitonic_load(BitonicArgs a, const uint64_t* __restrict__ src_k,
                                                      const uint32_t* __restrict__ src_v, uint64_t key_mask) {
  if (a.status && *a.status != SS_OK) return;
  const uint32_t n = valid_count(a);
  const uint64_t size = 1ull << a.log_n;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < size;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (i < n) {
      if (src_k) {
        a.keys[i] = src_k[i] & key_mask;
        a.vals[i] = src_v[i];
      }
    } else {
      a.keys[i] = ~0ull;
      a.vals[i] = ~0u;
    }
  }
}

// Stages s0..s1 inside one chunk of the array; for each stage the steps whose
// partner distance is below the chunk.  Chunks shorter than kChunk happen
// only when the whole array is shorter.  With `final` the chunk is written to
// the caller's output (entries below the valid count) instead of back.
__global__ __launch_bounds__(kLocalThreads) void k_bitonic_local(BitonicArgs a, uint32_t s0, uint32_t s1,
                                                                 bool final_pass) {
  __shared__ uint64_t sk[kChunk];
  __shared__ uint32_t sv[kChunk];
  if (a.status && *a.status != SS_OK) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t clog = a.log_n < kChunkLog ? a.log_n : kChunkLog;
  const uint32_t csize = 1u << clog;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) << clog;
#pragma unroll
  for (uint32_t m = 0; m < kLocalItems; ++m) {
    const uint32_t i = m * kLocalThreads + tid;
    if (i < csize) {
      sk[i] = a.keys[base + i];
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
        uint64_t k0 = sk[lo], k1 = sk[hi];
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
        a.out_keys[base + i] = sk[i];
        a.out_vals[base + i] = sv[i];
      }
    }
  } else {
#pragma unroll
    for (uint32_t m = 0; m < kLocalItems; ++m) {
      const uint32_t i = m * kLocalThreads + tid;
      if (i < csize) {
        a.keys[base + i] = sk[i];
        a.vals[base + i] = sv[i];
      }
    }
  }
}

// Steps j_hi, j_hi - 1, ..., j_hi - t + 1 of stage s (partner distances of
// at least one chunk).  Thread g owns the 2^t elements i0 + m 2^(j_hi - t),
// m < 2^t, where i0 is g with t zero bits inserted at bit j_hi - t.
template <uint32_t T>
__global__ __launch_bounds__(kGlobalThreads) void k_bitonic_global(BitonicArgs a, uint32_t s, uint32_t j_hi) {
  constexpr uint32_t E = 1u << T;
  if (a.status && *a.status != SS_OK) return;
  const uint64_t g = static_cast<uint64_t>(blockIdx.x) * kGlobalThreads + threadIdx.x;
  if (g >= (1ull << (a.log_n - T))) return;
  const uint32_t blo = j_hi - T;
  const uint64_t i0 = ((g >> blo) << (blo + T)) | (g & ((1ull << blo) - 1));
  const bool asc = ((i0 >> s) & 1) == 0;
  uint64_t k[E];
  uint32_t v[E];
#pragma unroll
  for (uint32_t m = 0; m < E; ++m) {
    k[m] = a.keys[i0 + (static_cast<uint64_t>(m) << blo)];
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
    a.keys[i0 + (static_cast<uint64_t>(m) << blo)] = k[m];
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

hipError_t launch_bitonic(const BitonicArgs& a, const uint64_t* src_k, const uint32_t* src_v, uint64_t key_mask,
                          hipStream_t s) {
  const uint64_t size = 1ull << a.log_n;
  const uint32_t load_grid = grid_for(size, 256) < 4096 ? grid_for(size, 256) : 4096;
  hipLaunchKernelGGL(k_bitonic_load, dim3(load_grid), dim3(256), 0, s, a, src_k, src_v, key_mask);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  const uint32_t clog = a.log_n < kChunkLog ? a.log_n : kChunkLog;
  const uint32_t chunks = static_cast<uint32_t>(size >> clog);
  hipLaunchKernelGGL(k_bitonic_local, dim3(chunks), dim3(kLocalThreads), 0, s, a, 1u, clog, a.log_n == clog);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  for (uint32_t st = clog + 1; st <= a.log_n; ++st) {
    uint32_t j = st;
    while (j > clog) {
      const uint32_t t = j - clog < kMaxFuse ? j - clog : kMaxFuse;
      const uint32_t grid = grid_for(size >> t, kGlobalThreads);
      if (t == 3) hipLaunchKernelGGL(k_bitonic_global<3>, dim3(grid), dim3(kGlobalThreads), 0, s, a, st, j);
      else if (t == 2) hipLaunchKernelGGL(k_bitonic_global<2>, dim3(grid), dim3(kGlobalThreads), 0, s, a, st, j);
      else hipLaunchKernelGGL(k_bitonic_global<1>, dim3(grid), dim3(kGlobalThreads), 0, s, a, st, j);
      if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
      j -= t;
    }
    hipLaunchKernelGGL(k_bitonic_local, dim3(chunks), dim3(kLocalThreads), 0, s, a, st, st, st == a.log_n);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ss

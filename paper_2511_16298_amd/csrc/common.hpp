// Device helpers shared by the splatsort kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include "splatsort.h"

namespace ss {

constexpr int kWave = 64;

// Look-back words.  32-bit form (sort passes): bits 30-31 hold the state,
// bits 0-29 the count.  64-bit form (the Gaussian scan): bits 62-63 state,
// bit 61 a sticky "invalid input" flag, bits 0-60 the count (saturating).
constexpr uint32_t kLbAgg32 = 1u << 30;
constexpr uint32_t kLbInc32 = 2u << 30;
constexpr uint32_t kLbMask32 = (1u << 30) - 1;
constexpr uint64_t kLbAgg64 = 1ull << 62;
constexpr uint64_t kLbInc64 = 2ull << 62;
constexpr uint64_t kLbBad64 = 1ull << 61;
constexpr uint64_t kLbMask64 = (1ull << 61) - 1;
// A published digit base (counts stay below 2^30).
constexpr uint32_t kBasePublished = 1u << 31;

// Look-back order.  Workgroup b takes tile b of the input and waits only on
// workgroups with smaller indices.  The dispatcher hands each XCD its
// workgroups in increasing index order, so the smallest undispatched
// workgroup always finds a slot once the running, smaller ones finish: no
// wait can block forever, and no atomic ticket (whose same-address atomics
// serialise at about 12 ns per workgroup) is needed.  Results do not depend
// on the dispatch order at all; the bounded spin below only guards progress.
//
// A bounded spin: after this many polls a waiting workgroup gives up, raises
// SS_ERR_TIMEOUT in the status word and leaves (its output is then invalid,
// but the grid always drains).  Far above any legitimate wait.
constexpr uint32_t kSpinLimit = 1u << 20;

// The spin limit a launch asked for (0: the default).
__device__ __forceinline__ uint32_t spin_limit_of(uint32_t asked) { return asked != 0 ? asked : kSpinLimit; }

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t popc_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// The lanes among `lanes` whose RB-bit digit equals this lane's (stable
// ranking inside a wave: this lane's rank is the number of them below it).
// For every digit bit b: t = 0 or ~0 (this lane's bit, sign-extended), m =
// the ballot of that bit; keep m where t is set and ~m elsewhere, i.e.
// mask & ~(m ^ t), which is one 3-input bitwise op per 32-lane half
// (truth table 0x90 over (mask, m, t)).  The empty asm keeps t opaque, so
// that the ballot is one compare of t rather than a fresh extraction of
// the bit from d.  Four VALU instructions per digit bit.
template <int RB>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t lanes) {
  uint32_t lo = static_cast<uint32_t>(lanes), hi = static_cast<uint32_t>(lanes >> 32);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    uint32_t t = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int>(d), b, 1));
    asm("" : "+v"(t));
    const uint64_t m = ballot(t != 0);
    lo = __builtin_amdgcn_bitop3_b32(lo, static_cast<uint32_t>(m), t, 0x90);
    hi = __builtin_amdgcn_bitop3_b32(hi, static_cast<uint32_t>(m >> 32), t, 0x90);
  }
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Cross-workgroup words are read and written with device-scope atomics so
// they are coherent across the XCDs' separate L2 caches.
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive scans over the 64 lanes of a wave with DPP lane moves instead of
// LDS permutes.  Inside each row of 16 lanes, four steps (row_shr:1, 2, 4, 8)
// add the value d lanes below; lanes below the row's start read 0 (bound_ctrl),
// the identity of both operations.  Then row_bcast:15 adds lane 15's prefix to
// rows 1 and 3, and row_bcast:31 lane 31's to rows 2 and 3.  Lanes outside a
// step's row or bank mask receive 0.
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ uint32_t dpp0(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROWS, BANKS, true));
}
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ uint64_t dpp0(uint64_t v) {
  return (static_cast<uint64_t>(dpp0<CTRL, ROWS, BANKS>(static_cast<uint32_t>(v >> 32))) << 32) |
         dpp0<CTRL, ROWS, BANKS>(static_cast<uint32_t>(v));
}
constexpr int kDppRowShr = 0x110, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit integers");
  using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
  U x = static_cast<U>(v);
  x += dpp0<kDppRowShr | 1, 0xF, 0xF>(x);
  x += dpp0<kDppRowShr | 2, 0xF, 0xF>(x);
  x += dpp0<kDppRowShr | 4, 0xF, 0xF>(x);
  x += dpp0<kDppRowShr | 8, 0xF, 0xF>(x);
  x += dpp0<kDppRowBcast15, 0xA, 0xF>(x);
  x += dpp0<kDppRowBcast31, 0xC, 0xF>(x);
  return static_cast<T>(x);
}

__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t x) {
  x = max(x, dpp0<kDppRowShr | 1, 0xF, 0xF>(x));
  x = max(x, dpp0<kDppRowShr | 2, 0xF, 0xF>(x));
  x = max(x, dpp0<kDppRowShr | 4, 0xF, 0xF>(x));
  x = max(x, dpp0<kDppRowShr | 8, 0xF, 0xF>(x));
  x = max(x, dpp0<kDppRowBcast15, 0xA, 0xF>(x));
  x = max(x, dpp0<kDppRowBcast31, 0xC, 0xF>(x));
  return x;
}

// Exclusive scan over a whole workgroup of THREADS threads (one value each).
// `s_tmp` holds THREADS / 64 values of LDS.  Returns the exclusive prefix and
// writes the workgroup total.  Contains two barriers.
template <typename T, int THREADS>
__device__ __forceinline__ T block_exclusive_scan(T v, T* s_tmp, T& total) {
  constexpr int kWaves = THREADS / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const T inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) s_tmp[wave] = inc;
  __syncthreads();
  T before = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const T x = s_tmp[w];
    before += (w < wave) ? x : T(0);
    sum += x;
  }
  __syncthreads();
  total = sum;
  return before + inc - v;
}

// Decoupled look-back for one digit (one calling thread per digit): adds up
// the digit's counts in workgroups 0 .. t-1 of `lb` ([workgroup][stride]
// words, this workgroup's aggregate already published) and publishes this
// workgroup's inclusive count.  Each round reads the words of
// kLookbackWindow predecessors at once (independent loads, so one memory
// latency per round) and consumes them nearest first, up to the first
// inclusive word; a word not yet published ends the round there.  Returns
// false after kSpinLimit fruitless rounds, having raised SS_ERR_TIMEOUT in
// *status (when not NULL).
constexpr int kLookbackWindow = 8;

// `first`: the chain's first workgroup (0, or a segment's first), which
// publishes its count as inclusive at once.  `spin_limit`: polls before
// giving up (kSpinLimit unless a caller asks for fewer).
__device__ __forceinline__ bool lookback_digit(uint32_t* lb, uint32_t t, uint32_t stride, uint32_t d, uint32_t own,
                                               uint32_t* status, uint32_t& excl, uint32_t first = 0,
                                               uint32_t spin_limit = kSpinLimit) {
  excl = 0;
  if (t == first) return true;
  int32_t kb = static_cast<int32_t>(t) - 1;  // nearest predecessor not yet consumed
  const int32_t lo = static_cast<int32_t>(first);
  uint32_t spins = 0;
  while (true) {
    uint32_t w[kLookbackWindow];
#pragma unroll
    for (int j = 0; j < kLookbackWindow; ++j)
      w[j] = kb - j >= lo ? ld_agent(&lb[static_cast<size_t>(kb - j) * stride + d]) : kLbInc32;
    uint32_t add = 0;
    int32_t used = 0;
    bool inc = false, stall = false;
#pragma unroll
    for (int j = 0; j < kLookbackWindow; ++j) {
      if (inc || stall) continue;
      if ((w[j] & ~kLbMask32) == 0) {
        stall = true;
      } else {
        add += w[j] & kLbMask32;
        ++used;
        inc = (w[j] & kLbInc32) != 0;
      }
    }
    excl += add;
    if (inc) break;
    kb -= used;
    if (stall) {
      if (++spins > spin_limit) {
        if (status) st_agent(status, static_cast<uint32_t>(SS_ERR_TIMEOUT));
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  st_agent(&lb[static_cast<size_t>(t) * stride + d], kLbInc32 | (excl + own));
  return true;
}

// The look-back above with 64-bit words that also carry a maximum: bits 0-29
// the count, bits 30-61 a value combined by max (0 = none), bits 62-63 the
// state.  Returns the exclusive count and maximum, and publishes this
// workgroup's inclusive word (own count and maximum `own_max`).
constexpr uint64_t kLbAggW = 1ull << 62;
constexpr uint64_t kLbIncW = 2ull << 62;
constexpr uint64_t kLbCountW = (1ull << 30) - 1;
constexpr uint64_t kLbMaxW = (1ull << 32) - 1;

__device__ __forceinline__ uint64_t lb_word(uint64_t state, uint32_t count, uint32_t mx) {
  return state | (static_cast<uint64_t>(mx) << 30) | count;
}

__device__ __forceinline__ bool lookback_digit_max(uint64_t* lb, uint32_t t, uint32_t stride, uint32_t d,
                                                   uint32_t own, uint32_t own_max, uint32_t* status,
                                                   uint32_t& excl, uint32_t& excl_max, uint32_t first = 0,
                                                   uint32_t spin_limit = kSpinLimit) {
  excl = 0;
  excl_max = 0;
  if (t == first) return true;
  int32_t kb = static_cast<int32_t>(t) - 1;
  const int32_t lo = static_cast<int32_t>(first);
  uint32_t spins = 0;
  while (true) {
    uint64_t w[kLookbackWindow];
#pragma unroll
    for (int j = 0; j < kLookbackWindow; ++j)
      w[j] = kb - j >= lo ? ld_agent(&lb[static_cast<size_t>(kb - j) * stride + d]) : kLbIncW;
    uint32_t add = 0, mx = 0;
    int32_t used = 0;
    bool inc = false, stall = false;
#pragma unroll
    for (int j = 0; j < kLookbackWindow; ++j) {
      if (inc || stall) continue;
      if ((w[j] >> 62) == 0) {
        stall = true;
      } else {
        add += static_cast<uint32_t>(w[j] & kLbCountW);
        const uint32_t m = static_cast<uint32_t>((w[j] >> 30) & kLbMaxW);
        mx = m > mx ? m : mx;
        ++used;
        inc = (w[j] >> 62) == 2;
      }
    }
    excl += add;
    excl_max = mx > excl_max ? mx : excl_max;
    if (inc) break;
    kb -= used;
    if (stall) {
      if (++spins > spin_limit) {
        if (status) st_agent(status, static_cast<uint32_t>(SS_ERR_TIMEOUT));
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  st_agent(&lb[static_cast<size_t>(t) * stride + d],
           lb_word(kLbIncW, excl + own, own_max > excl_max ? own_max : excl_max));
  return true;
}

}  // namespace ss

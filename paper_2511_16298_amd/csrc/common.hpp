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

// Decoupled look-back for one digit by a group of G consecutive lanes of one
// wave (one group per digit): adds up the digit's counts in workgroups
// first .. t-1 of `lb` ([workgroup][stride] words, this workgroup's aggregate
// already published).  Each round, lane s of the group reads the words of
// predecessors kb - 8s - j (j < 8) at once, independent loads, so a round
// costs one memory latency and covers 8G predecessors.  Every lane sums its
// words nearest first, up to the first inclusive or not yet published one;
// the group then takes its lanes in order up to the first that stopped.  An
// inclusive word ends the look-back; an unpublished one ends the round there
// (the round after restarts at it).  `first`: the chain's first workgroup,
// which published its count as inclusive at once; words before it read as
// inclusive zeros.  Returns the exclusive count (and, with 64-bit words, the
// largest carried maximum) in every lane of the group; returns false after
// spin_limit fruitless rounds, having raised SS_ERR_TIMEOUT in *status (when
// not NULL).  The caller publishes the inclusive word.
constexpr int kLookbackWindow = 8;

// 64-bit look-back words that also carry a maximum: bits 0-29 the count,
// bits 30-61 a value combined by max (0 = none), bits 62-63 the state.
constexpr uint64_t kLbAggW = 1ull << 62;
constexpr uint64_t kLbIncW = 2ull << 62;
constexpr uint64_t kLbCountW = (1ull << 30) - 1;
constexpr uint64_t kLbMaxW = (1ull << 32) - 1;

__device__ __forceinline__ uint64_t lb_word(uint64_t state, uint32_t count, uint32_t mx) {
  return state | (static_cast<uint64_t>(mx) << 30) | count;
}

struct LbWords32 {
  using W = uint32_t;
  static constexpr bool kMax = false;
  static constexpr W kBefore = kLbInc32;
  __device__ static bool published(W w) { return (w & ~kLbMask32) != 0; }
  __device__ static bool inclusive(W w) { return (w & kLbInc32) != 0; }
  __device__ static uint32_t count(W w) { return w & kLbMask32; }
  __device__ static uint32_t maximum(W) { return 0; }
};
struct LbWords64 {
  using W = uint64_t;
  static constexpr bool kMax = true;
  static constexpr W kBefore = kLbIncW;
  __device__ static bool published(W w) { return (w >> 62) != 0; }
  __device__ static bool inclusive(W w) { return (w >> 62) == 2; }
  __device__ static uint32_t count(W w) { return static_cast<uint32_t>(w & kLbCountW); }
  __device__ static uint32_t maximum(W w) { return static_cast<uint32_t>((w >> 30) & kLbMaxW); }
};

template <int G, typename P>
__device__ __forceinline__ bool lookback_group(typename P::W* lb, uint32_t t, uint32_t stride, uint32_t d,
                                               uint32_t* status, uint32_t& excl, uint32_t& excl_max,
                                               uint32_t first, uint32_t spin_limit) {
  static_assert(G >= 1 && G <= kWave && kWave % G == 0, "a group lies inside one wave");
  constexpr int W = kLookbackWindow;
  const uint32_t lane = lane_id();
  const uint32_t s = lane % G;
  const uint32_t base = lane - s;
  excl = 0;
  excl_max = 0;
  if (t == first) return true;
  int32_t kb = static_cast<int32_t>(t) - 1;  // nearest predecessor not yet consumed
  const int32_t lo = static_cast<int32_t>(first);
  uint32_t spins = 0;
  while (true) {
    typename P::W w[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int32_t k = kb - static_cast<int32_t>(s) * W - j;
      w[j] = k >= lo ? ld_agent(&lb[static_cast<size_t>(k) * stride + d]) : P::kBefore;
    }
    uint32_t sum = 0, mx = 0, used = 0, st = 0;  // st: 0 all consumed, 1 inclusive met, 2 unpublished met
#pragma unroll
    for (int j = 0; j < W; ++j) {
      if (st != 0) continue;
      if (!P::published(w[j])) {
        st = 2;
      } else {
        sum += P::count(w[j]);
        if (P::kMax) mx = max(mx, P::maximum(w[j]));
        ++used;
        if (P::inclusive(w[j])) st = 1;
      }
    }
    // the group's lanes in order, up to the first that stopped
    uint32_t add = 0, amx = 0, taken = 0, stop = 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const uint32_t sk = G == 1 ? sum : static_cast<uint32_t>(__shfl(static_cast<int>(sum), base + k, kWave));
      const uint32_t pk = G == 1 ? (used | st << 8)
                                 : static_cast<uint32_t>(__shfl(static_cast<int>(used | st << 8), base + k, kWave));
      uint32_t mk = 0;
      if (P::kMax) mk = G == 1 ? mx : static_cast<uint32_t>(__shfl(static_cast<int>(mx), base + k, kWave));
      if (stop == 0) {
        add += sk;
        amx = max(amx, mk);
        taken += pk & 0xFFu;
        stop = pk >> 8;
      }
    }
    excl += add;
    excl_max = max(excl_max, amx);
    if (stop == 1) break;
    kb -= static_cast<int32_t>(taken);
    if (stop == 2) {
      if (++spins > spin_limit) {
        if (status && s == 0) st_agent(status, static_cast<uint32_t>(SS_ERR_TIMEOUT));
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return true;
}

}  // namespace ss

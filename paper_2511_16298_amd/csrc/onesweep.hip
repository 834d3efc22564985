// One digit pass of the stable LSD radix sort of (key, 32-bit value) pairs
// (paper: Background, "Sorting" -- by tile, then by depth; Design, "Sorting
// Optimizations in Context of 3DGS" -- the original method sorts a 64-bit
// integer key).  Single-pass ("onesweep") scatter: the global digit totals
// are known beforehand (gathered while the pairs were produced), so a
// workgroup needs only the counts of its digits in earlier workgroups, which
// it gets by a decoupled look-back, and then scatters its tile straight to the
// output.  One read and one write of every pair per pass.
//
// Three forms of the item: a key with a 32-bit value (kPassKV, both key
// widths); a packed 64-bit pair alone (kPassItems: tile, depth field and
// index in one word, see PackedPairs); and the last pass over packed pairs
// (kPassUnpack), which writes the pairs back as 64-bit keys (tile << 32 |
// depth bits) and 32-bit indices and, while it writes them, the tile ranges:
// a pair whose tile differs from its predecessor's starts a range.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

// Workgroup of THREADS threads (256 or 512: 4 or 8 waves), ITEMS pairs per
// thread.  Pairs are loaded wave-striped: wave w owns the contiguous segment
// [w * 64 * ITEMS, (w + 1) * 64 * ITEMS) of the tile and lane l holds elements
// j * 64 + l, so every load instruction reads 64 consecutive pairs.
//
// Stable ranking in wave64: for item slot j, RB ballots give each lane the
// mask of lanes holding the same digit; its rank among them is the popcount
// of that mask below the lane, plus the wave's running count of the digit
// kept in LDS (read by all lanes, then advanced by the lowest lane of each
// digit group).  Slots are visited in order j = 0, 1, ..., so ranks follow
// the input order inside the wave; waves are then offset by the counts of
// earlier waves, and digits by a workgroup scan.  The tile is permuted into
// digit order in LDS -- keys first, then values through the same buffer, to
// keep LDS small (160 KB per CU holds four 256 x 16 tiles of 64-bit keys, or
// two 512 x 16 ones) -- and written out so that runs of one digit land on
// consecutive addresses.
template <typename K, int RB, int ITEMS, int THREADS, int MODE>
struct PassSmem {
  // keys, then values (as uint32; with 32-bit keys, values and second values
  // as pairs of uint32)
  K buf[THREADS * ITEMS * (sizeof(K) == 4 ? 2 : 1)];
  uint32_t wcnt[(THREADS / kWave) << RB];
  uint32_t dstart[1 << RB];
  uint32_t cnt[1 << RB];    // the tile's count of each digit
  uint32_t gofs[1 << RB];
  // kPassUnpack: per digit, 1 + the largest tile part below the digit among
  // the pairs of earlier workgroups (0: none)
  uint32_t lbx[MODE == kPassUnpack ? (1 << RB) : 1];
  // segmented 64-bit passes: each frame's first tile workgroup; the
  // segmented depth sort: each frame's first Gaussian
  uint32_t aux[kMaxFrames + 1];
  unsigned long long tmp[THREADS / kWave];
  uint32_t timeout;
  uint32_t drop;     // 32-bit keys: this pass drops culled Gaussians
  uint32_t ticket;   // persistent passes: the workgroup's current ticket
};

// Where a workgroup's tile sits in a segmented pass (a frame's first tile
// workgroup, the frame's digit bases, its first global tile); the whole
// sort is one segment otherwise.
struct SegCtx {
  uint32_t first;
  const uint32_t* bases;
  uint32_t tile_base;  // 64-bit unpacking: the frame's first tile; 32-bit
                       // segmented: the frame's first Gaussian
  uint32_t hist_off;   // 32-bit segmented: the frame's histograms
};

// Largest f < n_frames with first[f] <= x (first[] non-decreasing).
__device__ __forceinline__ uint32_t segment_of(const uint32_t* first, uint32_t n_frames, uint32_t x) {
  uint32_t lo = 0, hi = n_frames;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The digit of key k at bit `shift`.  Packed items keep their tile field in
// the high word (shift >= 32): one 32-bit field extract instead of a 64-bit
// shift and a mask.
template <typename K, int MODE, int RB>
__device__ __forceinline__ uint32_t key_digit(K k, uint32_t shift) {
  if constexpr (sizeof(K) == 8 && MODE != kPassKV)
    return __builtin_amdgcn_ubfe(static_cast<uint32_t>(k >> 32), shift - 32, RB);
  else
    return static_cast<uint32_t>(k >> shift) & ((1u << RB) - 1u);
}

// The tile body, in two parts: the loads, then ranking and scatter.  FULL:
// every one of the TILE slots holds a pair (all tiles but the last, unless
// items are dropped), so no per-item bounds tests are needed.  `dropped`
// (32-bit keys): culled items an earlier pass dropped, all of digit 255.
template <typename K, int RB, int ITEMS, int THREADS, int MODE, bool FULL>
__device__ __forceinline__ void pass_load(const PassArgs& a, PassSmem<K, RB, ITEMS, THREADS, MODE>& sm,
                                          uint32_t base, uint32_t n, uint32_t dropped, uint32_t hist_off,
                                          K (&k)[ITEMS], uint32_t (&v)[ITEMS], uint32_t (&dg)[ITEMS]) {
  constexpr int BINS = 1 << RB;
  const int tid = threadIdx.x;
  // 32-bit keys: global total of digit tid (summed over the histogram
  // copies), whose exclusive prefix over the digits is the digit's first
  // output slot; parked in LDS so that no register holds it through the
  // ranking
  if constexpr (sizeof(K) == 4) {
    if (tid < BINS) {
      uint32_t gtot = 0;
#pragma unroll
      for (uint32_t c = 0; c < kHistCopies; ++c) gtot += a.hist[static_cast<size_t>(c) * a.hist_stride + hist_off + tid];
      // culled Gaussians dropped by an earlier pass (all of digit 255)
      if (tid == BINS - 1) gtot -= dropped;
      sm.gofs[tid] = gtot;
    }
  }

  // ---- load (wave-striped) ----
  const K* __restrict__ kin = static_cast<const K*>(a.kin);
  const uint32_t lane = lane_id();
  const uint32_t wave = tid / kWave;
  const uint32_t seg = base + wave * (kWave * ITEMS);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t idx = seg + j * kWave + lane;
    if (FULL || idx < n) {
      k[j] = kin[idx];
      v[j] = MODE == kPassKV ? a.vin[idx] : 0u;
      dg[j] = key_digit<K, MODE, RB>(k[j], a.shift);
    } else {
      k[j] = 0;
      v[j] = 0;
      dg[j] = BINS;  // not a pair
    }
  }
}

// kPassUnpack: the pair at output position o is the first of its tile when
// its predecessor's tile tp is smaller; then o starts tile t, ends tp, and
// every tile between them is empty at o.
__device__ __forceinline__ void range_boundary(uint32_t* __restrict__ ranges, int64_t tp, uint32_t t, uint32_t o) {
  if (tp >= 0) ranges[2 * tp + 1] = o;
  for (int64_t e = tp + 1; e < static_cast<int64_t>(t); ++e) {
    ranges[2 * e] = o;
    ranges[2 * e + 1] = o;
  }
  ranges[2 * static_cast<size_t>(t)] = o;
}

template <typename K, int RB, int ITEMS, int THREADS, int MODE, bool FULL>
__device__ __forceinline__ void pass_rest(const PassArgs& a, PassSmem<K, RB, ITEMS, THREADS, MODE>& sm, uint32_t t,
                                          uint32_t base, uint32_t n, K (&k)[ITEMS], uint32_t (&v)[ITEMS],
                                          uint32_t (&dg)[ITEMS], const SegCtx& sc) {
  constexpr int WAVES = THREADS / kWave;
  constexpr int BINS = 1 << RB;
  constexpr int TILE = THREADS * ITEMS;
  const int tid = threadIdx.x;
  const uint32_t wave = tid / kWave;
  // kPassUnpack: the depth field's form, read now (uniform scalar loads) and
  // used only when writing
  uint32_t top_max = 0, top_min = 0;
  if constexpr (MODE == kPassUnpack) {
    top_max = a.packed.depth_top[0];
    top_min = a.packed.depth_top[1];
  }

  // ---- stable rank inside the wave ----
  // peers = valid lanes whose digit equals this lane's
  uint32_t* wc = sm.wcnt + wave * BINS;
  uint32_t pos[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const bool valid = FULL || dg[j] < BINS;
    const uint64_t peers = match_digit<RB>(dg[j], FULL ? ~0ull : ballot(valid));
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

  // ---- per digit: offsets of the waves, workgroup count, publish ----
  uint32_t bcnt = 0;
  if (tid < BINS) {
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t c = sm.wcnt[w * BINS + tid];
      sm.wcnt[w * BINS + tid] = bcnt;
      bcnt += c;
    }
    // kPassUnpack publishes after the permute, with its largest tile part
    if (MODE != kPassUnpack)
      st_agent(&a.lookback[static_cast<size_t>(t) * BINS + tid], (t == sc.first ? kLbInc32 : kLbAgg32) | bcnt);
  }
  uint32_t gbase, lexcl;
  uint32_t tile_pairs = 0;  // 32-bit keys: valid items of the tile (some may be dropped)
  if constexpr (sizeof(K) == 4) {
    // one scan for both prefixes over the digits: the global digit bases
    // (high word) and this tile's digit starts (low word); neither carries
    const uint32_t gtot = tid < BINS ? sm.gofs[tid] : 0u;
    unsigned long long total;
    const unsigned long long both = block_exclusive_scan<unsigned long long, THREADS>(
        (static_cast<unsigned long long>(gtot) << 32) | bcnt, sm.tmp, total);
    gbase = static_cast<uint32_t>(both >> 32);
    lexcl = static_cast<uint32_t>(both);
    tile_pairs = static_cast<uint32_t>(total);
  } else {
    uint32_t total;
    lexcl = block_exclusive_scan<uint32_t, THREADS>(bcnt, reinterpret_cast<uint32_t*>(sm.tmp), total);
    gbase = 0;  // 64-bit keys: published digit bases, read at the look-back
  }
  if (tid < BINS) {
    sm.dstart[tid] = lexcl;
    sm.cnt[tid] = bcnt;
    if constexpr (sizeof(K) == 4) sm.gofs[tid] = gbase + sc.tile_base;
  }
  __syncthreads();

  // ---- permute the keys into digit order in LDS ----
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (FULL || dg[j] < BINS) {
      pos[j] += sm.dstart[dg[j]] + wc[dg[j]];
      sm.buf[pos[j]] = k[j];
    }
  }
  // 32-bit keys: the second value, loaded now (into the registers the keys
  // leave free) so that its latency hides behind the look-back
  uint32_t pl[ITEMS];
  if constexpr (sizeof(K) == 4) {
    if (a.pin != nullptr) {
      const uint32_t seg = base + wave * (kWave * ITEMS) + lane_id();
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) pl[j] = (FULL || dg[j] < BINS) ? a.pin[seg + j * kWave] : 0u;
    }
  }
  // kPassUnpack: the digit's largest tile part in this workgroup is that of
  // its last slot (the input is in order of the lower tile bits); 1 + it,
  // or 0 for a digit without pairs here
  const uint32_t lowmask = a.low_bits >= 32 ? ~0u : (1u << a.low_bits) - 1u;
  auto own_max_of = [&](uint32_t start, uint32_t count) -> uint32_t {
    return count == 0 ? 0u
                      : 1u + (static_cast<uint32_t>(sm.buf[start + count - 1] >> a.packed.tile_shift) & lowmask);
  };
  if constexpr (MODE == kPassUnpack) {
    __syncthreads();
    if (tid < BINS)
      st_agent(&a.lookback64[static_cast<size_t>(t) * BINS + tid],
               lb_word(t == sc.first ? kLbIncW : kLbAggW, bcnt, own_max_of(lexcl, bcnt)));
  }

  // ---- decoupled look-back: pairs of digit d in earlier workgroups ----
  // G consecutive lanes per digit: two where the workgroup has the threads
  // (16 predecessors per round), except in 16-item passes over pairs, whose
  // long chains of tiles measured faster with one; more lanes spread each
  // load over more rows of the look-back words and measured slower
  constexpr int G = sizeof(K) == 8 && ITEMS >= 16 ? 1 : THREADS / BINS > 2 ? 2 : THREADS / BINS;
  static_assert(G >= 1 && THREADS % BINS == 0, "whole lane groups per digit");
  if (tid < BINS * G) {
    const uint32_t d = static_cast<uint32_t>(tid) / G;
    const uint32_t limit = spin_limit_of(a.spin_limit);
    uint32_t gb;
    if constexpr (sizeof(K) == 8) {
      // published by workgroup 0 of the chain's first pass, long before any
      // workgroup gets here
      uint32_t w = ld_agent(&sc.bases[d]), spins = 0;
      while ((w & kBasePublished) == 0) {
        if (++spins > limit) {
          sm.timeout = 1;
          if (a.status) st_agent(a.status, static_cast<uint32_t>(SS_ERR_TIMEOUT));
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        w = ld_agent(&sc.bases[d]);
      }
      gb = w & ~kBasePublished;
    } else {
      gb = sm.gofs[d];  // the digit's global base, from the scan
    }
    const uint32_t count = sm.cnt[d], start = sm.dstart[d];
    uint32_t excl = 0, excl_max = 0;
    bool ok;
    if constexpr (MODE == kPassUnpack)
      ok = lookback_group<G, LbWords64>(a.lookback64, t, BINS, d, a.status, excl, excl_max, sc.first, limit);
    else
      ok = lookback_group<G, LbWords32>(a.lookback, t, BINS, d, a.status, excl, excl_max, sc.first, limit);
    if (!ok) {
      sm.timeout = 1;
    } else if (static_cast<uint32_t>(tid) % G == 0) {
      // the group's first lane publishes the inclusive word (the chain's
      // first workgroup published its count as inclusive already)
      if (t != sc.first) {
        if constexpr (MODE == kPassUnpack) {
          const uint32_t om = own_max_of(start, count);
          st_agent(&a.lookback64[static_cast<size_t>(t) * BINS + d],
                   lb_word(kLbIncW, excl + count, om > excl_max ? om : excl_max));
        } else {
          st_agent(&a.lookback[static_cast<size_t>(t) * BINS + d], kLbInc32 | (excl + count));
        }
      }
      if constexpr (MODE == kPassUnpack) sm.lbx[d] = excl != 0 ? excl_max : 0u;
      sm.gofs[d] = gb + excl - start;
    }
  }
  __syncthreads();
  if (sm.timeout) return;

  // ---- write keys: LDS slot i goes to global position gofs[digit] + i ----
  K* __restrict__ kout = static_cast<K*>(a.kout);
  // pairs held in LDS: the whole tile, or the valid ones of a partial tile
  // (the tail; with 32-bit keys also a tile with dropped items)
  const uint32_t valid_n = FULL ? TILE
                           : sizeof(K) == 4 ? tile_pairs
                                            : ((n - base) < static_cast<uint32_t>(TILE) ? (n - base) : TILE);
  if constexpr (MODE == kPassUnpack) {
    // packed pair -> (tile << 32 | depth bits, index); tile ranges on the way
    const uint32_t S = a.packed.tile_shift, ib = a.packed.idx_bits;
    uint32_t ebase;
    const bool trimmed = packed_depth_trimmed(top_max, top_min, a.packed, &ebase);
    const uint64_t pmask = (1ull << S) - 1;
    const uint32_t imask = ib >= 32 ? ~0u : (1u << ib) - 1u;
    // one loop per form of the depth field, so that neither carries the
    // other's test per item
    auto write_all = [&](auto trim) {
      constexpr bool kTrimmed = decltype(trim)::value;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = j * THREADS + tid;
        if (FULL || i < valid_n) {
          const uint64_t item = sm.buf[i];
          const uint32_t d = key_digit<K, MODE, RB>(item, a.shift);
          const uint32_t o = sm.gofs[d] + i;
          if (o < n) {
            const uint32_t tile = sc.tile_base + (static_cast<uint32_t>(item >> 32) >> (S - 32));
            const uint64_t payload = item & pmask;
            const uint32_t hi = static_cast<uint32_t>(payload >> ib);
            const uint32_t dbits = kTrimmed ? hi + ebase : a.packed.depth_sorted[hi];
            kout[o] = (static_cast<uint64_t>(tile) << 32) | dbits;
            a.vout[o] = static_cast<uint32_t>(payload) & imask;
            // predecessor: the slot before, inside this digit's run; else the
            // last pair of the digit in earlier workgroups; else (the digit's
            // first pair overall) left to k_ranges_fix
            int64_t tp = -1;
            bool known = true;
            if (i > sm.dstart[d]) {
              tp = static_cast<int64_t>(sc.tile_base + (static_cast<uint32_t>(sm.buf[i - 1] >> 32) >> (S - 32)));
            } else {
              const uint32_t lx = sm.lbx[d];
              known = lx != 0;
              tp = sc.tile_base + ((static_cast<int64_t>(d) << a.low_bits) | static_cast<int64_t>(lx - 1u));
            }
            if (known && tp != static_cast<int64_t>(tile)) range_boundary(a.ranges, tp, tile, o);
          }
        }
      }
    };
    if (trimmed) write_all(std::true_type{});
    else write_all(std::false_type{});
    return;
  }
  // Packed pairs in 16-item tiles (the shape for 2^23 pairs and more, which
  // outgrow the caches before the next pass reads them back): non-temporal
  // stores, measured faster there (large-6m passes 293 -> 285 us) and slower
  // on smaller frames, whose outputs the next pass still finds in cache, and
  // in key + value passes, whose values would stay cached without their keys
  constexpr bool kStreamStores = MODE == kPassItems && ITEMS == 16;
  uint32_t dst[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t i = j * THREADS + tid;
    dst[j] = 0xFFFFFFFFu;
    if (FULL || i < valid_n) {
      const K key = sm.buf[i];
      const uint32_t d = key_digit<K, MODE, RB>(key, a.shift);
      const uint32_t o = sm.gofs[d] + i;
      if (o < n) {
        if constexpr (kStreamStores) __builtin_nontemporal_store(key, &kout[o]);
        else kout[o] = key;
        dst[j] = o;
      }
    }
  }
  if constexpr (MODE == kPassItems) return;
  __syncthreads();

  // ---- values through the same buffer (with a second value: both as a
  // pair, in one round) ----
  if constexpr (sizeof(K) == 4) {
    if (a.pin != nullptr) {
      uint2* s_two = reinterpret_cast<uint2*>(sm.buf);
#pragma unroll
      for (int j = 0; j < ITEMS; ++j)
        if (FULL || dg[j] < BINS) s_two[pos[j]] = make_uint2(v[j], pl[j]);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = j * THREADS + tid;
        if (dst[j] != 0xFFFFFFFFu) {
          const uint2 vp = s_two[i];
          a.vout[dst[j]] = vp.x;
          a.pout[dst[j]] = vp.y;
        }
      }
      return;
    }
  }
  uint32_t* s_val = reinterpret_cast<uint32_t*>(sm.buf);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (FULL || dg[j] < BINS) s_val[pos[j]] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t i = j * THREADS + tid;
    if (dst[j] != 0xFFFFFFFFu) a.vout[dst[j]] = s_val[i];
  }
}

template <typename K, int RB, int ITEMS, int THREADS, int MODE, bool FULL>
__device__ __forceinline__ void pass_tile(const PassArgs& a, PassSmem<K, RB, ITEMS, THREADS, MODE>& sm, uint32_t t,
                                          uint32_t base, uint32_t n, uint32_t dropped, const SegCtx& sc) {
  K k[ITEMS];
  uint32_t v[ITEMS];
  uint32_t dg[ITEMS];
  pass_load<K, RB, ITEMS, THREADS, MODE, FULL>(a, sm, base, n, dropped, sc.hist_off, k, v, dg);
  pass_rest<K, RB, ITEMS, THREADS, MODE, FULL>(a, sm, t, base, n, k, v, dg, sc);
}

// The extra workgroup of a chain's first 64-bit pass: digit bases of
// publish_passes passes from the histogram copies, published with bit 31 set
// (the current pass's first, since this launch's tiles need those now).
template <int RB, int THREADS>
__device__ __forceinline__ void publish_bases(const PassArgs& a, uint32_t* s_tmp) {
  constexpr int BINS = 1 << RB;
  const int tid = threadIdx.x;
  if (a.fault == SS_FAULT_WITHHOLD_BASES) return;
  for (uint32_t q = 0; q < a.publish_passes; ++q) {
    uint32_t tot = 0;
    if (tid < BINS) {
#pragma unroll
      for (uint32_t c = 0; c < kHistCopies; ++c)
        tot += a.hist[static_cast<size_t>(c) * a.hist_stride + q * BINS + tid];
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_scan<uint32_t, THREADS>(tot, s_tmp, all);
    if (tid < BINS) st_agent(&a.bases[q * BINS + tid], ex | kBasePublished);
  }
}

// The depth sort's first pass, workgroup 0, after its tile: the largest and
// smallest top byte of the depth keys of Gaussians with pairs (positive
// depths have a top byte below 128; culled keys sit in bin 255).
template <int THREADS>
__device__ __forceinline__ void store_depth_top(const PassArgs& a, uint32_t* s2) {
  __syncthreads();
  if (threadIdx.x == 0) {
    s2[0] = 0;
    s2[1] = 0xFF;
  }
  __syncthreads();
  if (threadIdx.x < 128) {
    uint32_t c = 0;
#pragma unroll
    for (uint32_t k = 0; k < kHistCopies; ++k) c += a.hist_top[static_cast<size_t>(k) * a.hist_stride + threadIdx.x];
    if (c != 0) {
      atomicMax(&s2[0], static_cast<uint32_t>(threadIdx.x));
      atomicMin(&s2[1], static_cast<uint32_t>(threadIdx.x));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.depth_top_out[0] = s2[0];
    a.depth_top_out[1] = s2[1] <= s2[0] ? s2[1] : 0u;
  }
}

template <typename K, int RB, int ITEMS, int THREADS, int MODE, bool DROP>
__device__ __forceinline__ bool onesweep_body(const PassArgs& a, PassSmem<K, RB, ITEMS, THREADS, MODE>& sm,
                                              uint32_t t);

// Segmented: publishing workgroup f computes frame f's digit bases for
// publish_passes passes (from the frame's histograms) and offsets them by the
// frame's first pair.
template <int RB, int THREADS>
__device__ __forceinline__ void publish_bases_seg(const PassArgs& a, uint32_t f, uint32_t* s_tmp) {
  constexpr int BINS = 1 << RB;
  const int tid = threadIdx.x;
  if (a.fault == SS_FAULT_WITHHOLD_BASES) return;
  const uint32_t first = a.seg_base[f];
  const size_t fo = static_cast<size_t>(f) * a.bases_frame_stride;
  for (uint32_t q = 0; q < a.publish_passes; ++q) {
    uint32_t tot = 0;
    if (tid < BINS) {
#pragma unroll
      for (uint32_t c = 0; c < kHistCopies; ++c)
        tot += a.hist[static_cast<size_t>(c) * a.hist_stride + fo + q * BINS + tid];
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_scan<uint32_t, THREADS>(tot, s_tmp, all);
    if (tid < BINS) st_agent(&a.bases[fo + q * BINS + tid], (first + ex) | kBasePublished);
  }
}

// DROP (32-bit keys, the depth sort's first pass): may drop the culled
// Gaussians (the decision is known only after the loads).  Workgroup b is
// tile b (after the publishing workgroups).
template <typename K, int RB, int ITEMS, int THREADS, int MODE, bool DROP>
__global__ __launch_bounds__(THREADS) void k_onesweep(PassArgs a) {
  __shared__ PassSmem<K, RB, ITEMS, THREADS, MODE> sm;
  if (a.status && *a.status != SS_OK) return;
  onesweep_body<K, RB, ITEMS, THREADS, MODE, DROP>(a, sm, blockIdx.x);
  if constexpr (sizeof(K) == 4) {
    if (a.depth_top_out != nullptr && blockIdx.x == 0) store_depth_top<THREADS>(a, sm.dstart);
  }
}

// Persistent form (64-bit keys, 512 threads, a.tickets): tickets in order
// until one lies past the last tile.  A ticket is taken only by a running
// workgroup, so every ticket a tile waits on (publishers, earlier tiles) is
// held by one that runs too.  The loop would keep more registers live than
// the one-tile kernel's; the bounds hold it to the waves per SIMD that the
// tile's LDS allows anyway (4 with 16 items, 6 with 8).
template <typename K, int RB, int ITEMS, int THREADS, int MODE>
__global__ __launch_bounds__(THREADS, ITEMS >= 16 ? 4 : 6) void k_onesweep_persistent(PassArgs a) {
  __shared__ PassSmem<K, RB, ITEMS, THREADS, MODE> sm;
  if (a.status && *a.status != SS_OK) return;
  while (true) {
    if (threadIdx.x == 0)
      sm.ticket = a.status && ld_agent(a.status) != SS_OK ? 0xFFFFFFFFu : atomicAdd(a.tickets, 1u);
    __syncthreads();
    const uint32_t t = sm.ticket;
    if (t == 0xFFFFFFFFu || !onesweep_body<K, RB, ITEMS, THREADS, MODE, false>(a, sm, t)) break;
    __syncthreads();  // every thread is done with this ticket's LDS
  }
}

// Workgroup (or ticket) t.  Returns false when t lies past the pass's last
// tile (a persistent workgroup then stops taking tickets).
template <typename K, int RB, int ITEMS, int THREADS, int MODE, bool DROP>
__device__ __forceinline__ bool onesweep_body(const PassArgs& a, PassSmem<K, RB, ITEMS, THREADS, MODE>& sm,
                                              uint32_t t) {
  constexpr int TILE = THREADS * ITEMS;
  const uint32_t n = a.num_pairs ? *a.num_pairs : a.n_fixed;
  const int tid = threadIdx.x;
  if (tid == 0) sm.timeout = 0;
  for (int i = tid; i < (THREADS / kWave) << RB; i += THREADS) sm.wcnt[i] = 0;
  __syncthreads();
  // In a chain's first 64-bit pass workgroup 0 only publishes the digit
  // bases (dispatched first, it has them out before any tile needs them, and
  // no tile's look-back waits on it); tile b is then workgroup b + 1.  A
  // segmented chain has one publishing workgroup per frame.
  SegCtx sc{0u, a.bases, 0u, 0u};
  uint32_t base = 0, end = n;
  if constexpr (sizeof(K) == 8) {
    const uint32_t publishers = a.publish_passes == 0 ? 0u : a.seg_wgs != nullptr ? a.seg_frames : 1u;
    if (t < publishers) {
      if (a.seg_wgs != nullptr)
        publish_bases_seg<RB, THREADS>(a, t, reinterpret_cast<uint32_t*>(sm.tmp));
      else
        publish_bases<RB, THREADS>(a, reinterpret_cast<uint32_t*>(sm.tmp));
      return true;
    }
    t -= publishers;
    if (a.seg_wgs != nullptr) {
      // this workgroup's frame, and its tile inside the frame's pairs
      for (uint32_t i = tid; i <= a.seg_frames; i += THREADS) sm.aux[i] = a.seg_wgs[i];
      __syncthreads();
      if (t >= sm.aux[a.seg_frames]) return false;   // more workgroups than the frames' tiles
      const uint32_t f = segment_of(sm.aux, a.seg_frames, t);
      sc.first = sm.aux[f];
      sc.bases = a.bases + static_cast<size_t>(f) * a.bases_frame_stride;
      if (MODE == kPassUnpack) sc.tile_base = a.table[f].tile_base;
      base = a.seg_base[f] + (t - sc.first) * TILE;
      end = a.seg_base[f + 1];
    } else {
      base = t * TILE;
    }
  } else {
    base = t * TILE;
    if (a.depth_seg) {
      // this workgroup's frame and its tile inside the frame's Gaussians:
      // the frames' first tile workgroups by a scan of their tile counts
      // (parked in the permute buffer, free until the tile is ranked)
      static_assert(THREADS >= kMaxFrames, "one frame per thread in the scan");
      uint32_t* s_wgs = reinterpret_cast<uint32_t*>(sm.buf);
      for (uint32_t i = tid; i <= a.n_frames; i += THREADS) sm.aux[i] = i < a.n_frames ? a.table[i].gauss_base : n;
      __syncthreads();
      const uint32_t nf = static_cast<uint32_t>(tid) < a.n_frames ? sm.aux[tid + 1] - sm.aux[tid] : 0u;
      uint32_t tiles_all;
      const uint32_t first_wg = block_exclusive_scan<uint32_t, THREADS>(
          (nf + TILE - 1) / TILE, reinterpret_cast<uint32_t*>(sm.tmp), tiles_all);
      if (static_cast<uint32_t>(tid) <= a.n_frames) s_wgs[tid] = static_cast<uint32_t>(tid) < a.n_frames ? first_wg : tiles_all;
      __syncthreads();
      if (t >= tiles_all) return false;  // more workgroups than the frames' tiles (uniform)
      const uint32_t f = segment_of(s_wgs, a.n_frames, t);
      sc.first = s_wgs[f];
      sc.tile_base = sm.aux[f];
      sc.hist_off = f * 4u * 256u;
      base = sm.aux[f] + (t - s_wgs[f]) * TILE;
      end = sm.aux[f + 1];
      __syncthreads();  // s_wgs is the permute buffer
    }
  }
  if (base >= end) return false;  // uniform over the workgroup
  if constexpr (!DROP) {
    const uint32_t dropped = sizeof(K) == 4 && a.n_total != 0 ? a.n_total - n : 0u;
    if (end - base >= static_cast<uint32_t>(TILE))
      pass_tile<K, RB, ITEMS, THREADS, MODE, true>(a, sm, t, base, end, dropped, sc);
    else
      pass_tile<K, RB, ITEMS, THREADS, MODE, false>(a, sm, t, base, end, dropped, sc);
  } else {
    // the loads go out before the drop decision (one thread's reads of the
    // culled count), which only marks the culled as not pairs
    K k[ITEMS];
    uint32_t v[ITEMS];
    uint32_t dg[ITEMS];
    pass_load<K, RB, ITEMS, THREADS, MODE, false>(a, sm, base, n, 0u, 0u, k, v, dg);
    if (tid == 0) {
      // drop when the culled are more than n / 16 (the same decision in
      // every workgroup)
      uint32_t c = 0;
#pragma unroll
      for (uint32_t i = 0; i < kHistCopies; ++i) c += a.culled[static_cast<size_t>(i) * a.hist_stride];
      const bool d = static_cast<unsigned long long>(c) * 16 > n;
      if (t == 0) st_agent(a.kept, d ? n - c : n);
      sm.drop = d;
    }
    __syncthreads();
    if (sm.drop) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j)
        if (k[j] == 0xFFFFFFFFu) dg[j] = 1u << RB;  // culled Gaussian: not a pair
    }
    // a full tile that drops nothing is ranked without validity tests where
    // the second variant fits the registers (up to 12 items per thread)
    if constexpr (ITEMS <= 12) {
      if (n - base >= static_cast<uint32_t>(TILE) && !sm.drop) {
        pass_rest<K, RB, ITEMS, THREADS, MODE, true>(a, sm, t, base, n, k, v, dg, sc);
        return true;
      }
    }
    pass_rest<K, RB, ITEMS, THREADS, MODE, false>(a, sm, t, base, n, k, v, dg, sc);
  }
  return true;
}

// Workgroups of this kernel that the device holds at once (persistent
// passes), from its occupancy and the device's CU count; 0 if unknown.
template <typename K, int RB, int ITEMS, int THREADS, int MODE>
uint32_t resident_workgroups() {
  static const uint32_t n = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_onesweep_persistent<K, RB, ITEMS, THREADS, MODE>), THREADS,
            0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0u;
    return static_cast<uint32_t>(per_cu > 0 && cus > 0 ? per_cu * cus : 0);
  }();
  return n;
}

template <typename K, int RB, int ITEMS, int THREADS, int MODE>
hipError_t pass_launch(const PassArgs& a, uint32_t nblocks, hipStream_t s) {
  const uint32_t publishers = a.publish_passes == 0 ? 0u : a.seg_wgs != nullptr ? a.seg_frames : 1u;
  uint32_t grid = nblocks + (sizeof(K) == 8 ? publishers : 0u);
  if constexpr (sizeof(K) == 8 && THREADS == 512) {
    if (a.tickets != nullptr) {
      const uint32_t r = resident_workgroups<K, RB, ITEMS, THREADS, MODE>();
      if (r == 0) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_onesweep_persistent<K, RB, ITEMS, THREADS, MODE>), dim3(grid < r ? grid : r),
                         dim3(THREADS), 0, s, a);
      return hipGetLastError();
    }
  }
  if (a.tickets != nullptr) return hipErrorInvalidValue;  // persistent: 512-thread 64-bit passes only
  if constexpr (sizeof(K) == 4) {
    if (a.culled != nullptr) {
      hipLaunchKernelGGL((k_onesweep<K, RB, ITEMS, THREADS, MODE, true>), dim3(grid), dim3(THREADS), 0, s, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_onesweep<K, RB, ITEMS, THREADS, MODE, false>), dim3(grid), dim3(THREADS), 0, s, a);
  return hipGetLastError();
}

// One workgroup: the boundary at each digit's first pair (its predecessor
// lies in the previous non-empty digit's run) and the tiles after the last
// pair; with no pairs every range is [0, 0).  `bins`: the digits of the last
// pass's instantiation (every one of their bases is published).
__global__ __launch_bounds__(256) void k_ranges_fix(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ num_pairs,
                                                    const uint32_t* __restrict__ status,
                                                    const uint32_t* __restrict__ bases, uint32_t bins,
                                                    uint32_t num_tiles, uint32_t* __restrict__ ranges) {
  if (status && *status != SS_OK) return;
  const uint32_t m = *num_pairs;
  for (uint32_t d = threadIdx.x; d < bins; d += blockDim.x) {
    const uint32_t o = bases[d] & ~kBasePublished;
    const uint32_t next = d + 1 < bins ? bases[d + 1] & ~kBasePublished : m;
    if (next > o && o < m) {
      const int64_t tp = o == 0 ? -1 : static_cast<int64_t>(keys[o - 1] >> 32);
      const uint32_t tile = static_cast<uint32_t>(keys[o] >> 32);
      if (tp != static_cast<int64_t>(tile)) range_boundary(ranges, tp, tile, o);
    }
  }
  // after the last pair (tile tl): tl ends at m, later tiles are [m, m)
  const int64_t tl = m == 0 ? -1 : static_cast<int64_t>(keys[m - 1] >> 32);
  if (threadIdx.x == 0 && tl >= 0) ranges[2 * tl + 1] = m;
  for (int64_t e = tl + 1 + threadIdx.x; e < static_cast<int64_t>(num_tiles); e += blockDim.x) {
    ranges[2 * e] = m;
    ranges[2 * e + 1] = m;
  }
}

// One workgroup per frame of a segmented batch: the frame's tiles before its
// first pair start (and end) at its first pair, each digit's first pair
// starts a range, and the tiles after its last pair are empty at its end.
__global__ __launch_bounds__(256) void k_ranges_fix_seg(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ status,
                                                        const uint32_t* __restrict__ bases, uint32_t bins,
                                                        uint32_t frame_stride, const uint32_t* __restrict__ seg_base,
                                                        const FrameInfo* __restrict__ table,
                                                        uint32_t* __restrict__ ranges) {
  if (status && *status != SS_OK) return;
  const uint32_t f = blockIdx.x;
  const uint32_t lo = seg_base[f], hi = seg_base[f + 1];
  const uint32_t t0 = table[f].tile_base, t1 = t0 + table[f].tiles_x * table[f].tiles_y;
  const uint32_t* b = bases + static_cast<size_t>(f) * frame_stride;
  for (uint32_t d = threadIdx.x; d < bins; d += blockDim.x) {
    const uint32_t o = b[d] & ~kBasePublished;
    const uint32_t next = d + 1 < bins ? b[d + 1] & ~kBasePublished : hi;
    if (next > o && o < hi) {
      const uint32_t tile = static_cast<uint32_t>(keys[o] >> 32);
      if (tile < t0 || tile >= t1) continue;  // not this frame's: never so for a sorted frame
      if (o == lo) {
        // the frame's first pair: its lower tiles are empty at lo
        for (uint32_t e = t0; e < tile; ++e) {
          ranges[2 * e] = lo;
          ranges[2 * e + 1] = lo;
        }
        ranges[2 * tile] = lo;
      } else {
        const int64_t tp = static_cast<int64_t>(keys[o - 1] >> 32);
        if (tp >= t0 && tp < tile) range_boundary(ranges, tp, tile, o);
      }
    }
  }
  // after the frame's last pair (tile tl): tl ends at hi, later tiles are [hi, hi)
  int64_t tl = hi == lo ? static_cast<int64_t>(t0) - 1 : static_cast<int64_t>(keys[hi - 1] >> 32);
  if (tl >= static_cast<int64_t>(t1)) tl = static_cast<int64_t>(t1) - 1;  // (as above)
  if (threadIdx.x == 0 && tl >= static_cast<int64_t>(t0)) ranges[2 * tl + 1] = hi;
  for (int64_t e = tl + 1 + threadIdx.x; e < static_cast<int64_t>(t1); e += blockDim.x) {
    ranges[2 * e] = hi;
    ranges[2 * e + 1] = hi;
  }
}

}  // namespace

bool pass_config_supported(int radix_bits, int items, int threads) {
  const bool rb_ok = radix_bits == 4 || radix_bits == 6 || radix_bits == 8;
  const bool it_ok = items == 8 || items == 12 || items == 16;
  const bool th_ok = threads == 256 || (threads == 512 && (items == 8 || items == 16));
  return rb_ok && it_ok && th_ok;
}

bool packed_pass_supported(int radix_bits, int items, int threads) {
  return threads == 512 && (items == 8 || items == 16) && radix_bits >= 4 && radix_bits <= 8;
}

int narrow_pass_bits(int bits, int key_bytes, int radix_bits, int items, int threads) {
  // compiled narrow widths: 64-bit keys, 4..7-bit passes of 512 threads
  if (key_bytes != 8 || radix_bits < 5 || radix_bits > 8 || threads != 512 || (items != 8 && items != 16)) return 0;
  if (bits <= 4) return 4;
  return bits < radix_bits ? bits : 0;
}

hipError_t launch_pass(const PassArgs& a, int key_bytes, int radix_bits, int items, int threads, uint32_t nblocks,
                       hipStream_t s, int mode) {
  if (nblocks == 0) return hipSuccess;
#define SS_PASS_CASE(K, RB, IT, TH)                                                                        \
  if (mode == kPassKV && key_bytes == sizeof(K) && radix_bits == RB && items == IT && threads == TH) \
    return pass_launch<K, RB, IT, TH, kPassKV>(a, nblocks, s);
  SS_PASS_CASE(uint64_t, 8, 16, 256) SS_PASS_CASE(uint64_t, 8, 12, 256) SS_PASS_CASE(uint64_t, 8, 8, 256)
  SS_PASS_CASE(uint64_t, 6, 16, 256) SS_PASS_CASE(uint64_t, 6, 12, 256) SS_PASS_CASE(uint64_t, 6, 8, 256)
  SS_PASS_CASE(uint64_t, 4, 16, 256) SS_PASS_CASE(uint64_t, 4, 12, 256) SS_PASS_CASE(uint64_t, 4, 8, 256)
  SS_PASS_CASE(uint64_t, 8, 16, 512) SS_PASS_CASE(uint64_t, 8, 8, 512)
  SS_PASS_CASE(uint64_t, 7, 16, 512) SS_PASS_CASE(uint64_t, 7, 8, 512)
  SS_PASS_CASE(uint64_t, 6, 16, 512) SS_PASS_CASE(uint64_t, 6, 8, 512)
  SS_PASS_CASE(uint64_t, 5, 16, 512) SS_PASS_CASE(uint64_t, 5, 8, 512)
  SS_PASS_CASE(uint64_t, 4, 16, 512) SS_PASS_CASE(uint64_t, 4, 8, 512)
  // the Gaussian depth sort's shapes
  SS_PASS_CASE(uint32_t, 8, 16, 512) SS_PASS_CASE(uint32_t, 8, 8, 512) SS_PASS_CASE(uint32_t, 8, 4, 1024)
#undef SS_PASS_CASE
  // packed pairs: 512-thread shapes, 4..8-bit digits
#define SS_PACKED_CASE(RB, IT)                                                      \
  if (key_bytes == 8 && radix_bits == RB && items == IT && threads == 512) {        \
    if (mode == kPassItems) return pass_launch<uint64_t, RB, IT, 512, kPassItems>(a, nblocks, s);   \
    if (mode == kPassUnpack) return pass_launch<uint64_t, RB, IT, 512, kPassUnpack>(a, nblocks, s); \
  }
  SS_PACKED_CASE(8, 16) SS_PACKED_CASE(8, 8) SS_PACKED_CASE(7, 16) SS_PACKED_CASE(7, 8)
  SS_PACKED_CASE(6, 16) SS_PACKED_CASE(6, 8) SS_PACKED_CASE(5, 16) SS_PACKED_CASE(5, 8)
  SS_PACKED_CASE(4, 16) SS_PACKED_CASE(4, 8)
#undef SS_PACKED_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_ranges_fix_seg(const uint64_t* keys, const uint32_t* status, const uint32_t* bases, uint32_t bins,
                                 uint32_t frame_stride, const uint32_t* seg_base, const FrameInfo* table,
                                 uint32_t n_frames, uint32_t* ranges, hipStream_t s) {
  if (n_frames == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ranges_fix_seg, dim3(n_frames), dim3(256), 0, s, keys, status, bases, bins, frame_stride,
                     seg_base, table, ranges);
  return hipGetLastError();
}

hipError_t launch_ranges_fix(const uint64_t* keys, const uint32_t* num_pairs, const uint32_t* status,
                             const uint32_t* bases, uint32_t bins, uint32_t num_tiles, uint32_t* ranges,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_ranges_fix, dim3(1), dim3(256), 0, s, keys, num_pairs, status, bases, bins, num_tiles,
                     ranges);
  return hipGetLastError();
}

}  // namespace ss

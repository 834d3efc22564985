// One digit pass of the stable LSD radix sort of (64-bit key, 32-bit value)
// pairs (paper: Background, "Sorting" -- by tile, then by depth; Design,
// "Sorting Optimizations in Context of 3DGS" -- the original method sorts a
// 64-bit integer key).  Single-pass ("onesweep") scatter: the global digit
// counts are known beforehand (gathered while the pairs were produced), so a
// workgroup needs only the counts of its digit in earlier workgroups, which it
// gets by a decoupled look-back, and then scatters its tile straight to the
// output.  One read and one write of every pair per pass.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

// Workgroup of 256 threads (4 waves), ITEMS pairs per thread.  Pairs are
// loaded wave-striped: wave w owns the contiguous segment
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
// digit order in LDS and written out so that runs of one digit land on
// consecutive addresses.
template <int RB, int ITEMS>
__global__ __launch_bounds__(kPassThreads) void k_onesweep(PassArgs a) {
  constexpr int THREADS = kPassThreads;
  constexpr int WAVES = THREADS / kWave;
  constexpr int BINS = 1 << RB;
  constexpr uint32_t DMASK = BINS - 1;
  constexpr int TILE = THREADS * ITEMS;
  constexpr int DPT = (BINS + THREADS - 1) / THREADS;  // digits per thread
  static_assert(BINS <= THREADS * DPT, "digit ownership");

  __shared__ uint64_t s_keys[TILE];
  __shared__ uint32_t s_vals[TILE];
  __shared__ uint32_t s_wcnt[WAVES * BINS];
  __shared__ uint32_t s_dstart[BINS];
  __shared__ uint32_t s_gofs[BINS];
  __shared__ uint32_t s_tmp[WAVES];
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t s_timeout;

  if (a.status && *a.status != SS_OK) return;
  const uint32_t n = a.num_pairs ? *a.num_pairs : a.n_fixed;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_ticket = atomicAdd(a.ticket, 1u);
    s_timeout = 0;
  }
  for (int i = tid; i < WAVES * BINS; i += THREADS) s_wcnt[i] = 0;
  __syncthreads();
  const uint32_t t = s_ticket;
  const uint32_t base = t * TILE;
  if (base >= n) return;  // uniform over the workgroup

  // ---- global digit totals (sum of the histogram copies) ----
  uint32_t gcnt[DPT];
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = tid * DPT + i;
    uint32_t s = 0;
    if (d < BINS)
      for (uint32_t c = 0; c < kHistCopies; ++c) s += a.hist[c * a.hist_stride + d];
    gcnt[i] = s;
  }

  // ---- load (wave-striped) ----
  const uint32_t lane = lane_id();
  const uint32_t wave = tid / kWave;
  const uint32_t seg = base + wave * (kWave * ITEMS);
  uint64_t k[ITEMS];
  uint32_t v[ITEMS];
  uint32_t dg[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint32_t idx = seg + j * kWave + lane;
    if (idx < n) {
      k[j] = a.kin[idx];
      v[j] = a.vin[idx];
      dg[j] = static_cast<uint32_t>(k[j] >> a.shift) & DMASK;
    } else {
      k[j] = 0;
      v[j] = 0;
      dg[j] = BINS;  // not a pair
    }
  }

  // ---- stable rank inside the wave ----
  uint32_t* wc = s_wcnt + wave * BINS;
  uint32_t rank[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const bool valid = dg[j] < BINS;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const bool bit = (dg[j] >> b) & 1u;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    uint32_t r = 0;
    if (valid) {
      const uint32_t old = wc[dg[j]];
      const uint32_t below = popc_below(peers);
      r = old + below;
      __builtin_amdgcn_wave_barrier();
      if (below == 0) wc[dg[j]] = old + static_cast<uint32_t>(__popcll(peers));
    }
    __builtin_amdgcn_wave_barrier();
    rank[j] = r;
  }
  __syncthreads();

  // ---- per digit: offsets of the waves, workgroup count, publish ----
  uint32_t bcnt[DPT];
  uint32_t tsum = 0, gsum = 0;
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int d = tid * DPT + i;
    uint32_t s = 0;
    if (d < BINS) {
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_wcnt[w * BINS + d];
        s_wcnt[w * BINS + d] = s;
        s += c;
      }
      st_agent(&a.lookback[static_cast<size_t>(t) * BINS + d], (t == 0 ? kLbInc32 : kLbAgg32) | s);
    }
    bcnt[i] = s;
    tsum += s;
    gsum += gcnt[i];
  }
  uint32_t total;
  const uint32_t lexcl = block_exclusive_scan<uint32_t, THREADS>(tsum, s_tmp, total);
  const uint32_t gexcl = block_exclusive_scan<uint32_t, THREADS>(gsum, s_tmp, total);
  {
    uint32_t run = lexcl;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = tid * DPT + i;
      if (d < BINS) s_dstart[d] = run;
      run += bcnt[i];
    }
  }
  __syncthreads();

  // ---- permute the tile into digit order in LDS ----
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (dg[j] < BINS) {
      const uint32_t pos = s_dstart[dg[j]] + wc[dg[j]] + rank[j];
      s_keys[pos] = k[j];
      s_vals[pos] = v[j];
    }
  }

  // ---- decoupled look-back: pairs of digit d in earlier workgroups ----
  {
    uint32_t grun = gexcl;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int d = tid * DPT + i;
      if (d < BINS) {
        uint32_t excl = 0;
        if (t > 0) {
          int32_t kb = static_cast<int32_t>(t) - 1;
          uint32_t spins = 0;
          while (true) {
            const uint32_t w = ld_agent(&a.lookback[static_cast<size_t>(kb) * BINS + d]);
            if ((w & ~kLbMask32) == 0) {
              if (++spins > kSpinLimit) {
                s_timeout = 1;
                if (a.status) st_agent(a.status, static_cast<uint32_t>(SS_ERR_TIMEOUT));
                break;
              }
              __builtin_amdgcn_s_sleep(1);
              continue;
            }
            excl += w & kLbMask32;
            if (w & kLbInc32) break;
            --kb;
          }
          st_agent(&a.lookback[static_cast<size_t>(t) * BINS + d], kLbInc32 | (excl + bcnt[i]));
        }
        s_gofs[d] = grun + excl - s_dstart[d];
      }
      grun += gcnt[i];
    }
  }
  __syncthreads();
  if (s_timeout) return;

  // ---- write out: LDS slot i goes to global position gofs[digit] + i ----
  const uint32_t valid_n = (n - base) < static_cast<uint32_t>(TILE) ? (n - base) : TILE;
  for (uint32_t i = tid; i < valid_n; i += THREADS) {
    const uint64_t key = s_keys[i];
    const uint32_t d = static_cast<uint32_t>(key >> a.shift) & DMASK;
    const uint32_t o = s_gofs[d] + i;
    if (o < n) {
      a.kout[o] = key;
      a.vout[o] = s_vals[i];
    }
  }
}

template <int RB, int ITEMS>
hipError_t pass_launch(const PassArgs& a, uint32_t nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_onesweep<RB, ITEMS>), dim3(nblocks), dim3(kPassThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

bool pass_config_supported(int radix_bits, int items) {
  const bool rb_ok = radix_bits == 4 || radix_bits == 6 || radix_bits == 8;
  const bool it_ok = items == 8 || items == 12 || items == 16;
  return rb_ok && it_ok;
}

hipError_t launch_pass(const PassArgs& a, int radix_bits, int items, uint32_t nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
#define SS_PASS_CASE(RB, IT) \
  if (radix_bits == RB && items == IT) return pass_launch<RB, IT>(a, nblocks, s);
  SS_PASS_CASE(8, 16) SS_PASS_CASE(8, 12) SS_PASS_CASE(8, 8)
  SS_PASS_CASE(6, 16) SS_PASS_CASE(6, 12) SS_PASS_CASE(6, 8)
  SS_PASS_CASE(4, 16) SS_PASS_CASE(4, 12) SS_PASS_CASE(4, 8)
#undef SS_PASS_CASE
  return hipErrorInvalidValue;
}

}  // namespace ss

// Internal launch interface between the host ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "splatsort.h"

namespace ss {

// Gaussians per workgroup of the fused count / scan / duplicate kernel.
constexpr uint32_t kCountTile = 1024;
// Histogram copies: workgroups spread their global atomics over this many
// copies to cut same-address contention; passes sum the copies.
constexpr uint32_t kHistCopies = 8;

struct CountDupArgs {
  const ss_gaussian2d* gaussians;
  uint32_t n;
  uint32_t tiles_x, tiles_y;
  uint32_t capacity;        // pairs that may be written; 0 with dup = false
  uint32_t npasses;         // sort passes whose digit histograms are gathered
  uint32_t* tiles_touched;  // optional [n]
  uint32_t* offsets;        // optional [n]
  uint64_t* keys;           // [capacity] unsorted pairs
  uint32_t* values;
  uint32_t* ticket;         // zeroed counter
  uint64_t* lookback;       // zeroed [nblocks]
  uint32_t* hist;           // zeroed [kHistCopies][npasses][bins]
  uint32_t* num_pairs;
  uint32_t* status;
  uint32_t nblocks;
};

struct PassArgs {
  const void* kin;            // uint64_t or uint32_t keys
  const uint32_t* vin;
  void* kout;
  uint32_t* vout;
  const uint32_t* num_pairs;  // device M; NULL means n_fixed
  uint32_t n_fixed;
  uint32_t* status;           // device status word or NULL
  uint32_t shift;             // first key bit of this digit
  const uint32_t* bases;      // [bins] exclusive prefix of this pass's digit totals
  uint32_t* ticket;           // zeroed counter
  uint32_t* lookback;         // zeroed [nblocks][bins]
};

struct HistArgs {
  const uint64_t* keys;
  uint32_t n;
  uint32_t npasses;
  uint32_t* hist;             // zeroed [kHistCopies][npasses][bins]
};

// Zeroes `bytes` (a multiple of 16) at p and, if not NULL, the word `extra`.
hipError_t launch_clear(void* p, size_t bytes, uint32_t* extra, hipStream_t s);
hipError_t launch_count_dup(const CountDupArgs& a, int radix_bits, bool dup, hipStream_t s);
hipError_t launch_ranges(const uint64_t* keys, const uint32_t* num_pairs, const uint32_t* status,
                         uint32_t capacity, uint32_t num_tiles, uint32_t* ranges, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_hist(const HistArgs& a, int radix_bits, hipStream_t s);
// bases[p][d] = sum over histogram copies and digits d' < d of hist[c][p][d'].
hipError_t launch_digit_bases(const uint32_t* hist, uint32_t npasses, uint32_t* bases, int radix_bits,
                              hipStream_t s);
hipError_t launch_pass(const PassArgs& a, int key_bytes, int radix_bits, int items, int threads, uint32_t nblocks,
                       hipStream_t s);

// Sort-pass configurations (radix width, items per thread, workgroup size)
// compiled into the library.
bool pass_config_supported(int radix_bits, int items, int threads);

}  // namespace ss

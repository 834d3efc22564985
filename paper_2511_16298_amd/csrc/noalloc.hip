// ss_sort_frame for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid it): the
// workspace is a fixed array in the library's own device memory instead of
// a caller buffer.  Every call on one GPU uses that GPU's copy of the array,
// so calls that overlap on one GPU race; the array keeps the last call's
// contents, and the sort clears what it needs with its own fill kernel.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>

#include "splatsort.h"

namespace {

// The library-owned workspace: one per GPU, held until the process ends.
static __device__ __align__(256) unsigned char scratch[SS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device
// with that device current (each GPU holds its own copy at its own address;
// in host code the array's name is only a stand-in).
ss_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return SS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[dev] == nullptr) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return SS_ERR_HIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return SS_ERR_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr) return SS_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SS_OK;
}

}  // namespace

extern "C" {

ss_status ss_sort_frame_noalloc(const ss_frame* frame, const ss_frame_out* out, void* stream,
                                const ss_options* options) {
  // the depth-first path only (the default): the others build host tables
  if (options != nullptr && options->struct_size >= offsetof(ss_options, spin_limit) &&
      ((options->algorithm != SS_ALGO_AUTO && options->algorithm != SS_ALGO_DEPTH_FIRST) ||
       (options->flags & (SS_FLAG_UNSORTED | SS_FLAG_KEY32_LOSSY)) != 0))
    return SS_ERR_UNSUPPORTED;
  if (out == nullptr) return SS_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  const ss_status st = ss_workspace_bytes(frame, out->pair_capacity, options, &need);
  if (st != SS_OK) return st;
  if (need > SS_NOALLOC_SCRATCH_BYTES) return SS_ERR_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipDevice_t dev = -1;
  if (hipStreamGetDevice(s, &dev) != hipSuccess) return SS_ERR_HIP;
  void* ws = nullptr;
  const ss_status ss = scratch_on(static_cast<int>(dev), &ws);
  if (ss != SS_OK) return ss;
  return ss_sort_frame(frame, out, ws, SS_NOALLOC_SCRATCH_BYTES, stream, options);
}

}  // extern "C"

// Plans: a fixed batch shape whose whole pipeline is captured once into a
// HIP graph and replayed; optional autotuning of the pass configuration by
// timing every compiled candidate on the caller's data.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stddef.h>

#include <new>
#include <string>
#include <vector>

#include "splatsort.h"
#include "tunecache.hpp"

struct ss_plan {
  std::vector<ss_frame> frames;
  ss_batch_out out{};
  void* workspace = nullptr;
  size_t workspace_bytes = 0;
  ss_options options{};
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<double> candidate_ms;   // empty when the choice came from the tune cache
};

namespace {

struct Candidate {
  uint32_t radix_bits, items, threads, flags;
};

// Every pass configuration compiled into the library, and the 512-thread
// ones again as persistent passes.
const Candidate kCandidates[] = {
    {8, 16, 512, 0}, {8, 8, 512, 0},  {6, 16, 512, 0}, {6, 8, 512, 0},  {4, 16, 512, 0},
    {8, 16, 256, 0}, {8, 12, 256, 0}, {8, 8, 256, 0},  {6, 16, 256, 0}, {4, 16, 256, 0},
    {8, 16, 512, SS_FLAG_PERSISTENT}, {8, 8, 512, SS_FLAG_PERSISTENT}, {6, 16, 512, SS_FLAG_PERSISTENT},
};

ss_options with(const ss_options& base, const Candidate& c) {
  ss_options o = base;
  o.struct_size = sizeof(ss_options);
  o.radix_bits = c.radix_bits;
  o.items_per_thread = c.items;
  o.workgroup_size = c.threads;
  o.flags = (base.flags & ~SS_FLAG_PERSISTENT) | c.flags;  // the caller's other flags stay
  o.timer = nullptr;
  return o;
}

void destroy(ss_plan* p) {
  if (p == nullptr) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  delete p;
}

// Mean milliseconds per launch of one configuration (after one warm-up).
// The batch's status word is out.status, or else the first word of the
// workspace (where the depth-first layout keeps it).
ss_status time_candidate(ss_plan* p, const ss_options& o, uint32_t repeats, hipStream_t s, double* ms,
                         ss_status* device_status) {
  const uint32_t n = static_cast<uint32_t>(p->frames.size());
  ss_status st = ss_sort_batch(p->frames.data(), n, &p->out, p->workspace, p->workspace_bytes, s, &o);
  if (st != SS_OK) return st;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return SS_ERR_HIP;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return SS_ERR_HIP;
  }
  st = SS_OK;
  if (hipEventRecord(a, s) != hipSuccess) st = SS_ERR_HIP;
  for (uint32_t i = 0; st == SS_OK && i < repeats; ++i)
    st = ss_sort_batch(p->frames.data(), n, &p->out, p->workspace, p->workspace_bytes, s, &o);
  if (st == SS_OK && hipEventRecord(b, s) != hipSuccess) st = SS_ERR_HIP;
  if (st == SS_OK && hipEventSynchronize(b) != hipSuccess) st = SS_ERR_HIP;
  float t = 0.0f;
  if (st == SS_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) st = SS_ERR_HIP;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = static_cast<double>(t) / repeats;
  // a candidate that stopped early on a device error (look-back timeout,
  // capacity, bad input) would time as the fastest: read its status word
  if (st == SS_OK) {
    uint32_t dev_status = SS_ERR_HIP;
    const uint32_t* word = p->out.status ? p->out.status : static_cast<const uint32_t*>(p->workspace);
    if (hipMemcpyAsync(&dev_status, word, sizeof(dev_status), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = SS_ERR_HIP;
    else
      *device_status = static_cast<ss_status>(dev_status);
  }
  return st;
}

uint32_t log2_ceil(uint64_t x) {
  uint32_t b = 0;
  while ((1ull << b) < x && b < 63) ++b;
  return b;
}

// The tune-cache key of a plan's batch on the stream's device.
bool plan_tune_key(const ss_plan* p, hipStream_t s, ss::TuneKey* k) {
  int dev = 0;
  if (s != nullptr) {
    hipDevice_t d = 0;
    if (hipStreamGetDevice(s, &d) != hipSuccess) return false;
    dev = static_cast<int>(d);
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return false;
  }
  hipDeviceProp_t prop;
  int runtime = 0;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess || hipRuntimeGetVersion(&runtime) != hipSuccess) return false;
  uint64_t n = 0, tiles = 0, max_tiles = 0;
  for (const ss_frame& f : p->frames) {
    uint32_t tx = 0, ty = 0, kb = 0;
    if (ss_frame_geometry(&f, &tx, &ty, &kb) != SS_OK) return false;
    const uint64_t t = static_cast<uint64_t>(tx) * ty;
    n += f.num_gaussians;
    tiles += t;
    if (t > max_tiles) max_tiles = t;
  }
  k->arch = ss::tune_arch_token(prop.gcnArchName);
  k->runtime = runtime;
  k->abi = ss_abi_version();
  k->frames_log2 = log2_ceil(p->frames.size());
  k->gaussians_log2 = log2_ceil(n);
  k->pairs_log2 = log2_ceil(p->out.pair_capacity);
  k->tile_bits = log2_ceil(tiles);
  k->frame_tile_bits = log2_ceil(max_tiles);
  return true;
}

}  // namespace

extern "C" {

ss_status ss_plan_workspace_bytes(const ss_frame* frames, uint32_t n_frames, uint32_t pair_capacity,
                                  size_t* bytes) {
  if (bytes == nullptr) return SS_ERR_INVALID_ARGUMENT;
  size_t best = 0;
  ss_options base{};
  base.struct_size = sizeof(ss_options);
  for (const Candidate& c : kCandidates) {
    const ss_options o = with(base, c);
    size_t b = 0;
    const ss_status st = ss_batch_workspace_bytes(frames, n_frames, pair_capacity, &o, &b);
    if (st != SS_OK) return st;
    if (b > best) best = b;
  }
  *bytes = best;
  return SS_OK;
}

ss_status ss_plan_create(ss_plan** plan, const ss_plan_desc* desc, void* stream) {
  // callers built before tune_cache existed pass the shorter struct
  if (plan == nullptr || desc == nullptr || desc->struct_size < offsetof(ss_plan_desc, tune_cache))
    return SS_ERR_INVALID_ARGUMENT;
  const char* cache = desc->struct_size >= sizeof(ss_plan_desc) ? desc->tune_cache : nullptr;
  if (desc->frames == nullptr || desc->n_frames == 0) return SS_ERR_INVALID_ARGUMENT;
  ss_plan* p = new (std::nothrow) ss_plan;
  if (p == nullptr) return SS_ERR_HIP;
  p->frames.assign(desc->frames, desc->frames + desc->n_frames);
  p->out = desc->out;
  p->workspace = desc->workspace;
  p->workspace_bytes = desc->workspace_bytes;
  p->options = desc->options;
  p->options.struct_size = sizeof(ss_options);
  p->options.timer = nullptr;
  const hipStream_t s = static_cast<hipStream_t>(stream);

  // validate the starting configuration without launching anything
  size_t need = 0;
  ss_status st = ss_batch_workspace_bytes(p->frames.data(), desc->n_frames, p->out.pair_capacity, &p->options,
                                          &need);
  if (st == SS_OK && desc->workspace_bytes < need) st = SS_ERR_WORKSPACE;
  // a cached choice for this device, runtime and batch size skips the timing
  ss::TuneKey key;
  const bool keyed = st == SS_OK && desc->autotune && cache != nullptr && plan_tune_key(p, s, &key);
  bool tuned = false;
  if (keyed) {
    ss::TuneChoice c;
    if (ss::tune_cache_lookup(cache, key, &c)) {
      const ss_options o = with(p->options, Candidate{c.radix_bits, c.items, c.threads, c.flags});
      size_t b = 0;
      if (ss_batch_workspace_bytes(p->frames.data(), desc->n_frames, p->out.pair_capacity, &o, &b) == SS_OK &&
          b <= desc->workspace_bytes) {
        p->options = o;
        tuned = true;
      }
    }
  }
  if (st == SS_OK && desc->autotune && !tuned) {
    const uint32_t repeats = desc->tune_repeats ? desc->tune_repeats : 5;
    double best = 1e30;
    ss_options chosen = p->options;
    for (const Candidate& c : kCandidates) {
      const ss_options o = with(p->options, c);
      size_t b = 0;
      if (ss_batch_workspace_bytes(p->frames.data(), desc->n_frames, p->out.pair_capacity, &o, &b) != SS_OK ||
          b > desc->workspace_bytes)
        continue;
      double ms = 0.0;
      ss_status dev = SS_OK;
      st = time_candidate(p, o, repeats, s, &ms, &dev);
      if (st != SS_OK) break;
      if (dev != SS_OK) {
        // a device error is the data's (capacity, bad depth) or a timeout: the
        // candidate is not chosen; its time is reported as negative
        p->candidate_ms.push_back(-1.0);
        continue;
      }
      p->candidate_ms.push_back(ms);
      if (ms < best) {
        best = ms;
        chosen = o;
      }
    }
    p->options = chosen;
    if (st == SS_OK && keyed && best < 1e30)
      (void)ss::tune_cache_store(cache, key, ss::TuneChoice{chosen.radix_bits, chosen.items_per_thread,
                                                            chosen.workgroup_size,
                                                            chosen.flags & SS_FLAG_PERSISTENT, best});
  }
  if (st == SS_OK && hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)
    st = SS_ERR_HIP;
  if (st == SS_OK && hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    st = SS_ERR_HIP;
  if (st == SS_OK) {
    const ss_status launched = ss_sort_batch(p->frames.data(), desc->n_frames, &p->out, p->workspace,
                                             p->workspace_bytes, p->capture_stream, &p->options);
    const hipError_t ended = hipStreamEndCapture(p->capture_stream, &p->graph);
    if (launched != SS_OK) st = launched;
    else if (ended != hipSuccess) st = SS_ERR_HIP;
  }
  if (st == SS_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) st = SS_ERR_HIP;
  if (st != SS_OK) {
    destroy(p);
    return st;
  }
  *plan = p;
  return SS_OK;
}

ss_status ss_plan_launch(ss_plan* plan, void* stream) {
  if (plan == nullptr || plan->exec == nullptr) return SS_ERR_INVALID_ARGUMENT;
  return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? SS_OK : SS_ERR_HIP;
}

ss_status ss_plan_config(const ss_plan* plan, ss_options* chosen, double* candidate_ms, uint32_t* n) {
  if (plan == nullptr) return SS_ERR_INVALID_ARGUMENT;
  if (chosen) *chosen = plan->options;
  if (n != nullptr) {
    const uint32_t have = static_cast<uint32_t>(plan->candidate_ms.size());
    const uint32_t k = candidate_ms ? (*n < have ? *n : have) : 0;
    for (uint32_t i = 0; i < k; ++i) candidate_ms[i] = plan->candidate_ms[i];
    *n = have;
  }
  return SS_OK;
}

void ss_plan_destroy(ss_plan* plan) { destroy(plan); }

}  // extern "C"

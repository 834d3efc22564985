// Serving: frame-sort requests arrive over time; a scheduler thread admits
// them against an HBM budget (a caller-owned arena), packs the admitted ones
// into one segmented sort per round (continuous batching: requests that
// arrive while others run join the next round), keeps up to n_streams
// rounds in flight, and completes each request when its round's event
// fires.  Results stay in the arena until the caller releases them.
//
// Rounds in flight are queued back to back on ONE in-order stream, never run
// side by side: their passes wait on earlier workgroups (decoupled
// look-back), and the eight XCDs dispatch their share of each grid on their
// own, so two such kernels running at once can fill one XCD with waiting
// workgroups of the first whose predecessor is queued on an XCD full of
// waiting workgroups of the second, and the other way round: a circular
// wait that only the bounded spin (SS_ERR_TIMEOUT) ends.  The sizing counts
// (no inter-workgroup waits) run on their own stream and overlap the rounds;
// results are read back on a third stream, so that a finished round's
// read-back does not queue behind the round after it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "splatsort.h"

namespace {

using ss::Arena;
using ss::kArenaAlign;
size_t round_up(size_t x) { return ss::arena_round_up(x); }

double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

struct Round;

struct Request {
  uint64_t ticket = 0;
  ss_frame frame{};
  uint32_t tiles = 0;
  int64_t pairs = -1;        // known after sizing
  ss_status status = SS_OK;
  bool done = false;
  double submit_us = 0, start_us = 0, done_us = 0;
  std::shared_ptr<Round> round;
  uint32_t index = 0;        // frame index inside its round
};

// One segmented sort: its workspace (freed at completion) and its outputs
// (freed when every request of the round has been released).
struct Round {
  std::vector<Request*> reqs;
  size_t ws_off = 0, ws_bytes = 0, out_off = 0, out_bytes = 0;
  uint32_t capacity = 0, total_tiles = 0;
  int stream = -1;                 // the round's slot
  hipEvent_t done_event = nullptr;
  uint32_t unreleased = 0;
  // host copies read back at completion
  std::vector<uint32_t> frame_pairs, frame_base;
  std::vector<uint32_t> tile_base;
  uint32_t status = SS_OK;
  // device pointers inside the arena
  uint64_t* keys = nullptr;
  uint32_t* values = nullptr;
  uint32_t* ranges = nullptr;
  uint32_t* d_frame_pairs = nullptr;
  uint32_t* d_frame_base = nullptr;
  uint32_t* d_scalars = nullptr;  // num_pairs, status
};

}  // namespace

struct ss_server {
  char* arena_ptr = nullptr;
  Arena arena;
  ss_server_desc desc{};
  hipStream_t sort_stream = nullptr;      // every round, in order
  std::vector<bool> busy;                 // round slots (n_streams)
  hipStream_t count_stream = nullptr;     // sizing counts
  hipStream_t readback_stream = nullptr;  // completed rounds' small read-backs
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::vector<std::shared_ptr<Round>> inflight;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread worker;
  // statistics
  uint64_t rounds = 0, admitted = 0, completed = 0, rejected = 0;
  double busy_frames = 0;
};

namespace {

// Pair counts of the pending requests that do not have one yet (one batched
// count, synchronous on the count stream).  Called without the lock held.
void size_requests(ss_server* s, const std::vector<Request*>& todo) {
  if (todo.empty()) return;
  std::vector<ss_frame> frames;
  for (Request* r : todo) frames.push_back(r->frame);
  const uint32_t n = static_cast<uint32_t>(frames.size());
  size_t ws = 0;
  ss_status st = ss_batch_count_workspace_bytes(frames.data(), n, &ws);
  const size_t scratch = round_up(ws) + round_up((n + 2) * sizeof(uint32_t));
  size_t off = 0;
  bool have = false;
  if (st == SS_OK) {
    std::lock_guard<std::mutex> g(s->mu);
    have = s->arena.alloc(scratch, &off);
  }
  if (st != SS_OK || !have) {
    for (Request* r : todo) r->pairs = -1;  // retry next round
    return;
  }
  char* base = s->arena_ptr + off;
  uint32_t* d_counts = reinterpret_cast<uint32_t*>(base + round_up(ws));
  st = ss_batch_count_pairs(frames.data(), n, d_counts, d_counts + n, d_counts + n + 1, base, ws, s->count_stream);
  std::vector<uint32_t> host(n + 2, 0);
  if (st == SS_OK &&
      hipMemcpyAsync(host.data(), d_counts, (n + 2) * sizeof(uint32_t), hipMemcpyDeviceToHost, s->count_stream) !=
          hipSuccess)
    st = SS_ERR_HIP;
  if (st == SS_OK && hipStreamSynchronize(s->count_stream) != hipSuccess) st = SS_ERR_HIP;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->arena.release(off, scratch);
  }
  for (uint32_t i = 0; i < n; ++i) {
    if (st != SS_OK) {
      todo[i]->status = st;
      todo[i]->pairs = 0;
    } else if (host[n + 1] == SS_ERR_INVALID_INPUT || host[n + 1] == SS_ERR_OVERFLOW) {
      // find the offending frames individually next time: count them alone
      todo[i]->pairs = n == 1 ? 0 : -2;
      if (n == 1) todo[i]->status = static_cast<ss_status>(host[n + 1]);
    } else {
      todo[i]->pairs = host[i];
    }
  }
}

// Bytes a round needs: workspace (released at completion) and outputs.
void round_bytes(const std::vector<Request*>& rs, const ss_server_desc& d, size_t* ws, size_t* out, uint32_t* cap,
                 uint32_t* tiles, ss_status* st) {
  std::vector<ss_frame> frames;
  uint64_t m = 0, t = 0;
  for (Request* r : rs) {
    frames.push_back(r->frame);
    m += static_cast<uint64_t>(r->pairs);
    t += r->tiles;
  }
  *cap = m > SS_MAX_PAIR_CAPACITY ? SS_MAX_PAIR_CAPACITY : static_cast<uint32_t>(m);
  *tiles = static_cast<uint32_t>(t);
  *st = ss_batch_workspace_bytes(frames.data(), static_cast<uint32_t>(frames.size()), *cap, &d.options, ws);
  const size_t n = rs.size();
  *out = round_up(static_cast<size_t>(*cap) * 8) + round_up(static_cast<size_t>(*cap) * 4) +
         round_up(static_cast<size_t>(t) * 8) + round_up(n * 4) * 2 + round_up(16);
  if (m > SS_MAX_PAIR_CAPACITY) *st = SS_ERR_BUDGET;
}

void complete_round(ss_server* s, const std::shared_ptr<Round>& rd) {
  // read back per-frame counts, bases and the status (small, synchronous)
  const size_t n = rd->reqs.size();
  rd->frame_pairs.assign(n, 0);
  rd->frame_base.assign(n, 0);
  uint32_t sc[2] = {0, SS_ERR_HIP};
  // the round's event has fired: its outputs are complete
  const hipStream_t st = s->readback_stream;
  bool ok = hipMemcpyAsync(rd->frame_pairs.data(), rd->d_frame_pairs, n * 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipMemcpyAsync(rd->frame_base.data(), rd->d_frame_base, n * 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipMemcpyAsync(sc, rd->d_scalars, 8, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipStreamSynchronize(st) == hipSuccess;
  const double t = now_us();
  std::lock_guard<std::mutex> g(s->mu);
  rd->status = ok ? sc[1] : static_cast<uint32_t>(SS_ERR_HIP);
  s->arena.release(rd->ws_off, rd->ws_bytes);
  s->busy[rd->stream] = false;
  (void)hipEventDestroy(rd->done_event);
  rd->done_event = nullptr;
  for (Request* r : rd->reqs) {
    r->done = true;
    r->done_us = t;
    r->status = static_cast<ss_status>(rd->status);
    ++s->completed;
  }
  s->cv_done.notify_all();
}

void worker_loop(ss_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // 1. completions
    std::vector<std::shared_ptr<Round>> finished;
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
      if (hipEventQuery((*it)->done_event) == hipSuccess) {
        finished.push_back(*it);
        it = s->inflight.erase(it);
      } else {
        ++it;
      }
    }
    if (!finished.empty()) {
      lk.unlock();
      for (auto& rd : finished) complete_round(s, rd);
      lk.lock();
      continue;
    }
    if (s->stopping && s->pending.empty() && s->inflight.empty()) break;
    // 2. a free stream and work waiting: size, admit, launch
    int free_stream = -1;
    for (size_t i = 0; i < s->busy.size(); ++i)
      if (!s->busy[i]) {
        free_stream = static_cast<int>(i);
        break;
      }
    if (free_stream >= 0 && !s->pending.empty()) {
      std::vector<Request*> cand;
      for (Request* r : s->pending) {
        if (cand.size() >= s->desc.max_batch_frames) break;
        cand.push_back(r);
      }
      std::vector<Request*> todo;
      for (Request* r : cand)
        if (r->pairs < 0) todo.push_back(r);
      lk.unlock();
      if (!todo.empty()) {
        // a round with a bad frame is sized frame by frame
        bool split = false;
        size_requests(s, todo);
        for (Request* r : todo) split |= r->pairs == -2;
        if (split)
          for (Request* r : todo) {
            std::vector<Request*> one{r};
            size_requests(s, one);
          }
      }
      lk.lock();
      // requests that failed sizing complete at once
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        Request* r = *it;
        if (r->pairs >= 0 && r->status != SS_OK) {
          r->done = true;
          r->done_us = now_us();
          ++s->completed;
          it = s->pending.erase(it);
          s->cv_done.notify_all();
        } else {
          ++it;
        }
      }
      // admit the longest prefix whose round fits the arena now
      std::vector<Request*> take;
      size_t ws_b = 0, out_b = 0, ws_off = 0, out_off = 0;
      uint32_t cap = 0, tiles = 0;
      for (Request* r : s->pending) {
        if (take.size() >= s->desc.max_batch_frames || r->pairs < 0) break;
        take.push_back(r);
      }
      bool never_fits = false;
      const uint32_t k = ss::admit_prefix(
          s->arena, static_cast<uint32_t>(take.size()),
          [&](uint32_t n, size_t* ws, size_t* out) {
            std::vector<Request*> prefix(take.begin(), take.begin() + n);
            ss_status bst;
            round_bytes(prefix, s->desc, ws, out, &cap, &tiles, &bst);
            return bst == SS_OK;
          },
          &ws_off, &ws_b, &out_off, &out_b, &never_fits);
      const bool got = k > 0;
      if (got) {
        take.resize(k);  // cap and tiles are those of this prefix (the last one sized)
      } else {
        if (!take.empty() && never_fits) {
          // alone in an empty arena it could never fit: reject
          Request* r = take[0];
          r->status = SS_ERR_BUDGET;
          r->done = true;
          r->done_us = now_us();
          ++s->rejected;
          ++s->completed;
          s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
          s->cv_done.notify_all();
        }
        take.clear();
      }
      if (got) {
        auto rd = std::make_shared<Round>();
        rd->reqs = take;
        rd->ws_off = ws_off;
        rd->ws_bytes = ws_b;
        rd->out_off = out_off;
        rd->out_bytes = out_b;
        rd->capacity = cap;
        rd->total_tiles = tiles;
        rd->stream = free_stream;
        rd->unreleased = static_cast<uint32_t>(take.size());
        char* o = s->arena_ptr + out_off;
        rd->keys = reinterpret_cast<uint64_t*>(o);
        o += round_up(static_cast<size_t>(cap) * 8);
        rd->values = reinterpret_cast<uint32_t*>(o);
        o += round_up(static_cast<size_t>(cap) * 4);
        rd->ranges = reinterpret_cast<uint32_t*>(o);
        o += round_up(static_cast<size_t>(tiles) * 8);
        rd->d_frame_pairs = reinterpret_cast<uint32_t*>(o);
        o += round_up(take.size() * 4);
        rd->d_frame_base = reinterpret_cast<uint32_t*>(o);
        o += round_up(take.size() * 4);
        rd->d_scalars = reinterpret_cast<uint32_t*>(o);
        uint32_t tb = 0;
        std::vector<ss_frame> frames;
        for (size_t i = 0; i < take.size(); ++i) {
          Request* r = take[i];
          r->round = rd;
          r->index = static_cast<uint32_t>(i);
          r->start_us = now_us();
          rd->tile_base.push_back(tb);
          tb += r->tiles;
          frames.push_back(r->frame);
          s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
        }
        s->busy[free_stream] = true;
        ++s->rounds;
        s->admitted += take.size();
        s->busy_frames += static_cast<double>(take.size());
        lk.unlock();
        ss_batch_out out{};
        out.pair_capacity = cap;
        out.keys = rd->keys;
        out.values = rd->values;
        out.tile_ranges = rd->ranges;
        out.frame_pairs = rd->d_frame_pairs;
        out.frame_pair_base = rd->d_frame_base;
        out.num_pairs = rd->d_scalars;
        out.status = rd->d_scalars + 1;
        const hipStream_t st = s->sort_stream;
        ss_status ls = ss_sort_batch(frames.data(), static_cast<uint32_t>(frames.size()), &out,
                                     s->arena_ptr + ws_off, ws_b, st, &s->desc.options);
        if (ls == SS_OK && hipEventCreateWithFlags(&rd->done_event, hipEventDisableTiming) != hipSuccess)
          ls = SS_ERR_HIP;
        if (ls == SS_OK && hipEventRecord(rd->done_event, st) != hipSuccess) ls = SS_ERR_HIP;
        lk.lock();
        if (ls != SS_OK) {
          // launch failed: complete the round's requests with the error at once
          if (rd->done_event) (void)hipEventDestroy(rd->done_event);
          rd->done_event = nullptr;
          s->arena.release(ws_off, ws_b);
          s->busy[free_stream] = false;
          for (Request* r : take) {
            r->status = ls;
            r->done = true;
            r->done_us = now_us();
            ++s->completed;
          }
          s->cv_done.notify_all();
        } else {
          s->inflight.push_back(rd);
        }
        continue;
      }
    }
    // 3. nothing to do right now: wait briefly for arrivals or completions
    if (s->inflight.empty() && (s->pending.empty() || free_stream < 0))
      s->cv_work.wait_for(lk, std::chrono::microseconds(200));
    else
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

ss_status ss_server_create(ss_server** server, void* arena, size_t arena_bytes, const ss_server_desc* desc) {
  if (server == nullptr || arena == nullptr || arena_bytes < kArenaAlign) return SS_ERR_INVALID_ARGUMENT;
  if (reinterpret_cast<uintptr_t>(arena) % kArenaAlign != 0) return SS_ERR_INVALID_ARGUMENT;
  if (desc == nullptr || desc->struct_size < sizeof(ss_server_desc)) return SS_ERR_INVALID_ARGUMENT;
  if (desc->max_batch_frames == 0 || desc->max_batch_frames > SS_MAX_BATCH_FRAMES) return SS_ERR_INVALID_ARGUMENT;
  if (desc->n_streams == 0 || desc->n_streams > 8) return SS_ERR_INVALID_ARGUMENT;
  // the options must describe a valid batched configuration (all zero = defaults)
  ss_options opts = desc->options;
  if (opts.struct_size == 0) opts.struct_size = sizeof(ss_options);
  opts.timer = nullptr;
  ss_frame probe{16, 16, 16, 0, nullptr};
  size_t b = 0;
  const ss_status ost = ss_batch_workspace_bytes(&probe, 1, 0, &opts, &b);
  if (ost != SS_OK) return ost;
  ss_server* s = new (std::nothrow) ss_server;
  if (s == nullptr) return SS_ERR_HIP;
  s->arena_ptr = static_cast<char*>(arena);
  s->arena.reset(arena_bytes & ~(kArenaAlign - 1));
  s->desc = *desc;
  s->desc.options = opts;
  const bool ok = hipStreamCreateWithFlags(&s->count_stream, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&s->sort_stream, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&s->readback_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    if (s->readback_stream) (void)hipStreamDestroy(s->readback_stream);
    if (s->sort_stream) (void)hipStreamDestroy(s->sort_stream);
    if (s->count_stream) (void)hipStreamDestroy(s->count_stream);
    delete s;
    return SS_ERR_HIP;
  }
  s->busy.assign(desc->n_streams, false);
  s->worker = std::thread(worker_loop, s);
  *server = s;
  return SS_OK;
}

ss_status ss_server_submit(ss_server* s, const ss_frame* frame, uint64_t* ticket) {
  if (s == nullptr || frame == nullptr || ticket == nullptr) return SS_ERR_INVALID_ARGUMENT;
  uint32_t tx = 0, ty = 0, kb = 0;
  const ss_status st = ss_frame_geometry(frame, &tx, &ty, &kb);
  if (st != SS_OK) return st;
  auto r = std::make_unique<Request>();
  r->frame = *frame;
  r->tiles = tx * ty;
  r->submit_us = now_us();
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stopping) return SS_ERR_INVALID_ARGUMENT;
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->pending.push_back(r.get());
  s->requests.emplace(r->ticket, std::move(r));
  s->cv_work.notify_one();
  return SS_OK;
}

ss_status ss_server_wait(ss_server* s, uint64_t ticket, ss_result* out) {
  if (s == nullptr || out == nullptr) return SS_ERR_INVALID_ARGUMENT;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return SS_ERR_INVALID_ARGUMENT;
  Request* r = it->second.get();
  s->cv_done.wait(lk, [&] { return r->done; });
  *out = ss_result{};
  out->status = r->status;
  out->submit_us = r->submit_us;
  out->start_us = r->start_us;
  out->done_us = r->done_us;
  if (r->status == SS_OK && r->round) {
    Round* rd = r->round.get();
    const uint32_t base = rd->frame_base[r->index];
    out->num_pairs = rd->frame_pairs[r->index];
    out->keys = rd->keys + base;
    out->values = rd->values + base;
    out->tile_ranges = rd->ranges + 2 * static_cast<size_t>(rd->tile_base[r->index]);
    out->tile_base = rd->tile_base[r->index];
    out->pair_base = base;
    out->round_frames = static_cast<uint32_t>(rd->reqs.size());
  }
  return SS_OK;
}

ss_status ss_server_release(ss_server* s, uint64_t ticket) {
  if (s == nullptr) return SS_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end() || !it->second->done) return SS_ERR_INVALID_ARGUMENT;
  std::shared_ptr<Round> rd = it->second->round;
  s->requests.erase(it);
  if (rd && --rd->unreleased == 0) s->arena.release(rd->out_off, rd->out_bytes);
  s->cv_work.notify_one();
  return SS_OK;
}

ss_status ss_server_stats(ss_server* s, ss_server_counters* out) {
  if (s == nullptr || out == nullptr) return SS_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(s->mu);
  out->rounds = s->rounds;
  out->admitted = s->admitted;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->pending = s->pending.size();
  out->arena_used = s->arena.used();
  out->mean_round_frames = s->rounds ? s->busy_frames / static_cast<double>(s->rounds) : 0.0;
  return SS_OK;
}

void ss_server_destroy(ss_server* s) {
  if (s == nullptr) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamDestroy(s->readback_stream);
  (void)hipStreamDestroy(s->sort_stream);
  (void)hipStreamDestroy(s->count_stream);
  delete s;
}

}  // extern "C"

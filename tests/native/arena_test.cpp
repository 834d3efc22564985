// Host-only test of the server's arena allocator and admission rule
// (paper_2511_16298_amd/csrc/arena.hpp), built with sanitizers by
// tests/test_host_runtime_cpu.py.  Prints OK and exits 0 when every check
// holds.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "arena.hpp"

using ss::Arena;

static int g_fail = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                      \
    }                                                                \
  } while (0)

// Reference: one flag per 256-byte unit, first fit by a linear scan.
struct Model {
  std::vector<char> used;
  explicit Model(size_t units) : used(units, 0) {}
  bool alloc(size_t units, size_t* at) {
    size_t run = 0;
    for (size_t i = 0; i < used.size(); ++i) {
      run = used[i] ? 0 : run + 1;
      if (run == units) {
        *at = i + 1 - units;
        for (size_t j = *at; j <= i; ++j) used[j] = 1;
        return true;
      }
    }
    return false;
  }
  void release(size_t at, size_t units) {
    for (size_t j = at; j < at + units; ++j) used[j] = 0;
  }
  size_t free_runs() const {
    size_t runs = 0;
    for (size_t i = 0; i < used.size(); ++i)
      if (!used[i] && (i == 0 || used[i - 1])) ++runs;
    return runs;
  }
  size_t used_units() const {
    size_t u = 0;
    for (char c : used) u += c;
    return u;
  }
};

static void test_random_against_model(unsigned seed) {
  std::mt19937_64 rng(seed);
  const size_t units = 512;
  Arena a;
  a.reset(units * ss::kArenaAlign + 100);  // a ragged size rounds down
  CHECK(a.size() == units * ss::kArenaAlign);
  Model m(units);
  struct Block { size_t off, bytes; };
  std::vector<Block> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t bytes = rng() % 4 == 0 ? 0 : 1 + rng() % (40 * ss::kArenaAlign);
      const size_t u = ss::arena_round_up(bytes ? bytes : ss::kArenaAlign) / ss::kArenaAlign;
      size_t off = 0, at = 0;
      const bool got = a.alloc(bytes, &off);
      const bool mgot = m.alloc(u, &at);
      CHECK(got == mgot);
      if (got && mgot) {
        CHECK(off == at * ss::kArenaAlign);
        CHECK(off % ss::kArenaAlign == 0);
        live.push_back({off, bytes});
      }
    } else {
      const size_t i = rng() % live.size();
      const Block b = live[i];
      live[i] = live.back();
      live.pop_back();
      a.release(b.off, b.bytes);
      m.release(b.off / ss::kArenaAlign, ss::arena_round_up(b.bytes ? b.bytes : ss::kArenaAlign) / ss::kArenaAlign);
    }
    CHECK(a.used() == m.used_units() * ss::kArenaAlign);
    CHECK(a.free_blocks() == m.free_runs());  // neighbours always coalesce
  }
  for (const Block& b : live) a.release(b.off, b.bytes);
  CHECK(a.used() == 0);
  CHECK(a.free_blocks() == 1 && a.largest_free() == a.size());
}

// Admission: requests with fixed workspace/output sizes per frame; a round of
// the first k has ws = sum of ws and out = sum of out.
static void test_admission() {
  const size_t U = ss::kArenaAlign;
  std::vector<size_t> ws = {10 * U, 20 * U, 30 * U, 40 * U}, out = {5 * U, 5 * U, 5 * U, 5 * U};
  auto sizes = [&](uint32_t k, size_t* w, size_t* o) {
    *w = *o = 0;
    for (uint32_t i = 0; i < k; ++i) {
      *w += ws[i];
      *o += out[i];
    }
    return true;
  };
  size_t wo, wb, oo, ob;
  bool never;
  {
    Arena a;
    a.reset(1000 * U);
    CHECK(ss::admit_prefix(a, 4, sizes, &wo, &wb, &oo, &ob, &never) == 4);  // everything fits
    CHECK(wb == 100 * U && ob == 20 * U && !never);
    CHECK(a.used() == 120 * U);
  }
  {
    Arena a;
    a.reset(70 * U);   // 10+20+30 = 60 ws + 15 out = 75 > 70; two frames: 30 + 10 = 40
    CHECK(ss::admit_prefix(a, 4, sizes, &wo, &wb, &oo, &ob, &never) == 2);
    CHECK(wb == 30 * U && ob == 10 * U && a.used() == 40 * U && !never);
    // the rest waits: with 30 units left only a round of frame 3 alone (ws 30 + out 5) would need 35
    std::vector<size_t> ws2 = {30 * U}, out2 = {5 * U};
    auto one = [&](uint32_t, size_t* w, size_t* o) { *w = ws2[0]; *o = out2[0]; return true; };
    CHECK(ss::admit_prefix(a, 1, one, &wo, &wb, &oo, &ob, &never) == 0);
    CHECK(!never && a.used() == 40 * U);       // nothing left allocated by the failed attempt
  }
  {
    Arena a;
    a.reset(12 * U);   // frame 0 alone needs 15: can never fit
    CHECK(ss::admit_prefix(a, 4, sizes, &wo, &wb, &oo, &ob, &never) == 0);
    CHECK(never && a.used() == 0);
  }
  {
    Arena a;
    a.reset(100 * U);
    auto impossible = [&](uint32_t, size_t* w, size_t* o) { *w = *o = U; return false; };
    CHECK(ss::admit_prefix(a, 3, impossible, &wo, &wb, &oo, &ob, &never) == 0);
    CHECK(never && a.used() == 0);
  }
  {
    // workspace fits but the outputs do not: the workspace block is given back
    Arena a;
    a.reset(16 * U);
    size_t hold = 0;
    CHECK(a.alloc(4 * U, &hold));
    auto big_out = [&](uint32_t, size_t* w, size_t* o) { *w = 10 * U; *o = 5 * U; return true; };
    CHECK(ss::admit_prefix(a, 1, big_out, &wo, &wb, &oo, &ob, &never) == 0);
    CHECK(!never && a.used() == 4 * U && a.free_blocks() == 1);
  }
}

// A fake-clock run of the scheduler's admission over a FIFO: each admitted
// round holds its workspace for `dur` ticks and its outputs until released
// one tick after completion; every request is eventually admitted in FIFO
// order and the arena returns to empty.
static void test_fake_clock_fifo(unsigned seed) {
  std::mt19937_64 rng(seed);
  const size_t U = ss::kArenaAlign;
  Arena a;
  a.reset(400 * U);
  struct Req { size_t ws, out; int arrive; };
  std::vector<Req> reqs;
  for (int i = 0; i < 300; ++i) reqs.push_back({(1 + rng() % 60) * U, (1 + rng() % 30) * U, static_cast<int>(i / 3)});
  struct Live { size_t ws_off, ws, out_off, out; int done; };
  std::vector<Live> live;
  size_t next = 0;
  int admitted_rounds = 0;
  for (int t = 0; t < 100000 && (next < reqs.size() || !live.empty()); ++t) {
    for (size_t i = 0; i < live.size();) {
      if (live[i].done == t) a.release(live[i].ws_off, live[i].ws);
      if (live[i].done + 1 == t) {
        a.release(live[i].out_off, live[i].out);
        live[i] = live.back();
        live.pop_back();
      } else {
        ++i;
      }
    }
    uint32_t waiting = 0;
    while (next + waiting < reqs.size() && reqs[next + waiting].arrive <= t && waiting < 8) ++waiting;
    if (waiting == 0 || live.size() >= 2) continue;   // two streams
    size_t wo, wb, oo, ob;
    bool never;
    auto sizes = [&](uint32_t k, size_t* w, size_t* o) {
      *w = *o = 0;
      for (uint32_t i = 0; i < k; ++i) {
        *w += reqs[next + i].ws;
        *o += reqs[next + i].out;
      }
      return true;
    };
    const uint32_t k = ss::admit_prefix(a, waiting, sizes, &wo, &wb, &oo, &ob, &never);
    CHECK(!never);
    if (k) {
      live.push_back({wo, wb, oo, ob, t + 1 + static_cast<int>(rng() % 5)});
      next += k;
      ++admitted_rounds;
    }
    CHECK(a.used() <= a.size());
  }
  CHECK(next == reqs.size());
  CHECK(live.empty() && a.used() == 0);
  CHECK(admitted_rounds > 0 && admitted_rounds < static_cast<int>(reqs.size()));  // some rounds batched
}

int main() {
  for (unsigned s = 1; s <= 5; ++s) test_random_against_model(s);
  test_admission();
  for (unsigned s = 1; s <= 5; ++s) test_fake_clock_fifo(s);
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("OK\n");
  return 0;
}

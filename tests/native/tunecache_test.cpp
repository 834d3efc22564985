// Host-only test of the plans' autotune cache
// (paper_2511_16298_amd/csrc/tunecache.hpp), built with sanitizers by
// tests/test_host_runtime_cpu.py.  Takes a scratch directory; prints OK and
// exits 0 when every check holds.
#include <stdio.h>
#include <stdlib.h>

#include <string>

#include "tunecache.hpp"

using ss::TuneChoice;
using ss::TuneKey;

static int g_fail = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                             \
    }                                                                       \
  } while (0)

static std::string slurp(const std::string& path) {
  std::string s;
  FILE* f = fopen(path.c_str(), "r");
  if (f == nullptr) return s;
  int ch;
  while ((ch = fgetc(f)) != EOF) s.push_back(static_cast<char>(ch));
  fclose(f);
  return s;
}

static size_t count(const std::string& s, const std::string& sub) {
  size_t n = 0;
  for (size_t at = s.find(sub); at != std::string::npos; at = s.find(sub, at + 1)) ++n;
  return n;
}

static TuneKey key(uint32_t pairs_log2, const char* arch = "gfx950") {
  TuneKey k;
  k.arch = ss::tune_arch_token(arch);
  k.runtime = 70226015;
  k.abi = 3;
  k.frames_log2 = 6;
  k.gaussians_log2 = 26;
  k.pairs_log2 = pairs_log2;
  k.tile_bits = 19;
  k.frame_tile_bits = 13;
  return k;
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  const std::string dir = argv[1];
  const std::string path = dir + "/tune.txt";
  TuneChoice c;

  // architecture tokens
  CHECK(ss::tune_arch_token("gfx950:sramecc+:xnack-") == "gfx950");
  CHECK(ss::tune_arch_token("") == "unknown");
  CHECK(ss::tune_arch_token(nullptr) == "unknown");
  CHECK(ss::tune_arch_token("a b") == "a");
  CHECK(ss::tune_arch_token("x=y") == "xy");

  // no file, no path
  CHECK(!ss::tune_cache_lookup(path.c_str(), key(28), &c));
  CHECK(!ss::tune_cache_lookup(nullptr, key(28), &c));
  CHECK(!ss::tune_cache_store(nullptr, key(28), c));
  CHECK(!ss::tune_cache_store("", key(28), c));

  // store, then look up
  CHECK(ss::tune_cache_store(path.c_str(), key(28), TuneChoice{8, 16, 512, 0, 4.5}));
  CHECK(ss::tune_cache_lookup(path.c_str(), key(28), &c));
  CHECK(c.radix_bits == 8 && c.items == 16 && c.threads == 512 && c.flags == 0 && c.ms > 4.49 && c.ms < 4.51);
  // other keys miss: pair bucket, architecture
  CHECK(!ss::tune_cache_lookup(path.c_str(), key(27), &c));
  CHECK(!ss::tune_cache_lookup(path.c_str(), key(28, "gfx942"), &c));

  // a second key, then replacing the first: one line each
  CHECK(ss::tune_cache_store(path.c_str(), key(27), TuneChoice{6, 8, 512, 8, 1.25}));
  CHECK(ss::tune_cache_store(path.c_str(), key(28), TuneChoice{4, 16, 256, 0, 3.0}));
  std::string text = slurp(path);
  CHECK(count(text, "\n") == 2);
  CHECK(ss::tune_cache_lookup(path.c_str(), key(28), &c) && c.radix_bits == 4 && c.threads == 256);
  CHECK(ss::tune_cache_lookup(path.c_str(), key(27), &c) && c.radix_bits == 6 && c.flags == 8);

  // foreign and broken lines: ignored by lookups, kept by updates; a
  // duplicate of a key is collapsed into one line on the next store
  {
    FILE* f = fopen(path.c_str(), "a");
    CHECK(f != nullptr);
    if (f) {
      fprintf(f, "# a comment line\n");
      fprintf(f, "%s = 8 16\n", key(26).str().c_str());            // too few fields
      fprintf(f, "%s = 8 16 512 0 1.0 junk\n", key(25).str().c_str());  // trailing junk
      fprintf(f, "%s = 8 8 512 0 2.0\n", key(27).str().c_str());    // duplicate of key(27): last wins
      fprintf(f, "no newline at the end");
      fclose(f);
    }
  }
  CHECK(!ss::tune_cache_lookup(path.c_str(), key(26), &c));
  CHECK(!ss::tune_cache_lookup(path.c_str(), key(25), &c));
  CHECK(ss::tune_cache_lookup(path.c_str(), key(27), &c) && c.items == 8 && c.flags == 0);
  CHECK(ss::tune_cache_store(path.c_str(), key(27), TuneChoice{8, 16, 512, 8, 0.5}));
  text = slurp(path);
  CHECK(count(text, "# a comment line\n") == 1);
  CHECK(count(text, "no newline at the end\n") == 1);
  CHECK(count(text, key(27).str() + " = ") == 1);
  CHECK(ss::tune_cache_lookup(path.c_str(), key(27), &c) && c.items == 16 && c.flags == 8);
  CHECK(ss::tune_cache_lookup(path.c_str(), key(28), &c) && c.radix_bits == 4);

  // an unwritable location: the store fails and leaves nothing behind
  const std::string bad = dir + "/missing-dir/tune.txt";
  CHECK(!ss::tune_cache_store(bad.c_str(), key(28), TuneChoice{8, 16, 512, 0, 1.0}));
  CHECK(!ss::tune_cache_lookup(bad.c_str(), key(28), &c));
  CHECK(slurp(path + ".tmp").empty());

  if (g_fail == 0) printf("OK\n");
  return g_fail == 0 ? 0 : 1;
}

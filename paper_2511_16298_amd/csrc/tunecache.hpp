// Host-only autotune cache for plans: the pass configuration a plan chose,
// per device architecture, HIP runtime version, library ABI version and
// batch size bucket, kept one entry per line in a small text file so that
// later plans of the same shape skip the timing.  Free of HIP, so that it
// can be built and tested on its own (with sanitizers) on any host.
//
// Line format (fields separated by single spaces):
//   ss-tune 1 <arch> <runtime> <abi> <frames_log2> <gaussians_log2>
//             <pairs_log2> <tile_bits> <frame_tile_bits> = <radix_bits>
//             <items> <threads> <flags> <ms>
// Lines that do not parse are ignored by lookups and kept by updates.
#pragma once

#include <stdint.h>
#include <stdio.h>

#include <string>
#include <vector>

namespace ss {

struct TuneKey {
  std::string arch;          // device architecture name (no spaces; see tune_arch_token)
  int32_t runtime = 0;       // HIP runtime version
  uint32_t abi = 0;          // library ABI version
  uint32_t frames_log2 = 0, gaussians_log2 = 0, pairs_log2 = 0, tile_bits = 0, frame_tile_bits = 0;

  std::string str() const {
    char buf[160];
    snprintf(buf, sizeof(buf), "%d %u %u %u %u %u %u", runtime, abi, frames_log2, gaussians_log2, pairs_log2,
             tile_bits, frame_tile_bits);
    return "ss-tune 1 " + arch + " " + buf;
  }
};

struct TuneChoice {
  uint32_t radix_bits = 0, items = 0, threads = 0, flags = 0;
  double ms = 0.0;
};

// The architecture token of a device name such as "gfx950:sramecc+:xnack-":
// up to the first ':' or blank, other characters kept if printable; never
// empty ("unknown").
inline std::string tune_arch_token(const char* name) {
  std::string s;
  for (const char* c = name; c != nullptr && *c != 0 && *c != ':' && *c != ' ' && s.size() < 64; ++c)
    if (*c > ' ' && *c < 127 && *c != '=') s.push_back(*c);
  return s.empty() ? std::string("unknown") : s;
}

namespace tune_detail {

inline bool read_lines(const char* path, std::vector<std::string>* lines) {
  FILE* f = fopen(path, "r");
  if (f == nullptr) return false;
  std::string cur;
  int ch;
  while ((ch = fgetc(f)) != EOF) {
    if (ch == '\n') {
      lines->push_back(cur);
      cur.clear();
    } else if (cur.size() < 4096) {
      cur.push_back(static_cast<char>(ch));
    }
  }
  if (!cur.empty()) lines->push_back(cur);
  fclose(f);
  return true;
}

// Splits "<key> = <choice>"; true when the line is an entry whose choice parses.
inline bool parse_entry(const std::string& line, std::string* key, TuneChoice* c) {
  const size_t eq = line.find(" = ");
  if (eq == std::string::npos || line.compare(0, 10, "ss-tune 1 ") != 0) return false;
  *key = line.substr(0, eq);
  unsigned rb = 0, it = 0, th = 0, fl = 0;
  double ms = 0.0;
  char tail = 0;
  if (sscanf(line.c_str() + eq + 3, "%u %u %u %u %lf %c", &rb, &it, &th, &fl, &ms, &tail) != 5) return false;
  c->radix_bits = rb;
  c->items = it;
  c->threads = th;
  c->flags = fl;
  c->ms = ms;
  return true;
}

}  // namespace tune_detail

// The cached choice for `k`, if the file has one (the last such line wins).
inline bool tune_cache_lookup(const char* path, const TuneKey& k, TuneChoice* out) {
  if (path == nullptr || *path == 0) return false;
  std::vector<std::string> lines;
  if (!tune_detail::read_lines(path, &lines)) return false;
  const std::string want = k.str();
  bool found = false;
  for (const std::string& l : lines) {
    std::string key;
    TuneChoice c;
    if (tune_detail::parse_entry(l, &key, &c) && key == want) {
      *out = c;
      found = true;
    }
  }
  return found;
}

// Records `c` for `k`: the file's other lines stay, an entry of the same key
// is replaced.  Written to "<path>.tmp" and renamed over the file, so a
// reader sees the old file or the new one.  False if the file could not be
// written (the plan itself does not depend on it).
inline bool tune_cache_store(const char* path, const TuneKey& k, const TuneChoice& c) {
  if (path == nullptr || *path == 0) return false;
  std::vector<std::string> lines;
  tune_detail::read_lines(path, &lines);  // a missing file is an empty one
  const std::string want = k.str();
  char val[96];
  snprintf(val, sizeof(val), "%u %u %u %u %.6f", c.radix_bits, c.items, c.threads, c.flags, c.ms);
  const std::string entry = want + " = " + val;
  bool replaced = false;
  for (std::string& l : lines) {
    std::string key;
    TuneChoice old;
    if (tune_detail::parse_entry(l, &key, &old) && key == want) {
      l = replaced ? std::string() : entry;  // later duplicates dropped below
      replaced = true;
    }
  }
  if (!replaced) lines.push_back(entry);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (f == nullptr) return false;
  bool ok = true;
  for (const std::string& l : lines)
    if (!l.empty()) ok = ok && fprintf(f, "%s\n", l.c_str()) >= 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace ss

// Plain CPU oracle of the per-frame tile-and-depth sort of 3D Gaussian
// Splatting.  TEST INFRASTRUCTURE ONLY: nothing in the product library links,
// loads or calls this file; the tests, the smoke check and the benchmark's
// CPU baseline do.  It is written to be read against the paper, not to be
// fast: one thread, plain loops, std::exclusive_scan and std::stable_sort.
//
// Paper passages followed (arXiv 2511.16298):
//  * Background, "Duplication with Tiles": the image is cut into 16x16 tiles,
//    each projected Gaussian is bounded by an axis-aligned box, and it is
//    duplicated once per tile the box meets; each duplicate is a key-value
//    pair keyed by tile id and depth.
//  * Background, "Sorting": pairs are ordered by tile, then by depth.
//  * Design, "Sorting Optimizations in Context of 3DGS": the original method
//    uses a 64-bit integer key built from tile number and depth; only the tile
//    part of the key is needed to find each tile's range afterwards.
//  * Design, table of grouped preprocessing outputs: the duplication step
//    reads exactly the 2D mean, the depth and the radius of each Gaussian;
//    rendering also reads the conic-and-opacity and colour groups.
//  * Background, "Rendering", and Design, "Efficient Tile-Based Rendering":
//    every 16x16 tile composites its sorted Gaussians per pixel by alpha
//    blending, with the compositing rule of 3D Gaussian Splatting (Kerbl et
//    al. 2023), which the paper builds on (oracle_render).
//
// Readings where the paper is silent (each one also listed with the design
// notes of the repository):
//  * the box is open, (cx - r, cx + r) on each axis, and meets tile t when it
//    overlaps the half-open pixel span [16 t, 16 t + 16);
//  * radius 0 means culled (no pair at all);
//  * tile id = ty * tiles_x + tx (row-major), in the key's high 32 bits;
//    depth enters as its raw IEEE-754 bits in the low 32 bits;
//  * ascending order; equal keys keep duplication order (increasing index);
//  * a tile without pairs gets the empty range [p, p) with p = number of
//    pairs of lower tiles, so the ranges partition [0, M).
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

constexpr int64_t kFixed = 16;  // mean units per pixel

// floor(a / b) for b > 0, exact for negative a.
int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if (a % b != 0 && a < 0) --q;
  return q;
}

// ceil(a / b) for b > 0.
int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }

int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

bool valid_frame(const oracle_frame* f) {
  if (f == nullptr) return false;
  if (f->tile_px != 16) return false;
  if (f->width < 1 || f->height < 1) return false;
  if (f->width > (1u << 20) || f->height > (1u << 20)) return false;
  if (f->num_gaussians > 0 && f->gaussians == nullptr) return false;
  return true;
}

struct Rect {
  int64_t x0, x1, y0, y1;
};

// Overlap of Gaussian g's bounding box with the tile grid, in tile indices,
// half-open.  In fixed-point units a tile spans 16 * 16 = 256 units.  Tile tx
// meets the open box (X - R, X + R) iff 256 tx < X + R and X - R < 256 tx + 256,
// i.e. floor((X - R) / 256) <= tx < ceil((X + R) / 256).
Rect overlap_rect(const oracle_gaussian& g, int64_t tiles_x, int64_t tiles_y) {
  const int64_t span = kFixed * 16;
  const int64_t R = kFixed * static_cast<int64_t>(g.radius);
  const int64_t X = g.mean_x, Y = g.mean_y;
  Rect r;
  r.x0 = clamp64(floor_div(X - R, span), 0, tiles_x);
  r.x1 = clamp64(ceil_div(X + R, span), 0, tiles_x);
  r.y0 = clamp64(floor_div(Y - R, span), 0, tiles_y);
  r.y1 = clamp64(ceil_div(Y + R, span), 0, tiles_y);
  return r;
}

uint64_t rect_area(const oracle_gaussian& g, const Rect& r) {
  if (g.radius == 0) return 0;                    // culled by definition
  if (r.x1 <= r.x0 || r.y1 <= r.y0) return 0;    // box misses the image
  return static_cast<uint64_t>(r.x1 - r.x0) * static_cast<uint64_t>(r.y1 - r.y0);
}

uint32_t depth_bits(float d) {
  uint32_t b;
  std::memcpy(&b, &d, sizeof b);
  return b;
}

bool depth_ok(float d) { return std::isfinite(d) && d > 0.0f; }

struct Pair {
  uint64_t key;
  uint32_t value;
};

}  // namespace

extern "C" {

int oracle_tile_grid(const oracle_frame* f, uint32_t* tiles_x, uint32_t* tiles_y) {
  if (!valid_frame(f) || tiles_x == nullptr || tiles_y == nullptr) return ORACLE_ERR_INVALID_ARGUMENT;
  *tiles_x = static_cast<uint32_t>(ceil_div(f->width, f->tile_px));
  *tiles_y = static_cast<uint32_t>(ceil_div(f->height, f->tile_px));
  return ORACLE_OK;
}

int oracle_count(const oracle_frame* f, uint32_t* tiles_touched, uint32_t* rects) {
  uint32_t tx, ty;
  int st = oracle_tile_grid(f, &tx, &ty);
  if (st != ORACLE_OK) return st;
  for (uint32_t g = 0; g < f->num_gaussians; ++g) {
    const Rect r = overlap_rect(f->gaussians[g], tx, ty);
    const uint64_t area = rect_area(f->gaussians[g], r);
    if (tiles_touched) tiles_touched[g] = static_cast<uint32_t>(area);  // area <= 2^32
    if (rects) {
      rects[4 * (size_t)g + 0] = static_cast<uint32_t>(r.x0);
      rects[4 * (size_t)g + 1] = static_cast<uint32_t>(r.x1);
      rects[4 * (size_t)g + 2] = static_cast<uint32_t>(r.y0);
      rects[4 * (size_t)g + 3] = static_cast<uint32_t>(r.y1);
    }
  }
  return ORACLE_OK;
}

int oracle_scan(const uint32_t* counts, uint32_t n, uint64_t* offsets, uint64_t* total) {
  if ((n > 0 && (counts == nullptr || offsets == nullptr)) || total == nullptr) return ORACLE_ERR_INVALID_ARGUMENT;
  std::vector<uint64_t> wide(counts, counts + n);
  std::exclusive_scan(wide.begin(), wide.end(), offsets, uint64_t{0});
  *total = n == 0 ? 0 : offsets[n - 1] + wide[n - 1];
  return ORACLE_OK;
}

int oracle_duplicate(const oracle_frame* f, const uint64_t* offsets, uint64_t m,
                     uint64_t* keys, uint32_t* values) {
  uint32_t tiles_x, tiles_y;
  int st = oracle_tile_grid(f, &tiles_x, &tiles_y);
  if (st != ORACLE_OK) return st;
  for (uint32_t g = 0; g < f->num_gaussians; ++g) {
    const oracle_gaussian& G = f->gaussians[g];
    const Rect r = overlap_rect(G, tiles_x, tiles_y);
    if (rect_area(G, r) == 0) continue;
    uint64_t pos = offsets[g];
    for (int64_t ty = r.y0; ty < r.y1; ++ty) {
      for (int64_t tx = r.x0; tx < r.x1; ++tx) {
        if (pos >= m) return ORACLE_ERR_CAPACITY;
        const uint64_t tile = static_cast<uint64_t>(ty) * tiles_x + static_cast<uint64_t>(tx);
        keys[pos] = (tile << 32) | depth_bits(G.depth);
        values[pos] = g;
        ++pos;
      }
    }
  }
  return ORACLE_OK;
}

int oracle_sort(uint64_t* keys, uint32_t* values, uint64_t m) {
  std::vector<Pair> pairs(m);
  for (uint64_t i = 0; i < m; ++i) pairs[i] = Pair{keys[i], values[i]};
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const Pair& a, const Pair& b) { return a.key < b.key; });
  for (uint64_t i = 0; i < m; ++i) {
    keys[i] = pairs[i].key;
    values[i] = pairs[i].value;
  }
  return ORACLE_OK;
}

int oracle_ranges(const uint64_t* keys, uint64_t m, uint64_t num_tiles, uint32_t* ranges) {
  if (ranges == nullptr && num_tiles > 0) return ORACLE_ERR_INVALID_ARGUMENT;
  const uint64_t unset = ~uint64_t{0};
  std::vector<uint64_t> start(num_tiles, unset), end(num_tiles, unset);
  for (uint64_t i = 0; i < m; ++i) {
    const uint64_t t = keys[i] >> 32;
    if (t >= num_tiles) return ORACLE_ERR_INVALID_ARGUMENT;
    if (i == 0 || (keys[i - 1] >> 32) != t) start[t] = i;
    if (i + 1 == m || (keys[i + 1] >> 32) != t) end[t] = i + 1;
  }
  // Empty tiles: the range starts where the next non-empty tile starts.
  uint64_t next = m;
  for (uint64_t t = num_tiles; t-- > 0;) {
    if (start[t] == unset) {
      start[t] = end[t] = next;
    } else {
      next = start[t];
    }
  }
  for (uint64_t t = 0; t < num_tiles; ++t) {
    ranges[2 * t] = static_cast<uint32_t>(start[t]);
    ranges[2 * t + 1] = static_cast<uint32_t>(end[t]);
  }
  return ORACLE_OK;
}

int oracle_sort_frame(const oracle_frame* f, uint64_t capacity,
                      uint32_t* tiles_touched, uint64_t* offsets,
                      uint64_t* unsorted_keys, uint32_t* unsorted_values,
                      uint64_t* keys, uint32_t* values, uint32_t* ranges,
                      uint64_t* num_pairs) {
  uint32_t tiles_x, tiles_y;
  int st = oracle_tile_grid(f, &tiles_x, &tiles_y);
  if (st != ORACLE_OK || num_pairs == nullptr) return ORACLE_ERR_INVALID_ARGUMENT;
  const uint32_t n = f->num_gaussians;

  std::vector<uint32_t> cnt(n);
  oracle_count(f, cnt.data(), nullptr);
  for (uint32_t g = 0; g < n; ++g)
    if (cnt[g] > 0 && !depth_ok(f->gaussians[g].depth)) return ORACLE_ERR_INVALID_INPUT;

  std::vector<uint64_t> off(n);
  uint64_t m = 0;
  oracle_scan(cnt.data(), n, off.data(), &m);
  *num_pairs = m;
  if (tiles_touched) std::copy(cnt.begin(), cnt.end(), tiles_touched);
  if (offsets) std::copy(off.begin(), off.end(), offsets);
  if (m > 0xFFFFFFFFull) return ORACLE_ERR_OVERFLOW;
  if (m > capacity) return ORACLE_ERR_CAPACITY;

  std::vector<uint64_t> k(m);
  std::vector<uint32_t> v(m);
  oracle_duplicate(f, off.data(), m, k.data(), v.data());
  if (unsorted_keys) std::copy(k.begin(), k.end(), unsorted_keys);
  if (unsorted_values) std::copy(v.begin(), v.end(), unsorted_values);

  oracle_sort(k.data(), v.data(), m);
  if (keys) std::copy(k.begin(), k.end(), keys);
  if (values) std::copy(v.begin(), v.end(), values);

  if (ranges) oracle_ranges(k.data(), m, static_cast<uint64_t>(tiles_x) * tiles_y, ranges);
  return ORACLE_OK;
}

int oracle_render(const oracle_frame* f, const float* conic_opacity, const float* rgb, const uint32_t* values,
                  const uint32_t* ranges, const double background[3], int exact, double* out_color,
                  double* out_T, uint32_t* n_contrib, double* margin) {
  uint32_t tiles_x, tiles_y;
  if (oracle_tile_grid(f, &tiles_x, &tiles_y) != ORACLE_OK || background == nullptr) return ORACLE_ERR_INVALID_ARGUMENT;
  if (f->num_gaussians > 0 && (conic_opacity == nullptr || rgb == nullptr)) return ORACLE_ERR_INVALID_ARGUMENT;
  const uint64_t W = f->width, H = f->height;
  const double kMinAlpha = 1.0 / 255.0, kMaxAlpha = 0.99, kMinT = 1e-4;
  for (uint64_t y = 0; y < H; ++y) {
    for (uint64_t x = 0; x < W; ++x) {
      const uint64_t tile = (y / 16) * tiles_x + x / 16;
      const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
      double T = 1.0, c[3] = {0.0, 0.0, 0.0}, m = 1.0;
      uint32_t k = 0;
      for (uint32_t i = start; i < end; ++i) {
        const uint32_t g = values[i];
        const oracle_gaussian& G = f->gaussians[g];
        const double dx = G.mean_x / 16.0 - (static_cast<double>(x) + 0.5);
        const double dy = G.mean_y / 16.0 - (static_cast<double>(y) + 0.5);
        const double a = conic_opacity[4 * g], b = conic_opacity[4 * g + 1], cc = conic_opacity[4 * g + 2];
        const double q = a * dx * dx + 2.0 * b * dx * dy + cc * dy * dy;
        double alpha = conic_opacity[4 * g + 3] * std::exp(-0.5 * q);
        if (!exact) {
          if (q < 0.0) continue;
          alpha = std::min(kMaxAlpha, alpha);
          m = std::min(m, std::fabs(alpha - kMinAlpha) / kMinAlpha);
          if (alpha < kMinAlpha) continue;
          const double next = T * (1.0 - alpha);
          m = std::min(m, std::fabs(next - kMinT) / kMinT);
          if (next < kMinT) break;
        }
        for (int ch = 0; ch < 3; ++ch) c[ch] += rgb[4 * g + ch] * alpha * T;
        T *= 1.0 - alpha;
        ++k;
      }
      const uint64_t px = y * W + x;
      if (out_color)
        for (int ch = 0; ch < 3; ++ch) out_color[ch * W * H + px] = c[ch] + T * background[ch];
      if (out_T) out_T[px] = T;
      if (n_contrib) n_contrib[px] = k;
      if (margin) margin[px] = m;
    }
  }
  return ORACLE_OK;
}

}  // extern "C"

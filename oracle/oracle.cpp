// Plain CPU oracle of the per-frame tile-and-depth sort of 3D Gaussian
// Splatting.  TEST INFRASTRUCTURE ONLY: nothing in the product library links,
// loads or calls this file; the tests, the smoke check and the benchmark's
// CPU baseline do.  It is written to be read against the paper, not to be
// fast: one thread, plain loops, std::exclusive_scan and std::stable_sort.
// (oracle_sort_frame_mt repeats the same steps on several threads, only to
// time the CPU beside the GPU; it defines nothing.)
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

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <parallel/algorithm>
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

// The same steps on several host threads, for timing the CPU beside the GPU
// only (the tests check it against oracle_sort_frame before it is timed):
// the count and duplicate loops split over the Gaussians with OpenMP (each
// Gaussian writes its own segment [offsets[g], offsets[g] + count[g])), the
// scan and the range scan stay sequential, and the sort is libstdc++'s
// parallel-mode stable sort.  The result is the same pairs in the same order.
int oracle_sort_frame_mt(const oracle_frame* f, uint64_t capacity, uint64_t* keys, uint32_t* values,
                         uint32_t* ranges, uint64_t* num_pairs, int threads) {
  uint32_t tiles_x, tiles_y;
  int st = oracle_tile_grid(f, &tiles_x, &tiles_y);
  if (st != ORACLE_OK || num_pairs == nullptr || threads < 1) return ORACLE_ERR_INVALID_ARGUMENT;
  omp_set_num_threads(threads);
  const int64_t n = f->num_gaussians;

  std::vector<uint32_t> cnt(n);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t g = 0; g < n; ++g) {
    const oracle_gaussian& G = f->gaussians[g];
    cnt[g] = static_cast<uint32_t>(rect_area(G, overlap_rect(G, tiles_x, tiles_y)));
    if (cnt[g] > 0 && !depth_ok(G.depth)) bad = 1;
  }
  if (bad) return ORACLE_ERR_INVALID_INPUT;

  std::vector<uint64_t> off(n);
  uint64_t m = 0;
  oracle_scan(cnt.data(), static_cast<uint32_t>(n), off.data(), &m);
  *num_pairs = m;
  if (m > 0xFFFFFFFFull) return ORACLE_ERR_OVERFLOW;
  if (m > capacity) return ORACLE_ERR_CAPACITY;

  std::vector<Pair> pairs(m);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t g = 0; g < n; ++g) {
    if (cnt[g] == 0) continue;
    const oracle_gaussian& G = f->gaussians[g];
    const Rect r = overlap_rect(G, tiles_x, tiles_y);
    uint64_t pos = off[g];
    for (int64_t ty = r.y0; ty < r.y1; ++ty)
      for (int64_t tx = r.x0; tx < r.x1; ++tx) {
        const uint64_t t = static_cast<uint64_t>(tiles_x) * static_cast<uint64_t>(ty) + static_cast<uint64_t>(tx);
        pairs[pos++] = Pair{(t << 32) | depth_bits(G.depth), static_cast<uint32_t>(g)};
      }
  }
  __gnu_parallel::stable_sort(pairs.begin(), pairs.end(),
                              [](const Pair& x, const Pair& y) { return x.key < y.key; });
  std::vector<uint64_t> k(m);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < static_cast<int64_t>(m); ++i) {
    k[i] = pairs[i].key;
    if (keys) keys[i] = pairs[i].key;
    if (values) values[i] = pairs[i].value;
  }
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

// Associated Legendre function P_l^m(x), m >= 0, with the Condon-Shortley
// phase (-1)^m, by the standard recurrences.
static double assoc_legendre(int l, int m, double x) {
  double pmm = 1.0;
  if (m > 0) {
    const double s = std::sqrt(std::max(0.0, 1.0 - x * x));
    double f = 1.0;
    for (int i = 1; i <= m; ++i) {
      pmm *= -f * s;
      f += 2.0;
    }
  }
  if (l == m) return pmm;
  double pmmp1 = x * (2 * m + 1) * pmm;
  if (l == m + 1) return pmmp1;
  double pll = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pll = (x * (2 * ll - 1) * pmmp1 - (ll + m - 1) * pmm) / (ll - m);
    pmm = pmmp1;
    pmmp1 = pll;
  }
  return pll;
}

static double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

void oracle_sh_basis(const double d[3], double out[16]) {
  // real SH: Y_l0 = K_l0 P_l^0(cos t); Y_lm = sqrt(2) K_lm cos(m phi) P_l^m(cos t)
  // and Y_l,-m = sqrt(2) K_lm sin(m phi) P_l^m(cos t), m > 0, with
  // K_lm = sqrt((2l + 1) / (4 pi) (l - m)! / (l + m)!); cos t = z, phi = atan2(y, x)
  const double pi = 3.14159265358979323846;
  const double ct = d[2], phi = std::atan2(d[1], d[0]);
  int idx = 0;
  for (int l = 0; l <= 3; ++l) {
    for (int m = -l; m <= l; ++m) {
      const int am = std::abs(m);
      const double K = std::sqrt((2 * l + 1) / (4 * pi) * factorial(l - am) / factorial(l + am));
      const double P = assoc_legendre(l, am, ct);
      double y;
      if (m == 0) y = K * P;
      else if (m > 0) y = std::sqrt(2.0) * K * std::cos(m * phi) * P;
      else y = std::sqrt(2.0) * K * std::sin(am * phi) * P;
      out[idx++] = y;
    }
  }
}

int oracle_preprocess(const oracle_camera* cam, uint32_t n, const float* mean3d_opacity, const float* cov3d,
                      const float* sh, oracle_gaussian* records, double* conic_opacity, double* rgb,
                      double* margin) {
  if (cam == nullptr || cam->sh_degree > 3 || (n > 0 && (mean3d_opacity == nullptr || cov3d == nullptr)))
    return ORACLE_ERR_INVALID_ARGUMENT;
  if (cam->sh_degree > 0 || rgb != nullptr)
    if (n > 0 && sh == nullptr) return ORACLE_ERR_INVALID_ARGUMENT;
  const double* V = cam->view;
  for (uint32_t g = 0; g < n; ++g) {
    const double p[3] = {mean3d_opacity[4 * g], mean3d_opacity[4 * g + 1], mean3d_opacity[4 * g + 2]};
    const double opacity = mean3d_opacity[4 * g + 3];
    double t[3];
    for (int r = 0; r < 3; ++r) t[r] = V[4 * r] * p[0] + V[4 * r + 1] * p[1] + V[4 * r + 2] * p[2] + V[4 * r + 3];
    oracle_gaussian rec{0, 0, static_cast<float>(t[2]), 0};
    double co[4] = {0, 0, 0, 0}, col[3] = {0, 0, 0}, mg[3] = {1, 1, 1};
    bool culled = t[2] <= cam->near_plane;
    double a = 0, b = 0, c = 0, det = 0, x = 0, y = 0;
    if (!culled) {
      x = cam->fx * t[0] / t[2] + cam->cx;
      y = cam->fy * t[1] / t[2] + cam->cy;
      // projection Jacobian at t, with x/z and y/z clamped to 1.3 tan(fov/2)
      const double lx = 1.3 * cam->tan_fovx, ly = 1.3 * cam->tan_fovy;
      const double tx = std::min(lx, std::max(-lx, t[0] / t[2])) * t[2];
      const double ty = std::min(ly, std::max(-ly, t[1] / t[2])) * t[2];
      const double J[2][3] = {{cam->fx / t[2], 0.0, -cam->fx * tx / (t[2] * t[2])},
                              {0.0, cam->fy / t[2], -cam->fy * ty / (t[2] * t[2])}};
      const float* cv = cov3d + 8 * g;
      const double S[3][3] = {{cv[0], cv[1], cv[2]}, {cv[1], cv[3], cv[4]}, {cv[2], cv[4], cv[5]}};
      double M[2][3];  // J R
      for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k) M[i][k] = J[i][0] * V[k] + J[i][1] * V[4 + k] + J[i][2] * V[8 + k];
      double C[2][2];  // M S M^T
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) acc += M[i][k] * S[k][l] * M[j][l];
          C[i][j] = acc;
        }
      a = C[0][0] + 0.3;
      b = C[0][1];
      c = C[1][1] + 0.3;
      det = a * c - b * b;
      if (det == 0.0) culled = true;
    }
    if (!culled) {
      const double mid = 0.5 * (a + c);
      const double l1 = mid + std::sqrt(std::max(0.1, mid * mid - det));
      const double l2 = mid - std::sqrt(std::max(0.1, mid * mid - det));
      const double r3 = 3.0 * std::sqrt(std::max(l1, l2));
      rec.radius = static_cast<uint32_t>(std::ceil(r3));
      mg[2] = std::fabs(r3 - std::nearbyint(r3));
      const double X = std::min(1073741824.0, std::max(-1073741824.0, 16.0 * x));
      const double Y = std::min(1073741824.0, std::max(-1073741824.0, 16.0 * y));
      rec.mean_x = static_cast<int32_t>(std::nearbyint(X));   // current rounding mode: half to even
      rec.mean_y = static_cast<int32_t>(std::nearbyint(Y));
      mg[0] = std::fabs(std::fabs(X - std::floor(X)) - 0.5);
      mg[1] = std::fabs(std::fabs(Y - std::floor(Y)) - 0.5);
      co[0] = c / det;
      co[1] = -b / det;
      co[2] = a / det;
      co[3] = opacity;
      // colour from the spherical harmonics of the viewing direction
      double d[3] = {p[0] - cam->cam_pos[0], p[1] - cam->cam_pos[1], p[2] - cam->cam_pos[2]};
      const double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (double& v : d) v /= len;
      double basis[16];
      oracle_sh_basis(d, basis);
      const int nb = (static_cast<int>(cam->sh_degree) + 1) * (static_cast<int>(cam->sh_degree) + 1);
      for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < nb; ++k) acc += sh[48 * static_cast<size_t>(g) + 3 * k + ch] * basis[k];
        col[ch] = std::max(0.0, acc);
      }
    } else {
      rec.mean_x = rec.mean_y = 0;
      rec.radius = 0;
    }
    if (records) records[g] = rec;
    if (conic_opacity)
      for (int i = 0; i < 4; ++i) conic_opacity[4 * static_cast<size_t>(g) + i] = co[i];
    if (rgb) {
      for (int i = 0; i < 3; ++i) rgb[4 * static_cast<size_t>(g) + i] = col[i];
      rgb[4 * static_cast<size_t>(g) + 3] = 0.0;
    }
    if (margin)
      for (int i = 0; i < 3; ++i) margin[3 * static_cast<size_t>(g) + i] = mg[i];
  }
  return ORACLE_OK;
}

}  // extern "C"

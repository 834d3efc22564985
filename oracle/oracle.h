/* Plain CPU oracle of the per-frame tile-and-depth sort of 3D Gaussian
 * Splatting.  TEST INFRASTRUCTURE ONLY: the product library never links,
 * loads or calls it.  Only the tests, the smoke check and the CPU baseline
 * of the benchmark use it.
 *
 * What it computes (paper: Background, "Duplication with Tiles" and
 * "Sorting"; Design, "Sorting Optimizations in Context of 3DGS"): the list of
 * all (tile, Gaussian) pairs whose 16x16-pixel tile meets the Gaussian's
 * axis-aligned bounding box, ordered by tile, then by depth, then by Gaussian
 * index, as 64-bit keys (tile << 32 | depth bits) with 32-bit index values,
 * plus each tile's [start, end) range into that list.
 *
 * This header defines its own types; it shares nothing with the GPU library.
 * Status numbers equal the GPU library's status codes so results compare.
 */
#ifndef SPLAT_ORACLE_H
#define SPLAT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_ERR_INVALID_ARGUMENT = 1,
  ORACLE_ERR_CAPACITY = 3,
  ORACLE_ERR_OVERFLOW = 4,
  ORACLE_ERR_INVALID_INPUT = 5
};

/* One projected Gaussian: mean in signed 1/16-pixel fixed point, FP32 view
 * depth, radius in whole pixels (0 = culled).  16 bytes. */
typedef struct {
  int32_t mean_x;
  int32_t mean_y;
  float depth;
  uint32_t radius;
} oracle_gaussian;

typedef struct {
  uint32_t width;   /* pixels, 1 .. 2^20 */
  uint32_t height;  /* pixels, 1 .. 2^20 */
  uint32_t tile_px; /* must be 16 */
  uint32_t num_gaussians;
  const oracle_gaussian* gaussians;
} oracle_frame;

/* a0: tile grid size; partial edge tiles count. */
int oracle_tile_grid(const oracle_frame* f, uint32_t* tiles_x, uint32_t* tiles_y);

/* a1: per-Gaussian overlap rectangle [x0,x1) x [y0,y1) in tiles and its area.
 * rects may be NULL; otherwise rects[4g..4g+3] = x0, x1, y0, y1. */
int oracle_count(const oracle_frame* f, uint32_t* tiles_touched, uint32_t* rects);

/* a2: exclusive prefix sum of the counts, and the total M. */
int oracle_scan(const uint32_t* counts, uint32_t n, uint64_t* offsets, uint64_t* total);

/* a3: one (key, value) pair per touched tile, Gaussian by Gaussian, tiles of a
 * Gaussian in row-major order.  keys/values hold m entries. */
int oracle_duplicate(const oracle_frame* f, const uint64_t* offsets, uint64_t m,
                     uint64_t* keys, uint32_t* values);

/* a4: stable sort of the pairs by the full 64-bit key, in place. */
int oracle_sort(uint64_t* keys, uint32_t* values, uint64_t m);

/* a5: ranges[2t], ranges[2t+1] = start, end of tile t in the sorted keys.
 * Tiles with no pair get start = end = the number of pairs of lower tiles. */
int oracle_ranges(const uint64_t* keys, uint64_t m, uint64_t num_tiles, uint32_t* ranges);

/* Whole frame: a1..a5.  Any output pointer except num_pairs may be NULL.
 * keys/values must hold capacity entries; unsorted_* receive the a3 order.
 * Returns ORACLE_ERR_OVERFLOW if M > 2^32-1, ORACLE_ERR_CAPACITY if
 * M > capacity (num_pairs is still written), ORACLE_ERR_INVALID_INPUT if a
 * Gaussian that touches a tile has a depth that is not positive and finite. */
int oracle_sort_frame(const oracle_frame* f, uint64_t capacity,
                      uint32_t* tiles_touched, uint64_t* offsets,
                      uint64_t* unsorted_keys, uint32_t* unsorted_values,
                      uint64_t* keys, uint32_t* values, uint32_t* ranges,
                      uint64_t* num_pairs);

/* Render (the step after the sort; paper: Background, "Rendering", and
 * Design, "Efficient Tile-Based Rendering"): every pixel of a tile composites
 * the tile's Gaussians front to back, in the order of the sorted values,
 * by alpha blending as in 3D Gaussian Splatting (Kerbl et al. 2023):
 *   pixel (x, y) is sampled at its centre (x + 1/2, y + 1/2), in the frame in
 *   which a Gaussian's mean is (mean_x / 16, mean_y / 16);
 *   d = mean - sample; q = a dx^2 + 2 b dx dy + c dy^2 with (a, b, c) the
 *   conic (inverse 2D covariance); alpha = opacity * exp(-q / 2);
 *   colour += rgb * alpha * T, then T *= 1 - alpha, starting from T = 1;
 *   the result is colour + T * background.
 * The 3DGS rasteriser's thresholds apply unless exact != 0: a Gaussian with
 * q < 0 is skipped, alpha is capped at 0.99, a Gaussian with alpha < 1/255
 * is skipped, and a pixel stops (without that Gaussian) once T (1 - alpha)
 * would drop below 1e-4.  Arithmetic in double.
 *
 * conic_opacity[4g..4g+3] = a, b, c, opacity; rgb[4g..4g+2] = colour.
 * values/ranges are a sorted frame (oracle_sort_frame).  Outputs per pixel,
 * row-major, colour planar [3][H][W]: out_color, out_T (final T), n_contrib
 * (Gaussians composited) and margin (the smallest relative distance of an
 * evaluated alpha to 1/255 or of T (1 - alpha) to 1e-4; 1 if none) -- any
 * output may be NULL. */
int oracle_render(const oracle_frame* f, const float* conic_opacity, const float* rgb, const uint32_t* values,
                  const uint32_t* ranges, const double background[3], int exact, double* out_color,
                  double* out_T, uint32_t* n_contrib, double* margin);

/* Preprocess (the step before the sort; paper: Background, "Preprocessing",
 * and Design, "Variable Packing" with its input and output group tables):
 * 3D Gaussians (mean and opacity, 3D covariance, spherical-harmonic colour)
 * and a pinhole camera in; per Gaussian out the 16-byte record of the sort
 * (2D mean in 1/16 px, depth, radius), the conic and opacity, and the colour.
 * It follows 3D Gaussian Splatting (Kerbl et al. 2023), which the paper
 * builds on:
 *   t = R p + T (camera frame); culled (radius 0) when t.z <= near;
 *   pixel = (fx t.x / t.z + cx, fy t.y / t.z + cy);
 *   2D covariance = J R S R^T J^T + 0.3 I, with the projection's Jacobian J at
 *   t, its x/z and y/z clamped to 1.3 tan(fov/2) on each axis;
 *   culled when that covariance is singular; conic = its inverse;
 *   radius = ceil(3 sqrt(largest eigenvalue)), the eigenvalue taken as
 *   mid + sqrt(max(0.1, mid^2 - det)), mid = half the trace;
 *   colour = max(0, 1/2 + sum over SH degrees <= sh_degree of coefficient *
 *   real spherical harmonic (with the Condon-Shortley phase) of the unit
 *   direction from the camera centre to p).
 * mean3d_opacity [n][4]; cov3d [n][8] = xx, xy, xz, yy, yz, zz, -, -;
 * sh [n][48] = 16 coefficients x RGB, in (l, m = -l..l) order.  Outputs:
 * records (mean rounded half-to-even to 1/16 px), conic_opacity [n][4],
 * rgb [n][4] (double), and margin [n][3]: the distance of 16 x and 16 y to
 * a rounding boundary (in 1/16 px) and of 3 sqrt(eigenvalue) to an integer;
 * culled Gaussians get radius 0, zero conic and colour.  Arithmetic in
 * double; any output may be NULL. */
typedef struct {
  double view[12];            /* [R | T], row-major 3 x 4 */
  double fx, fy, cx, cy;      /* focal lengths and principal point, pixels */
  double tan_fovx, tan_fovy;  /* half-angle tangents */
  double cam_pos[3];          /* camera centre in world coordinates */
  double near_plane;
  uint32_t sh_degree;         /* 0 .. 3 */
} oracle_camera;

int oracle_preprocess(const oracle_camera* cam, uint32_t n, const float* mean3d_opacity, const float* cov3d,
                      const float* sh, oracle_gaussian* records, double* conic_opacity, double* rgb,
                      double* margin);

/* oracle_sort_frame on `threads` host threads (OpenMP count and duplicate
 * loops, parallel-mode stable sort), for timing the CPU beside the GPU only.
 * Outputs keys, values (may be NULL) and ranges (may be NULL) as
 * oracle_sort_frame does, with the same statuses. */
int oracle_sort_frame_mt(const oracle_frame* f, uint64_t capacity, uint64_t* keys, uint32_t* values,
                         uint32_t* ranges, uint64_t* num_pairs, int threads);

/* The real spherical harmonics (Condon-Shortley phase) used above, degree
 * <= 3, at unit direction d: out[16] in (l, m = -l..l) order. */
void oracle_sh_basis(const double d[3], double out[16]);

#ifdef __cplusplus
}
#endif

#endif

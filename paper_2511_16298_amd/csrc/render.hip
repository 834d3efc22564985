// Rendering: per-tile alpha blending over the sorted tile lists (paper:
// Background, "Rendering"; Design, "Efficient Tile-Based Rendering" -- one
// workgroup per 16x16 tile, several pixels per thread, colour channels
// unrolled).  On MI355X one wave64 owns one tile: lane l holds the four
// pixels l, l + 64, l + 128, l + 192 of the tile (rows l/16, l/16 + 4, ...).
// Every 64 list entries the lanes load one Gaussian each (mean, conic and
// opacity, colour) and store its nine per-Gaussian values in the wave's own
// LDS slots; the wave then walks them in order, all lanes reading the same
// slot (a broadcast read, on the LDS pipe rather than the vector ALU), and
// every lane blends its four pixels.  The wave leaves the list once all 256
// pixels have stopped, tested every fourth Gaussian.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

constexpr uint32_t kRenderWaves = 4;  // tiles per workgroup
constexpr float kMaxAlpha = 0.99f;
constexpr float kMinAlpha = 1.0f / 255.0f;
constexpr float kMinT = 1e-4f;
// opacity * exp(-q / 2) = 2^(log2(opacity) - q log2(e) / 2): the factor is
// folded into the conic and log2(opacity) into the dx term once per
// Gaussian, so a pixel evaluates 2^p, p = log2(o) + a' dx^2 + 2 b' dx dy + c' dy^2
constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2

// A tile's Gaussian batch in LDS: 64 slots of nine values.
struct RenderSlots {
  float4 geo[kWave];   // mean x, mean y, -log2(e)/2 * (conic a, conic b)
  float4 mix[kWave];   // -log2(e)/2 * conic c, log2(opacity), red, green
  float blue[kWave];
};

// Gaussians blended between two tests of the wave's live pixels.  A batch's
// slots past its last entry hold a Gaussian that changes no pixel (opacity 0:
// log2 = -inf, so 2^p = 0), so every batch walks whole groups; a stopped pixel
// is left unchanged by further Gaussians, so testing once a group only adds
// work, never changes the image.
constexpr uint32_t kGroup = 4;

// Blends the Gaussian of slot j into the lane's four pixels.  `counted`
// (uniform): slot j holds a list entry, not padding (for the statistics).
template <bool EXACT, bool STATS>
__device__ __forceinline__ void blend(const RenderSlots& sl, uint32_t j, bool counted, float sx, const float (&sy)[4],
                                      float (&T)[4], float (&cr)[4], float (&cg)[4], float (&cb)[4], uint32_t (&n)[4],
                                      uint32_t& evals) {
  const float4 g0 = sl.geo[j], g1 = sl.mix[j];
  const float Gx = g0.x, Gy = g0.y, A = g0.z, B = g0.w, C = g1.x, O = g1.y;
  const float R = g1.z, Gc = g1.w, Bl = sl.blue[j];
  // p = log2(o) - q log2(e) / 2 with q = A dx^2 + 2 B dx dy + C dy^2, as
  // (log2(o) + A' dx^2) + dy (2 B' dx + C' dy): the dx terms are shared by
  // the lane's four pixels (one column); q >= 0 is p <= log2(o)
  const float dx = Gx - sx;
  const float qa = fmaf(A * dx, dx, O);
  const float qb = 2.0f * B * dx;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float dy = Gy - sy[k];
    const float q = fmaf(dy, fmaf(C, dy, qb), qa);  // = p
    const float e = __builtin_amdgcn_exp2f(q);
    if (EXACT) {
      const float w = e * T[k];
      cr[k] = fmaf(R, w, cr[k]);
      cg[k] = fmaf(Gc, w, cg[k]);
      cb[k] = fmaf(Bl, w, cb[k]);
      T[k] = fmaf(-e, T[k], T[k]);
      if (STATS) n[k] += counted ? 1u : 0u;
    } else {
      const float alpha = fminf(kMaxAlpha, e);
      if (STATS) evals += counted && T[k] > 0.0f ? 1u : 0u;
      // a stopped pixel needs no test here: its T is negative, so is next,
      // which reads as a stop again and leaves it unchanged
      const float ae = (q <= O && alpha >= kMinAlpha) ? alpha : 0.0f;
      const float next = fmaf(-ae, T[k], T[k]);
      const bool stop = next < kMinT;  // also true for a pixel already stopped
      const float w = stop ? 0.0f : ae * T[k];
      cr[k] = fmaf(R, w, cr[k]);
      cg[k] = fmaf(Gc, w, cg[k]);
      cb[k] = fmaf(Bl, w, cb[k]);
      T[k] = stop ? -fabsf(T[k]) : next;
      if (STATS) n[k] += w != 0.0f ? 1u : 0u;
    }
  }
  if (EXACT && STATS) evals += counted ? 4u : 0u;
}

// EXACT: no thresholds.  STATS: also count the Gaussians composited per pixel
// and the evaluations per tile.  A pixel that has stopped keeps its T with the
// sign bit set (T > 0 means live), so the thresholds cost selects, not
// branches, and the lanes never diverge.  The plain kernels are held to 64
// VGPRs, eight waves per SIMD: a full-HD frame's 8,160 tile waves are then all
// resident at once, which beats both fewer resident waves and fewer registers
// spent on the next batch's loads.
template <bool EXACT, bool STATS>
__global__ __launch_bounds__(kRenderWaves * kWave) __attribute__((amdgpu_waves_per_eu(STATS ? 1 : 8, 8))) void k_render(RenderArgs a) {
  __shared__ RenderSlots slots[kRenderWaves];
  if (a.status && *a.status != SS_OK) return;
  const uint32_t lane = lane_id();
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // uniform over the wave: the list bounds are scalar loads
  const uint32_t tile = blockIdx.x * kRenderWaves + wave;
  if (tile >= a.tiles_x * a.tiles_y) return;
  RenderSlots& sl = slots[wave];
  const uint32_t tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];

  // sample points of this lane's four pixels
  const float sx = static_cast<float>(tx * 16 + (lane & 15)) + 0.5f;
  float sy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) sy[k] = static_cast<float>(ty * 16 + (lane >> 4) + 4 * k) + 0.5f;

  float T[4], cr[4], cg[4], cb[4];
  uint32_t n[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T[k] = 1.0f;
    cr[k] = cg[k] = cb[k] = 0.0f;
    n[k] = 0;
  }
  uint32_t evals = 0;

  // The next batch's Gaussians are loaded while the wave walks the current
  // one, so the gathers' latency hides behind the blending.
  int2 m = make_int2(0, 0);
  float4 co = make_float4(0.0f, 0.0f, 0.0f, 0.0f), cl = co;
  if (start + lane < end) {
    const uint32_t gi = a.values[start + lane];
    m = *reinterpret_cast<const int2*>(a.gaussians + gi);
    co = reinterpret_cast<const float4*>(a.conic_opacity)[gi];
    cl = reinterpret_cast<const float4*>(a.rgb)[gi];
  }
  bool live = true;
  for (uint32_t b = start; b < end && live; b += kWave) {
    // one Gaussian per lane into the wave's slots; padding past the end
    const bool valid = b + lane < end;
    sl.geo[lane] = make_float4(valid ? static_cast<float>(m.x) * (1.0f / 16.0f) : 0.0f,
                               valid ? static_cast<float>(m.y) * (1.0f / 16.0f) : 0.0f,
                               valid ? -kHalfLog2e * co.x : 0.0f, valid ? -kHalfLog2e * co.y : 0.0f);
    // log2(opacity); opacity in (0, 1]
    sl.mix[lane] = make_float4(valid ? -kHalfLog2e * co.z : 0.0f,
                               valid ? __builtin_amdgcn_logf(co.w) : -__builtin_inff(), valid ? cl.x : 0.0f,
                               valid ? cl.y : 0.0f);
    sl.blue[lane] = valid ? cl.z : 0.0f;
    const uint32_t nb = b + kWave;
    if (nb + lane < end) {
      const uint32_t gi = a.values[nb + lane];
      m = *reinterpret_cast<const int2*>(a.gaussians + gi);
      co = reinterpret_cast<const float4*>(a.conic_opacity)[gi];
      cl = reinterpret_cast<const float4*>(a.rgb)[gi];
    }
    // the slots are this wave's alone and its LDS accesses complete in
    // order, so the reads below see the stores above without a barrier
    __builtin_amdgcn_wave_barrier();
    const uint32_t count = end - b < kWave ? end - b : kWave;
    for (uint32_t j = 0; j < count; j += kGroup) {
#pragma unroll
      for (uint32_t u = 0; u < kGroup; ++u)
        blend<EXACT, STATS>(sl, j + u, j + u < count, sx, sy, T, cr, cg, cb, n, evals);
      if (!EXACT) {
        live = ballot(fmaxf(fmaxf(T[0], T[1]), fmaxf(T[2], T[3])) > 0.0f) != 0;
        if (!live) break;
      }
    }
    // the next batch's stores follow this batch's reads
    __builtin_amdgcn_wave_barrier();
  }

  const uint32_t W = a.width, H = a.height;
  const size_t plane = static_cast<size_t>(W) * H;
  const uint32_t px = tx * 16 + (lane & 15);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t py = ty * 16 + (lane >> 4) + 4 * k;
    const float t = fabsf(T[k]);
    if (px < W && py < H) {
      const size_t o = static_cast<size_t>(py) * W + px;
      a.color[o] = cr[k] + t * a.bg[0];
      a.color[plane + o] = cg[k] + t * a.bg[1];
      a.color[2 * plane + o] = cb[k] + t * a.bg[2];
      if (a.T) a.T[o] = t;
      if (STATS && a.contrib) a.contrib[o] = n[k];
    }
  }
  if (STATS && a.tile_evals) {
    // sum over the wave of the per-lane evaluation counts
    uint32_t e = evals;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) e += __shfl_xor(e, d, kWave);
    if (lane == 0) a.tile_evals[tile] = e;
  }
}

}  // namespace

hipError_t launch_render(const RenderArgs& a, bool exact, hipStream_t s) {
  const uint32_t tiles = a.tiles_x * a.tiles_y;
  const uint32_t blocks = (tiles + kRenderWaves - 1) / kRenderWaves;
  if (blocks == 0) return hipSuccess;
  const dim3 g(blocks), t(kRenderWaves * kWave);
  const bool stats = a.contrib != nullptr || a.tile_evals != nullptr;
  if (exact && stats) hipLaunchKernelGGL((k_render<true, true>), g, t, 0, s, a);
  else if (exact) hipLaunchKernelGGL((k_render<true, false>), g, t, 0, s, a);
  else if (stats) hipLaunchKernelGGL((k_render<false, true>), g, t, 0, s, a);
  else hipLaunchKernelGGL((k_render<false, false>), g, t, 0, s, a);
  return hipGetLastError();
}

}  // namespace ss

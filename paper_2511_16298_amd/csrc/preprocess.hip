// Preprocess: 3D Gaussians and a pinhole camera to the sort's 16-byte records,
// the conic and opacity, and the colour (paper: Background, "Preprocessing";
// Design, "Variable Packing" and its input/output group tables -- mean and
// opacity, 3D covariance, spherical-harmonic coefficients in; mean, depth,
// radius / conic and opacity / colour out -- following 3D Gaussian Splatting):
//   t = R p + T; culled when t.z <= near;
//   pixel = (fx t.x / t.z + cx, fy t.y / t.z + cy), stored in 1/16 px,
//     rounded half to even;
//   2D covariance = J R S R^T J^T + 0.3 I, J the projection's Jacobian at t
//     with t.x / t.z and t.y / t.z clamped to 1.3 tan(fov / 2);
//   culled when it is singular; conic = its inverse;
//   radius = ceil(3 sqrt(mid + sqrt(max(0.1, mid^2 - det)))), mid = trace / 2;
//   colour = max(0, 1/2 + sum of SH coefficients times the real harmonics
//     (Condon-Shortley phase) of the direction from the camera to p).
// One thread per Gaussian; a memory-bound stream of 240 bytes in and 48 out.
// The 192 bytes of SH coefficients per Gaussian are the bulk.  Loaded one
// row per lane they would touch 64 rows 192 bytes apart per instruction;
// each wave instead reads its 64 rows as two contiguous 6-KB blocks of 32
// rows (1 KB per load instruction, and no cache line shared between the
// blocks, so every line is fetched once), transposes each block through LDS
// with rows padded to 13 float4 (16 consecutive rows start in distinct bank
// groups, so the 16-byte row reads do not conflict), and the block's 32 lanes
// read their rows back.  All loads of a wave are issued before its first
// wait; 26 KB of LDS and 94 VGPRs leave five waves per SIMD.
#include "common.hpp"
#include "internal.hpp"

namespace ss {
namespace {

// Real spherical harmonics with the Condon-Shortley phase, degree <= 3, in
// (l, m = -l..l) order, as constant x polynomial in the unit direction:
// l = 0: 1 / (2 sqrt(pi)); l = 1: sqrt(3 / (4 pi)) (-y, z, -x);
// l = 2: sqrt(15 / pi) / 2 (xy, -yz), sqrt(5 / pi) / 4 (2z^2 - x^2 - y^2),
//        -sqrt(15 / pi) / 2 xz, sqrt(15 / pi) / 4 (x^2 - y^2);
// l = 3: -sqrt(35 / (2 pi)) / 4 y (3x^2 - y^2), sqrt(105 / pi) / 2 xyz,
//        -sqrt(21 / (2 pi)) / 4 y (4z^2 - x^2 - y^2),
//        sqrt(7 / pi) / 4 z (2z^2 - 3x^2 - 3y^2),
//        -sqrt(21 / (2 pi)) / 4 x (4z^2 - x^2 - y^2),
//        sqrt(105 / pi) / 4 z (x^2 - y^2), -sqrt(35 / (2 pi)) / 4 x (x^2 - 3y^2).
constexpr float kY00 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kY2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kY2c = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float kY3a = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float kY3b = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float kY3c = 0.45704579946446572f;  // sqrt(21 / (2 pi)) / 4
constexpr float kY3d = 0.37317633259011540f;  // sqrt(7 / pi) / 4
constexpr float kY3e = 1.4453057213202769f;   // sqrt(105 / pi) / 4

// a c - b^2 with the rounding error of b^2 put back (Kahan's 2x2
// determinant): close to correctly rounded even when the two terms nearly
// cancel, which they do for elongated footprints.
__device__ __forceinline__ float det2(float a, float b, float c) {
  const float w = b * b;
  const float e = fmaf(-b, b, w);
  return fmaf(a, c, -w) + e;
}

constexpr uint32_t kThreads = 256;
constexpr uint32_t kStageRows = 32;    // SH rows per LDS stage
constexpr uint32_t kRowSlots = 13;     // float4 per padded LDS row (12 + 1)

__global__ __launch_bounds__(kThreads) void k_preprocess(PreprocessArgs a) {
  __shared__ float4 lds[kThreads / kWave][kStageRows * kRowSlots];
  const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const uint32_t g = blockIdx.x * kThreads + threadIdx.x;
  const uint32_t wave_first = g - lane;
  const uint32_t nb = (a.cam.sh_degree + 1) * (a.cam.sh_degree + 1);
  float4 po = make_float4(0.f, 0.f, 0.f, 0.f), s0 = po, s1 = po;
  if (g < a.n) {
    po = reinterpret_cast<const float4*>(a.mean3d_opacity)[g];
    s0 = reinterpret_cast<const float4*>(a.cov3d)[2 * static_cast<size_t>(g)];
    s1 = reinterpret_cast<const float4*>(a.cov3d)[2 * static_cast<size_t>(g) + 1];
  }
  // stage s holds rows 32 s .. 32 s + 31 of the wave, a contiguous 6-KB
  // block: its float4 f = 64 q + lane (q < 6) is part f % 12 of local row f / 12
  const float4* src = reinterpret_cast<const float4*>(a.sh) + static_cast<size_t>(wave_first) * 12;
  float4 ld[12];
#pragma unroll
  for (uint32_t st = 0; st < 2; ++st)
#pragma unroll
    for (uint32_t q = 0; q < 6; ++q) {
      const uint32_t f = kWave * q + lane, row = kStageRows * st + f / 12, part = f % 12;
      ld[6 * st + q] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (wave_first + row < a.n && 4 * part < 3 * nb) ld[6 * st + q] = src[384 * st + f];
    }
  float4 shr[12];
#pragma unroll
  for (uint32_t st = 0; st < 2; ++st) {
#pragma unroll
    for (uint32_t q = 0; q < 6; ++q) {
      const uint32_t f = kWave * q + lane;
      lds[wave][(f / 12) * kRowSlots + f % 12] = ld[6 * st + q];
    }
    __syncthreads();
    if (lane / kStageRows == st) {
#pragma unroll
      for (uint32_t q = 0; q < 12; ++q) shr[q] = lds[wave][(lane % kStageRows) * kRowSlots + q];
    }
    __syncthreads();
  }
  if (g >= a.n) return;
  const ss_camera& c = a.cam;
  const float tx0 = c.view[0] * po.x + c.view[1] * po.y + c.view[2] * po.z + c.view[3];
  const float ty0 = c.view[4] * po.x + c.view[5] * po.y + c.view[6] * po.z + c.view[7];
  const float tz = c.view[8] * po.x + c.view[9] * po.y + c.view[10] * po.z + c.view[11];

  int4 rec = make_int4(0, 0, __float_as_int(tz), 0);
  float4 co = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 col = make_float4(0.f, 0.f, 0.f, 0.f);
  bool culled = tz <= c.near_plane;
  float a2 = 0.f, b2 = 0.f, c2 = 0.f, det = 0.f, x = 0.f, y = 0.f;
  if (!culled) {
    const float iz = 1.0f / tz;
    x = c.fx * tx0 * iz + c.cx;
    y = c.fy * ty0 * iz + c.cy;
    const float lx = 1.3f * c.tan_fovx, ly = 1.3f * c.tan_fovy;
    const float ux = fminf(lx, fmaxf(-lx, tx0 * iz));
    const float uy = fminf(ly, fmaxf(-ly, ty0 * iz));
    // J = [[fx/z, 0, -fx u_x/z], [0, fy/z, -fy u_y/z]] (u = clamped t.xy / z);  M = J R
    const float j00 = c.fx * iz, j02 = -j00 * ux;
    const float j11 = c.fy * iz, j12 = -j11 * uy;
    float M[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      M[0][k] = j00 * c.view[k] + j02 * c.view[8 + k];
      M[1][k] = j11 * c.view[4 + k] + j12 * c.view[8 + k];
    }
    const float S[3][3] = {{s0.x, s0.y, s0.z}, {s0.y, s0.w, s1.x}, {s0.z, s1.x, s1.y}};
    float MS[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) MS[i][k] = M[i][0] * S[0][k] + M[i][1] * S[1][k] + M[i][2] * S[2][k];
    a2 = MS[0][0] * M[0][0] + MS[0][1] * M[0][1] + MS[0][2] * M[0][2] + 0.3f;
    b2 = MS[0][0] * M[1][0] + MS[0][1] * M[1][1] + MS[0][2] * M[1][2];
    c2 = MS[1][0] * M[1][0] + MS[1][1] * M[1][1] + MS[1][2] * M[1][2] + 0.3f;
    det = det2(a2, b2, c2);
    if (det == 0.0f) culled = true;
  }
  if (!culled) {
    // largest eigenvalue: mid + sqrt(mid^2 - det), with mid^2 - det formed as
    // ((a - c) / 2)^2 + b^2 (the same quantity without the cancellation)
    const float mid = 0.5f * (a2 + c2), hd = 0.5f * (a2 - c2);
    const float l1 = mid + sqrtf(fmaxf(0.1f, fmaf(hd, hd, b2 * b2)));
    rec.w = static_cast<int>(static_cast<uint32_t>(ceilf(3.0f * sqrtf(l1))));
    const float X = fminf(1073741824.0f, fmaxf(-1073741824.0f, 16.0f * x));
    const float Y = fminf(1073741824.0f, fmaxf(-1073741824.0f, 16.0f * y));
    rec.x = static_cast<int>(rintf(X));  // round half to even
    rec.y = static_cast<int>(rintf(Y));
    const float idet = 1.0f / det;
    co = make_float4(c2 * idet, -b2 * idet, a2 * idet, po.w);

    float dx = po.x - c.cam_pos[0], dy = po.y - c.cam_pos[1], dz = po.z - c.cam_pos[2];
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= il;
    dy *= il;
    dz *= il;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float Yb[16] = {kY00,
                          -kY1 * dy, kY1 * dz, -kY1 * dx,
                          kY2a * dx * dy, -kY2a * dy * dz, kY2b * (2.0f * zz - xx - yy), -kY2a * dx * dz,
                          kY2c * (xx - yy),
                          -kY3a * dy * (3.0f * xx - yy), kY3b * dx * dy * dz,
                          -kY3c * dy * (4.0f * zz - xx - yy), kY3d * dz * (2.0f * zz - 3.0f * xx - 3.0f * yy),
                          -kY3c * dx * (4.0f * zz - xx - yy), kY3e * dz * (xx - yy),
                          -kY3a * dx * (xx - 3.0f * yy)};
    float v[48];
#pragma unroll
    for (uint32_t q = 0; q < 12; ++q) {
      const float4 t4 = shr[q];
      v[4 * q] = t4.x;
      v[4 * q + 1] = t4.y;
      v[4 * q + 2] = t4.z;
      v[4 * q + 3] = t4.w;
    }
    float r = 0.5f, gg = 0.5f, bb = 0.5f;
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
      // terms beyond nb are dropped by selects (their bytes may hold anything)
      r = k < nb ? fmaf(v[3 * k], Yb[k], r) : r;
      gg = k < nb ? fmaf(v[3 * k + 1], Yb[k], gg) : gg;
      bb = k < nb ? fmaf(v[3 * k + 2], Yb[k], bb) : bb;
    }
    col = make_float4(fmaxf(0.f, r), fmaxf(0.f, gg), fmaxf(0.f, bb), 0.f);
  }
  reinterpret_cast<int4*>(a.records)[g] = rec;
  reinterpret_cast<float4*>(a.conic_opacity)[g] = co;
  reinterpret_cast<float4*>(a.rgb)[g] = col;
}

}  // namespace

hipError_t launch_preprocess(const PreprocessArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_preprocess, dim3((a.n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace ss

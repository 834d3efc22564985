"""Seeded synthetic inputs for the tile-and-depth sort of 3D Gaussian Splatting.

This module only draws input records: projected Gaussians (fixed-point mean,
FP32 depth, integer radius) for a frame, batches of frames and request
arrival traces.  It holds none of the sort's arithmetic (no tile overlap, no
scan, no keys), so both the CPU oracle and the GPU path can take their inputs
from here without sharing any of the method's code.

The paper's trained scenes (Tanks&Temples Train/Truck, DeepBlending Playroom;
Evaluation, "Datasets") are not available, so these distributions stand in for
them.  Image sizes bracket the paper's (980x545 to 1264x832, Evaluation table
of per-stage latency) and the pair counts span its random key-value sweep
(0.5M to 17M pairs, Evaluation, "Datasets").

Random numbers
--------------
All draws come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: element ``i`` of the stream with start state ``s`` is
``mix64(s + (i + 1) * GOLDEN)``, where ``mix64`` is the published SplitMix64
output function.  A stream's start state is derived from ``(seed, ids...)`` by
chaining the same function, so every variable of every frame has its own
stream and any element can be drawn on its own.  Arithmetic is numpy uint64
with wrap-around.

Derived variates (documented so the inputs can be reproduced elsewhere):

* uniform double in [0, 1):   ``(x >> 11) * 2**-53``
* uniform double in (0, 1]:   ``((x >> 11) + 1) * 2**-53``
* uniform integer in [0, n):  ``((x >> 32) * n) >> 32``  (n < 2**32)
* standard normal:            Box-Muller, ``sqrt(-2 ln u1) * cos(2 pi u2)`` with
                              u1 in (0, 1] and u2 in [0, 1)
* lround(v) for v >= 0:       ``floor(v + 0.5)``
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

#: record layout shared by every consumer: 16 bytes, little endian.
#: mean_x/mean_y: signed 1/16-pixel fixed point; depth: FP32; radius: pixels.
RECORD_DTYPE = np.dtype([("mean_x", "<i4"), ("mean_y", "<i4"),
                         ("depth", "<f4"), ("radius", "<u4")])
assert RECORD_DTYPE.itemsize == 16

#: fixed-point scale of the mean (units per pixel)
FIXED_POINT = 16


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, *ids: int) -> int:
    """Start state of the stream named by ``(seed, ids...)``."""
    k = seed & _MASK64
    for i in ids:
        k = _mix64_int(k + ((int(i) + 1) * int(GOLDEN)))
    return k


def raw_u64(key: int, n: int, start: int = 0) -> np.ndarray:
    """Elements ``start .. start+n-1`` of the SplitMix64 stream ``key``."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = np.uint64(key) + idx * GOLDEN
    return _mix64(s)


def uniform01(key: int, n: int) -> np.ndarray:
    """Doubles in [0, 1)."""
    return (raw_u64(key, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform01_open0(key: int, n: int) -> np.ndarray:
    """Doubles in (0, 1]."""
    return ((raw_u64(key, n) >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * (2.0 ** -53)


def uniform_int(key: int, n: int, bound: int) -> np.ndarray:
    """Integers in [0, bound) (Lemire's multiply-shift on the high 32 bits)."""
    if not 0 < bound < (1 << 32):
        raise ValueError("bound must be in (0, 2^32)")
    hi = raw_u64(key, n) >> np.uint64(32)
    with np.errstate(over="ignore"):
        return ((hi * np.uint64(bound)) >> np.uint64(32)).astype(np.int64)


def normal(key: int, n: int) -> np.ndarray:
    """Standard normals by Box-Muller (cosine branch) from two sub-streams."""
    u1 = uniform01_open0(stream_key(key, 0), n)
    u2 = uniform01(stream_key(key, 1), n)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def lround_nonneg(v: np.ndarray) -> np.ndarray:
    return np.floor(v + 0.5)


# ----------------------------------------------------------------------------
# frame specifications
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class FrameSpec:
    """Distribution of one frame's projected Gaussians."""
    width: int
    height: int
    n: int
    radius: str = "lognormal"        # "lognormal" or "pareto"
    sigma_mu: float = math.log(3.0)  # lognormal sigma: exp(mu + s z)
    sigma_s: float = 0.6
    pareto_alpha: float = 1.8        # pareto sigma: u^(-1/alpha), x_m = 1 px
    radius_cap: int = 64
    depth_lo: float = 0.2
    depth_hi: float = 100.0
    blob_fraction: float = 0.0       # share of means drawn around blob centres
    n_blobs: int = 8
    blob_std_px: float = 80.0


# stream ids of the per-Gaussian variables
_V_MX, _V_MY, _V_SEL, _V_BLOB, _V_BX, _V_BY, _V_SIGMA, _V_DEPTH, _V_CENTRES = range(9)


def make_frame(spec: FrameSpec, seed: int, frame_index: int = 0) -> np.ndarray:
    """Draw ``spec.n`` records for frame ``frame_index`` of stream ``seed``.

    Means are integer-uniform over the image in 1/16 px (``[0, 16 W)``); a
    ``blob_fraction`` share (chosen per Gaussian) is instead placed at
    ``centre + round_half_even(16 * std * z)`` around one of ``n_blobs``
    centres, without clamping, so some fall off the image.  Radii are
    ``clamp(lround(3 sigma), 1, cap)``; depths ``float32(exp(U(ln lo, ln hi)))``.
    """
    n = int(spec.n)
    key = stream_key(seed, frame_index)
    fw = FIXED_POINT * spec.width
    fh = FIXED_POINT * spec.height
    mx = uniform_int(stream_key(key, _V_MX), n, fw)
    my = uniform_int(stream_key(key, _V_MY), n, fh)
    if spec.blob_fraction > 0.0 and n > 0:
        sel = uniform01(stream_key(key, _V_SEL), n) < spec.blob_fraction
        which = uniform_int(stream_key(key, _V_BLOB), n, spec.n_blobs)
        ckey = stream_key(key, _V_CENTRES)
        cx = uniform_int(stream_key(ckey, 0), spec.n_blobs, fw)
        cy = uniform_int(stream_key(ckey, 1), spec.n_blobs, fh)
        scale = FIXED_POINT * spec.blob_std_px
        bx = cx[which] + np.rint(scale * normal(stream_key(key, _V_BX), n)).astype(np.int64)
        by = cy[which] + np.rint(scale * normal(stream_key(key, _V_BY), n)).astype(np.int64)
        mx = np.where(sel, bx, mx)
        my = np.where(sel, by, my)
    if spec.radius == "lognormal":
        sigma = np.exp(spec.sigma_mu + spec.sigma_s * normal(stream_key(key, _V_SIGMA), n))
    elif spec.radius == "pareto":
        sigma = uniform01_open0(stream_key(key, _V_SIGMA), n) ** (-1.0 / spec.pareto_alpha)
    else:
        raise ValueError(spec.radius)
    radius = np.clip(lround_nonneg(3.0 * sigma), 1, spec.radius_cap)
    lo, hi = math.log(spec.depth_lo), math.log(spec.depth_hi)
    depth = np.exp(lo + (hi - lo) * uniform01(stream_key(key, _V_DEPTH), n)).astype(np.float32)

    rec = np.empty(n, dtype=RECORD_DTYPE)
    rec["mean_x"] = mx.astype(np.int32)
    rec["mean_y"] = my.astype(np.int32)
    rec["depth"] = depth
    rec["radius"] = radius.astype(np.uint32)
    return rec


_V_S1, _V_S2, _V_THETA, _V_OPACITY, _V_RGB = range(16, 21)


def make_render_attrs(records: np.ndarray, seed: int, frame_index: int = 0) -> tuple:
    """Per-Gaussian render inputs for ``records`` (frame ``frame_index`` of
    stream ``seed``): ``(conic_opacity, rgb)``, float32 [N, 4] each.

    The 2D covariance has principal standard deviations s1 = (r/3) U(0.6, 1)
    and s2 = s1 U(0.25, 1) (so the record's radius r still bounds 3 s1) at an
    angle U(0, pi); the conic is its inverse (a, b, c) = (Syy, -Sxy, Sxx)/det.
    Opacity U(0.05, 0.99); colour U(0, 1) per channel; the fourth colour
    component is 0."""
    n = len(records)
    key = stream_key(seed, frame_index, 1 << 23)
    r = records["radius"].astype(np.float64)
    s1 = np.maximum(r, 1.0) / 3.0 * (0.6 + 0.4 * uniform01(stream_key(key, _V_S1), n))
    s2 = s1 * (0.25 + 0.75 * uniform01(stream_key(key, _V_S2), n))
    th = math.pi * uniform01(stream_key(key, _V_THETA), n)
    cs, sn = np.cos(th), np.sin(th)
    sxx = s1 * s1 * cs * cs + s2 * s2 * sn * sn
    syy = s1 * s1 * sn * sn + s2 * s2 * cs * cs
    sxy = (s1 * s1 - s2 * s2) * sn * cs
    det = sxx * syy - sxy * sxy
    conic_opacity = np.empty((n, 4), np.float32)
    conic_opacity[:, 0] = syy / det
    conic_opacity[:, 1] = -sxy / det
    conic_opacity[:, 2] = sxx / det
    conic_opacity[:, 3] = 0.05 + 0.94 * uniform01(stream_key(key, _V_OPACITY), n)
    rgb = np.zeros((n, 4), np.float32)
    rgb[:, :3] = uniform01(stream_key(key, _V_RGB), 3 * n).reshape(n, 3)
    return conic_opacity, rgb


# ----------------------------------------------------------------------------
# 3D scenes (inputs of the preprocessing step)
# ----------------------------------------------------------------------------

_V_P3, _V_SCALE, _V_QUAT, _V_OPAC3, _V_SH = range(32, 37)


@dataclasses.dataclass(frozen=True)
class Camera:
    """Pinhole camera looking down +z from the origin (world = camera frame
    up to ``view``): pixel = focal * (x / z, y / z) + centre."""
    width: int
    height: int
    focal: float
    near: float = 0.2
    sh_degree: int = 3

    @property
    def view(self) -> np.ndarray:
        """World-to-camera [R | t], 3 x 4 (identity here)."""
        v = np.zeros((3, 4), np.float64)
        v[:3, :3] = np.eye(3)
        return v

    @property
    def tan_fov(self) -> tuple:
        return self.width / (2.0 * self.focal), self.height / (2.0 * self.focal)


def make_scene(n: int, cam: Camera, seed: int) -> dict:
    """``n`` 3D Gaussians in front of ``cam``: positions uniform in the view
    frustum between depth 1 and 50 (10 % placed up to 1.5x beyond the image
    edges, 2 % behind the near plane), log-normal scales (median 0.0015 z, about
    2 px on screen),
    uniformly random rotations (normalised Gaussian quaternions), opacity
    U(0.05, 0.99), degree-3 SH coefficients N(0, 0.3) with the DC term
    N(0.5, 0.5).  Returns float32 arrays: mean3d_opacity [n, 4], cov3d [n, 8]
    (xx, xy, xz, yy, yz, zz, 0, 0) and sh [n, 48] (16 coefficients x RGB)."""
    key = stream_key(seed, 0, 1 << 24)
    u = uniform01(stream_key(key, _V_P3), 3 * n).reshape(n, 3)
    z = np.exp(np.log(1.0) + (np.log(50.0) - np.log(1.0)) * u[:, 2])
    tx, ty = cam.tan_fov
    spread = np.where(uniform01(stream_key(key, _V_P3 + 100), n) < 0.1, 1.5, 1.0)
    x = (2.0 * u[:, 0] - 1.0) * tx * z * spread
    y = (2.0 * u[:, 1] - 1.0) * ty * z * spread
    z = np.where(uniform01(stream_key(key, _V_P3 + 200), n) < 0.02, -z, z)
    sc = 0.0015 * np.abs(z)[:, None] * np.exp(0.5 * normal(stream_key(key, _V_SCALE), 3 * n).reshape(n, 3))
    q = normal(stream_key(key, _V_QUAT), 4 * n).reshape(n, 4)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, qx, qy, qz = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.stack([np.stack([1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - w * qz), 2 * (qx * qz + w * qy)], -1),
                  np.stack([2 * (qx * qy + w * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - w * qx)], -1),
                  np.stack([2 * (qx * qz - w * qy), 2 * (qy * qz + w * qx), 1 - 2 * (qx * qx + qy * qy)], -1)], 1)
    M = R * sc[:, None, :]
    S = M @ np.transpose(M, (0, 2, 1))
    m3 = np.zeros((n, 4), np.float32)
    m3[:, 0], m3[:, 1], m3[:, 2] = x, y, z
    m3[:, 3] = 0.05 + 0.94 * uniform01(stream_key(key, _V_OPAC3), n)
    cov = np.zeros((n, 8), np.float32)
    cov[:, 0], cov[:, 1], cov[:, 2] = S[:, 0, 0], S[:, 0, 1], S[:, 0, 2]
    cov[:, 3], cov[:, 4], cov[:, 5] = S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]
    sh = (0.3 * normal(stream_key(key, _V_SH), 48 * n)).reshape(n, 16, 3)
    sh[:, 0, :] = 0.5 + 0.5 * normal(stream_key(key, _V_SH + 100), 3 * n).reshape(n, 3)
    return {"mean3d_opacity": m3, "cov3d": cov, "sh": sh.reshape(n, 48).astype(np.float32)}


def band_frames(records: np.ndarray, width: int, height: int, bands: int) -> list:
    """One frame cut into ``bands`` bands of whole tile rows (as equal as the
    row count allows), each as a frame of its own: the same records with
    mean_y moved up by the band's first pixel row, so that the band's tiles
    are tiles 0 .. of the cut frame and everything else falls outside it.
    Returns [(band_height, first_tile_row, records)].  Sorting band b and
    adding first_tile_row * tiles_x to its tile ids gives the band's share of
    the whole frame's output."""
    ty = -(-height // 16)
    bounds = [ty * b // bands for b in range(bands + 1)]
    out = []
    for b in range(bands):
        r0, r1 = bounds[b], bounds[b + 1]
        if r1 == r0:
            continue
        rec = np.array(records, copy=True)
        rec["mean_y"] = rec["mean_y"].astype(np.int64) - 256 * r0
        h = min(16 * r1, height) - 16 * r0
        out.append((h, r0, rec))
    return out


def camera_params(cam: Camera, view=None, cam_pos=(0.0, 0.0, 0.0)) -> dict:
    """The camera as the float32 values a device call receives (principal point
    at the image centre, fx = fy = focal); both the device path and the CPU
    check are given exactly these numbers."""
    tx, ty = cam.tan_fov
    v = cam.view if view is None else view
    f = lambda x: float(np.float32(x))  # noqa: E731
    return {"view": [f(x) for x in np.asarray(v).reshape(12)], "fx": f(cam.focal), "fy": f(cam.focal),
            "cx": f(cam.width / 2), "cy": f(cam.height / 2), "tan_fovx": f(tx), "tan_fovy": f(ty),
            "cam_pos": [f(x) for x in cam_pos], "near_plane": f(cam.near), "sh_degree": cam.sh_degree}


def pose_scene(scene: dict, seed: int, centre=(1.5, -2.0, 0.7)) -> tuple:
    """The same Gaussians seen by a rotated camera at ``centre``: a uniformly
    random rotation R (normalised Gaussian quaternion), world points
    p_w = R^T p + centre and covariances R^T S R, so that the view [R | -R
    centre] maps them back in front of the camera.  Returns (scene in world
    coordinates, float32 view 3 x 4, centre)."""
    q = normal(stream_key(seed, 77), 4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    C = np.asarray(centre, np.float64)
    view = np.zeros((3, 4))
    view[:, :3] = R
    view[:, 3] = -R @ C
    view = view.astype(np.float32)
    m3 = scene["mean3d_opacity"].astype(np.float64)
    out = dict(scene)
    pw = m3[:, :3] @ R + C          # rows: (R^T p)^T = p^T R
    out["mean3d_opacity"] = np.concatenate([pw, m3[:, 3:]], 1).astype(np.float32)
    cv = scene["cov3d"].astype(np.float64)
    S = np.stack([np.stack([cv[:, 0], cv[:, 1], cv[:, 2]], -1), np.stack([cv[:, 1], cv[:, 3], cv[:, 4]], -1),
                  np.stack([cv[:, 2], cv[:, 4], cv[:, 5]], -1)], 1)
    Sw = np.einsum("ji,njk,kl->nil", R, S, R)
    c8 = np.zeros_like(scene["cov3d"])
    c8[:, 0], c8[:, 1], c8[:, 2] = Sw[:, 0, 0], Sw[:, 0, 1], Sw[:, 0, 2]
    c8[:, 3], c8[:, 4], c8[:, 5] = Sw[:, 1, 1], Sw[:, 1, 2], Sw[:, 2, 2]
    out["cov3d"] = c8
    return out, view, tuple(float(np.float32(c)) for c in C)


#: the preprocessing workload: a full-HD view of 10^6 Gaussians (seed 1006)
SCENE_CAMERA = Camera(1920, 1080, focal=1400.0)
SCENE_SEED = 1006


# ----------------------------------------------------------------------------
# the benchmark workloads
# ----------------------------------------------------------------------------

#: base seed of workload k is 1000 + k
SEED_BASE = 1000

SMALL = FrameSpec(256, 256, 10_000)                                   # 256 tiles
FULL_HD = FrameSpec(1920, 1080, 1_000_000, sigma_mu=math.log(2.0), sigma_s=0.8,
                    blob_fraction=0.2)                                 # 8,160 tiles
LARGE = FrameSpec(1920, 1080, 6_000_000, radius="pareto", radius_cap=256,
                  depth_lo=0.1, depth_hi=500.0)                        # heavy tail

#: the three single-frame workloads by name
FRAME_WORKLOADS = {"small-256x256": (SMALL, SEED_BASE + 0),
                   "fullhd-1m": (FULL_HD, SEED_BASE + 1),
                   "large-6m": (LARGE, SEED_BASE + 2)}

#: supplementary: the heavy-tailed frame scaled to about 10^8 pairs (about
#: 1.2 GB of keys and values per sort pass)
SUPPLEMENTARY_WORKLOADS = {"large-2b-22m": (dataclasses.replace(LARGE, n=21_800_000), SEED_BASE + 2)}


def workload(name: str) -> tuple:
    """(FrameSpec, seed) of a single-frame workload, core or supplementary."""
    if name in FRAME_WORKLOADS:
        return FRAME_WORKLOADS[name]
    return SUPPLEMENTARY_WORKLOADS[name]

BATCH_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080))
BATCH_N_RANGE = (50_000, 2_000_000)


def scaled(spec: FrameSpec, n: int) -> FrameSpec:
    """Same distributions with a different Gaussian count."""
    return dataclasses.replace(spec, n=int(n))


def batch_frame_spec(seed: int, frame_index: int,
                     n_range: Sequence[int] = BATCH_N_RANGE) -> FrameSpec:
    """Frame ``frame_index`` of a batch: resolution uniform over three sizes,
    N log-uniform over ``n_range``, other distributions as the full-HD frame."""
    key = stream_key(seed, frame_index, 1 << 20)
    r = int(uniform_int(stream_key(key, 0), 1, len(BATCH_RESOLUTIONS))[0])
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    u = float(uniform01(stream_key(key, 1), 1)[0])
    n = int(math.floor(math.exp(lo + (hi - lo) * u)))
    w, h = BATCH_RESOLUTIONS[r]
    return dataclasses.replace(FULL_HD, width=w, height=h, n=n)


def batch_frame(seed: int, frame_index: int, n_range: Sequence[int] = BATCH_N_RANGE) -> tuple:
    """Frame ``frame_index`` of batch stream ``seed`` as ``(width, height, records)``."""
    spec = batch_frame_spec(seed, frame_index, n_range)
    return spec.width, spec.height, make_frame(spec, seed, frame_index)


def make_batch(n_frames: int, seed: int = SEED_BASE + 3,
               n_range: Sequence[int] = BATCH_N_RANGE) -> List[tuple]:
    """``n_frames`` uneven frames as ``(width, height, records)`` tuples."""
    return [batch_frame(seed, f, n_range) for f in range(n_frames)]


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: exponential gaps -ln(u)/rate."""
    expect = int(rate_per_s * duration_s * 1.5 + 64)
    gaps = -np.log(uniform01_open0(stream_key(seed, 1 << 21), expect)) / rate_per_s
    t = np.cumsum(gaps)
    while t[-1] < duration_s:   # rare: extend the stream
        more = -np.log(uniform01_open0(stream_key(seed, 1 << 21, len(t)), expect)) / rate_per_s
        t = np.concatenate([t, t[-1] + np.cumsum(more)])
    return t[t < duration_s]


def sort_sweep_pairs(m: int, key_bits: int, seed: int) -> tuple:
    """Random pairs for the sort-only sweep: keys uniform over [0, 2^key_bits),
    values 0..m-1 (the paper's random key-value datasets, Evaluation)."""
    k = raw_u64(stream_key(seed, 1 << 22), m)
    if key_bits < 64:
        k = k >> np.uint64(64 - key_bits)
    return k, np.arange(m, dtype=np.uint32)

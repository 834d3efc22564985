"""CPU oracle of the per-frame tile-and-depth sort (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product: the two share no code.  Inputs come
from ``synth`` (seeded records only).

The arithmetic lives in ``oracle.cpp`` (plain C++, one thread); this module
builds it with g++ and wraps it with numpy arrays.  ``sort_batch`` composes
single-frame results into the batched layout (frame-major pairs, global tile
ids ``tile_base[f] + t``, frame-local values, global ranges).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SS_ORACLE_LIB selects another build of the same source (the sanitizer
# run of the pins builds one with -fsanitize=address,undefined)
LIB_PATH = os.environ.get("SS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.cpp")

OK, ERR_INVALID_ARGUMENT, ERR_CAPACITY, ERR_OVERFLOW, ERR_INVALID_INPUT = 0, 1, 3, 4, 5


def build(src: str = SRC_PATH, out: str = LIB_PATH, extra=()) -> str:
    """Compile the oracle into a shared library (g++, C++17)."""
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-I", HERE, *extra, src, "-o", out + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


class _Frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("tile_px", ctypes.c_uint32), ("num_gaussians", ctypes.c_uint32),
                ("gaussians", ctypes.c_void_p)]


_P = ctypes.c_void_p
_U64 = ctypes.c_uint64


class _Camera(ctypes.Structure):
    _fields_ = [("view", ctypes.c_double * 12), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("tan_fovx", ctypes.c_double),
                ("tan_fovy", ctypes.c_double), ("cam_pos", ctypes.c_double * 3), ("near_plane", ctypes.c_double),
                ("sh_degree", ctypes.c_uint32)]


def camera(view, fx, fy, cx, cy, tan_fovx, tan_fovy, cam_pos, near, sh_degree) -> _Camera:
    c = _Camera()
    v = np.asarray(view, np.float64).reshape(12)
    for i in range(12):
        c.view[i] = v[i]
    c.fx, c.fy, c.cx, c.cy, c.tan_fovx, c.tan_fovy = fx, fy, cx, cy, tan_fovx, tan_fovy
    for i in range(3):
        c.cam_pos[i] = cam_pos[i]
    c.near_plane, c.sh_degree = near, sh_degree
    return c


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    fp = ctypes.POINTER(_Frame)
    lib.oracle_tile_grid.argtypes = [fp, _P, _P]
    lib.oracle_count.argtypes = [fp, _P, _P]
    lib.oracle_scan.argtypes = [_P, ctypes.c_uint32, _P, _P]
    lib.oracle_duplicate.argtypes = [fp, _P, _U64, _P, _P]
    lib.oracle_sort.argtypes = [_P, _P, _U64]
    lib.oracle_ranges.argtypes = [_P, _U64, _U64, _P]
    lib.oracle_sort_frame.argtypes = [fp, _U64, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.oracle_sort_frame_mt.argtypes = [fp, _U64, _P, _P, _P, _P, ctypes.c_int]
    lib.oracle_render.argtypes = [fp, _P, _P, _P, _P, _P, ctypes.c_int, _P, _P, _P, _P]
    lib.oracle_preprocess.argtypes = [ctypes.POINTER(_Camera), ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P]
    lib.oracle_sh_basis.argtypes = [_P, _P]
    lib.oracle_sh_basis.restype = None
    for f in (lib.oracle_tile_grid, lib.oracle_count, lib.oracle_scan, lib.oracle_duplicate,
              lib.oracle_sort, lib.oracle_ranges, lib.oracle_sort_frame, lib.oracle_sort_frame_mt, lib.oracle_render,
              lib.oracle_preprocess):
        f.restype = ctypes.c_int
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _frame(width: int, height: int, records: np.ndarray, tile_px: int = 16) -> _Frame:
    rec = np.ascontiguousarray(records)
    assert rec.dtype.itemsize == 16
    return _Frame(width, height, tile_px, len(rec), rec.ctypes.data if len(rec) else None), rec


@dataclasses.dataclass
class FrameResult:
    status: int
    tiles_x: int
    tiles_y: int
    num_pairs: int
    tiles_touched: np.ndarray
    offsets: np.ndarray
    unsorted_keys: np.ndarray
    unsorted_values: np.ndarray
    keys: np.ndarray
    values: np.ndarray
    ranges: np.ndarray     # (T, 2) uint32

    @property
    def num_tiles(self) -> int:
        return self.tiles_x * self.tiles_y


def tile_grid(width: int, height: int, tile_px: int = 16):
    fr, _ = _frame(width, height, np.zeros(0, dtype=np.dtype((np.void, 16))), tile_px)
    tx, ty = ctypes.c_uint32(), ctypes.c_uint32()
    st = lib().oracle_tile_grid(ctypes.byref(fr), ctypes.addressof(tx), ctypes.addressof(ty))
    if st != OK:
        raise ValueError(f"invalid frame geometry {width}x{height}/{tile_px}")
    return tx.value, ty.value


def count(width: int, height: int, records: np.ndarray, tile_px: int = 16):
    """Counting alone: (tiles_touched[N], rects[N,4] = x0, x1, y0, y1)."""
    fr, rec = _frame(width, height, records, tile_px)
    n = len(rec)
    cnt = np.zeros(n, np.uint32)
    rects = np.zeros((n, 4), np.uint32)
    st = lib().oracle_count(ctypes.byref(fr), _ptr(cnt), _ptr(rects))
    if st != OK:
        raise ValueError(f"oracle_count status {st}")
    return cnt, rects


def scan(counts: np.ndarray):
    """The scan alone: (offsets[N] uint64, total)."""
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    off = np.zeros(len(c), np.uint64)
    tot = ctypes.c_uint64()
    st = lib().oracle_scan(_ptr(c), len(c), _ptr(off), ctypes.addressof(tot))
    assert st == OK
    return off, tot.value


def duplicate(width: int, height: int, records: np.ndarray, offsets: np.ndarray, num_pairs: int,
              tile_px: int = 16):
    """Duplication alone: the unsorted (keys, values) from the scan's offsets."""
    fr, rec = _frame(width, height, records, tile_px)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    k = np.zeros(num_pairs, np.uint64)
    v = np.zeros(num_pairs, np.uint32)
    st = lib().oracle_duplicate(ctypes.byref(fr), _ptr(off), num_pairs, _ptr(k), _ptr(v))
    if st != OK:
        raise ValueError(f"oracle_duplicate status {st}")
    return k, v


def sort_pairs(keys: np.ndarray, values: np.ndarray):
    """The sort alone on copies: stable sort by the 64-bit key."""
    k = np.array(keys, dtype=np.uint64, copy=True)
    v = np.array(values, dtype=np.uint32, copy=True)
    assert lib().oracle_sort(_ptr(k), _ptr(v), len(k)) == OK
    return k, v


def ranges(sorted_keys: np.ndarray, num_tiles: int) -> np.ndarray:
    """Range identification alone: (T, 2) start/end."""
    k = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    r = np.zeros((num_tiles, 2), np.uint32)
    st = lib().oracle_ranges(_ptr(k), len(k), num_tiles, _ptr(r))
    if st != OK:
        raise ValueError(f"oracle_ranges status {st}")
    return r


def sort_frame(width: int, height: int, records: np.ndarray, tile_px: int = 16,
               capacity: Optional[int] = None, stages: bool = True) -> FrameResult:
    """Whole frame: count, scan, duplicate, sort, ranges.  With ``capacity=None`` the pair buffers are sized
    to the exact M (a first call counts).  ``stages`` also returns the
    per-Gaussian counts, offsets and the unsorted duplication order."""
    fr, rec = _frame(width, height, records, tile_px)
    n = len(rec)
    if tile_px != 16 or width < 1 or height < 1:
        tx = ty = 0
    else:
        tx, ty = tile_grid(width, height, tile_px)
    m_out = ctypes.c_uint64()
    if capacity is None:
        cnt = np.zeros(n, np.uint32)
        st = lib().oracle_count(ctypes.byref(fr), _ptr(cnt), None)
        if st != OK:
            return FrameResult(st, tx, ty, 0, *(np.zeros(0),) * 7)
        capacity = int(cnt.astype(np.uint64).sum())
        capacity = min(capacity, 0xFFFFFFFF)
    cap = int(capacity)
    cnt = np.zeros(n, np.uint32) if stages else None
    off = np.zeros(n, np.uint64) if stages else None
    uk = np.zeros(cap, np.uint64) if stages else None
    uv = np.zeros(cap, np.uint32) if stages else None
    k = np.zeros(cap, np.uint64)
    v = np.zeros(cap, np.uint32)
    r = np.zeros((tx * ty, 2), np.uint32)
    st = lib().oracle_sort_frame(ctypes.byref(fr), cap, _ptr(cnt), _ptr(off), _ptr(uk), _ptr(uv),
                                 _ptr(k), _ptr(v), _ptr(r), ctypes.addressof(m_out))
    m = int(m_out.value)
    mm = min(m, cap)
    empty = np.zeros(0)
    return FrameResult(st, tx, ty, m,
                       cnt if cnt is not None else empty, off if off is not None else empty,
                       uk[:mm] if uk is not None else empty, uv[:mm] if uv is not None else empty,
                       k[:mm], v[:mm], r)


def sort_frame_mt(width: int, height: int, records: np.ndarray, threads: int,
                  capacity: Optional[int] = None) -> FrameResult:
    """``sort_frame`` (without the stage outputs) on ``threads`` host threads
    (oracle_sort_frame_mt): the CPU timing baseline beside the GPU, the same
    result."""
    fr, rec = _frame(width, height, records, 16)
    n = len(rec)
    tx, ty = tile_grid(width, height, 16)
    if capacity is None:
        cnt = np.zeros(n, np.uint32)
        st = lib().oracle_count(ctypes.byref(fr), _ptr(cnt), None)
        if st != OK:
            return FrameResult(st, tx, ty, 0, *(np.zeros(0),) * 7)
        capacity = min(int(cnt.astype(np.uint64).sum()), 0xFFFFFFFF)
    cap = int(capacity)
    k = np.zeros(cap, np.uint64)
    v = np.zeros(cap, np.uint32)
    r = np.zeros((tx * ty, 2), np.uint32)
    m_out = ctypes.c_uint64()
    st = lib().oracle_sort_frame_mt(ctypes.byref(fr), cap, _ptr(k), _ptr(v), _ptr(r), ctypes.addressof(m_out),
                                    int(threads))
    m = int(m_out.value)
    mm = min(m, cap)
    empty = np.zeros(0)
    return FrameResult(st, tx, ty, m, empty, empty, empty, empty, k[:mm], v[:mm], r)


@dataclasses.dataclass
class RenderResult:
    status: int
    color: np.ndarray      # float64 [3, H, W]
    T: np.ndarray          # float64 [H, W], final transmittance
    n_contrib: np.ndarray  # uint32 [H, W], Gaussians composited
    margin: np.ndarray     # float64 [H, W], closest relative distance to a threshold


def render(width: int, height: int, records: np.ndarray, conic_opacity: np.ndarray, rgb: np.ndarray,
           values: np.ndarray, ranges: np.ndarray, background=(0.0, 0.0, 0.0), exact: bool = False) -> RenderResult:
    """Alpha blending of every tile's sorted Gaussians (oracle_render).
    ``conic_opacity`` and ``rgb`` are float32 [N, 4]; ``values``/``ranges`` a
    sorted frame."""
    fr, rec = _frame(width, height, records)
    co = np.ascontiguousarray(conic_opacity, dtype=np.float32).reshape(-1, 4)
    cl = np.ascontiguousarray(rgb, dtype=np.float32).reshape(-1, 4)
    vals = np.ascontiguousarray(values, dtype=np.uint32)
    rng = np.ascontiguousarray(ranges, dtype=np.uint32)
    bg = np.ascontiguousarray(background, dtype=np.float64)
    color = np.zeros((3, height, width), np.float64)
    T = np.zeros((height, width), np.float64)
    k = np.zeros((height, width), np.uint32)
    margin = np.zeros((height, width), np.float64)
    st = lib().oracle_render(ctypes.byref(fr), _ptr(co), _ptr(cl), _ptr(vals), _ptr(rng), _ptr(bg), int(exact),
                             _ptr(color), _ptr(T), _ptr(k), _ptr(margin))
    return RenderResult(st, color, T, k, margin)


@dataclasses.dataclass
class PreprocessResult:
    status: int
    records: np.ndarray        # RECORD-like structured array (mean_x, mean_y, depth, radius)
    conic_opacity: np.ndarray  # float64 [n, 4]
    rgb: np.ndarray            # float64 [n, 4]
    margin: np.ndarray         # float64 [n, 3]: rounding margins of 16x, 16y, 3 sqrt(lambda)


def preprocess(cam: _Camera, mean3d_opacity: np.ndarray, cov3d: np.ndarray, sh: np.ndarray) -> PreprocessResult:
    """3D Gaussians to sort records, conic/opacity and colour (oracle_preprocess)."""
    m3 = np.ascontiguousarray(mean3d_opacity, dtype=np.float32).reshape(-1, 4)
    cv = np.ascontiguousarray(cov3d, dtype=np.float32).reshape(-1, 8)
    shc = np.ascontiguousarray(sh, dtype=np.float32).reshape(-1, 48)
    n = len(m3)
    rec = np.zeros(n, dtype=np.dtype([("mean_x", "<i4"), ("mean_y", "<i4"), ("depth", "<f4"), ("radius", "<u4")]))
    co = np.zeros((n, 4), np.float64)
    rgb = np.zeros((n, 4), np.float64)
    mg = np.zeros((n, 3), np.float64)
    st = lib().oracle_preprocess(ctypes.byref(cam), n, _ptr(m3), _ptr(cv), _ptr(shc), _ptr(rec), _ptr(co), _ptr(rgb),
                                 _ptr(mg))
    return PreprocessResult(st, rec, co, rgb, mg)


def sh_basis(direction) -> np.ndarray:
    """The 16 real spherical harmonics (degree <= 3) at a unit direction."""
    d = np.ascontiguousarray(direction, dtype=np.float64).reshape(3)
    out = np.zeros(16, np.float64)
    lib().oracle_sh_basis(_ptr(d), _ptr(out))
    return out


@dataclasses.dataclass
class BatchResult:
    num_pairs: np.ndarray      # per frame
    pair_base: np.ndarray      # first pair of each frame
    tile_base: np.ndarray      # first global tile of each frame
    keys: np.ndarray           # global tile ids in the high 32 bits
    values: np.ndarray         # frame-local Gaussian indices
    ranges: np.ndarray         # (sum T, 2), global pair indices


def sort_batch(frames: Sequence[tuple]) -> BatchResult:
    """Batched layout from single-frame results: frame f's pairs form one
    contiguous segment starting at the sum of earlier frames' M; its tiles
    are renumbered tile_base[f] + t with tile_base the exclusive sum of T."""
    outs: List[FrameResult] = []
    for (w, h, rec) in frames:
        res = sort_frame(w, h, rec, stages=False)
        if res.status != OK:
            raise ValueError(f"frame status {res.status}")
        outs.append(res)
    ms = np.array([o.num_pairs for o in outs], np.uint64)
    ts = np.array([o.num_tiles for o in outs], np.uint64)
    pair_base = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.uint64) if outs else np.zeros(0, np.uint64)
    tile_base = np.concatenate([[0], np.cumsum(ts)[:-1]]).astype(np.uint64) if outs else np.zeros(0, np.uint64)
    keys, vals, rngs = [], [], []
    for f, o in enumerate(outs):
        keys.append(o.keys + (np.uint64(tile_base[f]) << np.uint64(32)))
        vals.append(o.values)
        rngs.append(o.ranges.astype(np.uint64) + pair_base[f])
    cat = (lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt))
    return BatchResult(ms, pair_base, tile_base, cat(keys, np.uint64), cat(vals, np.uint32),
                       cat(rngs, np.uint64).reshape(-1, 2).astype(np.uint32))


# ----------------------------------------------------------------------------
# The paper's key normalisation (Design, "Sorting Optimizations in Context of
# 3DGS"): the 64-bit (tile, depth) key replaced by one 32-bit float holding 20
# bits of tile number and the depth brought below 2^10.  Reading: k = FP32
# value of tile * 2^10 + min(depth, largest float below 2^10), rounded toward
# zero (so k never reaches the next tile's first key); pairs ordered by
# (k, Gaussian index).

#: largest float32 below 2^10
KEY32_DEPTH_CAP = np.float32(1024.0) - np.float32(2.0 ** -14)


def key32_normalized(keys: np.ndarray) -> np.ndarray:
    """Bits (uint32) of the normalised float key of each 64-bit frame key.

    The sum is formed in float64 and then rounded toward zero to float32.
    That equals rounding the exact sum toward zero: tile * 2^10 and every
    float32 at or below 2^30 + 2^10 are float64 values, and float64 rounding
    is monotonic, so it can only land on a float32 value F that exceeds the
    exact sum if the exact sum lies within half a float64 unit below F; but
    F - tile * 2^10 - depth is a multiple of the last bit of depth, which is
    at least 2^-23 of depth and far larger than that."""
    k = np.asarray(keys, dtype=np.uint64)
    tile = (k >> np.uint64(32)).astype(np.float64)
    depth = (k & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    d = np.minimum(depth, KEY32_DEPTH_CAP).astype(np.float64)
    exact = tile * 1024.0 + d
    f = exact.astype(np.float32)                                  # nearest
    f = np.where(f.astype(np.float64) > exact, np.nextafter(f, np.float32(0)), f)  # toward zero
    return f.astype(np.float32).view(np.uint32)


def sort_frame_key32(width: int, height: int, records: np.ndarray) -> FrameResult:
    """The frame sorted by the normalised 32-bit key: the frame's pairs (from
    ``sort_frame``) reordered by (k, value); keys stay the exact 64-bit keys,
    ranges are recomputed from them (k keeps the tiles in order)."""
    r = sort_frame(width, height, records, stages=False)
    if r.status != OK:
        return r
    k32 = key32_normalized(r.keys)
    order = np.lexsort((r.values, k32))      # primary k32, then value
    keys, values = r.keys[order], r.values[order]
    return dataclasses.replace(r, keys=keys, values=values, ranges=ranges(keys, r.num_tiles))

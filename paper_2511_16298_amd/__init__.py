"""splatsort for MI355X: the per-frame tile-and-depth sort of 3D Gaussian
Splatting (arXiv 2511.16298, Background, "Duplication with Tiles" and
"Sorting"), as a HIP library with a C ABI.

This module marshals torch tensors into the C ABI (``_abi``); torch supplies
device memory and the stream, the HIP kernels do all the work.  Integer
buffers use signed torch dtypes of the same width (keys int64 = uint64 bits,
values and ranges int32 = uint32 bits).
"""
from __future__ import annotations

import contextlib
import ctypes
import dataclasses
from typing import Optional

from . import _abi
from ._abi import (SS_ALGO_AUTO, SS_ALGO_BITONIC, SS_ALGO_DEPTH_FIRST, SS_ALGO_DIRECT, SS_ALGO_TILE_FIRST, SS_OK,
                   SplatSortError, check,
                   make_options, ss_batch_out, ss_frame, ss_frame_out)

__all__ = ["FrameSorter", "BatchSorter", "Plan", "Server", "Renderer", "render_attrs_to_device",
           "Preprocessor", "PreprocessOutput", "camera", "sort_frame",
           "count_pairs", "sort_pairs", "copy_bytes", "Timer",
           "records_to_device", "SplatSortError", "geometry", "SS_ALGO_AUTO", "SS_ALGO_DEPTH_FIRST",
           "SS_ALGO_DIRECT", "SS_ALGO_BITONIC", "SS_ALGO_TILE_FIRST"]


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _allocating_on(stream):
    """Context in which torch allocates for ``stream``: temporaries that the
    kernels on that stream use are then not handed out again before those
    kernels have finished, even when ``stream`` is not the current stream."""
    if stream is None:
        return contextlib.nullcontext()
    return _torch().cuda.stream(stream)


def records_to_device(records, device="cuda"):
    """A numpy array of 16-byte records (``synth.RECORD_DTYPE``) as an (N, 4)
    int32 device tensor."""
    import numpy as np
    torch = _torch()
    a = np.ascontiguousarray(records).view(np.int32).reshape(-1, 4)
    return torch.from_numpy(a.copy()).to(device)


def _frame(records, width: int, height: int, tile_px: int = 16) -> ss_frame:
    n = 0 if records is None else int(records.shape[0])
    if records is not None and n > 0:
        torch = _torch()
        if records.dtype != torch.int32 or records.dim() != 2 or records.shape[1] != 4 or not records.is_contiguous():
            raise ValueError("records must be a contiguous (N, 4) int32 tensor")
    f = ss_frame()
    f.width, f.height, f.tile_px, f.num_gaussians = width, height, tile_px, n
    f.gaussians = records.data_ptr() if n > 0 else None
    return f


def geometry(width: int, height: int, tile_px: int = 16):
    """(tiles_x, tiles_y, key_bits) of a frame."""
    f = ss_frame()
    f.width, f.height, f.tile_px, f.num_gaussians, f.gaussians = width, height, tile_px, 0, None
    st, tx, ty, kb = _abi.ss_frame_geometry(f)
    check(st, "ss_frame_geometry")
    return tx, ty, kb


class Timer:
    """Per-kernel HIP-event timing (``ss_timer``)."""

    def __init__(self, max_launches: int = 4096):
        st, h = _abi.ss_timer_create(max_launches)
        check(st, "ss_timer_create")
        self.handle = h

    def reset(self):
        check(_abi.ss_timer_reset(self.handle), "ss_timer_reset")

    def read(self, kind: int):
        """(total milliseconds, launches) of one kernel kind; the stream must
        have been synchronised."""
        st, ms, n = _abi.ss_timer_read(self.handle, kind)
        check(st, "ss_timer_read")
        return ms, n

    def close(self):
        if self.handle:
            _abi.ss_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class FrameOutput:
    keys: "object"            # int64 [capacity] (uint64 bits)
    values: "object"          # int32 [capacity] (uint32 bits)
    tile_ranges: "object"     # int32 [T, 2]
    num_pairs: "object"       # int32 [1] device scalar
    status: "object"          # int32 [1] device scalar
    tiles_touched: "object" = None
    offsets: "object" = None

    def result(self):
        """Synchronise and return (status, M)."""
        return int(self.status.item()), int(self.num_pairs.item()) & 0xFFFFFFFF


class FrameSorter:
    """Pre-allocated outputs and workspace for repeated ``ss_sort_frame`` calls
    on frames of one shape (the device-resident buffers of a serving loop or
    a benchmark)."""

    def __init__(self, width: int, height: int, num_gaussians: int, pair_capacity: int,
                 radix_bits: int = 0, items_per_thread: int = 0, stages: bool = False,
                 device="cuda", unsorted: bool = False, workgroup_size: int = 0, algorithm: int = 0,
                 key32: bool = False, drop_culled: bool = False, persistent: bool = False,
                 spin_limit: int = 0, fault: int = 0):
        torch = _torch()
        self.width, self.height = width, height
        self.num_gaussians = num_gaussians
        self.capacity = int(pair_capacity)
        self.tiles_x, self.tiles_y, self.key_bits = geometry(width, height)
        self.num_tiles = self.tiles_x * self.tiles_y
        flags = ((_abi.SS_FLAG_UNSORTED if unsorted else 0) | (_abi.SS_FLAG_KEY32_LOSSY if key32 else 0)
                 | (_abi.SS_FLAG_DROP_CULLED if drop_culled else 0)
                 | (_abi.SS_FLAG_PERSISTENT if persistent else 0))
        self.options = make_options(radix_bits, items_per_thread, flags=flags,
                                    workgroup_size=workgroup_size, algorithm=algorithm,
                                    spin_limit=spin_limit, fault=fault)
        probe = ss_frame()
        probe.width, probe.height, probe.tile_px, probe.num_gaussians = width, height, 16, num_gaussians
        probe.gaussians = 16 if num_gaussians else None   # only shape matters here
        st, ws = _abi.ss_workspace_bytes(probe, self.capacity, self.options)
        check(st, "ss_workspace_bytes")
        self.workspace_bytes = ws
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        cap = max(self.capacity, 1)
        n = max(num_gaussians, 1)
        self.out = FrameOutput(
            keys=torch.empty(cap, dtype=torch.int64, device=device),
            values=torch.empty(cap, dtype=torch.int32, device=device),
            tile_ranges=torch.empty((self.num_tiles, 2), dtype=torch.int32, device=device),
            num_pairs=torch.zeros(1, dtype=torch.int32, device=device),
            status=torch.zeros(1, dtype=torch.int32, device=device),
            tiles_touched=torch.empty(n, dtype=torch.int32, device=device) if stages else None,
            offsets=torch.empty(n, dtype=torch.int32, device=device) if stages else None)
        o = ss_frame_out()
        o.pair_capacity = self.capacity
        o.keys = self.out.keys.data_ptr()
        o.values = self.out.values.data_ptr()
        o.tile_ranges = self.out.tile_ranges.data_ptr()
        o.tiles_touched = self.out.tiles_touched.data_ptr() if stages else None
        o.offsets = self.out.offsets.data_ptr() if stages else None
        o.num_pairs = self.out.num_pairs.data_ptr()
        o.status = self.out.status.data_ptr()
        self._cout = o

    def __call__(self, records, stream=None, timer: Optional[Timer] = None) -> FrameOutput:
        """Enqueue ``ss_sort_frame`` on ``stream`` (default: torch's current
        stream).  Raises on a synchronous error; device errors land in
        ``out.status``."""
        if int(records.shape[0]) != self.num_gaussians:
            raise ValueError("records do not match the sorter's Gaussian count")
        f = _frame(records, self.width, self.height)
        self.options.timer = timer.handle if timer is not None else None
        st = _abi.ss_sort_frame(f, self._cout, self.workspace.data_ptr(), self.workspace_bytes,
                                _stream_handle(stream), self.options)
        check(st, "ss_sort_frame")
        return self.out


class BatchSorter:
    """Pre-allocated buffers for ``ss_sort_batch`` over frames of fixed shapes
    ``[(width, height, num_gaussians), ...]`` (one segmented sort)."""

    def __init__(self, shapes, pair_capacity: int, radix_bits: int = 0, items_per_thread: int = 0,
                 workgroup_size: int = 0, device="cuda", plan_workspace: bool = False, drop_culled: bool = False,
                 persistent: bool = False, spin_limit: int = 0, fault: int = 0):
        import numpy as np
        torch = _torch()
        self.shapes = [tuple(int(x) for x in s) for s in shapes]
        self.capacity = int(pair_capacity)
        flags = (_abi.SS_FLAG_DROP_CULLED if drop_culled else 0) | (_abi.SS_FLAG_PERSISTENT if persistent else 0)
        self.options = make_options(radix_bits, items_per_thread, workgroup_size=workgroup_size,
                                    flags=flags, spin_limit=spin_limit, fault=fault)
        tiles = [geometry(w, h)[0] * geometry(w, h)[1] for (w, h, _) in self.shapes]
        self.tile_base = np.concatenate([[0], np.cumsum(tiles)[:-1]]).astype(np.int64)
        self.num_tiles = int(sum(tiles))
        probe = []
        for (w, h, n) in self.shapes:
            f = ss_frame()
            f.width, f.height, f.tile_px, f.num_gaussians = w, h, 16, n
            f.gaussians = 16 if n else None
            probe.append(f)
        if plan_workspace:
            st, ws = _abi.ss_plan_workspace_bytes(probe, self.capacity)
            check(st, "ss_plan_workspace_bytes")
        else:
            st, ws = _abi.ss_batch_workspace_bytes(probe, self.capacity, self.options)
            check(st, "ss_batch_workspace_bytes")
        self.workspace_bytes = ws
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        cap = max(self.capacity, 1)
        nf = len(self.shapes)
        self.keys = torch.empty(cap, dtype=torch.int64, device=device)
        self.values = torch.empty(cap, dtype=torch.int32, device=device)
        self.tile_ranges = torch.empty((self.num_tiles, 2), dtype=torch.int32, device=device)
        self.frame_pairs = torch.zeros(nf, dtype=torch.int32, device=device)
        self.frame_pair_base = torch.zeros(nf, dtype=torch.int32, device=device)
        self.num_pairs = torch.zeros(1, dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        o = ss_batch_out()
        o.pair_capacity = self.capacity
        o.keys, o.values = self.keys.data_ptr(), self.values.data_ptr()
        o.tile_ranges = self.tile_ranges.data_ptr()
        o.frame_pairs, o.frame_pair_base = self.frame_pairs.data_ptr(), self.frame_pair_base.data_ptr()
        o.num_pairs, o.status = self.num_pairs.data_ptr(), self.status.data_ptr()
        self._cout = o

    def __call__(self, records_list, stream=None, timer: Optional[Timer] = None):
        if len(records_list) != len(self.shapes):
            raise ValueError("one records tensor per frame")
        frames = []
        for rec, (w, h, n) in zip(records_list, self.shapes):
            if int(rec.shape[0]) != n:
                raise ValueError("records do not match the frame shape")
            frames.append(_frame(rec, w, h))
        self.options.timer = timer.handle if timer is not None else None
        st = _abi.ss_sort_batch(frames, self._cout, self.workspace.data_ptr(), self.workspace_bytes,
                                _stream_handle(stream), self.options)
        check(st, "ss_sort_batch")
        return self

    def result(self):
        """Synchronise and return (status, total pairs)."""
        return int(self.status.item()), int(self.num_pairs.item()) & 0xFFFFFFFF

    def frames_for(self, records_list):
        return [_frame(rec, w, h) for rec, (w, h, _) in zip(records_list, self.shapes)]


class Plan:
    """A BatchSorter's pipeline captured into a HIP graph (``ss_plan_*``) for
    fixed record tensors; ``autotune`` times every compiled pass configuration
    first.  The sorter must have been made with ``plan_workspace=True``.
    ``tune_cache``: a file that keeps the autotuned choice per device and
    batch size (a later plan of the same size skips the timing)."""

    def __init__(self, sorter: BatchSorter, records_list, autotune: bool = True, tune_repeats: int = 0,
                 stream=None, tune_cache=None):
        self.sorter = sorter
        self.records = list(records_list)   # keep the captured inputs alive
        st, h = _abi.ss_plan_create(sorter.frames_for(self.records), sorter._cout, sorter.workspace.data_ptr(),
                                    sorter.workspace_bytes, _stream_handle(stream), int(autotune), tune_repeats,
                                    sorter.options, tune_cache=tune_cache)
        check(st, "ss_plan_create")
        self.handle = h

    def launch(self, stream=None):
        check(_abi.ss_plan_launch(self.handle, _stream_handle(stream)), "ss_plan_launch")
        return self.sorter

    def config(self):
        st, o, ms = _abi.ss_plan_config(self.handle)
        check(st, "ss_plan_config")
        return {"radix_bits": o.radix_bits, "items_per_thread": o.items_per_thread,
                "workgroup_size": o.workgroup_size, "persistent": bool(o.flags & _abi.SS_FLAG_PERSISTENT),
                "candidate_ms": ms}

    def close(self):
        if getattr(self, "handle", None):
            _abi.ss_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """``ss_server_*``: continuous-batching frame-sort service over a device
    arena (a torch uint8 tensor owned by this object)."""

    def __init__(self, arena_bytes: int, max_batch_frames: int = 64, n_streams: int = 2, device="cuda",
                 radix_bits: int = 0, items_per_thread: int = 0, workgroup_size: int = 0):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        opts = make_options(radix_bits, items_per_thread, workgroup_size=workgroup_size)
        st, h = _abi.ss_server_create(self.arena.data_ptr(), int(arena_bytes), max_batch_frames, n_streams, opts)
        check(st, "ss_server_create")
        self.handle = h

    def submit(self, records, width: int, height: int) -> int:
        st, t = _abi.ss_server_submit(self.handle, _frame(records, width, height))
        check(st, "ss_server_submit")
        return t

    def wait(self, ticket: int):
        st, r = _abi.ss_server_wait(self.handle, ticket)
        check(st, "ss_server_wait")
        return r

    def release(self, ticket: int):
        check(_abi.ss_server_release(self.handle, ticket), "ss_server_release")

    def stats(self):
        st, c = _abi.ss_server_stats(self.handle)
        check(st, "ss_server_stats")
        return {k: getattr(c, k) for k, _ in c._fields_}

    def result_arrays(self, r, num_tiles: int):
        """Host copies of a completed result: keys with the frame's own tile
        ids, values, and frame-local ranges (the device arrays live inside
        the arena, so they are slices of it)."""
        import numpy as np
        base = self.arena.data_ptr()
        m = int(r.num_pairs)

        def grab(ptr, nbytes):
            off = int(ptr) - base
            return self.arena[off:off + nbytes].cpu().numpy()
        k = grab(r.keys, 8 * m).view(np.uint64).copy()
        v = grab(r.values, 4 * m).view(np.uint32).copy()
        rg = grab(r.tile_ranges, 8 * num_tiles).view(np.uint32).reshape(num_tiles, 2).copy()
        k -= np.uint64(int(r.tile_base)) << np.uint64(32)
        rg -= np.uint32(int(r.pair_base))
        return k, v, rg

    def close(self):
        if getattr(self, "handle", None):
            _abi.ss_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count_pairs(records, width: int, height: int, stream=None):
    """Counting and scan: (tiles_touched, offsets, num_pairs, status) device tensors."""
    torch = _torch()
    dev = records.device
    f = _frame(records, width, height)
    n = max(int(records.shape[0]), 1)
    probe = f
    st, ws = _abi.ss_workspace_bytes(probe, 0, None)
    check(st, "ss_workspace_bytes")
    with _allocating_on(stream):
        work = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
        tt = torch.empty(n, dtype=torch.int32, device=dev)
        off = torch.empty(n, dtype=torch.int32, device=dev)
        m = torch.zeros(1, dtype=torch.int32, device=dev)
        s = torch.zeros(1, dtype=torch.int32, device=dev)
    st = _abi.ss_count_pairs(f, tt.data_ptr(), off.data_ptr(), m.data_ptr(), s.data_ptr(),
                             work.data_ptr(), ws, _stream_handle(stream))
    check(st, "ss_count_pairs")
    return tt, off, m, s


def sort_frame(records, width: int, height: int, capacity: Optional[int] = None, stream=None,
               radix_bits: int = 0, items_per_thread: int = 0, stages: bool = False):
    """Whole frame.  With ``capacity=None`` a first call counts the pairs and
    one 4-byte read-back sizes the buffers exactly.  Returns the sorter's
    FrameOutput (slice ``[:M]`` after ``result()``)."""
    if capacity is None:
        _, _, m, s = count_pairs(records, width, height, stream)
        st = int(s.item())
        if st != SS_OK:
            raise SplatSortError(st, "ss_count_pairs")
        capacity = int(m.item()) & 0xFFFFFFFF
    sorter = FrameSorter(width, height, int(records.shape[0]), capacity, radix_bits, items_per_thread,
                         stages, device=records.device)
    return sorter(records, stream)


def sort_pairs(keys, values, key_bits: int, stream=None, radix_bits: int = 0, items_per_thread: int = 0,
               timer: Optional[Timer] = None, workgroup_size: int = 0, algorithm: int = 0):
    """The sort alone: stable sort of (int64 keys, int32 values) by key bits
    [0, key_bits) (``SS_ALGO_BITONIC``: by (key bits, value)).  Returns new
    (keys, values) tensors."""
    torch = _torch()
    n = int(keys.shape[0])
    opts = make_options(radix_bits, items_per_thread, timer.handle if timer is not None else None,
                        workgroup_size=workgroup_size, algorithm=algorithm)
    st, ws = _abi.ss_sort_pairs_workspace_bytes(n, key_bits, opts)
    check(st, "ss_sort_pairs_workspace_bytes")
    with _allocating_on(stream):
        work = torch.empty(max(ws, 256), dtype=torch.uint8, device=keys.device)
        ko = torch.empty_like(keys)
        vo = torch.empty_like(values)
    st = _abi.ss_sort_pairs(keys.data_ptr(), values.data_ptr(), n, key_bits, ko.data_ptr(), vo.data_ptr(),
                            work.data_ptr(), ws, _stream_handle(stream), opts)
    check(st, "ss_sort_pairs")
    return ko, vo


@dataclasses.dataclass
class RenderOutput:
    color: "object"        # float32 [3, H, W]
    T: "object"            # float32 [H, W] or None
    contrib: "object"      # int32 [H, W] or None
    tile_evals: "object"   # int32 [T] or None


class Renderer:
    """Pre-allocated outputs for repeated ``ss_render_frame`` calls on frames
    of one size (alpha blending over a sorted frame's tile lists)."""

    def __init__(self, width: int, height: int, device="cuda", want_T: bool = False,
                 want_contrib: bool = False, want_tile_evals: bool = False):
        torch = _torch()
        self.width, self.height = width, height
        tx, ty, _ = geometry(width, height)
        self.out = RenderOutput(
            torch.empty((3, height, width), dtype=torch.float32, device=device),
            torch.empty((height, width), dtype=torch.float32, device=device) if want_T else None,
            torch.empty((height, width), dtype=torch.int32, device=device) if want_contrib else None,
            torch.empty(tx * ty, dtype=torch.int32, device=device) if want_tile_evals else None)

    def __call__(self, records, conic_opacity, rgb, values, tile_ranges, status=None, background=(0.0, 0.0, 0.0),
                 exact: bool = False, stream=None, timer: Optional[Timer] = None) -> RenderOutput:
        def ptr(t):
            return None if t is None else t.data_ptr()
        f = _frame(records, self.width, self.height)
        o = self.out
        d = _abi.make_render_desc(ptr(conic_opacity), ptr(rgb), ptr(values), ptr(tile_ranges), ptr(o.color),
                                  ptr(status), background, exact, ptr(o.T), ptr(o.contrib), ptr(o.tile_evals),
                                  timer.handle if timer is not None else None)
        check(_abi.ss_render_frame(f, d, _stream_handle(stream)), "ss_render_frame")
        return o


def render_attrs_to_device(conic_opacity, rgb, device="cuda"):
    """float32 [N, 4] numpy arrays as device tensors."""
    import numpy as np
    torch = _torch()
    return (torch.from_numpy(np.ascontiguousarray(conic_opacity, dtype=np.float32)).to(device),
            torch.from_numpy(np.ascontiguousarray(rgb, dtype=np.float32)).to(device))


def camera(view, fx: float, fy: float, cx: float, cy: float, tan_fovx: float, tan_fovy: float, cam_pos,
           near_plane: float = 0.2, sh_degree: int = 3) -> _abi.ss_camera:
    """A pinhole camera for ``Preprocessor``: ``view`` = [R | T] (3 x 4,
    world to camera), focal lengths and principal point in pixels, tangents
    of the half field of view, camera centre in world coordinates."""
    return _abi.make_camera(view, fx, fy, cx, cy, tan_fovx, tan_fovy, cam_pos, near_plane, sh_degree)


@dataclasses.dataclass
class PreprocessOutput:
    records: object        # (N, 4) int32: ss_gaussian2d (mean_x, mean_y, depth bits, radius)
    conic_opacity: object  # (N, 4) float32
    rgb: object            # (N, 4) float32


class Preprocessor:
    """Pre-allocated outputs for repeated ``ss_preprocess`` calls on up to
    ``capacity`` Gaussians: the projection of 3D Gaussians to the sort's
    records and the render's conic, opacity and colour."""

    def __init__(self, capacity: int, device="cuda"):
        torch = _torch()
        self.capacity = capacity
        self.out = PreprocessOutput(torch.empty((capacity, 4), dtype=torch.int32, device=device),
                                    torch.empty((capacity, 4), dtype=torch.float32, device=device),
                                    torch.empty((capacity, 4), dtype=torch.float32, device=device))

    def __call__(self, cam: _abi.ss_camera, mean3d_opacity, cov3d, sh, stream=None,
                 timer: Optional[Timer] = None) -> PreprocessOutput:
        torch = _torch()
        n = int(mean3d_opacity.shape[0])
        if n > self.capacity:
            raise ValueError(f"{n} Gaussians exceed the capacity {self.capacity}")
        for t, cols, name in ((mean3d_opacity, 4, "mean3d_opacity"), (cov3d, 8, "cov3d"), (sh, 48, "sh")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != cols or t.shape[0] != n \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous ({n}, {cols}) float32 tensor")
        o = self.out
        d = _abi.make_preprocess_desc(n, mean3d_opacity.data_ptr(), cov3d.data_ptr(), sh.data_ptr(),
                                      o.records.data_ptr(), o.conic_opacity.data_ptr(), o.rgb.data_ptr(),
                                      timer.handle if timer is not None else None)
        check(_abi.ss_preprocess(cam, d, _stream_handle(stream)), "ss_preprocess")
        return PreprocessOutput(o.records[:n], o.conic_opacity[:n], o.rgb[:n])

def copy_bytes(dst, src, nbytes: int, stream=None, timer: Optional[Timer] = None):
    opts = make_options(timer=timer.handle if timer is not None else None)
    check(_abi.ss_copy_bytes(dst.data_ptr(), src.data_ptr(), nbytes, _stream_handle(stream), opts),
          "ss_copy_bytes")

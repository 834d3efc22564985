"""ctypes declarations of the C ABI in include/splatsort.h (argument
marshalling only; every step of the sort runs in the HIP library).

Loading fails loudly when libsplatsort.so has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsplatsort.so")

SS_OK = 0
SS_ERR_INVALID_ARGUMENT = 1
SS_ERR_UNSUPPORTED = 2
SS_ERR_CAPACITY = 3
SS_ERR_OVERFLOW = 4
SS_ERR_INVALID_INPUT = 5
SS_ERR_WORKSPACE = 6
SS_ERR_HIP = 7
SS_ERR_BUDGET = 8
SS_ERR_TIMEOUT = 9

SS_KERNEL_CLEAR = 0
SS_KERNEL_COUNT_DUP = 1
SS_KERNEL_SORT_PASS = 2
SS_KERNEL_RANGES = 3
SS_KERNEL_COPY = 4
SS_KERNEL_HIST = 5
SS_KERNEL_DIGIT_BASES = 6
SS_KERNEL_DEPTH_PASS = 7
SS_KERNEL_EXPAND = 8
SS_KERNEL_RENDER = 9
SS_KERNEL_PREPROCESS = 10
SS_KERNEL_TILE_SORT = 11
SS_RENDER_EXACT = 1

SS_ALGO_AUTO = 0
SS_ALGO_DEPTH_FIRST = 1
SS_ALGO_DIRECT = 2
SS_ALGO_BITONIC = 3
SS_ALGO_TILE_FIRST = 4
SS_MAX_BATCH_FRAMES = 256

SS_FLAG_UNSORTED = 1
SS_FLAG_KEY32_LOSSY = 2
SS_FLAG_DROP_CULLED = 4
SS_FLAG_PERSISTENT = 8
SS_FAULT_NONE = 0
SS_FAULT_WITHHOLD_BASES = 1

SS_MAX_IMAGE_PX = 1048560
SS_MAX_PAIR_CAPACITY = (1 << 30) - 1
SS_NOALLOC_SCRATCH_BYTES = 128 << 20


class ss_frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("tile_px", ctypes.c_uint32), ("num_gaussians", ctypes.c_uint32),
                ("gaussians", ctypes.c_void_p)]


class ss_frame_out(ctypes.Structure):
    _fields_ = [("pair_capacity", ctypes.c_uint32),
                ("keys", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("tile_ranges", ctypes.c_void_p), ("tiles_touched", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("num_pairs", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class ss_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("radix_bits", ctypes.c_uint32),
                ("items_per_thread", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("timer", ctypes.c_void_p), ("workgroup_size", ctypes.c_uint32),
                ("algorithm", ctypes.c_uint32), ("spin_limit", ctypes.c_uint32), ("fault", ctypes.c_uint32)]


class ss_batch_out(ctypes.Structure):
    _fields_ = [("pair_capacity", ctypes.c_uint32),
                ("keys", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("tile_ranges", ctypes.c_void_p), ("frame_pairs", ctypes.c_void_p),
                ("frame_pair_base", ctypes.c_void_p), ("num_pairs", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


def make_options(radix_bits: int = 0, items_per_thread: int = 0, timer=None, flags: int = 0,
                 workgroup_size: int = 0, algorithm: int = 0, spin_limit: int = 0, fault: int = 0) -> ss_options:
    o = ss_options()
    o.struct_size = ctypes.sizeof(ss_options)
    o.radix_bits = radix_bits
    o.items_per_thread = items_per_thread
    o.flags = flags
    o.timer = timer
    o.workgroup_size = workgroup_size
    o.algorithm = algorithm
    o.spin_limit = spin_limit
    o.fault = fault
    return o


class SplatSortError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_SZ = ctypes.c_size_t


class ss_server_desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_batch_frames", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("options", ss_options)]


class ss_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("num_pairs", ctypes.c_uint32), ("keys", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("tile_ranges", ctypes.c_void_p), ("tile_base", ctypes.c_uint32),
                ("pair_base", ctypes.c_uint32), ("round_frames", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("submit_us", ctypes.c_double), ("start_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class ss_server_counters(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("pending", ctypes.c_uint64), ("arena_used", ctypes.c_uint64),
                ("mean_round_frames", ctypes.c_double)]


class ss_plan_desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_frames", ctypes.c_uint32),
                ("frames", ctypes.c_void_p), ("out", ss_batch_out), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("autotune", ctypes.c_uint32),
                ("tune_repeats", ctypes.c_uint32), ("options", ss_options), ("tune_cache", ctypes.c_char_p)]

class ss_render_desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("conic_opacity", ctypes.c_void_p), ("rgb", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("tile_ranges", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("background", ctypes.c_float * 3), ("out_color", ctypes.c_void_p), ("out_T", ctypes.c_void_p),
                ("out_contrib", ctypes.c_void_p), ("out_tile_evals", ctypes.c_void_p), ("timer", ctypes.c_void_p)]


class ss_camera(ctypes.Structure):
    _fields_ = [("view", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("tan_fovx", ctypes.c_float),
                ("tan_fovy", ctypes.c_float), ("cam_pos", ctypes.c_float * 3), ("near_plane", ctypes.c_float),
                ("sh_degree", ctypes.c_uint32)]


class ss_preprocess_desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("num_gaussians", ctypes.c_uint32),
                ("mean3d_opacity", ctypes.c_void_p), ("cov3d", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("out_records", ctypes.c_void_p), ("out_conic_opacity", ctypes.c_void_p),
                ("out_rgb", ctypes.c_void_p), ("timer", ctypes.c_void_p)]

_SIGNATURES = {
    "ss_abi_version": ([], _U32),
    "ss_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "ss_frame_geometry": ([ctypes.POINTER(ss_frame), _P, _P, _P], ctypes.c_int),
    "ss_workspace_bytes": ([ctypes.POINTER(ss_frame), _U32, ctypes.POINTER(ss_options),
                            ctypes.POINTER(_SZ)], ctypes.c_int),
    "ss_count_pairs": ([ctypes.POINTER(ss_frame), _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "ss_sort_frame": ([ctypes.POINTER(ss_frame), ctypes.POINTER(ss_frame_out), _P, _SZ, _P,
                       ctypes.POINTER(ss_options)], ctypes.c_int),
    "ss_sort_frame_noalloc": ([ctypes.POINTER(ss_frame), ctypes.POINTER(ss_frame_out), _P,
                               ctypes.POINTER(ss_options)], ctypes.c_int),
    "ss_batch_workspace_bytes": ([ctypes.POINTER(ss_frame), _U32, _U32, ctypes.POINTER(ss_options),
                                  ctypes.POINTER(_SZ)], ctypes.c_int),
    "ss_sort_batch": ([ctypes.POINTER(ss_frame), _U32, ctypes.POINTER(ss_batch_out), _P, _SZ, _P,
                       ctypes.POINTER(ss_options)], ctypes.c_int),
    "ss_plan_workspace_bytes": ([ctypes.POINTER(ss_frame), _U32, _U32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "ss_plan_create": ([ctypes.POINTER(_P), ctypes.POINTER(ss_plan_desc), _P], ctypes.c_int),
    "ss_plan_launch": ([_P, _P], ctypes.c_int),
    "ss_plan_config": ([_P, ctypes.POINTER(ss_options), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_U32)],
                       ctypes.c_int),
    "ss_plan_destroy": ([_P], None),
    "ss_batch_count_workspace_bytes": ([ctypes.POINTER(ss_frame), _U32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "ss_batch_count_pairs": ([ctypes.POINTER(ss_frame), _U32, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "ss_server_create": ([ctypes.POINTER(_P), _P, _SZ, ctypes.POINTER(ss_server_desc)], ctypes.c_int),
    "ss_server_submit": ([_P, ctypes.POINTER(ss_frame), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "ss_server_wait": ([_P, ctypes.c_uint64, ctypes.POINTER(ss_result)], ctypes.c_int),
    "ss_server_release": ([_P, ctypes.c_uint64], ctypes.c_int),
    "ss_server_stats": ([_P, ctypes.POINTER(ss_server_counters)], ctypes.c_int),
    "ss_server_destroy": ([_P], None),
    "ss_sort_pairs_workspace_bytes": ([_U32, _U32, ctypes.POINTER(ss_options), ctypes.POINTER(_SZ)],
                                      ctypes.c_int),
    "ss_sort_pairs": ([_P, _P, _U32, _U32, _P, _P, _P, _SZ, _P, ctypes.POINTER(ss_options)],
                      ctypes.c_int),
    "ss_copy_bytes": ([_P, _P, _SZ, _P, ctypes.POINTER(ss_options)], ctypes.c_int),
    "ss_render_frame": ([ctypes.POINTER(ss_frame), ctypes.POINTER(ss_render_desc), _P], ctypes.c_int),
    "ss_preprocess": ([ctypes.POINTER(ss_camera), ctypes.POINTER(ss_preprocess_desc), _P], ctypes.c_int),
    "ss_timer_create": ([ctypes.POINTER(_P), _U32], ctypes.c_int),
    "ss_timer_reset": ([_P], ctypes.c_int),
    "ss_timer_read": ([_P, _U32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_U32)], ctypes.c_int),
    "ss_timer_destroy": ([_P], None),
}

_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2511_16298_amd.build` (there is no fallback)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = h
    return _LIB


def status_string(status: int) -> str:
    return lib().ss_status_string(status).decode()


def check(status: int, what: str):
    if status != SS_OK:
        raise SplatSortError(status, what)


def declared_symbols():
    return sorted(_SIGNATURES)


# Thin wrappers with the C names -------------------------------------------------

def ss_abi_version() -> int:
    return lib().ss_abi_version()


def ss_status_string(status: int) -> str:
    return status_string(status)


def ss_frame_geometry(frame: ss_frame):
    tx, ty, kb = _U32(), _U32(), _U32()
    st = lib().ss_frame_geometry(ctypes.byref(frame), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(kb))
    return st, tx.value, ty.value, kb.value


def ss_workspace_bytes(frame: ss_frame, pair_capacity: int, options=None):
    n = _SZ()
    st = lib().ss_workspace_bytes(ctypes.byref(frame), pair_capacity,
                                  ctypes.byref(options) if options is not None else None, ctypes.byref(n))
    return st, n.value


def ss_count_pairs(frame: ss_frame, d_tiles_touched, d_offsets, d_num_pairs, d_status, workspace,
                   workspace_bytes, stream):
    return lib().ss_count_pairs(ctypes.byref(frame), d_tiles_touched, d_offsets, d_num_pairs, d_status,
                                workspace, workspace_bytes, stream)


def ss_sort_frame(frame: ss_frame, out: ss_frame_out, workspace, workspace_bytes, stream, options=None):
    return lib().ss_sort_frame(ctypes.byref(frame), ctypes.byref(out), workspace, workspace_bytes, stream,
                               ctypes.byref(options) if options is not None else None)


def ss_sort_frame_noalloc(frame: ss_frame, out: ss_frame_out, stream, options=None):
    return lib().ss_sort_frame_noalloc(ctypes.byref(frame), ctypes.byref(out), stream,
                                       ctypes.byref(options) if options is not None else None)


def _frames_array(frames):
    arr = (ss_frame * len(frames))()
    for i, f in enumerate(frames):
        arr[i] = f
    return arr


def ss_batch_workspace_bytes(frames, pair_capacity: int, options=None):
    arr = _frames_array(frames)
    b = _SZ()
    st = lib().ss_batch_workspace_bytes(arr, len(frames), pair_capacity,
                                        ctypes.byref(options) if options is not None else None, ctypes.byref(b))
    return st, b.value


def ss_sort_batch(frames, out: ss_batch_out, workspace, workspace_bytes, stream, options=None):
    arr = _frames_array(frames)
    return lib().ss_sort_batch(arr, len(frames), ctypes.byref(out), workspace, workspace_bytes, stream,
                               ctypes.byref(options) if options is not None else None)


def ss_plan_workspace_bytes(frames, pair_capacity: int):
    arr = _frames_array(frames)
    b = _SZ()
    st = lib().ss_plan_workspace_bytes(arr, len(frames), pair_capacity, ctypes.byref(b))
    return st, b.value


def ss_plan_create(frames, out: ss_batch_out, workspace, workspace_bytes, stream, autotune=0, tune_repeats=0,
                   options=None, tune_cache=None):
    arr = _frames_array(frames)
    d = ss_plan_desc()
    d.struct_size = ctypes.sizeof(ss_plan_desc)
    d.n_frames = len(frames)
    d.frames = ctypes.addressof(arr)
    d.out = out
    d.workspace = workspace
    d.workspace_bytes = workspace_bytes
    d.autotune = autotune
    d.tune_repeats = tune_repeats
    d.options = options if options is not None else make_options()
    d.tune_cache = os.fsencode(tune_cache) if tune_cache is not None else None
    h = _P()
    st = lib().ss_plan_create(ctypes.byref(h), ctypes.byref(d), stream)
    return st, h.value


def ss_plan_launch(plan, stream) -> int:
    return lib().ss_plan_launch(plan, stream)


def ss_plan_config(plan, max_candidates: int = 16):
    o = ss_options()
    ms = (ctypes.c_double * max_candidates)()
    n = _U32(max_candidates)
    st = lib().ss_plan_config(plan, ctypes.byref(o), ms, ctypes.byref(n))
    return st, o, [ms[i] for i in range(min(n.value, max_candidates))]


def ss_plan_destroy(plan) -> None:
    lib().ss_plan_destroy(plan)


def ss_batch_count_workspace_bytes(frames):
    arr = _frames_array(frames)
    b = _SZ()
    st = lib().ss_batch_count_workspace_bytes(arr, len(frames), ctypes.byref(b))
    return st, b.value


def ss_batch_count_pairs(frames, d_frame_pairs, d_num_pairs, d_status, workspace, workspace_bytes, stream):
    arr = _frames_array(frames)
    return lib().ss_batch_count_pairs(arr, len(frames), d_frame_pairs, d_num_pairs, d_status, workspace,
                                      workspace_bytes, stream)


def ss_server_create(arena, arena_bytes, max_batch_frames, n_streams, options=None):
    d = ss_server_desc()
    d.struct_size = ctypes.sizeof(ss_server_desc)
    d.max_batch_frames = max_batch_frames
    d.n_streams = n_streams
    d.reserved = 0
    d.options = options if options is not None else make_options()
    h = _P()
    st = lib().ss_server_create(ctypes.byref(h), arena, arena_bytes, ctypes.byref(d))
    return st, h.value


def ss_server_submit(server, frame: ss_frame):
    t = ctypes.c_uint64()
    st = lib().ss_server_submit(server, ctypes.byref(frame), ctypes.byref(t))
    return st, t.value


def ss_server_wait(server, ticket: int):
    r = ss_result()
    st = lib().ss_server_wait(server, ticket, ctypes.byref(r))
    return st, r


def ss_server_release(server, ticket: int) -> int:
    return lib().ss_server_release(server, ticket)


def ss_server_stats(server):
    c = ss_server_counters()
    st = lib().ss_server_stats(server, ctypes.byref(c))
    return st, c


def ss_server_destroy(server) -> None:
    lib().ss_server_destroy(server)


def ss_sort_pairs_workspace_bytes(n: int, key_bits: int, options=None):
    b = _SZ()
    st = lib().ss_sort_pairs_workspace_bytes(n, key_bits, ctypes.byref(options) if options is not None else None,
                                             ctypes.byref(b))
    return st, b.value


def ss_sort_pairs(keys_in, values_in, n, key_bits, keys_out, values_out, workspace, workspace_bytes, stream,
                  options=None):
    return lib().ss_sort_pairs(keys_in, values_in, n, key_bits, keys_out, values_out, workspace, workspace_bytes,
                               stream, ctypes.byref(options) if options is not None else None)


def make_render_desc(conic_opacity, rgb, values, tile_ranges, out_color, status=None, background=(0.0, 0.0, 0.0),
                     exact=False, out_T=None, out_contrib=None, out_tile_evals=None, timer=None) -> ss_render_desc:
    d = ss_render_desc()
    d.struct_size = ctypes.sizeof(ss_render_desc)
    d.flags = SS_RENDER_EXACT if exact else 0
    d.conic_opacity, d.rgb, d.values, d.tile_ranges = conic_opacity, rgb, values, tile_ranges
    d.status, d.out_color, d.out_T, d.out_contrib = status, out_color, out_T, out_contrib
    d.out_tile_evals, d.timer = out_tile_evals, timer
    for i in range(3):
        d.background[i] = float(background[i])
    return d


def ss_render_frame(frame, desc, stream):
    return lib().ss_render_frame(ctypes.byref(frame), ctypes.byref(desc), stream)


def make_camera(view, fx, fy, cx, cy, tan_fovx, tan_fovy, cam_pos, near_plane, sh_degree) -> ss_camera:
    """``view``: 12 floats, [R | T] row-major 3 x 4 (world to camera)."""
    c = ss_camera()
    v = [float(x) for x in (view.reshape(-1) if hasattr(view, "reshape") else view)]
    if len(v) != 12:
        raise ValueError("view must hold 12 values ([R | T], 3 x 4)")
    for i in range(12):
        c.view[i] = v[i]
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    c.tan_fovx, c.tan_fovy = float(tan_fovx), float(tan_fovy)
    for i in range(3):
        c.cam_pos[i] = float(cam_pos[i])
    c.near_plane, c.sh_degree = float(near_plane), int(sh_degree)
    return c


def make_preprocess_desc(n, mean3d_opacity, cov3d, sh, out_records, out_conic_opacity, out_rgb,
                         timer=None) -> ss_preprocess_desc:
    d = ss_preprocess_desc()
    d.struct_size = ctypes.sizeof(ss_preprocess_desc)
    d.num_gaussians = n
    d.mean3d_opacity, d.cov3d, d.sh = mean3d_opacity, cov3d, sh
    d.out_records, d.out_conic_opacity, d.out_rgb, d.timer = out_records, out_conic_opacity, out_rgb, timer
    return d


def ss_preprocess(camera, desc, stream):
    return lib().ss_preprocess(ctypes.byref(camera) if camera is not None else None,
                               ctypes.byref(desc) if desc is not None else None, stream)

def ss_copy_bytes(dst, src, nbytes, stream, options=None):
    return lib().ss_copy_bytes(dst, src, nbytes, stream, ctypes.byref(options) if options is not None else None)


def ss_timer_create(max_launches: int):
    h = _P()
    st = lib().ss_timer_create(ctypes.byref(h), max_launches)
    return st, h.value


def ss_timer_reset(timer) -> int:
    return lib().ss_timer_reset(timer)


def ss_timer_read(timer, kind: int):
    ms, n = ctypes.c_double(), _U32()
    st = lib().ss_timer_read(timer, kind, ctypes.byref(ms), ctypes.byref(n))
    return st, ms.value, n.value


def ss_timer_destroy(timer) -> None:
    lib().ss_timer_destroy(timer)

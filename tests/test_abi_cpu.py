"""The C-ABI library without a GPU: it loads, exports every function that
include/splatsort.h declares, and rejects bad arguments synchronously (no
compute calls are made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "splatsort.h")

from paper_2511_16298_amd import _abi  # noqa: E402


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?!typedef)[A-Za-z_][\w\s\*]*?\b(ss_\w+)\s*\(", text, flags=re.M):
        names.add(m.group(1))
    return names


def test_header_parsed():
    names = header_functions()
    assert {"ss_sort_frame", "ss_count_pairs", "ss_sort_pairs", "ss_workspace_bytes"} <= names


def test_every_declared_function_is_exported():
    out = subprocess.check_output(["nm", "-D", "--defined-only", _abi.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = header_functions() - exported
    assert not missing, missing
    lib = _abi.lib()
    for name in header_functions():
        assert hasattr(lib, name)


def test_binding_declares_exactly_the_header():
    assert set(_abi.declared_symbols()) == header_functions()


def test_abi_version_and_status_strings():
    assert _abi.ss_abi_version() == 1
    for s in range(10):
        assert _abi.ss_status_string(s) and "unknown" not in _abi.ss_status_string(s)
    assert "unknown" in _abi.ss_status_string(77)


def frame(w=1920, h=1080, n=0, ptr=None, tile=16):
    f = _abi.ss_frame()
    f.width, f.height, f.tile_px, f.num_gaussians = w, h, tile, n
    f.gaussians = ptr
    return f


@pytest.mark.parametrize("w,h,tx,ty,kb", [(1920, 1080, 120, 68, 45), (256, 256, 16, 16, 40),
                                          (16, 16, 1, 1, 32), (17, 16, 2, 1, 33), (1, 1, 1, 1, 32),
                                          (1048560, 1048560, 65535, 65535, 64)])
def test_geometry(w, h, tx, ty, kb):
    st, a, b, c = _abi.ss_frame_geometry(frame(w, h))
    assert st == _abi.SS_OK and (a, b, c) == (tx, ty, kb)


@pytest.mark.parametrize("f", [frame(0, 10), frame(10, 0), frame(1048561, 4), frame(tile=8),
                               frame(n=5, ptr=None), frame(n=5, ptr=8), frame(n=1 << 31, ptr=256)])
def test_bad_frames_rejected(f):
    assert _abi.ss_frame_geometry(f)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_workspace_bytes(f, 10)[0] == _abi.SS_ERR_INVALID_ARGUMENT


def fake_out(cap=100):
    o = _abi.ss_frame_out()
    o.pair_capacity = cap
    o.keys, o.values, o.tile_ranges = 1 << 20, 2 << 20, 3 << 20
    return o


def test_sort_frame_argument_errors_are_synchronous():
    f = frame(n=10, ptr=1 << 12)
    st, need = _abi.ss_workspace_bytes(f, 100)
    assert st == _abi.SS_OK and need > 0
    ws = 4 << 20
    # workspace too small / misaligned / missing
    assert _abi.ss_sort_frame(f, fake_out(), ws, need - 1, None) == _abi.SS_ERR_WORKSPACE
    assert _abi.ss_sort_frame(f, fake_out(), ws + 8, need, None) == _abi.SS_ERR_WORKSPACE
    assert _abi.ss_sort_frame(f, fake_out(), None, need, None) == _abi.SS_ERR_WORKSPACE
    # outputs
    o = fake_out()
    o.keys = None
    assert _abi.ss_sort_frame(f, o, ws, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    o = fake_out()
    o.tile_ranges = None
    assert _abi.ss_sort_frame(f, o, ws, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    o = fake_out()
    o.keys = (1 << 20) + 4
    assert _abi.ss_sort_frame(f, o, ws, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    o = fake_out(cap=_abi.SS_MAX_PAIR_CAPACITY + 1)
    assert _abi.ss_sort_frame(f, o, ws, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    # options
    for rb, it, fl, wg in [(5, 0, 0, 0), (9, 0, 0, 0), (0, 7, 0, 0), (0, 0, 16, 0), (0, 0, 0, 128),
                           (6, 12, 0, 512), (0, 12, 0, 512), (0, 0, 0, 1024)]:
        opt = _abi.make_options(rb, it, flags=fl, workgroup_size=wg)
        assert _abi.ss_sort_frame(f, fake_out(), ws, need, None, opt) == _abi.SS_ERR_UNSUPPORTED
    assert _abi.ss_sort_frame(f, fake_out(), ws, need, None,
                              _abi.make_options(fault=_abi.SS_FAULT_WITHHOLD_BASES + 1)) == _abi.SS_ERR_UNSUPPORTED
    bad = _abi.make_options()
    bad.struct_size = 4
    assert _abi.ss_sort_frame(f, fake_out(), ws, need, None, bad) == _abi.SS_ERR_INVALID_ARGUMENT
    # a caller built before spin_limit and fault existed: the shorter struct is
    # accepted and the fields it does not cover are not read
    old = _abi.make_options(fault=99)
    old.struct_size = _abi.ss_options.spin_limit.offset
    assert _abi.ss_workspace_bytes(f, 1000, old)[0] == _abi.SS_OK
    # count-only entry point
    assert _abi.ss_count_pairs(f, None, None, None, 1 << 10, ws, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_count_pairs(f, None, None, 1 << 10, 1 << 11, ws, 16, None) == _abi.SS_ERR_WORKSPACE


def test_sort_pairs_argument_errors():
    st, need = _abi.ss_sort_pairs_workspace_bytes(1000, 45)
    assert st == _abi.SS_OK
    for kb in (0, 65):
        assert _abi.ss_sort_pairs_workspace_bytes(10, kb)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    a, b, c, d = 1 << 20, 2 << 20, 3 << 20, 4 << 20
    assert _abi.ss_sort_pairs(a, b, 1000, 45, a, d, 8 << 20, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_sort_pairs(a, b, 1000, 45, c, d, 8 << 20, need - 1, None) == _abi.SS_ERR_WORKSPACE
    assert _abi.ss_sort_pairs(a + 4, b, 1000, 45, c, d, 8 << 20, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_copy_bytes(a, b, 15, None) == _abi.SS_ERR_INVALID_ARGUMENT


def test_workspace_grows_with_capacity_and_gaussians():
    f = frame(n=10_000, ptr=256)
    w1 = _abi.ss_workspace_bytes(f, 1000)[1]
    w2 = _abi.ss_workspace_bytes(f, 2_000_000)[1]
    assert w2 > w1 + 2_000_000 * 12
    assert _abi.ss_workspace_bytes(frame(n=10_000_000, ptr=256), 1000)[1] > w1
    assert _abi.ss_workspace_bytes(f, 1000, _abi.make_options(4))[1] != w1


def test_product_and_oracle_share_no_code():
    pkg = os.path.join(ROOT, "paper_2511_16298_amd")
    orc = os.path.join(ROOT, "oracle")
    for d, other in ((pkg, "oracle"), (orc, "paper_2511_16298_amd")):
        for dirpath, _, files in os.walk(d):
            for fn in files:
                if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                    txt = open(os.path.join(dirpath, fn)).read()
                    assert not re.search(rf"\bimport\s+{other}\b|\bfrom\s+{other}\b|{other}/", txt), (fn, other)
    # the product never includes the oracle header and vice versa
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".hip", ".hpp")):
                assert "oracle.h" not in open(os.path.join(dirpath, fn)).read()


def test_batch_argument_errors():
    fr = [frame(640, 360, n=100, ptr=1 << 12), frame(1280, 720, n=50, ptr=1 << 14)]
    st, need = _abi.ss_batch_workspace_bytes(fr, 1000)
    assert st == _abi.SS_OK and need > 0
    assert _abi.ss_batch_workspace_bytes([], 10)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_batch_workspace_bytes([frame()] * 257, 10)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_batch_workspace_bytes([fr[0], frame(0, 5)], 10)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_batch_workspace_bytes(fr, 10, _abi.make_options(algorithm=2))[0] == _abi.SS_ERR_UNSUPPORTED
    o = _abi.ss_batch_out()
    o.pair_capacity = 1000
    o.keys, o.values, o.tile_ranges = 1 << 20, 2 << 20, 3 << 20
    assert _abi.ss_sort_batch(fr, o, 4 << 20, need - 1, None) == _abi.SS_ERR_WORKSPACE
    o.tile_ranges = None
    assert _abi.ss_sort_batch(fr, o, 4 << 20, need, None) == _abi.SS_ERR_INVALID_ARGUMENT


def test_algorithm_option_validated():
    f = frame(n=10, ptr=1 << 12)
    assert _abi.ss_workspace_bytes(f, 100, _abi.make_options(algorithm=5))[0] == _abi.SS_ERR_UNSUPPORTED
    # tile-first: frames only
    assert _abi.ss_workspace_bytes(f, 100, _abi.make_options(algorithm=_abi.SS_ALGO_TILE_FIRST))[0] == _abi.SS_OK
    assert _abi.ss_batch_workspace_bytes([f, f], 100, _abi.make_options(algorithm=_abi.SS_ALGO_TILE_FIRST))[0] == \
        _abi.SS_ERR_UNSUPPORTED
    a = _abi.ss_workspace_bytes(f, 100, _abi.make_options(algorithm=1))
    b = _abi.ss_workspace_bytes(f, 100, _abi.make_options(algorithm=2))
    assert a[0] == b[0] == _abi.SS_OK and a[1] != b[1]


def test_bitonic_workspace_holds_the_padded_size():
    f = frame(n=10, ptr=1 << 12)
    direct = _abi.ss_workspace_bytes(f, 5000, _abi.make_options(algorithm=_abi.SS_ALGO_DIRECT))[1]
    bit = _abi.ss_workspace_bytes(f, 5000, _abi.make_options(algorithm=_abi.SS_ALGO_BITONIC))
    assert bit[0] == _abi.SS_OK and bit[1] >= 8192 * 12
    assert _abi.ss_workspace_bytes(f, 8192, _abi.make_options(algorithm=_abi.SS_ALGO_BITONIC))[1] == \
        _abi.ss_workspace_bytes(f, 5000, _abi.make_options(algorithm=_abi.SS_ALGO_BITONIC))[1]
    assert direct > 0
    # batches take the radix paths only
    assert _abi.ss_batch_workspace_bytes([frame(n=10, ptr=1 << 12)], 100,
                                         _abi.make_options(algorithm=_abi.SS_ALGO_BITONIC))[0] == \
        _abi.SS_ERR_UNSUPPORTED


def test_server_and_count_argument_errors():
    # rejected before any HIP call: no GPU needed
    assert _abi.ss_server_create(None, 1 << 20, 4, 1)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_server_create(1 << 20 | 8, 1 << 20, 4, 1)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_server_create(1 << 20, 1 << 20, 0, 1)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_server_create(1 << 20, 1 << 20, 257, 1)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_server_create(1 << 20, 1 << 20, 4, 0)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_server_create(1 << 20, 1 << 20, 4, 9)[0] == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_server_create(1 << 20, 1 << 20, 4, 1, _abi.make_options(5))[0] == _abi.SS_ERR_UNSUPPORTED
    fr = [frame(640, 360, n=100, ptr=1 << 12)]
    st, need = _abi.ss_batch_count_workspace_bytes(fr)
    assert st == _abi.SS_OK and need > 0
    assert _abi.ss_batch_count_pairs(fr, None, 1 << 10, 1 << 11, 1 << 20, need, None) == _abi.SS_ERR_INVALID_ARGUMENT
    assert _abi.ss_batch_count_pairs(fr, 1 << 9, 1 << 10, 1 << 11, 1 << 20, need - 1, None) == _abi.SS_ERR_WORKSPACE
    st, need = _abi.ss_plan_workspace_bytes(fr, 1000)
    assert st == _abi.SS_OK and need > 0


def test_render_argument_errors_are_synchronous():
    f = frame(64, 32, n=10, ptr=1 << 12)
    a = 1 << 20
    good = dict(conic_opacity=a, rgb=2 * a, values=3 * a, tile_ranges=4 * a, out_color=5 * a)

    def call(fr=f, struct_size=None, flags=0, **kw):
        args = dict(good)
        args.update(kw)
        d = _abi.make_render_desc(args["conic_opacity"], args["rgb"], args["values"], args["tile_ranges"],
                                  args["out_color"])
        d.flags = flags
        if struct_size is not None:
            d.struct_size = struct_size
        return _abi.ss_render_frame(fr, d, None)

    bad = _abi.SS_ERR_INVALID_ARGUMENT
    assert call(struct_size=8) == bad
    assert call(flags=2) == bad
    assert call(out_color=None) == bad
    assert call(tile_ranges=None) == bad
    assert call(conic_opacity=None) == bad and call(rgb=None) == bad and call(values=None) == bad
    assert call(conic_opacity=a + 8) == bad and call(rgb=2 * a + 4) == bad
    assert call(fr=frame(0, 32, n=10, ptr=1 << 12)) == bad


def test_preprocess_argument_errors_are_synchronous():
    a = 1 << 20
    good = dict(mean3d_opacity=a, cov3d=2 * a, sh=3 * a, out_records=4 * a, out_conic_opacity=5 * a, out_rgb=6 * a)
    view = [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]

    def cam(**kw):
        c = dict(view=view, fx=1000.0, fy=1000.0, cx=320.0, cy=240.0, tan_fovx=0.3, tan_fovy=0.2,
                 cam_pos=(0, 0, 0), near_plane=0.2, sh_degree=3)
        c.update(kw)
        return _abi.make_camera(**c)

    def call(c=None, n=10, struct_size=None, **kw):
        args = dict(good)
        args.update(kw)
        d = _abi.make_preprocess_desc(n, args["mean3d_opacity"], args["cov3d"], args["sh"], args["out_records"],
                                      args["out_conic_opacity"], args["out_rgb"])
        if struct_size is not None:
            d.struct_size = struct_size
        return _abi.ss_preprocess(c if c is not None else cam(), d, None)

    bad = _abi.SS_ERR_INVALID_ARGUMENT
    assert call(struct_size=8) == bad
    assert _abi.ss_preprocess(None, _abi.make_preprocess_desc(1, a, a, a, a, a, a), None) == bad
    assert _abi.ss_preprocess(cam(), None, None) == bad
    for k in good:
        assert call(**{k: None}) == bad, k
        assert call(**{k: good[k] + 4}) == bad, k
    assert call(n=1 << 31) == bad
    assert call(c=cam(sh_degree=4)) == bad
    assert call(c=cam(tan_fovx=0.0)) == bad and call(c=cam(tan_fovy=-1.0)) == bad
    assert call(c=cam(fx=float("inf"))) == bad and call(c=cam(near_plane=float("nan"))) == bad
    assert call(c=cam(view=view[:11] + [float("nan")])) == bad
    # nothing to do: no device call, no pointer needed
    assert call(n=0, **{k: None for k in good}) == _abi.SS_OK


def test_key32_option_rules():
    """The normalised 32-bit key: bitonic frames only, at most 2^20 tiles."""
    f = frame(n=10, ptr=1 << 12)
    K, U = _abi.SS_FLAG_KEY32_LOSSY, _abi.SS_FLAG_UNSORTED
    for algo in (_abi.SS_ALGO_AUTO, _abi.SS_ALGO_DEPTH_FIRST, _abi.SS_ALGO_DIRECT):
        assert _abi.ss_workspace_bytes(f, 100, _abi.make_options(flags=K, algorithm=algo))[0] == \
            _abi.SS_ERR_UNSUPPORTED
    assert _abi.ss_workspace_bytes(f, 100, _abi.make_options(flags=K | U, algorithm=_abi.SS_ALGO_BITONIC))[0] == \
        _abi.SS_ERR_UNSUPPORTED
    st, need = _abi.ss_workspace_bytes(f, 100, _abi.make_options(flags=K, algorithm=_abi.SS_ALGO_BITONIC))
    assert st == _abi.SS_OK
    assert need == _abi.ss_workspace_bytes(f, 100, _abi.make_options(algorithm=_abi.SS_ALGO_BITONIC))[1]
    opt = _abi.make_options(flags=K, algorithm=_abi.SS_ALGO_BITONIC)
    # 2^21 tiles: more than the key's 20 tile bits
    big = frame(w=16 * 2048, h=16 * 1024, n=10, ptr=1 << 12)
    st, need_big = _abi.ss_workspace_bytes(big, 100, opt)
    assert st == _abi.SS_OK
    assert _abi.ss_sort_frame(big, fake_out(), 4 << 20, need_big, None, opt) == _abi.SS_ERR_UNSUPPORTED
    # sort-only keys carry no (tile, depth) structure
    st, need_p = _abi.ss_sort_pairs_workspace_bytes(1000, 45, _abi.make_options(algorithm=_abi.SS_ALGO_BITONIC))
    assert st == _abi.SS_OK
    a, b, c, d = 1 << 20, 2 << 20, 3 << 20, 4 << 20
    assert _abi.ss_sort_pairs(a, b, 1000, 45, c, d, 8 << 20, need_p, None, opt) == _abi.SS_ERR_UNSUPPORTED



def test_noalloc_rejects_before_enqueueing():
    """The no-allocation entry point returns its argument errors before any
    GPU work: a workspace beyond its fixed array, an unsupported algorithm,
    missing outputs."""
    o = fake_out(cap=_abi.SS_MAX_PAIR_CAPACITY)
    big = frame(1920, 1080, 50_000_000, ptr=256)
    st, need = _abi.ss_workspace_bytes(big, o.pair_capacity, None)
    assert st == 0 and need > _abi.SS_NOALLOC_SCRATCH_BYTES
    assert _abi.ss_sort_frame_noalloc(big, o, None) == _abi.SS_ERR_WORKSPACE
    small = frame(256, 256, 1000, ptr=256)
    o2 = fake_out(cap=10_000)
    for algo in (_abi.SS_ALGO_DIRECT, _abi.SS_ALGO_BITONIC):
        assert _abi.ss_sort_frame_noalloc(small, o2, None, _abi.make_options(algorithm=algo)) == \
            _abi.SS_ERR_UNSUPPORTED
    assert _abi.ss_sort_frame_noalloc(small, o2, None, _abi.make_options(flags=_abi.SS_FLAG_UNSORTED)) == \
        _abi.SS_ERR_UNSUPPORTED

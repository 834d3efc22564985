"""GPU path against the CPU oracle, bit for bit (integer work: tolerance 0).

Every case runs the HIP library through its C ABI (via the thin binding) and
the oracle on the same seeded records.  Sizes span several workgroup tiles
and ragged tails; the full-size workloads run in the launch configuration
the benchmark times.
"""
import hashlib

import numpy as np
import pytest

import oracle
import pins
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_16298_amd as ss  # noqa: E402
from paper_2511_16298_amd import _abi  # noqa: E402


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


ALGOS = [ss.SS_ALGO_DEPTH_FIRST, ss.SS_ALGO_DIRECT, ss.SS_ALGO_BITONIC, ss.SS_ALGO_TILE_FIRST]


def gpu_frame(W, H, rec, capacity=None, radix_bits=0, items=0, stages=True, unsorted=False, algorithm=0,
              key32=False):
    d = ss.records_to_device(rec)
    if capacity is None:
        _, _, m, s = ss.count_pairs(d, W, H)
        assert int(s.item()) == 0
        capacity = int(m.item()) & 0xFFFFFFFF
    sorter = ss.FrameSorter(W, H, len(rec), capacity, radix_bits, items, stages=stages, unsorted=unsorted,
                            algorithm=algorithm, key32=key32)
    out = sorter(d)
    st, m = out.result()
    res = {"status": st, "M": m}
    if st == 0:
        res["keys"] = u64(out.keys)[:m]
        res["values"] = u32(out.values)[:m]
        res["ranges"] = u32(out.tile_ranges).reshape(-1, 2)
    if stages and len(rec):
        res["tiles_touched"] = u32(out.tiles_touched)[:len(rec)]
        res["offsets"] = u32(out.offsets)[:len(rec)]
    return res


def assert_same(W, H, rec, g, stages=True):
    o = oracle.sort_frame(W, H, rec)
    assert o.status == 0
    assert g["status"] == 0, _abi.status_string(g["status"])
    assert g["M"] == o.num_pairs
    assert np.array_equal(g["keys"], o.keys)
    assert np.array_equal(g["values"], o.values)
    assert np.array_equal(g["ranges"], o.ranges)
    if stages and len(rec):
        assert np.array_equal(g["tiles_touched"], o.tiles_touched)
        assert np.array_equal(g["offsets"], o.offsets.astype(np.uint32))
    return o


@pytest.mark.parametrize("algo", ALGOS)
def test_tiny_frames(algo):
    rs = np.random.default_rng(2024)
    for case in range(60):
        W, H, rec = pins.random_tiny_frame(rs)
        print(f"tiny case {case}: {W}x{H} n={len(rec)}", flush=True)
        assert_same(W, H, rec, gpu_frame(W, H, rec, algorithm=algo))


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("name", ["small-256x256", "fullhd-1m"])
def test_workload_frames(name, algo):
    spec, seed = synth.FRAME_WORKLOADS[name]
    rec = synth.make_frame(spec, seed)
    assert_same(spec.width, spec.height, rec, gpu_frame(spec.width, spec.height, rec, algorithm=algo))


@pytest.mark.parametrize("algo", ALGOS)
def test_large_frame_full_size(algo):
    spec, seed = synth.FRAME_WORKLOADS["large-6m"]
    rec = synth.make_frame(spec, seed)
    assert_same(spec.width, spec.height, rec,
                gpu_frame(spec.width, spec.height, rec, stages=False, algorithm=algo), stages=False)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("rb,items", [(8, 8), (8, 12), (6, 16), (4, 16), (4, 8)])
def test_radix_widths_and_tiles(rb, items, algo):
    spec, seed = synth.FRAME_WORKLOADS["fullhd-1m"]
    spec = synth.scaled(spec, 150_000)
    rec = synth.make_frame(spec, seed)
    assert_same(spec.width, spec.height, rec,
                gpu_frame(spec.width, spec.height, rec, radix_bits=rb, items=items, algorithm=algo))


def test_unsorted_stage_matches_duplication_order():
    spec, seed = synth.FRAME_WORKLOADS["fullhd-1m"]
    spec = synth.scaled(spec, 100_000)
    rec = synth.make_frame(spec, seed)
    o = oracle.sort_frame(spec.width, spec.height, rec)
    g = gpu_frame(spec.width, spec.height, rec, capacity=o.num_pairs, unsorted=True)
    assert g["M"] == o.num_pairs
    assert np.array_equal(g["keys"], o.unsorted_keys)
    assert np.array_equal(g["values"], o.unsorted_values)


def test_count_pairs_stage():
    spec, seed = synth.FRAME_WORKLOADS["large-6m"]
    spec = synth.scaled(spec, 300_001)
    rec = synth.make_frame(spec, seed)
    tt, off, m, s = ss.count_pairs(ss.records_to_device(rec), spec.width, spec.height)
    cnt, _ = oracle.count(spec.width, spec.height, rec)
    offs, tot = oracle.scan(cnt)
    assert int(s.item()) == 0 and int(m.item()) == tot
    assert np.array_equal(u32(tt), cnt) and np.array_equal(u32(off), offs.astype(np.uint32))


def blank(n):
    return np.zeros(n, dtype=synth.RECORD_DTYPE)


@pytest.mark.parametrize("algo", ALGOS)
def test_empty_and_degenerate_frames(algo):
    # no Gaussians
    assert_same(100, 70, blank(0), gpu_frame(100, 70, blank(0), capacity=0, algorithm=algo))
    # every radius 0: M = 0, all ranges empty
    rec = synth.make_frame(synth.scaled(synth.SMALL, 5000), 5)
    rec["radius"] = 0
    g = gpu_frame(256, 256, rec, capacity=0, algorithm=algo)
    assert g["M"] == 0 and not g["ranges"].any()
    # one tile (T = 1, 32-bit keys)
    rec = synth.make_frame(synth.FrameSpec(16, 9, 20_000), 6)
    assert_same(16, 9, rec, gpu_frame(16, 9, rec, algorithm=algo))
    # every pair in one tile of a large grid, equal depths (pure index order)
    rec = blank(70_001)
    rec["mean_x"], rec["mean_y"], rec["radius"], rec["depth"] = 16 * 700 + 8, 16 * 300 + 8, 1, 2.5
    assert_same(1920, 1080, rec, gpu_frame(1920, 1080, rec, algorithm=algo))
    # every Gaussian covers the whole grid
    rec = synth.make_frame(synth.FrameSpec(200, 120, 900), 8)
    rec["radius"] = 5000
    assert_same(200, 120, rec, gpu_frame(200, 120, rec, algorithm=algo))
    # a few Gaussians covering thousands of tiles among many small ones
    rec = synth.make_frame(synth.scaled(synth.FULL_HD, 30_000), 9)
    rec["radius"][::997] = 700
    assert_same(1920, 1080, rec, gpu_frame(1920, 1080, rec, algorithm=algo))


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("m", [4095, 4096, 4097, 3 * 4096 - 1, 3 * 4096 + 1, 1023, 1025, 8191, 8193, 2047, 2049])
def test_pair_counts_around_tile_sizes(m, algo):
    # m Gaussians of one tile each: M = m, spread over the grid
    rs = np.random.default_rng(m)
    rec = blank(m)
    rec["mean_x"] = 16 * (16 * rs.integers(0, 120, m) + 8)
    rec["mean_y"] = 16 * (16 * rs.integers(0, 68, m) + 8)
    rec["radius"] = 1
    rec["depth"] = rs.choice(np.float32([1.0, 2.0, 3.0]), m)
    assert_same(1920, 1080, rec, gpu_frame(1920, 1080, rec, algorithm=algo))


# (tiles_x, tiles_y, width and height trimmed by so many px): tile counts just
# below, at and above powers of two, where the number of tile-digit passes and
# the width of the last (narrowed) pass change: 255 / 256 / 257 tiles (one or
# two 8-bit passes, the second with 1 significant bit), 4,095 / 4,096 / 4,097,
# 65,535 / 65,536 / 65,792, and 16,777,215 / 16,781,312 (three or four passes).
TILE_GRIDS = [(15, 17, 0), (16, 16, 5), (257, 1, 3), (63, 65, 7), (64, 64, 0), (17, 241, 9),
              (255, 257, 0), (256, 256, 1), (257, 256, 0), (4097, 4095, 11), (4097, 4096, 0)]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("grid", TILE_GRIDS, ids=lambda g: f"{g[0]}x{g[1]}")
def test_tile_counts_around_powers_of_two(grid, algo):
    tx, ty, trim = grid
    W, H = 16 * tx - trim, 16 * ty - trim
    n = 30_000 if tx * ty > 4096 else 6_000
    rec = synth.make_frame(synth.FrameSpec(W, H, n, radius_cap=48), 4000 + tx + ty)
    print(f"tile grid {tx}x{ty} ({W}x{H} px), N={n}, algorithm {algo}", flush=True)
    assert_same(W, H, rec, gpu_frame(W, H, rec, stages=False, algorithm=algo), stages=False)


@pytest.mark.parametrize("algo", ALGOS)
def test_device_errors(algo):
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    o = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    # capacity one short
    g = gpu_frame(256, 256, rec, capacity=o.num_pairs - 1, algorithm=algo)
    assert g["status"] == _abi.SS_ERR_CAPACITY and g["M"] == o.num_pairs
    # a NaN or negative depth on a Gaussian that touches a tile
    for bad in (np.nan, -1.0, np.inf, 0.0):
        r2 = rec.copy()
        r2["depth"][1234] = bad
        assert gpu_frame(256, 256, r2, capacity=o.num_pairs, algorithm=algo)["status"] == _abi.SS_ERR_INVALID_INPUT
    # ... but not on a culled one
    r2 = rec.copy()
    r2["depth"][1234], r2["radius"][1234] = np.nan, 0
    g = gpu_frame(256, 256, r2, capacity=o.num_pairs, algorithm=algo)
    assert g["status"] == 0
    assert_same(256, 256, r2, g)
    # 2^32 pairs or more: 300 Gaussians covering 4096 x 4096 tiles
    rec = blank(300)
    rec["mean_x"] = rec["mean_y"] = 16 * 32768
    rec["radius"], rec["depth"] = 40000, 1.0
    g = gpu_frame(65536, 65536, rec, capacity=1000, stages=False, algorithm=algo)
    assert g["status"] == _abi.SS_ERR_OVERFLOW and g["M"] == 0xFFFFFFFF
    # a frame status is reset by the next call on the same buffers
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    d = ss.records_to_device(rec)
    sorter = ss.FrameSorter(256, 256, len(rec), o.num_pairs - 1, algorithm=algo)
    assert sorter(d).result()[0] == _abi.SS_ERR_CAPACITY
    sorter = ss.FrameSorter(256, 256, len(rec), o.num_pairs, algorithm=algo)
    r2 = rec.copy()
    r2["depth"][7] = np.nan
    assert sorter(ss.records_to_device(r2)).result()[0] == _abi.SS_ERR_INVALID_INPUT
    assert sorter(d).result()[0] == 0


@pytest.mark.parametrize("n,key_bits", [(1, 45), (4095, 13), (4097, 45), (100_003, 45), (65_536, 64),
                                        (50_000, 1), (300_000, 32)])
def test_sort_pairs_against_stable_argsort(n, key_bits):
    keys, vals = synth.sort_sweep_pairs(n, key_bits, seed=n + key_bits)
    if n > 10:  # force many ties
        keys[::3] = keys[0]
    vals = np.random.default_rng(n).permutation(n).astype(np.uint32)
    ko, vo = ss.sort_pairs(torch.from_numpy(keys.view(np.int64)).cuda(),
                           torch.from_numpy(vals.view(np.int32)).cuda(), key_bits)
    ok, ov = oracle.sort_pairs(keys, vals)
    assert np.array_equal(u64(ko), ok) and np.array_equal(u32(vo), ov)


@pytest.mark.parametrize("algo", ALGOS)
def test_repeated_runs_are_identical(algo):
    spec, seed = synth.FRAME_WORKLOADS["fullhd-1m"]
    rec = synth.make_frame(spec, seed)
    d = ss.records_to_device(rec)
    _, _, m, _ = ss.count_pairs(d, spec.width, spec.height)
    sorter = ss.FrameSorter(spec.width, spec.height, len(rec), int(m.item()), algorithm=algo)
    digests = set()
    for _ in range(10):
        out = sorter(d)
        torch.cuda.synchronize()
        h = hashlib.sha256()
        for t in (out.keys, out.values, out.tile_ranges, out.status):
            h.update(t.cpu().numpy().tobytes())
        digests.add(h.hexdigest())
    assert len(digests) == 1


@pytest.mark.parametrize("n,key_bits", [(1, 45), (4095, 13), (4097, 45), (100_003, 45), (65_536, 64),
                                        (300_000, 32), (1 << 20, 45)])
def test_bitonic_sort_pairs_orders_by_key_then_value(n, key_bits):
    keys, _ = synth.sort_sweep_pairs(n, key_bits, seed=n + key_bits + 1)
    if n > 10:
        keys[::3] = keys[0]
    vals = np.random.default_rng(n).permutation(n).astype(np.uint32)
    ko, vo = ss.sort_pairs(torch.from_numpy(keys.view(np.int64)).cuda(),
                           torch.from_numpy(vals.view(np.int32)).cuda(), key_bits, algorithm=ss.SS_ALGO_BITONIC)
    order = np.lexsort((vals, keys))
    assert np.array_equal(u64(ko), keys[order]) and np.array_equal(u32(vo), vals[order])


def assert_same_key32(W, H, rec, g):
    """The paper's normalised 32-bit key order (bitonic network), bit for bit
    against the oracle's definition of it; counts and offsets as usual."""
    o = oracle.sort_frame_key32(W, H, rec)
    assert o.status == 0
    assert g["status"] == 0, _abi.status_string(g["status"])
    assert g["M"] == o.num_pairs
    assert np.array_equal(g["keys"], o.keys)
    assert np.array_equal(g["values"], o.values)
    assert np.array_equal(g["ranges"], o.ranges)
    if len(rec):
        e = oracle.sort_frame(W, H, rec)
        assert np.array_equal(g["tiles_touched"], e.tiles_touched)
        assert np.array_equal(g["offsets"], e.offsets.astype(np.uint32))


def test_key32_tiny_and_boundary_frames():
    import key32_pins
    rs = np.random.default_rng(2025)
    frames = [pins.random_tiny_frame(rs) for _ in range(40)] + [key32_pins.high_tile_frame()]
    for case, (W, H, rec) in enumerate(frames):
        print(f"key32 case {case}: {W}x{H} n={len(rec)}", flush=True)
        assert_same_key32(W, H, rec, gpu_frame(W, H, rec, algorithm=ss.SS_ALGO_BITONIC, key32=True))


@pytest.mark.parametrize("name", ["small-256x256", "fullhd-1m"])
def test_key32_workloads(name):
    spec, seed = synth.workload(name)
    rec = synth.make_frame(spec, seed)
    print(f"key32 workload {name}", flush=True)
    assert_same_key32(spec.width, spec.height, rec,
                      gpu_frame(spec.width, spec.height, rec, algorithm=ss.SS_ALGO_BITONIC, key32=True))


@pytest.mark.parametrize("n", [0, 1, 37])
def test_count_pairs_in_the_sort_workspace(n):
    """ss_count_pairs runs in the workspace ss_workspace_bytes reports for
    capacity 0 (N = 0 included, where its own layout is the larger one)."""
    rec = synth.make_frame(synth.scaled(synth.SMALL, n), 77)[:n]
    d = ss.records_to_device(rec)
    tt, off, m, s = ss.count_pairs(d, 256, 256)
    assert int(s.item()) == 0
    o = oracle.sort_frame(256, 256, rec)
    assert int(m.item()) == o.num_pairs
    if n:
        assert np.array_equal(u32(tt)[:n], o.tiles_touched)


@pytest.mark.parametrize("n", [200_000, 3_000_000])
@pytest.mark.parametrize("culled_fraction", [0.0, 0.03, 0.5, 0.97, 1.0])
def test_culled_gaussians_with_and_without_dropping(culled_fraction, n):
    """Frames whose culled share (radius 0) is below and above the point
    (1/16) where SS_FLAG_DROP_CULLED makes the depth sort drop them, for both
    depth-tile shapes (below and above 2^21 Gaussians): the output is the same
    with and without the flag (culled Gaussians have no pairs)."""
    spec, seed = synth.workload("fullhd-1m")
    rec = synth.make_frame(synth.scaled(spec, n), 4600)
    rs = np.random.default_rng(4601)
    rec["radius"][rs.random(len(rec)) < culled_fraction] = 0
    print(f"culled {culled_fraction} n={n}", flush=True)
    o = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    d = ss.records_to_device(rec)
    for drop in (False, True):
        s = ss.FrameSorter(spec.width, spec.height, len(rec), o.num_pairs, drop_culled=drop)
        s(d)
        st, m = s.out.result()
        assert st == 0 and m == o.num_pairs, drop
        assert np.array_equal(u64(s.out.keys)[:m], o.keys), drop
        assert np.array_equal(u32(s.out.values)[:m], o.values), drop
        assert np.array_equal(u32(s.out.tile_ranges).reshape(-1, 2), o.ranges), drop


def depth_field_mode(tile_bits, n, depths):
    """Which depth field the packed 64-bit pairs carry for a single frame:
    'trimmed' (depth bits minus the smallest top byte << 24, when every
    depth that has pairs then fits the field), 'position' (the depth-order
    position, when they do not), or None (pairs not packed)."""
    idx_bits = int(np.ceil(np.log2(max(n, 1)))) if n > 1 else 0
    field = 64 - tile_bits - idx_bits
    if tile_bits == 0 or field < 27 or int(np.ceil(np.log2(max(n, 1)))) > field:
        return None
    top = np.asarray(depths, np.float32).view(np.uint32) >> 24
    span = int(top.max()) - int(top.min()) + 1
    return "trimmed" if field >= 32 or (span << 24) <= (1 << field) else "position"


# frames whose pairs travel packed, with depth ranges on both sides of the
# trimmed field's width: (tiles_x, tiles_y, N, depth_lo, depth_hi, expected field)
PACKED_CASES = [(256, 256, 1 << 21, 1.0, 100.0, "trimmed"),
                (256, 256, 1 << 21, 1e-3, 1e3, "position"),
                (120, 68, 5_000_000, 1e-4, 1e4, "trimmed"),
                (120, 68, 5_000_000, 1e-6, 1e6, "position")]


@pytest.mark.parametrize("case", PACKED_CASES, ids=lambda c: f"{c[0]}x{c[1]}-n{c[2]}-{c[5]}")
def test_packed_pairs_both_depth_fields(case):
    """Pairs carried through the tile passes as one 64-bit item: with the
    trimmed depth field, and with the depth-order position when the depths
    span more binades than the field holds (the last pass then reads each
    depth back); bit-exact against the oracle either way."""
    tx, ty, n, lo, hi, mode = case
    W, H = 16 * tx, 16 * ty
    rec = synth.make_frame(synth.FrameSpec(W, H, n, depth_lo=lo, depth_hi=hi), 7100 + tx)
    cnt, _ = oracle.count(W, H, rec)
    tile_bits = int(np.ceil(np.log2(tx * ty)))
    assert depth_field_mode(tile_bits, n, rec["depth"][cnt > 0]) == mode
    print(f"packed case {tx}x{ty} N={n} depth [{lo}, {hi}] -> {mode}", flush=True)
    assert_same(W, H, rec, gpu_frame(W, H, rec, stages=False), stages=False)


def top_byte_span(depths):
    """How many top-byte values (sign and 7 exponent bits) the depth keys
    take: 2 binades per value."""
    top = np.asarray(depths, np.float32).view(np.uint32) >> 24
    return 0 if len(top) == 0 else int(top.max()) - int(top.min()) + 1


# depth ranges from one binade to the whole float range: [2, 2^17) spans
# top bytes 64..71 (8 values), [1, 2^17) 63..71 (9)
DEPTH_RANGE_CASES = [(2.0, 131000.0, 8), (1.0, 131000.0, 9), (0.7, 0.71, 1), (1e-30, 1e30, 101)]


@pytest.mark.parametrize("case", DEPTH_RANGE_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
@pytest.mark.parametrize("drop", [False, True])
def test_depth_ranges_with_and_without_dropping(case, drop):
    """Depths over one binade up to nearly all of the float range, with a
    quarter of the Gaussians culled, with and without dropping them in the
    depth sort: bit-exact pairs and ranges."""
    lo, hi, span = case
    W, H, n = 1920, 1080, 300_000
    rec = synth.make_frame(synth.FrameSpec(W, H, n, depth_lo=lo, depth_hi=hi), 7300 + span)
    rec["radius"][::4] = 0
    cnt, _ = oracle.count(W, H, rec)
    assert top_byte_span(rec["depth"][cnt > 0]) == span
    print(f"depth [{lo}, {hi}] drop={drop}: top bytes span {span}", flush=True)
    o = oracle.sort_frame(W, H, rec, stages=False)
    s = ss.FrameSorter(W, H, n, o.num_pairs, drop_culled=drop)
    out = s(ss.records_to_device(rec))
    st, m = out.result()
    assert st == 0 and m == o.num_pairs
    assert np.array_equal(u64(out.keys)[:m], o.keys)
    assert np.array_equal(u32(out.values)[:m], o.values)
    assert np.array_equal(u32(out.tile_ranges).reshape(-1, 2), o.ranges)


@pytest.mark.parametrize("name", ["fullhd-1m", "large-6m", "one-pass", "capacity-tail"])
def test_persistent_passes_frame(name):
    """Persistent tile passes on single frames: several tiles per workgroup at
    full size, one tile pass (at most 256 tiles), and a capacity far above
    the pairs (tickets past the last tile end the loop)."""
    if name in synth.FRAME_WORKLOADS:
        spec, seed = synth.FRAME_WORKLOADS[name]
        W, H, rec = spec.width, spec.height, synth.make_frame(spec, seed)
    elif name == "one-pass":
        W, H, rec = 256, 256, synth.make_frame(synth.FrameSpec(256, 256, 40_000), 91)
    else:
        W, H, rec = 640, 360, synth.make_frame(synth.FrameSpec(640, 360, 30_000), 92)
    o = oracle.sort_frame(W, H, rec, stages=False)
    cap = o.num_pairs * (4 if name == "capacity-tail" else 1)
    s = ss.FrameSorter(W, H, len(rec), cap, persistent=True)
    out = s(ss.records_to_device(rec))
    st, m = out.result()
    assert st == 0 and m == o.num_pairs
    assert np.array_equal(u64(out.keys)[:m], o.keys)
    assert np.array_equal(u32(out.values)[:m], o.values)
    assert np.array_equal(u32(out.tile_ranges).reshape(-1, 2), o.ranges)


def test_timeout_raised_from_the_host_frame():
    """A single frame with its digit bases withheld: SS_ERR_TIMEOUT, every
    kernel finishing; then the hook off, exact."""
    W, H = 1920, 1080
    rec = synth.make_frame(synth.FrameSpec(W, H, 200_000), 93)
    o = oracle.sort_frame(W, H, rec, stages=False)
    d = ss.records_to_device(rec)
    bad = ss.FrameSorter(W, H, len(rec), o.num_pairs, spin_limit=32, fault=_abi.SS_FAULT_WITHHOLD_BASES)
    st, _ = bad(d).result()
    assert st == _abi.SS_ERR_TIMEOUT
    good = ss.FrameSorter(W, H, len(rec), o.num_pairs, spin_limit=32)
    out = good(d)
    st, m = out.result()
    assert st == 0 and m == o.num_pairs
    assert np.array_equal(u64(out.keys)[:m], o.keys)


@pytest.mark.parametrize("n", [8191, 8192, 8193, 20_000])
@pytest.mark.parametrize("depths", ["random", "low-byte", "ties"])
def test_tile_first_long_runs(n, depths):
    """Tile-first runs around and above what LDS holds (8,192 pairs), the
    longer ones sorted through the workspace chunk by chunk: one tile of a
    4 x 4 grid gets n pairs, every tile gets the 500 Gaussians that cover the
    grid.  Depths random, differing only in their low byte (one pass), or
    from a few values (index order decides)."""
    rs = np.random.default_rng(n + len(depths))
    rec = blank(n + 500)
    rec["mean_x"][:n] = rec["mean_y"][:n] = 16 * 24     # centre of tile (1, 1)
    rec["radius"][:n] = 1
    rec["mean_x"][n:] = rec["mean_y"][n:] = 16 * 32
    rec["radius"][n:] = 40                               # the whole 64 x 64 frame
    if depths == "random":
        rec["depth"] = rs.uniform(0.5, 300.0, n + 500).astype(np.float32)
    elif depths == "low-byte":
        rec["depth"] = (np.uint32(0x3F800000) + rs.integers(0, 256, n + 500).astype(np.uint32)).view(np.float32)
    else:
        rec["depth"] = rs.choice(np.float32([1.0, 2.0, 4.5]), n + 500)
    assert_same(64, 64, rec, gpu_frame(64, 64, rec, stages=False, algorithm=ss.SS_ALGO_TILE_FIRST), stages=False)


def test_frame_above_2_23_gaussians():
    """A single frame of more than 2^23 Gaussians (9M, of which 2% touch the
    image): the depth sort carries the packed rectangles past the size where
    batches stop doing so."""
    W, H, n = 1920, 1080, 9_000_000
    rec = synth.make_frame(synth.FrameSpec(W, H, 180_000), 9100)
    big = np.zeros(n, dtype=synth.RECORD_DTYPE)
    idx = np.random.default_rng(9101).choice(n, 180_000, replace=False)
    big[idx] = rec
    big["depth"][big["radius"] == 0] = 1.0
    assert_same(W, H, big, gpu_frame(W, H, big, stages=False), stages=False)


def tiny_path_frames():
    """Frames the two-kernel small-frame path takes (at most 256 tiles and
    16,384 Gaussians, no per-Gaussian outputs asked for), with its edges."""
    rs = np.random.default_rng(77)
    cases = []
    for i in range(80):
        W, H, rec = pins.random_tiny_frame(rs)
        cases.append((f"tiny{i}", W, H, rec))
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    cases.append(("small-256x256", spec.width, spec.height, synth.make_frame(spec, seed)))
    cases.append(("max-n", 256, 256, synth.make_frame(synth.scaled(synth.SMALL, 16_384), 11)))
    cases.append(("one-over-max-n", 256, 256, synth.make_frame(synth.scaled(synth.SMALL, 16_385), 12)))
    cases.append(("row", 4096, 16, synth.make_frame(synth.FrameSpec(4096, 16, 5000), 13)))
    cases.append(("column", 16, 4096, synth.make_frame(synth.FrameSpec(16, 4096, 5000), 14)))
    cases.append(("one-tile", 16, 9, synth.make_frame(synth.FrameSpec(16, 9, 16_384), 15)))
    cover = synth.make_frame(synth.FrameSpec(250, 250, 3000), 16)   # 3000 pairs in every tile
    cover["radius"] = 5000
    cases.append(("cover", 250, 250, cover))
    ties = cover.copy()
    ties["depth"] = np.float32(1.5)
    cases.append(("cover-ties", 250, 250, ties))
    one = blank(16_384)                                            # 16,384 pairs in one tile
    one["mean_x"], one["mean_y"], one["radius"] = 16 * 40 + 8, 16 * 100 + 8, 1
    one["depth"] = np.random.default_rng(3).choice(np.float32([1.0, 2.0, 3.0]), 16_384)
    cases.append(("one-tile-full", 256, 256, one))
    culled = synth.make_frame(synth.scaled(synth.SMALL, 4000), 17)
    culled["radius"] = 0
    cases.append(("all-culled", 256, 256, culled))
    cases.append(("empty", 100, 70, blank(0)))
    return cases


def test_small_frame_path():
    for name, W, H, rec in tiny_path_frames():
        print(f"small-frame path: {name} {W}x{H} N={len(rec)}", flush=True)
        cap = None if len(rec) else 0
        assert_same(W, H, rec, gpu_frame(W, H, rec, capacity=cap, stages=False), stages=False)


def test_small_frame_path_errors_and_reuse():
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    o = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    g = gpu_frame(256, 256, rec, capacity=o.num_pairs - 1, stages=False)
    assert g["status"] == _abi.SS_ERR_CAPACITY and g["M"] == o.num_pairs
    g = gpu_frame(256, 256, rec, capacity=100, stages=False)
    assert g["status"] == _abi.SS_ERR_CAPACITY and g["M"] == o.num_pairs
    for bad in (np.nan, -1.0, np.inf, 0.0):
        r2 = rec.copy()
        r2["depth"][4321] = bad
        assert gpu_frame(256, 256, r2, capacity=o.num_pairs, stages=False)["status"] == _abi.SS_ERR_INVALID_INPUT
    r2 = rec.copy()
    r2["depth"][4321], r2["radius"][4321] = np.nan, 0
    assert_same(256, 256, r2, gpu_frame(256, 256, r2, capacity=o.num_pairs, stages=False), stages=False)
    # the same buffers: an error, then a good frame
    d = ss.records_to_device(rec)
    sorter = ss.FrameSorter(256, 256, len(rec), o.num_pairs)
    bad = rec.copy()
    bad["depth"][9] = np.nan
    assert sorter(ss.records_to_device(bad)).result()[0] == _abi.SS_ERR_INVALID_INPUT
    out = sorter(d)
    assert out.result() == (0, o.num_pairs)
    assert np.array_equal(u64(out.keys)[:o.num_pairs], o.keys)
    assert np.array_equal(u32(out.values)[:o.num_pairs], o.values)
    assert np.array_equal(u32(out.tile_ranges).reshape(-1, 2), o.ranges)

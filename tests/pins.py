"""Independent pins of the CPU oracle.

Each check compares the oracle with something that is not the oracle: a
brute-force tile x Gaussian enumeration written from the problem statement
(Background, "Duplication with Tiles" and "Sorting"), closed forms (a 2D
difference array for per-tile counts, numpy's cumsum for the scan), a library
order (numpy lexsort on (key, value)), special cases that reduce to a plain
stable argsort of depth, and invariants of the output.  The checks raise
AssertionError; the mutation tests run them against oracles with planted
mistakes and expect at least one to fail.
"""
from __future__ import annotations

import bisect
import math
import struct

import numpy as np

import oracle
import synth


# ----------------------------------------------------------------------------
# brute force
# ----------------------------------------------------------------------------

def f32_bits(x: float) -> int:
    return struct.unpack("<I", struct.pack("<f", x))[0]


def touches(tile: int, centre: int, radius: int) -> bool:
    """Does the open interval (centre - 16 r, centre + 16 r) (1/16 px units)
    meet the half-open pixel span [16 tile, 16 tile + 16) (= [256 t, 256 t + 256))?"""
    R = 16 * radius
    return 256 * tile < centre + R and centre - R < 256 * tile + 256


def brute_force(width: int, height: int, rec: np.ndarray):
    """All (tile, Gaussian) pairs by enumeration, ordered by (tile, depth value,
    index) with Python's tuple sort.  Returns keys, values, ranges (T,2),
    per-Gaussian tile lists."""
    tx_n = -(-width // 16)
    ty_n = -(-height // 16)
    pairs = []
    per_g = []
    for g in range(len(rec)):
        X, Y = int(rec["mean_x"][g]), int(rec["mean_y"][g])
        r = int(rec["radius"][g])
        d = float(rec["depth"][g])
        tiles = []
        if r > 0:
            for ty in range(ty_n):
                if not touches(ty, Y, r):
                    continue
                for tx in range(tx_n):
                    if touches(tx, X, r):
                        tiles.append(ty * tx_n + tx)
        per_g.append(tiles)
        for t in tiles:
            pairs.append((t, d, g))
    pairs.sort()
    keys = np.array([(t << 32) | f32_bits(d) for (t, d, g) in pairs], dtype=np.uint64)
    vals = np.array([g for (_, _, g) in pairs], dtype=np.uint32)
    tile_of = [t for (t, _, _) in pairs]
    T = tx_n * ty_n
    rng = np.zeros((T, 2), np.uint32)
    for t in range(T):
        rng[t, 0] = bisect.bisect_left(tile_of, t)
        rng[t, 1] = bisect.bisect_right(tile_of, t)
    return keys, vals, rng, per_g


def random_tiny_frame(rs: np.random.Generator):
    """A tiny frame with every awkward feature: sizes that are not multiples of
    16, radius 0, radii larger than the image, means off the image, means on
    tile boundaries, and few distinct depths (so ties are common)."""
    W = int(rs.integers(1, 101))
    H = int(rs.integers(1, 101))
    n = int(rs.integers(0, 41))
    rec = np.zeros(n, dtype=synth.RECORD_DTYPE)
    aligned = rs.random(n) < 0.3
    mx = rs.integers(-16 * 40, 16 * (W + 40), n)
    my = rs.integers(-16 * 40, 16 * (H + 40), n)
    mx = np.where(aligned, (mx // 256) * 256 + rs.choice([0, 16 * 8], n), mx)
    my = np.where(aligned, (my // 256) * 256, my)
    rad = rs.integers(0, 24, n)
    rad = np.where(rs.random(n) < 0.1, 0, rad)
    rad = np.where(rs.random(n) < 0.05, 5000, rad)
    depths = rs.choice(np.array([0.5, 1.0, 1.0000001, 3.25, 80.0], np.float32), n)
    rec["mean_x"], rec["mean_y"], rec["radius"], rec["depth"] = mx, my, rad, depths
    return W, H, rec


def check_brute_force(cases: int = 150, seed: int = 7):
    rs = np.random.default_rng(seed)
    for _ in range(cases):
        W, H, rec = random_tiny_frame(rs)
        res = oracle.sort_frame(W, H, rec)
        assert res.status == oracle.OK
        k, v, rng, per_g = brute_force(W, H, rec)
        assert res.num_pairs == len(k), (W, H, res.num_pairs, len(k))
        assert np.array_equal(res.keys, k), (W, H)
        assert np.array_equal(res.values, v), (W, H)
        assert np.array_equal(res.ranges, rng), (W, H)
        # stage outputs: per-Gaussian counts and the duplication order (row-major tiles)
        cnt = np.array([len(t) for t in per_g], np.uint32)
        assert np.array_equal(res.tiles_touched, cnt)
        for g, tiles in enumerate(per_g):
            o = int(res.offsets[g])
            seg = res.unsorted_keys[o:o + len(tiles)]
            assert [int(x) >> 32 for x in seg] == tiles
            assert all(int(x) & 0xFFFFFFFF == f32_bits(float(rec["depth"][g])) for x in seg)
            assert all(int(x) == g for x in res.unsorted_values[o:o + len(tiles)])


# ----------------------------------------------------------------------------
# closed forms and invariants at larger sizes
# ----------------------------------------------------------------------------

def tile_counts_difference_array(width: int, height: int, rects: np.ndarray, cnt: np.ndarray):
    """Per-tile pair counts in O(N + T): +1/-1 at rectangle corners, then a
    2D prefix sum."""
    tx_n = -(-width // 16)
    ty_n = -(-height // 16)
    d = np.zeros((ty_n + 1, tx_n + 1), np.int64)
    live = cnt > 0
    x0, x1, y0, y1 = (rects[live, i].astype(np.int64) for i in range(4))
    np.add.at(d, (y0, x0), 1)
    np.add.at(d, (y0, x1), -1)
    np.add.at(d, (y1, x0), -1)
    np.add.at(d, (y1, x1), 1)
    return d.cumsum(0).cumsum(1)[:ty_n, :tx_n].reshape(-1)


def check_invariants(width: int, height: int, rec: np.ndarray, res=None):
    if res is None:
        res = oracle.sort_frame(width, height, rec)
    assert res.status == oracle.OK
    T = res.num_tiles
    M = res.num_pairs
    keys, vals, rng = res.keys, res.values, res.ranges
    cnt, rects = oracle.count(width, height, rec)
    # scan: exclusive prefix sum by a different routine, and the total
    c64 = cnt.astype(np.uint64)
    if len(cnt):
        assert np.array_equal(res.offsets, np.cumsum(c64) - c64)
        assert int(res.offsets[-1]) + int(cnt[-1]) == M
    else:
        assert M == 0
    # values are the multiset {g repeated cnt[g] times}
    assert np.array_equal(np.bincount(vals, minlength=len(rec)).astype(np.uint32)[:len(rec)], cnt)
    # keys non-decreasing; (key, value) strictly increasing; library order
    if M > 1:
        kk = keys.astype(np.uint64)
        assert np.all(kk[1:] >= kk[:-1])
        same = kk[1:] == kk[:-1]
        assert np.all(vals[1:][same] > vals[:-1][same])
        order = np.lexsort((vals, keys))
        assert np.array_equal(order, np.arange(M))
    # the sorted list is a permutation of the unsorted one
    if len(res.unsorted_keys):
        o = np.lexsort((res.unsorted_values, res.unsorted_keys))
        assert np.array_equal(res.unsorted_keys[o], keys)
        assert np.array_equal(res.unsorted_values[o], vals)
    # key trimming: only the low ceil(log2 T) + 32 bits may be non-zero
    tile_bits = 0 if T <= 1 else int(math.ceil(math.log2(T)))
    if M:
        assert int(keys.max()) >> (tile_bits + 32) == 0
    # low key bits are the depth bits of the value's Gaussian
    dbits = rec["depth"].view(np.uint32)
    assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.uint32), dbits[vals])
    # ranges partition [0, M) in tile order; lengths match a difference array
    assert rng.shape == (T, 2)
    assert rng[0, 0] == 0 and rng[-1, 1] == M
    assert np.array_equal(rng[1:, 0], rng[:-1, 1])
    assert np.all(rng[:, 1] >= rng[:, 0])
    per_tile = tile_counts_difference_array(width, height, rects, cnt)
    assert np.array_equal((rng[:, 1] - rng[:, 0]).astype(np.int64), per_tile)
    # every pair sits inside its tile's range
    tile_of = (keys >> np.uint64(32)).astype(np.int64)
    idx = np.arange(M)
    assert np.all(idx >= rng[tile_of, 0]) and np.all(idx < rng[tile_of, 1])


# ----------------------------------------------------------------------------
# special cases
# ----------------------------------------------------------------------------

def check_special_cases(seed: int = 11):
    rs = np.random.default_rng(seed)

    # one tile: the values are the stable argsort of depth over non-culled Gaussians
    n = 500
    rec = np.zeros(n, dtype=synth.RECORD_DTYPE)
    rec["mean_x"] = rs.integers(0, 16 * 12, n)
    rec["mean_y"] = rs.integers(0, 16 * 9, n)
    rec["radius"] = rs.integers(0, 4, n)
    rec["depth"] = rs.choice(np.array([1.0, 2.0, 2.5, 7.0], np.float32), n)
    res = oracle.sort_frame(12, 9, rec)
    live = np.nonzero(rec["radius"] > 0)[0]
    expect = live[np.argsort(rec["depth"][live], kind="stable")]
    assert res.num_tiles == 1 and np.array_equal(res.values, expect.astype(np.uint32))
    assert np.array_equal(res.ranges, np.array([[0, len(live)]], np.uint32))

    # every Gaussian covers the whole grid: each tile's list is the global order
    W, H, n = 100, 70, 300
    rec = np.zeros(n, dtype=synth.RECORD_DTYPE)
    rec["mean_x"] = 16 * 50
    rec["mean_y"] = 16 * 35
    rec["radius"] = rs.integers(120, 4000, n)
    rec["depth"] = rs.choice(np.array([0.25, 0.5, 0.75], np.float32), n)
    res = oracle.sort_frame(W, H, rec)
    T = res.num_tiles
    assert T == 7 * 5 and res.num_pairs == n * T
    order = np.argsort(rec["depth"], kind="stable").astype(np.uint32)
    for t in range(T):
        s, e = res.ranges[t]
        assert np.array_equal(res.values[s:e], order)

    # every depth equal: each tile lists its Gaussians by increasing index
    rec["depth"] = 3.0
    res = oracle.sort_frame(W, H, rec)
    for t in range(T):
        s, e = res.ranges[t]
        assert np.array_equal(res.values[s:e], np.arange(n, dtype=np.uint32))

    # every radius 0: no pairs, all ranges empty
    rec["radius"] = 0
    res = oracle.sort_frame(W, H, rec)
    assert res.num_pairs == 0 and not res.ranges.any()

    # no Gaussians at all
    res = oracle.sort_frame(W, H, np.zeros(0, dtype=synth.RECORD_DTYPE))
    assert res.status == oracle.OK and res.num_pairs == 0 and not res.ranges.any()

    # a Gaussian entirely off the image is culled
    rec = np.zeros(2, dtype=synth.RECORD_DTYPE)
    rec["mean_x"] = [-16 * 100, 16 * 5]
    rec["mean_y"] = [16 * 5, 16 * 5]
    rec["radius"] = [50, 1]
    rec["depth"] = [1.0, 2.0]
    res = oracle.sort_frame(32, 32, rec)
    assert list(res.tiles_touched) == [0, 1] and list(res.values) == [1]

    # radius 1 at a pixel centre inside tile (1, 0) touches that tile only;
    # on the tile boundary x = 16 px it touches the two tiles either side
    rec = np.zeros(2, dtype=synth.RECORD_DTYPE)
    rec["mean_x"] = [16 * 20 + 8, 16 * 16]
    rec["mean_y"] = [16 * 4, 16 * 4]
    rec["radius"] = [1, 1]
    rec["depth"] = [1.0, 1.0]
    res = oracle.sort_frame(48, 16, rec)
    assert list(res.tiles_touched) == [1, 2]
    assert list(res.unsorted_keys >> np.uint64(32)) == [1, 0, 1]

    # a box ending exactly on a tile edge does not touch the next tile
    # (open box): centre 8 px, radius 8 px ends at 16 px
    rec = np.zeros(1, dtype=synth.RECORD_DTYPE)
    rec["mean_x"], rec["mean_y"], rec["radius"], rec["depth"] = 16 * 8, 16 * 8, 8, 1.0
    res = oracle.sort_frame(48, 48, rec)
    assert list(res.tiles_touched) == [1]

    # capacity and invalid depth are reported
    rec = np.zeros(3, dtype=synth.RECORD_DTYPE)
    rec["mean_x"] = rec["mean_y"] = 16 * 8
    rec["radius"], rec["depth"] = 4, 1.0
    res = oracle.sort_frame(64, 64, rec, capacity=2)
    assert res.status == oracle.ERR_CAPACITY and res.num_pairs == 3
    rec["depth"][1] = np.float32(np.nan)
    assert oracle.sort_frame(64, 64, rec).status == oracle.ERR_INVALID_INPUT
    rec["depth"][1] = -1.0
    assert oracle.sort_frame(64, 64, rec).status == oracle.ERR_INVALID_INPUT
    rec["radius"][1] = 0   # a culled Gaussian's depth is never read
    assert oracle.sort_frame(64, 64, rec).status == oracle.OK


def check_depth_bits_order(seed: int = 3):
    """For positive finite floats the raw bit patterns order like the values,
    which is what lets the depth enter the integer key unchanged."""
    rs = np.random.default_rng(seed)
    d = np.exp(rs.uniform(np.log(1e-30), np.log(1e30), 20000)).astype(np.float32)
    d = np.concatenate([d, np.float32([np.finfo(np.float32).tiny, np.finfo(np.float32).max,
                                       np.float32(1e-45)])])
    by_val = np.argsort(d, kind="stable")
    by_bits = np.argsort(d.view(np.uint32), kind="stable")
    assert np.array_equal(by_val, by_bits)


def run_all_small():
    """The pin suite used against planted mistakes (fast subset)."""
    check_depth_bits_order()
    check_special_cases()
    check_brute_force(cases=80)
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    check_invariants(spec.width, spec.height, synth.make_frame(spec, seed))

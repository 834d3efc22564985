"""Independent checks of the frame order under the paper's normalised 32-bit
key (Design, "Sorting Optimizations in Context of 3DGS": 20 bits of tile
number and the depth brought below 2^10 in one float).

The reading: k = tile * 2^10 + min(depth, 1024 - 2^-14) rounded toward zero
to FP32, pairs ordered by (k, Gaussian index).  The checks compute k with
exact rational arithmetic (``fractions.Fraction``) and the largest float32 not
above it by bisection over float32 bit patterns, enumerate the pairs by brute
force, and test invariants that hold whatever the rounding details: the tile
blocks are those of the exact order, and inside a tile the order is the exact
depth order up to one unit in the last place of k.
"""
from fractions import Fraction

import numpy as np

import oracle
import pins
import synth

CAP = Fraction(1024) - Fraction(1, 1 << 14)


def f32_value(bits: int) -> Fraction:
    return Fraction(float(np.uint32(bits).view(np.float32)))


def largest_f32_at_most(x: Fraction) -> int:
    """Bits of the largest finite non-negative float32 <= x (x >= 0)."""
    lo, hi = 0, 0x7F7FFFFF
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if f32_value(mid) <= x:
            lo = mid
        else:
            hi = mid - 1
    return lo


def key32_exact(tile: int, depth: float) -> int:
    return largest_f32_at_most(Fraction(tile * 1024) + min(Fraction(depth), CAP))


def brute_force_key32(width, height, rec):
    """The exact pairs (by enumeration), reordered by (exact k, index) with
    Python's sort."""
    keys, vals, _, _ = pins.brute_force(width, height, rec)
    items = []
    for k, v in zip(keys.tolist(), vals.tolist()):
        depth = float(np.uint32(k & 0xFFFFFFFF).view(np.float32))
        items.append((f32_value(key32_exact(k >> 32, depth)), v, k))
    items.sort()
    return (np.array([k for (_, _, k) in items], np.uint64), np.array([v for (_, v, _) in items], np.uint32))


def high_tile_frame():
    """8,192 tiles (4,096 x 2): the last tile row, where one unit in the last
    place of k is 1/2.  Cases: depth 1023.99 in tile 8,190 (rounding to nearest
    would give exactly tile 8,191's first key), a depth beyond the cap (2000)
    in tile 8,189, depths 0.4, 0.2, 0.3 in tile 8,191 (one quantum: a tie), and
    depths 3.0 / 3.9 / 3.6 in tile 8,190 (3.9 and 3.6 share the quantum
    [3.5, 4) and keep index order, 3.9 first; 3.0 does not)."""
    W, H = 16 * 4096, 32
    specs = [  # (tile x in row 1, depth)
        (4095, 0.4), (4095, 0.2), (4094, 3.9), (4094, 3.6), (4094, 3.0),
        (4093, 5.0), (4094, 1023.99), (4093, 2000.0), (4095, 0.3)]
    rec = np.zeros(len(specs), dtype=synth.RECORD_DTYPE)
    for g, (tx, d) in enumerate(specs):
        rec["mean_x"][g] = 16 * (16 * tx + 8)
        rec["mean_y"][g] = 16 * 24
        rec["radius"][g] = 1
        rec["depth"][g] = d
    return W, H, rec


def check_brute_force(cases=120, seed=21):
    rs = np.random.default_rng(seed)
    frames = [pins.random_tiny_frame(rs) for _ in range(cases)] + [high_tile_frame()]
    for W, H, rec in frames:
        res = oracle.sort_frame_key32(W, H, rec)
        assert res.status == oracle.OK
        k, v = brute_force_key32(W, H, rec)
        assert np.array_equal(res.keys, k), (W, H)
        assert np.array_equal(res.values, v), (W, H)
        assert np.array_equal(res.ranges, oracle.sort_frame(W, H, rec).ranges), (W, H)


def check_high_tile_expectations():
    """The crafted frame's order written out by hand: tile 8,189 holds the
    capped depth after 5.0; tile 8,190 orders 3.0, then the tie {3.9 (g2),
    3.6 (g3)} by index, then 1023.99 last; tile 8,191 has the tie
    {0.4 (g0), 0.2 (g1), 0.3 (g8)} by index."""
    W, H, rec = high_tile_frame()
    res = oracle.sort_frame_key32(W, H, rec)
    tiles = (res.keys >> np.uint64(32)).tolist()
    assert tiles == [8189, 8189, 8190, 8190, 8190, 8190, 8191, 8191, 8191]
    assert res.values.tolist() == [5, 7, 4, 2, 3, 6, 0, 1, 8]


def quantum(tile: int) -> float:
    """Upper bound of one unit in the last place of k inside tile's range."""
    top = np.float32((tile + 1) * 1024.0)
    return float(np.spacing(top))


def check_invariants(name="fullhd-1m"):
    """On a workload: same tile blocks as the exact order, the same pairs per
    tile, and the depth order inside a tile violated by at most one quantum;
    where a tile's depths are all more than a quantum apart the order is the
    exact one."""
    spec, seed = synth.workload(name)
    rec = synth.make_frame(spec, seed)
    ex = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    lo = oracle.sort_frame_key32(spec.width, spec.height, rec)
    assert np.array_equal(lo.ranges, ex.ranges)
    tile = (lo.keys >> np.uint64(32)).astype(np.int64)
    depth = (lo.keys & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    q = np.array([quantum(t) for t in range(ex.num_tiles)])
    assert np.array_equal(tile, (ex.keys >> np.uint64(32)).astype(np.int64))
    for t in range(ex.num_tiles):
        a, b = lo.ranges[t]
        assert np.array_equal(np.sort(lo.values[a:b]), np.sort(ex.values[a:b]))
        # depth never falls by more than a quantum between two entries of a
        # tile: the running maximum minus the current depth stays <= q
        d = depth[a:b]
        assert np.all(np.maximum.accumulate(d) - d <= q[t] + 1e-12), t
    # tiles whose sorted depths are all more than a quantum apart keep the exact order
    for t in range(ex.num_tiles):
        a, b = ex.ranges[t]
        d = np.sort(depth[a:b])
        if b - a > 1 and np.all(np.diff(d) > q[t]):
            assert np.array_equal(lo.values[a:b], ex.values[a:b]), t


def check_separated_depths_equal_exact():
    """Special case: small tile ids (one unit in the last place of k at most
    2^-10) and depths on a 0.01 grid, all distinct: the lossy order is the
    exact order."""
    rs = np.random.default_rng(5)
    W, H, n = 64, 64, 300
    rec = np.zeros(n, dtype=synth.RECORD_DTYPE)
    rec["mean_x"] = rs.integers(0, 16 * W, n)
    rec["mean_y"] = rs.integers(0, 16 * H, n)
    rec["radius"] = rs.integers(1, 20, n)
    rec["depth"] = (rs.permutation(n) + 1) * 0.01
    ex = oracle.sort_frame(W, H, rec, stages=False)
    lo = oracle.sort_frame_key32(W, H, rec)
    assert np.array_equal(lo.keys, ex.keys) and np.array_equal(lo.values, ex.values)


def run_all_key32():
    check_brute_force()
    check_high_tile_expectations()
    check_separated_depths_equal_exact()
    check_invariants("small-256x256")
    check_invariants("fullhd-1m")

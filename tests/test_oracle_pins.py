"""The oracle against its independent pins (CPU only)."""
import numpy as np
import pytest

import oracle
import pins
import synth


def test_depth_bit_order_equals_value_order():
    pins.check_depth_bits_order()


def test_brute_force_tiny_frames():
    pins.check_brute_force(cases=300, seed=7)


def test_special_cases():
    pins.check_special_cases()


@pytest.mark.parametrize("name", ["small-256x256", "fullhd-1m"])
def test_invariants_workloads(name):
    spec, seed = synth.FRAME_WORKLOADS[name]
    pins.check_invariants(spec.width, spec.height, synth.make_frame(spec, seed))


def test_invariants_large_scaled_down():
    spec, seed = synth.FRAME_WORKLOADS["large-6m"]
    spec = synth.scaled(spec, 400_000)
    pins.check_invariants(spec.width, spec.height, synth.make_frame(spec, seed))


def test_stage_functions_compose():
    """Count, scan, duplicate, sort and ranges called one by one give the whole-frame result."""
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    res = oracle.sort_frame(spec.width, spec.height, rec)
    cnt, _ = oracle.count(spec.width, spec.height, rec)
    off, tot = oracle.scan(cnt)
    assert tot == res.num_pairs and np.array_equal(off, res.offsets)
    k, v = oracle.sort_pairs(res.unsorted_keys, res.unsorted_values)
    assert np.array_equal(k, res.keys) and np.array_equal(v, res.values)
    assert np.array_equal(oracle.ranges(k, res.num_tiles), res.ranges)


def test_batch_composition():
    frames = synth.make_batch(3, n_range=(2_000, 20_000))
    b = oracle.sort_batch(frames)
    for f, (w, h, rec) in enumerate(frames):
        one = oracle.sort_frame(w, h, rec, stages=False)
        s = int(b.pair_base[f])
        seg = slice(s, s + one.num_pairs)
        assert np.array_equal(b.values[seg], one.values)
        assert np.array_equal(b.keys[seg] - (np.uint64(b.tile_base[f]) << np.uint64(32)), one.keys)
        tb = int(b.tile_base[f])
        assert np.array_equal(b.ranges[tb:tb + one.num_tiles].astype(np.int64) - s,
                              one.ranges.astype(np.int64))
    assert b.ranges[0, 0] == 0 and b.ranges[-1, 1] == len(b.keys)
    assert np.array_equal(b.ranges[1:, 0], b.ranges[:-1, 1])

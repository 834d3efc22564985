"""The multi-threaded oracle variant (the CPU timing baseline beside the GPU)
gives exactly the plain oracle's result: same statuses, pairs, order and
ranges, at several thread counts."""
import numpy as np
import pytest

import oracle
import pins
import synth


def same(a, b):
    assert a.status == b.status
    assert a.num_pairs == b.num_pairs
    if a.status == oracle.OK:
        assert np.array_equal(a.keys, b.keys)
        assert np.array_equal(a.values, b.values)
        assert np.array_equal(a.ranges, b.ranges)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_tiny_frames(threads):
    rs = np.random.default_rng(31)
    for _ in range(40):
        W, H, rec = pins.random_tiny_frame(rs)
        same(oracle.sort_frame(W, H, rec, stages=False), oracle.sort_frame_mt(W, H, rec, threads))


@pytest.mark.parametrize("name", ["small-256x256", "fullhd-1m"])
def test_workloads(name):
    spec, seed = synth.workload(name)
    rec = synth.make_frame(spec, seed)
    plain = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    same(plain, oracle.sort_frame_mt(spec.width, spec.height, rec, 4))


def test_statuses():
    spec, seed = synth.workload("small-256x256")
    rec = synth.make_frame(spec, seed)
    plain = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    cap = plain.num_pairs - 1
    assert oracle.sort_frame_mt(spec.width, spec.height, rec, 2, capacity=cap).status == oracle.ERR_CAPACITY
    bad = rec.copy()
    bad["depth"][17] = -1.0
    bad["radius"][17] = 5
    assert oracle.sort_frame_mt(spec.width, spec.height, bad, 2).status == oracle.ERR_INVALID_INPUT
    empty = rec[:0]
    r = oracle.sort_frame_mt(spec.width, spec.height, empty, 2)
    assert r.status == oracle.OK and r.num_pairs == 0 and not r.ranges.any()

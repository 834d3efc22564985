"""The sharding design on the CPU oracle: a frame cut into bands of whole
tile rows, each band sorted as a frame of its own, gives the whole frame's
output once each band's tile ids are moved by its first tile row and its
ranges by the pairs of earlier bands (tile-row bands are the shards of one
frame across GPUs; the tile id is the major key)."""
import numpy as np
import pytest

import oracle
import pins
import synth


def assemble(width, height, rec, bands):
    tx = -(-width // 16)
    keys, vals, ranges, base = [], [], [], 0
    for h, r0, rb in synth.band_frames(rec, width, height, bands):
        o = oracle.sort_frame(width, h, rb, stages=False)
        assert o.status == oracle.OK
        keys.append(o.keys + (np.uint64(r0 * tx) << np.uint64(32)))
        vals.append(o.values)
        ranges.append(o.ranges.astype(np.int64) + base)
        base += o.num_pairs
    return np.concatenate(keys), np.concatenate(vals), np.concatenate(ranges)


@pytest.mark.parametrize("bands", [1, 2, 3, 8])
def test_bands_reassemble_the_frame(bands):
    spec, seed = synth.workload("small-256x256")
    rec = synth.make_frame(spec, seed)
    full = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    k, v, r = assemble(spec.width, spec.height, rec, bands)
    assert np.array_equal(k, full.keys) and np.array_equal(v, full.values)
    assert np.array_equal(r, full.ranges.astype(np.int64))


def test_bands_of_tiny_frames():
    """Heights that are not multiples of 16, more bands than tile rows,
    Gaussians spanning several bands, off-image means."""
    rs = np.random.default_rng(31)
    for _ in range(80):
        W, H, rec = pins.random_tiny_frame(rs)
        full = oracle.sort_frame(W, H, rec, stages=False)
        for bands in (2, 5, 9):
            k, v, r = assemble(W, H, rec, bands)
            assert np.array_equal(k, full.keys) and np.array_equal(v, full.values), (W, H, bands)
            assert np.array_equal(r, full.ranges.astype(np.int64)), (W, H, bands)

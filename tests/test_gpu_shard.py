"""One GPU's share of a frame sharded by tile-row bands, on the device:
every band of the heavy-tailed frame sorted alone equals the oracle's sort of
that band, and all bands sorted as one batch (global tile ids tile_base[f] + t
= the band's first tile row onwards) reproduce the whole frame's output bit
for bit."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_16298_amd as ss  # noqa: E402


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_band_shares_of_large_frame():
    spec, seed = synth.workload("large-6m")
    rec = synth.make_frame(spec, seed)
    for h, r0, rb in synth.band_frames(rec, spec.width, spec.height, 8):
        print(f"band from tile row {r0}, {spec.width}x{h}", flush=True)
        want = oracle.sort_frame(spec.width, h, rb, stages=False)
        d = ss.records_to_device(rb)
        for drop in (False, True):
            s = ss.FrameSorter(spec.width, h, len(rb), want.num_pairs, drop_culled=drop)
            s(d)
            st, m = s.out.result()
            assert st == 0 and m == want.num_pairs
            assert np.array_equal(u64(s.out.keys)[:m], want.keys)
            assert np.array_equal(u32(s.out.values)[:m], want.values)
            assert np.array_equal(u32(s.out.tile_ranges).reshape(-1, 2), want.ranges)


@pytest.mark.parametrize("drop", [False, True])
def test_bands_as_one_batch_equal_the_frame(drop):
    spec, seed = synth.workload("fullhd-1m")
    rec = synth.make_frame(spec, seed)
    full = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    bands = synth.band_frames(rec, spec.width, spec.height, 8)
    b = ss.BatchSorter([(spec.width, h, len(rb)) for (h, _, rb) in bands], full.num_pairs, drop_culled=drop)
    b([ss.records_to_device(rb) for (_, _, rb) in bands])
    st, m = b.result()
    assert st == 0 and m == full.num_pairs
    assert np.array_equal(u64(b.keys)[:m], full.keys)
    assert np.array_equal(u32(b.values)[:m], full.values)
    assert np.array_equal(u32(b.tile_ranges).reshape(-1, 2), full.ranges)

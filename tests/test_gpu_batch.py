"""Batched (segmented) sort on the GPU against the oracle's batched layout:
global tile ids tile_base[f] + t, frame-local values, frame-major segments,
global ranges.  Bit-exact."""
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


def run_batch(frames, capacity=None, **kw):
    if capacity is None:
        capacity = 0
        for (w, h, rec) in frames:
            cnt, _ = oracle.count(w, h, rec)
            capacity += int(cnt.astype(np.uint64).sum())
    b = ss.BatchSorter([(w, h, len(r)) for (w, h, r) in frames], capacity, **kw)
    recs = [ss.records_to_device(r) for (_, _, r) in frames]
    b(recs)
    st, m = b.result()
    return b, st, m


def check_against_oracle(frames, b, m):
    ref = oracle.sort_batch(frames)
    assert m == int(ref.num_pairs.sum())
    assert np.array_equal(u64(b.keys)[:m], ref.keys)
    assert np.array_equal(u32(b.values)[:m], ref.values)
    assert np.array_equal(u32(b.tile_ranges).reshape(-1, 2), ref.ranges)
    assert np.array_equal(u32(b.frame_pairs), ref.num_pairs.astype(np.uint32))
    assert np.array_equal(u32(b.frame_pair_base), ref.pair_base.astype(np.uint32))
    assert np.array_equal(b.tile_base, ref.tile_base.astype(np.int64))


@pytest.mark.parametrize("rb", [8, 4])
def test_small_batch(rb):
    frames = synth.make_batch(8, n_range=(5_000, 50_000))
    b, st, m = run_batch(frames, radix_bits=rb)
    assert st == 0
    check_against_oracle(frames, b, m)


def test_each_frame_alone_equals_its_segment():
    frames = synth.make_batch(5, seed=77, n_range=(20_000, 60_000))
    b, st, m = run_batch(frames)
    assert st == 0
    keys, vals = u64(b.keys)[:m], u32(b.values)[:m]
    base, cnt = u32(b.frame_pair_base), u32(b.frame_pairs)
    for f, (w, h, rec) in enumerate(frames):
        out = ss.sort_frame(ss.records_to_device(rec), w, h)
        st1, m1 = out.result()
        assert st1 == 0 and m1 == cnt[f]
        seg = slice(int(base[f]), int(base[f]) + m1)
        tb = np.uint64(int(b.tile_base[f])) << np.uint64(32)
        assert np.array_equal(keys[seg] - tb, u64(out.keys)[:m1])
        assert np.array_equal(vals[seg], u32(out.values)[:m1])


def test_batch_with_degenerate_frames():
    rs = np.random.default_rng(3)
    empty = np.zeros(0, dtype=synth.RECORD_DTYPE)
    culled = synth.make_frame(synth.FrameSpec(300, 200, 4000), 4)
    culled["radius"] = 0
    one_tile = synth.make_frame(synth.FrameSpec(12, 10, 3000), 5)
    normal = synth.make_frame(synth.FrameSpec(640, 360, 20000), 6)
    ties = synth.make_frame(synth.FrameSpec(100, 100, 5000), 7)
    ties["depth"] = rs.choice(np.float32([1.0, 2.0]), 5000)
    frames = [(64, 64, empty), (300, 200, culled), (12, 10, one_tile), (640, 360, normal), (100, 100, ties),
              (64, 64, empty)]
    b, st, m = run_batch(frames)
    assert st == 0
    check_against_oracle(frames, b, m)


def test_segmented_batch_frames_smaller_than_a_workgroup():
    """Many frames below 2,048 Gaussians between larger ones: one expansion
    workgroup spans several frames (the frames between its first and last
    count their tile digits straight into global memory); empty and
    one-Gaussian frames in the run."""
    rs = np.random.default_rng(11)
    frames = []
    for f in range(40):
        n = [0, 1, 7, 300, 900, 1500, 2047, 2049][f % 8] if f % 5 else int(rs.integers(3000, 12000))
        w, h = [(320, 180), (64, 48), (640, 360), (16, 16)][f % 4]
        frames.append((w, h, synth.make_frame(synth.FrameSpec(w, h, n), 500 + f)))
    for kw in ({}, {"radix_bits": 4}, {"items_per_thread": 8}):
        b, st, m = run_batch(frames, **kw)
        assert st == 0, kw
        check_against_oracle(frames, b, m)


def test_batch_of_256_frames():
    """The most frames a batch takes (256): the per-frame tables in LDS, one
    publishing workgroup and one range fix-up workgroup per frame; frames of
    0 to 3,000 Gaussians on grids of 1 to 8,160 tiles, some sharing an
    expansion workgroup with a dozen others."""
    rs = np.random.default_rng(256)
    sizes = [(16, 16), (64, 48), (320, 180), (640, 360), (1920, 1080), (1000, 16)]
    frames = []
    for f in range(256):
        w, h = sizes[int(rs.integers(len(sizes)))]
        n = int(rs.choice([0, 1, 17, 150, 600, 3000]))
        frames.append((w, h, synth.make_frame(synth.FrameSpec(w, h, n), 9000 + f)))
    for kw in ({}, {"persistent": True}):
        b, st, m = run_batch(frames, **kw)
        assert st == 0, kw
        check_against_oracle(frames, b, m)


def test_segmented_and_whole_batch_agree():
    """The same frames through the segmented tile passes (default) and the
    whole-batch ones (dropping culled Gaussians keeps the batch whole, as do
    256-thread passes): identical outputs, equal to the oracle's."""
    frames = synth.make_batch(7, seed=123, n_range=(4_000, 40_000))
    outs = []
    for kw in ({}, {"drop_culled": True}, {"workgroup_size": 256}):
        b, st, m = run_batch(frames, **kw)
        assert st == 0, kw
        check_against_oracle(frames, b, m)
        outs.append((u64(b.keys)[:m].copy(), u32(b.values)[:m].copy(), u32(b.tile_ranges).copy()))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)


def test_batch_frame_tile_limits():
    """A frame of exactly 2^16 tiles (4096 x 4096: the widest frame-local
    tile field of the segmented passes) and, in another batch, one of more
    (4200 x 4200, 69,169 tiles: the whole-batch passes)."""
    for big in (4096, 4200):
        frames = [(big, big, synth.make_frame(synth.FrameSpec(big, big, 30_000), 61)),
                  (640, 360, synth.make_frame(synth.FrameSpec(640, 360, 10_000), 62)),
                  (1280, 720, synth.make_frame(synth.FrameSpec(1280, 720, 5_000), 63))]
        b, st, m = run_batch(frames)
        assert st == 0, big
        check_against_oracle(frames, b, m)


def test_batch_wide_depth_ranges():
    """Frames whose depths span 2, 9 and 23 binades, through the segmented
    and the whole-batch tile passes."""
    frames = [(1280, 720, synth.make_frame(synth.FrameSpec(1280, 720, 40_000, depth_lo=1e-3, depth_hi=1e4), 81)),
              (640, 360, synth.make_frame(synth.FrameSpec(640, 360, 20_000, depth_lo=0.5, depth_hi=2.0), 82)),
              (1920, 1080, synth.make_frame(synth.FrameSpec(1920, 1080, 30_000), 83))]
    for kw in ({}, {"drop_culled": True}):
        b, st, m = run_batch(frames, **kw)
        assert st == 0, kw
        check_against_oracle(frames, b, m)


@pytest.mark.parametrize("drop", [False, True])
def test_persistent_passes_batch(drop):
    """Persistent tile passes (workgroups taking tiles by atomic ticket) over a
    segmented batch, and over a whole one: the same result."""
    frames = synth.make_batch(9, seed=321, n_range=(2_000, 60_000))
    b, st, m = run_batch(frames, persistent=True, drop_culled=drop)
    assert st == 0
    check_against_oracle(frames, b, m)


def test_timeout_raised_from_the_host():
    """With the digit bases withheld and a short spin limit every tile's wait
    ends in SS_ERR_TIMEOUT and every kernel still finishes; without the hook
    the same frames sort exactly."""
    frames = synth.make_batch(4, seed=322, n_range=(20_000, 60_000))
    for persistent in (False, True):
        b, st, m = run_batch(frames, persistent=persistent, spin_limit=32, fault=ss._abi.SS_FAULT_WITHHOLD_BASES)
        assert st == ss._abi.SS_ERR_TIMEOUT, persistent
        b, st, m = run_batch(frames, persistent=persistent, spin_limit=32)
        assert st == 0
        check_against_oracle(frames, b, m)


def test_batch_capacity_error():
    frames = synth.make_batch(3, n_range=(5_000, 9_000))
    total = sum(int(oracle.count(w, h, r)[0].astype(np.uint64).sum()) for (w, h, r) in frames)
    b, st, m = run_batch(frames, capacity=total - 1)
    assert st == ss._abi.SS_ERR_CAPACITY and m == total


def test_full_64_frame_batch_every_frame(batch64):
    """The 64-frame batch at full size (38.8M Gaussians, 182.9M pairs: the
    unpacked-rectangle path, since it holds more than 2^23 Gaussians): every
    frame's segment, frame-local ranges, pair count and first pair compared
    pair for pair with the oracle's result for that frame alone."""
    frames, refs = batch64
    ms = [int(r.num_pairs) for r in refs]
    b, st, m = run_batch(frames, capacity=sum(ms))
    assert st == 0 and m == sum(ms)
    keys, vals = u64(b.keys)[:m], u32(b.values)[:m]
    rng = u32(b.tile_ranges).reshape(-1, 2)
    base, cnt = u32(b.frame_pair_base).astype(np.int64), u32(b.frame_pairs).astype(np.int64)
    assert np.array_equal(cnt, np.array(ms, np.int64))
    assert np.array_equal(base, np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64))
    tile_base = 0
    for f, ref in enumerate(refs):
        assert int(b.tile_base[f]) == tile_base, f
        seg = slice(int(base[f]), int(base[f] + cnt[f]))
        tb = np.uint64(tile_base) << np.uint64(32)
        assert np.array_equal(keys[seg] - tb, ref.keys), f
        assert np.array_equal(vals[seg], ref.values), f
        t = ref.num_tiles
        assert np.array_equal(rng[tile_base:tile_base + t] - np.uint32(base[f]), ref.ranges), f
        tile_base += t
    assert tile_base == rng.shape[0]


def test_batch_with_unpacked_rectangles():
    """Frames wider or taller than 256 tiles: the depth sort carries no packed
    rectangles and expand gathers the 64-bit rectangles by index."""
    frames = [(4200, 200, synth.make_frame(synth.FrameSpec(4200, 200, 20_000), 41)),
              (640, 360, synth.make_frame(synth.FrameSpec(640, 360, 12_000), 42)),
              (300, 4500, synth.make_frame(synth.FrameSpec(300, 4500, 9_000), 43))]
    for rb in (8, 6):
        b, st, m = run_batch(frames, radix_bits=rb)
        assert st == 0
        check_against_oracle(frames, b, m)


def test_plan_graph_replays_match_eager():
    """A captured plan replayed several times, with eager work and host
    synchronisations between replays, equals the eager result every time."""
    frames = synth.make_batch(6, seed=91, n_range=(10_000, 40_000))
    capacity = sum(int(oracle.count(w, h, r)[0].astype(np.uint64).sum()) for (w, h, r) in frames)
    shapes = [(w, h, len(r)) for (w, h, r) in frames]
    recs = [ss.records_to_device(r) for (_, _, r) in frames]
    eager = ss.BatchSorter(shapes, capacity)
    eager(recs)
    st, m = eager.result()
    assert st == 0
    ref = (u64(eager.keys)[:m].copy(), u32(eager.values)[:m].copy(), u32(eager.tile_ranges).copy())
    sorter = ss.BatchSorter(shapes, capacity, plan_workspace=True)
    plan = ss.Plan(sorter, recs, autotune=True, tune_repeats=2)
    cfg = plan.config()
    assert len(cfg["candidate_ms"]) >= 5 and cfg["radix_bits"] in (4, 6, 8)
    for rep in range(4):
        sorter.keys.fill_(-1)
        sorter.values.fill_(-1)
        torch.cuda.synchronize()
        plan.launch()
        _ = (torch.arange(1000, device="cuda") * 3).sum().item()   # eager work between replays
        st, m2 = sorter.result()
        assert st == 0 and m2 == m, rep
        assert np.array_equal(u64(sorter.keys)[:m], ref[0]), rep
        assert np.array_equal(u32(sorter.values)[:m], ref[1]), rep
        assert np.array_equal(u32(sorter.tile_ranges), ref[2]), rep
    # new record contents at the same addresses are picked up by a replay
    frames2 = synth.make_batch(6, seed=91, n_range=(10_000, 40_000))
    for r in frames2:
        r[2]["depth"] = r[2]["depth"][::-1].copy()
    cap2 = sum(int(oracle.count(w, h, r)[0].astype(np.uint64).sum()) for (w, h, r) in frames2)
    assert cap2 == capacity
    for d, (_, _, r) in zip(recs, frames2):
        d.copy_(ss.records_to_device(r))
    plan.launch()
    st, m3 = sorter.result()
    assert st == 0
    ref2 = oracle.sort_batch(frames2)
    assert np.array_equal(u64(sorter.keys)[:m3], ref2.keys)
    assert np.array_equal(u32(sorter.values)[:m3], ref2.values)
    plan.close()


def test_plan_tune_cache(tmp_path):
    """The autotune cache: the first plan times the candidates and records the
    winner; a second plan of the same batch size takes it from the file
    without timing and sorts exactly; a batch of another size is timed and
    recorded beside it."""
    path = str(tmp_path / "tune.txt")

    def plan_for(frames):
        capacity = sum(int(oracle.count(w, h, r)[0].astype(np.uint64).sum()) for (w, h, r) in frames)
        shapes = [(w, h, len(r)) for (w, h, r) in frames]
        recs = [ss.records_to_device(r) for (_, _, r) in frames]
        sorter = ss.BatchSorter(shapes, capacity, plan_workspace=True)
        return sorter, ss.Plan(sorter, recs, autotune=True, tune_repeats=1, tune_cache=path)

    frames = synth.make_batch(5, seed=93, n_range=(10_000, 30_000))
    _, p1 = plan_for(frames)
    c1 = p1.config()
    assert len(c1["candidate_ms"]) >= 5
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("ss-tune 1 gfx")
    p1.close()
    sorter, p2 = plan_for(frames)
    c2 = p2.config()
    assert c2["candidate_ms"] == []
    assert {k: c2[k] for k in ("radix_bits", "items_per_thread", "workgroup_size", "persistent")} == \
        {k: c1[k] for k in ("radix_bits", "items_per_thread", "workgroup_size", "persistent")}
    p2.launch()
    st, m = sorter.result()
    assert st == 0
    check_against_oracle(frames, sorter, m)
    p2.close()
    _, p3 = plan_for(synth.make_batch(9, seed=94, n_range=(10_000, 30_000)))
    assert len(p3.config()["candidate_ms"]) >= 5
    assert len(open(path).read().splitlines()) == 2
    p3.close()

"""The serving loop on the GPU: every request's result, sorted in a round
with others, equals the frame sorted alone (tolerance 0); admission by HBM
budget waits for space and rejects what can never fit; a bad frame fails
only its own request."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_16298_amd as ss  # noqa: E402
from paper_2511_16298_amd import _abi  # noqa: E402


def frames_pool(k, seed, n_range=(3_000, 30_000)):
    return synth.make_batch(k, seed=seed, n_range=n_range)


def alone(w, h, rec):
    return oracle.sort_frame(w, h, rec, stages=False)


def test_results_in_the_mix_equal_alone():
    pool = frames_pool(12, 501)
    dev = [ss.records_to_device(r) for (_, _, r) in pool]
    srv = ss.Server(1 << 30, max_batch_frames=16, n_streams=2)
    rs = np.random.default_rng(1)
    order = rs.integers(0, len(pool), 60)
    tickets = [(srv.submit(dev[i], pool[i][0], pool[i][1]), i) for i in order]
    mixed = 0
    for t, i in tickets:
        r = srv.wait(t)
        assert r.status == 0, _abi.status_string(r.status)
        w, h, rec = pool[i]
        ref = alone(w, h, rec)
        assert r.num_pairs == ref.num_pairs
        k, v, rg = srv.result_arrays(r, ref.num_tiles)
        assert np.array_equal(k, ref.keys) and np.array_equal(v, ref.values) and np.array_equal(rg, ref.ranges)
        mixed += r.round_frames > 1
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 60 and st["pending"] == 0 and st["arena_used"] == 0
    assert mixed > 0, "no request was batched with another"
    srv.close()


def test_batch_sized_requests_in_the_mix_equal_alone(batch64):
    """Requests drawn from the batch distribution at full size (50k-2M
    Gaussians per frame, the served workload's frames), several rounds in
    flight (two) with up to 16 frames per round: every result equals
    the oracle's result for that frame alone, pair for pair."""
    frames, refs = batch64
    sizes = np.array([len(r) for (_, _, r) in frames])
    big = [int(i) for i in np.argsort(sizes)[::-1][:3]]      # the three largest frames (>= 1M Gaussians)
    assert sizes[big].min() >= 1_000_000
    rs = np.random.default_rng(11)
    order = big + [int(i) for i in rs.integers(0, len(frames), 33)] + big
    dev = {i: ss.records_to_device(frames[i][2]) for i in set(order)}
    srv = ss.Server(24 << 30, max_batch_frames=16, n_streams=2)
    tickets = [(srv.submit(dev[i], frames[i][0], frames[i][1]), i) for i in order]
    mixed = 0
    for t, i in tickets:
        r = srv.wait(t)
        assert r.status == 0, _abi.status_string(r.status)
        ref = refs[i]
        assert r.num_pairs == ref.num_pairs, i
        k, v, rg = srv.result_arrays(r, ref.num_tiles)
        assert np.array_equal(k, ref.keys), i
        assert np.array_equal(v, ref.values), i
        assert np.array_equal(rg, ref.ranges), i
        mixed += r.round_frames > 1
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(order) and st["pending"] == 0 and st["arena_used"] == 0
    assert mixed > 0, "no request was batched with another"
    srv.close()


def test_closed_loop_with_rounds_in_flight_drains_ok(batch64):
    """A closed loop of batch-sized requests (the served workload's frames,
    50k-2M Gaussians) with 48 outstanding and two rounds in flight, then the
    drain once submissions stop: every request ends OK (the drain's last
    rounds once ended in SS_ERR_TIMEOUT while rounds ran side by side on two
    streams), and every eighth result equals the oracle's for that frame."""
    frames, refs = batch64
    dev = [ss.records_to_device(r) for (_, _, r) in frames]
    srv = ss.Server(24 << 30, max_batch_frames=64, n_streams=2)
    order = [int(i) for i in np.random.default_rng(12).integers(0, len(frames), 240)]
    q = [(srv.submit(dev[i], frames[i][0], frames[i][1]), i) for i in order[:48]]
    nxt, done, big_rounds = 48, 0, 0
    while q:
        t, i = q.pop(0)
        r = srv.wait(t)
        assert r.status == 0, (done, _abi.status_string(r.status))
        big_rounds += r.round_frames >= 8
        if done % 8 == 0:
            ref = refs[i]
            assert r.num_pairs == ref.num_pairs, i
            k, v, rg = srv.result_arrays(r, ref.num_tiles)
            assert np.array_equal(k, ref.keys) and np.array_equal(v, ref.values) and np.array_equal(rg, ref.ranges), i
        srv.release(t)
        done += 1
        if nxt < len(order):
            j = order[nxt]
            q.append((srv.submit(dev[j], frames[j][0], frames[j][1]), j))
            nxt += 1
    st = srv.stats()
    assert done == len(order) and st["completed"] == len(order) and st["pending"] == 0 and st["arena_used"] == 0
    assert big_rounds > 0, "no round of eight frames or more"
    srv.close()


def test_budget_rejects_what_can_never_fit_and_waits_otherwise():
    big = synth.make_frame(synth.scaled(synth.FULL_HD, 200_000), 3)
    small = frames_pool(6, 502, n_range=(2_000, 4_000))
    d_big = ss.records_to_device(big)
    d_small = [ss.records_to_device(r) for (_, _, r) in small]
    srv = ss.Server(8 << 20, max_batch_frames=4, n_streams=1)   # 8 MiB: too small for the big frame
    t_big = srv.submit(d_big, 1920, 1080)
    ts = [(srv.submit(d, w, h), i) for d, (i, (w, h, _)) in zip(d_small, enumerate(small))]
    r = srv.wait(t_big)
    assert r.status == _abi.SS_ERR_BUDGET
    srv.release(t_big)
    # small ones complete; hold their results to force later rounds to wait for space
    results = []
    for t, i in ts:
        r = srv.wait(t)
        assert r.status == 0
        w, h, rec = small[i]
        ref = alone(w, h, rec)
        k, v, rg = srv.result_arrays(r, ref.num_tiles)
        assert np.array_equal(k, ref.keys) and np.array_equal(v, ref.values)
        results.append(t)
    for t in results:
        srv.release(t)
    assert srv.stats()["rejected"] == 1 and srv.stats()["arena_used"] == 0
    srv.close()


def test_bad_frame_fails_alone():
    pool = frames_pool(5, 503)
    bad = pool[2][2].copy()
    bad["depth"][17] = np.nan
    bad["radius"][17] = 5
    recs = [r for (_, _, r) in pool]
    recs[2] = bad
    dev = [ss.records_to_device(r) for r in recs]
    srv = ss.Server(1 << 28, max_batch_frames=8, n_streams=1)
    ts = [srv.submit(d, w, h) for d, (w, h, _) in zip(dev, pool)]
    for i, t in enumerate(ts):
        r = srv.wait(t)
        if i == 2:
            assert r.status == _abi.SS_ERR_INVALID_INPUT
        else:
            assert r.status == 0
            w, h, _ = pool[i]
            ref = alone(w, h, recs[i])
            k, v, _ = srv.result_arrays(r, ref.num_tiles)
            assert np.array_equal(k, ref.keys) and np.array_equal(v, ref.values)
        srv.release(t)
    srv.close()


def test_one_at_a_time_mode_and_drain_on_close():
    pool = frames_pool(4, 504)
    dev = [ss.records_to_device(r) for (_, _, r) in pool]
    srv = ss.Server(1 << 28, max_batch_frames=1, n_streams=1)
    ts = [srv.submit(d, w, h) for d, (w, h, _) in zip(dev, pool)]
    r = srv.wait(ts[-1])
    assert r.status == 0 and r.round_frames == 1
    srv.close()   # drains the rest without waiting on them from Python

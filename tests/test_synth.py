"""The seeded generator: determinism, stream independence, distributions."""
import math

import numpy as np

import synth


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    # (state += 0x9E3779B97F4A7C15; output = mix(state)).
    got = [int(x) for x in synth.raw_u64(0, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_same_seed_same_bytes_and_random_access():
    spec = synth.scaled(synth.FULL_HD, 5000)
    a = synth.make_frame(spec, 42)
    b = synth.make_frame(spec, 42)
    assert a.tobytes() == b.tobytes()
    assert synth.make_frame(spec, 43).tobytes() != a.tobytes()
    # element i of a stream does not depend on how many are drawn
    k = synth.stream_key(5, 1, 2)
    assert np.array_equal(synth.raw_u64(k, 10)[4:], synth.raw_u64(k, 6, start=4))


def test_distributions():
    spec, seed = synth.FRAME_WORKLOADS["fullhd-1m"]
    rec = synth.make_frame(synth.scaled(spec, 200_000), seed)
    r = rec["radius"].astype(np.float64)
    assert r.min() >= 1 and r.max() <= 64
    # median of 3 sigma with sigma lognormal(ln 2, 0.8) is 6
    assert abs(np.median(r) - 6.0) <= 1.0
    d = rec["depth"]
    assert d.min() >= np.float32(0.2) and d.max() <= np.float32(100.0)
    # log-uniform: median at sqrt(0.2 * 100)
    assert abs(np.median(d) - math.sqrt(20.0)) < 0.3
    # about 20 % of means sit in blobs; some of those fall off the image
    off = (rec["mean_x"] < 0) | (rec["mean_x"] >= 16 * 1920) | (rec["mean_y"] < 0) | (rec["mean_y"] >= 16 * 1080)
    assert 0.002 < off.mean() < 0.05
    # heavy tail of the large scene: Pareto(1.8) sigma, P(3 sigma >= 30) = 10^-1.8
    spec2, seed2 = synth.FRAME_WORKLOADS["large-6m"]
    r2 = synth.make_frame(synth.scaled(spec2, 200_000), seed2)["radius"]
    frac = (r2 >= 31).mean()   # lround(3 sigma) >= 31  <=>  3 sigma >= 30.5
    assert abs(frac - (3.0 / 30.5) ** 1.8) < 0.003
    assert r2.max() == 256


def test_batch_and_arrivals():
    specs = [synth.batch_frame_spec(synth.SEED_BASE + 3, f) for f in range(64)]
    sizes = {(s.width, s.height) for s in specs}
    assert sizes <= set(synth.BATCH_RESOLUTIONS) and len(sizes) == 3
    ns = np.array([s.n for s in specs])
    assert ns.min() >= 50_000 and ns.max() < 2_000_000
    frames = synth.make_batch(2, n_range=(1000, 2000))
    assert all(len(r) == s.n for (_, _, r), s in
               zip(frames, [synth.batch_frame_spec(synth.SEED_BASE + 3, f, (1000, 2000)) for f in range(2)]))
    t = synth.poisson_arrivals(1000.0, 5.0, 9)
    assert abs(len(t) - 5000) < 5 * math.sqrt(5000)
    assert np.all(np.diff(t) > 0) and t[-1] < 5.0

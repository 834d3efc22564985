"""GPU rendering against the render oracle (NEXT step after the sort).

The GPU sorts and renders in FP32; the oracle sorts and renders in FP64.
Tolerance per pixel and channel: 2e-6 + 2.4e-7 k, k = Gaussians composited
(threshold mode) or the tile list length (exact mode): the sample offsets are
exact in FP32 for these image sizes, alpha carries about 1e-6 relative error
(the quadratic form's roundings and exp's), and every compositing step adds
about one FP32 rounding (2^-23 relative) to T and to the colour, so the error
grows with the number of steps.  In threshold mode a pixel whose oracle
evaluation comes within 1e-4 (relative) of the 1/255 or 1e-4 threshold may
take the other branch in FP32; those pixels are left out, and every other
pixel must also composite exactly as many Gaussians as the oracle.
"""
import numpy as np
import pytest

import oracle
import pins
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_16298_amd as ss  # noqa: E402
from paper_2511_16298_amd import _abi  # noqa: E402

AMBIGUOUS = 1e-4


def gpu_render(W, H, rec, co, cl, bg, exact=False, tile_evals=False):
    d = ss.records_to_device(rec)
    out = ss.sort_frame(d, W, H) if len(rec) else None
    if out is not None:
        st, m = out.result()
        assert st == 0
        values, ranges, status = out.values, out.tile_ranges, out.status
    else:
        tx, ty, _ = ss.geometry(W, H)
        values = torch.zeros(1, dtype=torch.int32, device="cuda")
        ranges = torch.zeros((tx * ty, 2), dtype=torch.int32, device="cuda")
        status = None
    cod, cld = ss.render_attrs_to_device(co, cl)
    r = ss.Renderer(W, H, want_T=True, want_contrib=True, want_tile_evals=tile_evals)
    o = r(d, cod, cld, values, ranges, status, bg, exact)
    torch.cuda.synchronize()
    return (o.color.cpu().numpy().astype(np.float64), o.T.cpu().numpy().astype(np.float64),
            o.contrib.cpu().numpy().view(np.uint32), o.tile_evals.cpu().numpy().view(np.uint32) if tile_evals else None,
            ranges.cpu().numpy().view(np.uint32))


def compare(W, H, rec, co, cl, bg=(0.1, 0.2, 0.3), exact=False, min_ok=0.99):
    s = oracle.sort_frame(W, H, rec, stages=False)
    assert s.status == 0
    ref = oracle.render(W, H, rec, co, cl, s.values, s.ranges, bg, exact)
    assert ref.status == 0
    color, T, contrib, _, _ = gpu_render(W, H, rec, co, cl, bg, exact)
    ok = np.ones((H, W), bool) if exact else ref.margin >= AMBIGUOUS
    assert ok.mean() >= min_ok, ok.mean()
    k = ref.n_contrib.astype(np.float64)
    tol = 2e-6 + 2.4e-7 * k
    err = np.abs(color - ref.color).max(axis=0)
    bad = ok & (err > tol)
    assert not bad.any(), (int(bad.sum()), float(err[bad].max()), np.argwhere(bad)[:5])
    assert np.all(np.abs(T - ref.T)[ok] <= tol[ok])
    assert np.array_equal(contrib[ok], ref.n_contrib[ok])
    return ok


@pytest.mark.parametrize("exact", [False, True])
def test_small_workload(exact):
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    co, cl = synth.make_render_attrs(rec, seed)
    compare(spec.width, spec.height, rec, co, cl, exact=exact)


def test_fullhd_workload():
    spec, seed = synth.FRAME_WORKLOADS["fullhd-1m"]
    rec = synth.make_frame(spec, seed)
    co, cl = synth.make_render_attrs(rec, seed)
    ok = compare(spec.width, spec.height, rec, co, cl, bg=(0.0, 0.0, 0.0))
    print(f"fullhd render: {ok.mean():.5f} of pixels unambiguous", flush=True)


def test_tiny_frames_and_edges():
    rs = np.random.default_rng(77)
    for case in range(12):
        W, H, rec = pins.random_tiny_frame(rs)
        co, cl = synth.make_render_attrs(rec, 900 + case)
        print(f"tiny render {case}: {W}x{H} n={len(rec)}", flush=True)
        compare(W, H, rec, co, cl, exact=bool(case % 2), min_ok=0.0)


def test_empty_frame_is_background():
    rec = np.zeros(0, dtype=synth.RECORD_DTYPE)
    co = np.zeros((0, 4), np.float32)
    color, T, contrib, _, _ = gpu_render(40, 20, rec, co, co, (0.25, 0.5, 0.75))
    assert np.all(color[0] == 0.25) and np.all(color[1] == 0.5) and np.all(color[2] == 0.75)
    assert np.all(T == 1.0) and not contrib.any()


def test_exact_mode_evaluates_every_pixel_of_every_list():
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    co, cl = synth.make_render_attrs(rec, seed)
    _, _, _, evals, ranges = gpu_render(spec.width, spec.height, rec, co, cl, (0, 0, 0), exact=True,
                                        tile_evals=True)
    assert np.array_equal(evals.astype(np.int64), 256 * (ranges[:, 1].astype(np.int64) - ranges[:, 0]))


def test_failed_sort_writes_nothing():
    spec, seed = synth.FRAME_WORKLOADS["small-256x256"]
    rec = synth.make_frame(spec, seed)
    co, cl = synth.make_render_attrs(rec, seed)
    d = ss.records_to_device(rec)
    out = ss.sort_frame(d, spec.width, spec.height)
    out.result()
    bad = torch.full((1,), _abi.SS_ERR_CAPACITY, dtype=torch.int32, device="cuda")
    cod, cld = ss.render_attrs_to_device(co, cl)
    r = ss.Renderer(spec.width, spec.height)
    r.out.color.fill_(-7.0)
    r(d, cod, cld, out.values, out.tile_ranges, bad)
    torch.cuda.synchronize()
    assert bool(torch.all(r.out.color == -7.0))


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("name", ["small-256x256", "fullhd-1m"])
def test_plain_variant_matches_counting_variant(name, exact):
    """The kernel without the per-pixel and per-tile counters (the one a
    caller gets when it asks for neither) does the same arithmetic in the same
    order as the counting kernel, which the tests above compare with the
    oracle: colour and T must agree bit for bit.  The threshold-mode
    evaluation counts are bounded by the composited counts below and by 256
    evaluations per list entry above."""
    spec, seed = synth.FRAME_WORKLOADS[name]
    rec = synth.make_frame(spec, seed)
    co, cl = synth.make_render_attrs(rec, seed)
    d = ss.records_to_device(rec)
    out = ss.sort_frame(d, spec.width, spec.height)
    st, _ = out.result()
    assert st == 0
    cod, cld = ss.render_attrs_to_device(co, cl)
    bg = (0.1, 0.2, 0.3)
    plain = ss.Renderer(spec.width, spec.height, want_T=True)
    counting = ss.Renderer(spec.width, spec.height, want_T=True, want_contrib=True, want_tile_evals=True)
    a = plain(d, cod, cld, out.values, out.tile_ranges, out.status, bg, exact)
    b = counting(d, cod, cld, out.values, out.tile_ranges, out.status, bg, exact)
    torch.cuda.synchronize()
    assert torch.equal(a.color.view(torch.int32), b.color.view(torch.int32))
    assert torch.equal(a.T.view(torch.int32), b.T.view(torch.int32))
    if not exact:
        tx, ty, _ = ss.geometry(spec.width, spec.height)
        contrib = b.contrib.cpu().numpy().view(np.uint32).astype(np.int64)
        pad = np.zeros((ty * 16, tx * 16), np.int64)
        pad[:spec.height, :spec.width] = contrib
        per_tile = pad.reshape(ty, 16, tx, 16).sum(axis=(1, 3)).reshape(-1)
        evals = b.tile_evals.cpu().numpy().view(np.uint32).astype(np.int64)
        rng = out.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
        assert np.all(evals >= per_tile)
        assert np.all(evals <= 256 * (rng[:, 1] - rng[:, 0]))

"""Independent checks of the render oracle (NEXT step after the sort).

Each check states what the compositing rule fixes (paper: Background,
"Rendering"; the alpha-blending rule of 3D Gaussian Splatting it builds on)
and computes the expected pixel values its own way: closed forms for one,
two or a few Gaussians, the Gaussian density from the covariance matrix
(numpy matrix products and scipy's multivariate normal), and invariants of
the blending weights on a workload frame.  None re-types the oracle's loop.
"""
import numpy as np
from scipy.stats import multivariate_normal

import oracle
import synth

FIX = 16  # 1/16-pixel fixed point of the means


def frame_of(points, depths=None, radius=8):
    """Records for Gaussians at pixel positions ``points`` (floats, multiples
    of 1/16)."""
    n = len(points)
    rec = np.zeros(n, dtype=synth.RECORD_DTYPE)
    for i, (x, y) in enumerate(points):
        rec["mean_x"][i] = int(round(x * FIX))
        rec["mean_y"][i] = int(round(y * FIX))
    rec["depth"] = np.arange(1, n + 1, dtype=np.float32) if depths is None else np.asarray(depths, np.float32)
    rec["radius"] = radius
    return rec


def attrs(n, conic=(0.1, 0.0, 0.1), opacity=0.5, rgb=(0.2, 0.4, 0.6)):
    co = np.zeros((n, 4), np.float32)
    co[:, :3] = conic
    co[:, 3] = opacity
    cl = np.zeros((n, 4), np.float32)
    cl[:, :3] = rgb
    return co, cl


def render(W, H, rec, co, cl, bg=(0.0, 0.0, 0.0), exact=False):
    s = oracle.sort_frame(W, H, rec, stages=False)
    assert s.status == 0
    r = oracle.render(W, H, rec, co, cl, s.values, s.ranges, bg, exact)
    assert r.status == 0
    return r


def check_center_pixel():
    """A Gaussian centred on a pixel's sample point: q = 0, alpha = opacity,
    colour = alpha rgb + (1 - alpha) background, T = 1 - alpha."""
    rec = frame_of([(5.5, 7.5)])
    co, cl = attrs(1, opacity=0.5)
    bg = (0.1, 0.3, 0.9)
    r = render(32, 32, rec, co, cl, bg)
    want = 0.5 * np.array([0.2, 0.4, 0.6], np.float32).astype(np.float64) + 0.5 * np.array(bg)
    assert np.allclose(r.color[:, 7, 5], want, rtol=0, atol=1e-15), r.color[:, 7, 5]
    assert abs(r.T[7, 5] - 0.5) < 1e-15 and r.n_contrib[7, 5] == 1


def check_density_matches_covariance(seed=11):
    """Exact mode, one Gaussian: at every pixel of its tiles alpha equals
    opacity times the normal density ratio pdf(d) / pdf(0) for the covariance
    whose inverse is the conic (matrix form d^T K d; scipy for the density)."""
    rs = np.random.default_rng(seed)
    for _ in range(5):
        A = rs.normal(size=(2, 2))
        S = A @ A.T + 2.0 * np.eye(2)
        K = np.linalg.inv(S).astype(np.float32).astype(np.float64)   # the conic as stored
        cx, cy = 20 + rs.integers(0, 16 * 8) / 16.0, 18 + rs.integers(0, 16 * 8) / 16.0
        rec = frame_of([(cx, cy)], radius=12)
        co, cl = attrs(1, conic=(K[0, 0], K[0, 1], K[1, 1]), opacity=0.7, rgb=(1.0, 0.5, 0.25))
        r = render(48, 48, rec, co, cl, exact=True)
        mvn = multivariate_normal(mean=[0.0, 0.0], cov=np.linalg.inv(K))
        o = float(np.float32(0.7))
        covered = r.n_contrib > 0
        assert covered.sum() > 100
        for y, x in zip(*np.nonzero(covered)):
            d = np.array([cx - (x + 0.5), cy - (y + 0.5)])
            a_mat = o * np.exp(-0.5 * d @ K @ d)
            a_pdf = o * mvn.pdf(d) / mvn.pdf([0.0, 0.0])
            assert abs(a_mat - a_pdf) < 1e-12 * max(1.0, a_pdf)
            assert abs(r.color[0, y, x] - a_mat) < 1e-12, (x, y)
            assert abs(r.T[y, x] - (1.0 - a_mat)) < 1e-12


def check_front_to_back():
    """Two Gaussians on one sample point: the nearer one composites first,
    C = c1 a1 + c2 a2 (1 - a1) + (1 - a1)(1 - a2) bg, whatever their index."""
    c1, c2, bg = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0]), np.array([0.0, 1.0, 0.0])
    for depths, first in (([1.0, 2.0], 0), ([2.0, 1.0], 1)):
        rec = frame_of([(8.5, 8.5), (8.5, 8.5)], depths=depths)
        co, cl = attrs(2, opacity=0.5)
        co[1, 3] = 0.25
        cl[0, :3], cl[1, :3] = c1, c2
        r = render(16, 16, rec, co, cl, tuple(bg))
        a = [0.5, 0.25]
        f, s = first, 1 - first
        col = [c1, c2]
        want = col[f] * a[f] + col[s] * a[s] * (1 - a[f]) + (1 - a[f]) * (1 - a[s]) * bg
        assert np.allclose(r.color[:, 8, 8], want, rtol=0, atol=1e-15), (depths, r.color[:, 8, 8], want)


def check_thresholds():
    """The rasteriser's thresholds: alpha below 1/255 is skipped, alpha is
    capped at 0.99, q < 0 is skipped, and a pixel stops before the Gaussian
    that would take T below 1e-4."""
    bg = (0.5, 0.5, 0.5)
    # faint: skipped unless exact
    rec = frame_of([(4.5, 4.5)])
    co, cl = attrs(1, opacity=0.003, rgb=(1.0, 1.0, 1.0))
    r = render(16, 16, rec, co, cl, bg)
    assert r.n_contrib[4, 4] == 0 and r.T[4, 4] == 1.0 and np.all(r.color[:, 4, 4] == 0.5)
    r = render(16, 16, rec, co, cl, bg, exact=True)
    o = float(np.float32(0.003))
    assert abs(r.color[0, 4, 4] - (o + (1 - o) * 0.5)) < 1e-15
    # cap
    co, cl = attrs(1, opacity=1.0, rgb=(1.0, 1.0, 1.0))
    r = render(16, 16, rec, co, cl, (0.0, 0.0, 0.0))
    assert abs(r.color[0, 4, 4] - 0.99) < 1e-15 and abs(r.T[4, 4] - 0.01) < 1e-15
    # q < 0 (not positive definite)
    co, cl = attrs(1, conic=(-1.0, 0.0, -1.0), opacity=0.5)
    r = render(16, 16, frame_of([(4.0, 4.0)]), co, cl, bg)
    assert r.n_contrib.sum() == 0 and np.all(r.color == 0.5)
    # early stop: alpha 0.95 four times -> three composited, T = 0.05^3
    rec = frame_of([(4.5, 4.5)] * 4)
    co, cl = attrs(4, opacity=0.95, rgb=(1.0, 0.0, 0.0))
    r = render(16, 16, rec, co, cl, bg)
    a = float(np.float32(0.95))
    t3 = (1 - a) ** 3
    assert r.n_contrib[4, 4] == 3 and abs(r.T[4, 4] - t3) < 1e-15
    want = sum(a * (1 - a) ** i for i in range(3)) + t3 * 0.5
    assert abs(r.color[0, 4, 4] - want) < 1e-15


def check_tile_lists_bound_the_support():
    """Only a tile's list is composited: a Gaussian whose box stays inside
    tile (0, 0) leaves tile (1, 0) at the background even where its density
    would be high."""
    rec = frame_of([(8.0, 8.0)], radius=2)
    co, cl = attrs(1, conic=(1e-4, 0.0, 1e-4), opacity=0.9)
    r = render(32, 16, rec, co, cl, (0.25, 0.25, 0.25))
    assert r.n_contrib[:, :16].min() == 1 and r.n_contrib[:, 16:].max() == 0
    assert np.all(r.color[:, :, 16:] == 0.25)


def check_weight_invariants(name="small-256x256", samples=200, seed=5):
    """On a workload frame: in exact mode the weights alpha_i T_i and the
    final T sum to 1 (white Gaussians on a white background give exactly
    white), and T is the product of (1 - alpha_i) over the tile's list,
    recomputed here as exp(sum log1p(-alpha_i)) from the oracle's own sorted
    list; with thresholds T stays in [1e-4, 1]."""
    spec, fseed = synth.FRAME_WORKLOADS[name]
    rec = synth.make_frame(spec, fseed)
    co, cl = synth.make_render_attrs(rec, fseed)
    s = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
    white = np.zeros_like(cl)
    white[:, :3] = 1.0
    r = oracle.render(spec.width, spec.height, rec, co, white, s.values, s.ranges, (1.0, 1.0, 1.0), True)
    assert np.abs(r.color - 1.0).max() < 1e-12
    rs = np.random.default_rng(seed)
    tx = s.tiles_x
    for _ in range(samples):
        x, y = int(rs.integers(0, spec.width)), int(rs.integers(0, spec.height))
        t = (y // 16) * tx + x // 16
        g = s.values[s.ranges[t, 0]:s.ranges[t, 1]]
        dx = rec["mean_x"][g] / 16.0 - (x + 0.5)
        dy = rec["mean_y"][g] / 16.0 - (y + 0.5)
        K = co[g, :3].astype(np.float64)
        q = K[:, 0] * dx * dx + 2 * K[:, 1] * dx * dy + K[:, 2] * dy * dy
        alpha = co[g, 3].astype(np.float64) * np.exp(-0.5 * q)
        assert abs(r.T[y, x] - np.exp(np.sum(np.log1p(-alpha)))) < 1e-12
    rt = oracle.render(spec.width, spec.height, rec, co, cl, s.values, s.ranges)
    assert rt.T.min() >= 1e-4 and rt.T.max() <= 1.0


def run_all_render():
    check_center_pixel()
    check_density_matches_covariance()
    check_front_to_back()
    check_thresholds()
    check_tile_lists_bound_the_support()
    check_weight_invariants()

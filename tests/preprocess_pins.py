"""Independent checks of the preprocess oracle (the step before the sort).

Each check computes what the projection rule fixes its own way: the
spherical harmonics against scipy's complex harmonics and against sphere
quadrature, pixel positions by hand, the 2D covariance from a numerical
(finite-difference) Jacobian of the projection, radii from numpy's
eigenvalues or closed forms, the half-to-even rounding of the fixed-point
mean, culling, and invariants on a workload scene.
"""
import numpy as np
from scipy import special

import oracle
import synth


def cam_of(fx=1000.0, fy=900.0, cx=320.0, cy=240.0, tanx=0.4, tany=0.3, near=0.2, deg=3):
    v = np.zeros((3, 4))
    v[:3, :3] = np.eye(3)
    return oracle.camera(v, fx, fy, cx, cy, tanx, tany, (0.0, 0.0, 0.0), near, deg)


def one(p, cov, opacity=0.5, sh=None, cam=None):
    m3 = np.array([[p[0], p[1], p[2], opacity]], np.float32)
    cv = np.zeros((1, 8), np.float32)
    S = np.asarray(cov, np.float64)
    cv[0, :6] = S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]
    shc = np.zeros((1, 48), np.float32) if sh is None else np.asarray(sh, np.float32).reshape(1, 48)
    r = oracle.preprocess(cam or cam_of(), m3, cv, shc)
    assert r.status == 0
    return r, m3, cv


def check_sh_against_scipy(samples=50, seed=3):
    """Real harmonics = sqrt(2) Re / Im of scipy's complex ones (which carry
    the Condon-Shortley phase), Y_l0 = Y_l^0."""
    rs = np.random.default_rng(seed)
    for _ in range(samples):
        d = rs.normal(size=3)
        d /= np.linalg.norm(d)
        theta = np.arccos(d[2])             # polar
        phi = np.arctan2(d[1], d[0])        # azimuth
        got = oracle.sh_basis(d)
        want = []
        for l in range(4):
            for m in range(-l, l + 1):
                if hasattr(special, "sph_harm_y"):
                    y = special.sph_harm_y(l, abs(m), theta, phi)
                else:
                    y = special.sph_harm(abs(m), l, phi, theta)
                if m == 0:
                    want.append(y.real)
                elif m > 0:
                    want.append(np.sqrt(2.0) * y.real)
                else:
                    want.append(np.sqrt(2.0) * y.imag)
        assert np.allclose(got, want, rtol=0, atol=1e-12), (got, want)
    # degree 1 in closed form: sqrt(3 / 4 pi) (-y, z, -x)
    d = np.array([0.36, -0.48, 0.8])
    c1 = np.sqrt(3.0 / (4.0 * np.pi))
    assert np.allclose(oracle.sh_basis(d)[1:4], c1 * np.array([-d[1], d[2], -d[0]]), rtol=0, atol=1e-14)


def check_sh_orthonormal():
    """Gauss-Legendre x uniform-azimuth quadrature of Y_i Y_j over the sphere
    (exact for these degrees) gives the identity."""
    xs, ws = np.polynomial.legendre.leggauss(12)
    phis = np.arange(16) * (2 * np.pi / 16)
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        s = np.sqrt(1 - x * x)
        for ph in phis:
            y = oracle.sh_basis(np.array([s * np.cos(ph), s * np.sin(ph), x]))
            G += w * (2 * np.pi / 16) * np.outer(y, y)
    assert np.allclose(G, np.eye(16), atol=1e-12)


def check_projection_and_rounding():
    """Pixel = (fx x / z + cx, fy y / z + cy); the fixed-point mean rounds
    16 pixel half to even; the depth is z."""
    r, _, _ = one((0.0, 0.0, 5.0), np.eye(3) * 1e-4)
    assert r.records["mean_x"][0] == 16 * 320 and r.records["mean_y"][0] == 16 * 240
    assert r.records["depth"][0] == np.float32(5.0)
    r, _, _ = one((0.3, -0.2, 2.0), np.eye(3) * 1e-4)
    assert r.records["mean_x"][0] == round(16 * (1000 * 0.3 / 2 + 320))
    assert r.records["mean_y"][0] == round(16 * (900 * -0.2 / 2 + 240))
    # ties: 16 x = 0.5 -> 0 and 16 x = 1.5 -> 2 (fx = 1, cx = 0, z = 1)
    for xpix, want in ((0.5 / 16, 0), (1.5 / 16, 2), (2.5 / 16, 2)):
        r, _, _ = one((xpix, 0.0, 1.0), np.eye(3) * 1e-4, cam=cam_of(fx=1.0, cx=0.0, tanx=10.0))
        assert r.records["mean_x"][0] == want, (xpix, r.records["mean_x"][0])


def projection(p, fx, fy, cx, cy):
    return np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])


def check_covariance_from_numerical_jacobian(cases=20, seed=4):
    """Inside the clamp: the inverse conic equals Jn S Jn^T + 0.3 I, Jn the
    central-difference Jacobian of the projection; outside it, the same at
    the point moved onto the clamp boundary (same depth)."""
    rs = np.random.default_rng(seed)
    fx, fy, cx, cy, tx, ty = 1000.0, 900.0, 320.0, 240.0, 0.4, 0.3
    for case in range(cases):
        z = rs.uniform(1.0, 20.0)
        outside = case % 4 == 3
        u = rs.uniform(-0.9, 0.9, 2) * (np.array([2.5, 2.5]) if outside else 1.0)
        p = np.array([u[0] * tx * z, u[1] * ty * z, z], np.float32).astype(np.float64)
        A = rs.normal(size=(3, 3)) * 0.05
        S = (A @ A.T + 1e-4 * np.eye(3)).astype(np.float32).astype(np.float64)
        r, _, _ = one(p, S, cam=cam_of(fx, fy, cx, cy, tx, ty))
        q = p.copy()
        q[0] = np.clip(p[0] / p[2], -1.3 * tx, 1.3 * tx) * p[2]
        q[1] = np.clip(p[1] / p[2], -1.3 * ty, 1.3 * ty) * p[2]
        h = 1e-6 * np.abs(q[2])
        Jn = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (projection(q + e, fx, fy, cx, cy) - projection(q - e, fx, fy, cx, cy)) / (2 * h)
        C = Jn @ S @ Jn.T + 0.3 * np.eye(2)
        a, b, c = r.conic_opacity[0, :3]
        K = np.array([[a, b], [b, c]])
        assert np.allclose(np.linalg.inv(K), C, rtol=1e-6, atol=1e-9), (case, np.linalg.inv(K), C)
        # radius from numpy's eigenvalues when the 0.1 floor is inactive
        ev = np.linalg.eigvalsh(C)
        mid = 0.5 * np.trace(C)
        if mid * mid - np.linalg.det(C) > 0.1:
            assert r.records["radius"][0] == int(np.ceil(3 * np.sqrt(ev.max()))), case


def check_radius_floor_and_culling():
    """An isotropic Gaussian on the axis: covariance s I projects to
    (f s / z)^2 I + 0.3 I, whose eigenvalue gap is 0, so the radius uses the
    0.1 floor: ceil(3 sqrt(lambda + sqrt(0.1))).  Depth at or before the near
    plane culls; a singular covariance is impossible after the 0.3."""
    f, s, z = 1000.0, 0.0104, 4.0     # f s / z = 2.6: the floor moves the radius from 8 to 9
    r, _, _ = one((0.0, 0.0, z), np.eye(3) * s * s, cam=cam_of(fx=f, fy=f))
    lam = (f / z) ** 2 * float(np.float32(s * s)) + 0.3
    assert int(np.ceil(3 * np.sqrt(lam))) == 8
    assert r.records["radius"][0] == int(np.ceil(3 * np.sqrt(lam + np.sqrt(0.1)))) == 9
    for zz, culled in ((0.19, True), (0.1, True), (-3.0, True), (0.2001, False)):
        r, _, _ = one((0.0, 0.0, zz), np.eye(3) * 1e-4)
        assert (r.records["radius"][0] == 0) == culled, zz
        if culled:
            assert not r.conic_opacity.any() and not r.rgb.any()


def check_colour():
    """Degree 0: 1/2 + sh0 / (2 sqrt(pi)), clamped at 0; higher degrees add
    the harmonics of the viewing direction; sh_degree masks the rest."""
    sh = np.zeros(48)
    sh[0:3] = [1.0, -3.0, 0.25]
    r, _, _ = one((0.0, 0.0, 3.0), np.eye(3) * 1e-4, sh=sh, cam=cam_of(deg=0))
    c0 = 0.5 / np.sqrt(np.pi)
    assert np.allclose(r.rgb[0, :3], [0.5 + c0, 0.0, 0.5 + 0.25 * c0], rtol=0, atol=1e-14)
    sh = np.random.default_rng(9).normal(size=48)
    p = np.array([0.4, -0.3, 2.0], np.float32).astype(np.float64)
    d = p / np.linalg.norm(p)
    Y = oracle.sh_basis(d)
    co = sh.reshape(16, 3).astype(np.float32).astype(np.float64)
    for deg in range(4):
        r, _, _ = one(p, np.eye(3) * 1e-4, sh=sh, cam=cam_of(deg=deg))
        nb = (deg + 1) ** 2
        want = np.maximum(0.0, 0.5 + Y[:nb] @ co[:nb])
        assert np.allclose(r.rgb[0, :3], want, atol=1e-9), deg


def check_scene_invariants(n=20000, seed=5):
    """Workload scene: the conic is positive definite and its inverse has both
    eigenvalues >= 0.3; radii bound 3 standard deviations; colours >= 0; the
    culled ones are exactly the points at or before the near plane."""
    cam = synth.SCENE_CAMERA
    sc = synth.make_scene(n, cam, seed)
    tx, ty = cam.tan_fov
    c = oracle.camera(cam.view, cam.focal, cam.focal, cam.width / 2, cam.height / 2, tx, ty, (0, 0, 0),
                      cam.near, cam.sh_degree)
    r = oracle.preprocess(c, sc["mean3d_opacity"], sc["cov3d"], sc["sh"])
    live = r.records["radius"] > 0
    assert np.array_equal(~live, sc["mean3d_opacity"][:, 2].astype(np.float64) <= cam.near)
    a, b, cc = r.conic_opacity[live, 0], r.conic_opacity[live, 1], r.conic_opacity[live, 2]
    det = a * cc - b * b
    assert np.all(a > 0) and np.all(det > 0)
    inv_a, inv_c = cc / det, a / det   # diagonal of the 2D covariance
    assert np.all(inv_a >= 0.3 - 1e-9) and np.all(inv_c >= 0.3 - 1e-9)
    rad = r.records["radius"][live].astype(np.float64)
    assert np.all(rad >= 3 * np.sqrt(np.maximum(inv_a, inv_c)) - 1e-9)
    assert np.all(r.rgb >= 0.0)


def run_all_preprocess():
    check_sh_against_scipy()
    check_sh_orthonormal()
    check_projection_and_rounding()
    check_covariance_from_numerical_jacobian()
    check_radius_floor_and_culling()
    check_colour()
    check_scene_invariants()

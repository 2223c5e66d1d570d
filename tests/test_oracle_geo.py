"""Pins for the oracle's geometry-consistency loss (Sec. 3.2, Eq. 3) between
consecutive flow sets, and the full loss (Eq. 4).

Each test states the mistake it is there to catch.
"""

import numpy as np
import pytest
from scipy.ndimage import map_coordinates
from scipy.spatial.transform import Rotation

import oracle
from tests.test_oracle_flowsets import knots_of
from tests.test_oracle_pins import mkwin


def geo_window(W, H, f, refs, rho, theta, cx=None, cy=None):
    e = np.zeros(0)
    return mkwin(W, H, f, refs, e, e, e, e, rho, theta, cx=cx, cy=cy)


def _project(win, f):
    """scipy reference of pair f: rotation from scipy's rotation vector, the
    point's z and its projection."""
    rho = np.asarray(win.rho, np.float64)
    th = np.asarray(win.theta, np.float64)
    K = knots_of(win.refs)
    d = K[f + 1] - K[f]
    Rm = Rotation.from_rotvec(d * th[f, 3:]).as_matrix()
    xs, ys = np.meshgrid(np.arange(win.width, dtype=np.float64),
                         np.arange(win.height, dtype=np.float64))
    X = np.stack([(xs - win.cx) / win.fx, (ys - win.cy) / win.fy, np.ones_like(xs)], -1)
    X = X / rho[f][..., None]
    P = X @ Rm.T + d * th[f, :3]
    z = P[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        xp = win.fx * P[..., 0] / z + win.cx
        yp = win.fy * P[..., 1] / z + win.cy
    ok = (rho[f] > 0) & (z > 0) & (xp >= 0) & (xp <= win.width - 1) & (yp >= 0) & \
        (yp <= win.height - 1)
    return z, xp, yp, ok


def scipy_geo(win):
    """L_geo from scipy's rotation and order-1 (bilinear) interpolation."""
    rho = np.asarray(win.rho, np.float64)
    F = rho.shape[0]
    total, pairs = 0.0, []
    for f in range(F - 1):
        z, xp, yp, ok = _project(win, f)
        Db = 1.0 / rho[f + 1]
        Dp = map_coordinates(Db, [yp[ok], xp[ok]], order=1, mode="nearest")
        term = np.abs(z[ok] - Dp) / (z[ok] + Dp)
        m = term.mean() if ok.any() else 0.0
        pairs.append((m, ok.sum()))
        total += m
    return total / (F - 1), np.array(pairs)


def smooth_rho(rng, F, W, H, lo=0.5, hi=1.5):
    xs, ys = np.meshgrid(np.arange(W), np.arange(H))
    out = []
    for _ in range(F):
        g = sum(rng.uniform(0.2, 0.5) * np.exp(-((xs - rng.uniform(0, W)) ** 2 +
                                                 (ys - rng.uniform(0, H)) ** 2) / rng.uniform(20, 80))
                for _ in range(3))
        out.append(lo + (hi - lo) * g / max(g.max(), 1e-9))
    return np.stack(out)


# ---------------------------------------------------------------------------
# Identity and closed forms.  Catches: a depth that is not 1/rho, a pose that
# is not the identity at zero motion, a wrong normaliser, a wrong V.
# ---------------------------------------------------------------------------

def test_identity_pose_and_equal_depths_give_zero():
    rng = np.random.default_rng(1)
    W, H = 30, 22
    rho = smooth_rho(rng, 1, W, H)
    win = geo_window(W, H, 25.0, [0.0, 0.5, 1.0], np.repeat(rho, 2, 0), np.zeros((2, 6)))
    g = oracle.geo(win, grad=True)
    # exact: zero motion maps every pixel onto itself, border pixels included
    assert g["loss"] == 0.0
    np.testing.assert_array_equal(g["pairs"], [[0.0, W * H]])


@pytest.mark.parametrize("tz", [0.3, -0.4])
def test_pure_z_translation_constant_depths_closed_form(tz):
    """Constant depths Da, Db and translation tz: D_{0->1} = Da + tz and
    D'_1 = Db, so every visible pixel gives |Da + tz - Db| / (Da + tz + Db);
    the image zooms about the principal point by Da / (Da + tz), so for
    tz < 0 exactly the pixels with |x - c| Da/(Da + tz) inside the box stay."""
    W, H, f = 41, 31, 30.0
    Da, Db = 2.0, 1.7
    refs = [0.0, 0.5, 1.0]
    delta = 0.5                                      # segment 0 = [0, 0.5]
    theta = np.zeros((2, 6))
    theta[0, 2] = tz / delta
    rho = np.stack([np.full((H, W), 1 / Da), np.full((H, W), 1 / Db)])
    win = geo_window(W, H, f, refs, rho, theta)
    g = oracle.geo(win)
    want = abs(Da + tz - Db) / (Da + tz + Db)
    s = Da / (Da + tz)
    xs = (np.arange(W) - (W - 1) / 2) * s + (W - 1) / 2
    ys = (np.arange(H) - (H - 1) / 2) * s + (H - 1) / 2
    nx = ((xs >= 0) & (xs <= W - 1)).sum()
    ny = ((ys >= 0) & (ys <= H - 1)).sum()
    assert g["pairs"][0, 1] == nx * ny
    if tz > 0:
        assert nx * ny == W * H
    else:
        assert nx * ny < W * H
    assert abs(g["loss"] - want) < 1e-13


def test_roll_about_optical_axis_keeps_depth():
    """Rotation about the optical axis leaves z unchanged: every visible pixel
    gives |Da - Db| / (Da + Db); the visible pixels are those whose rotated
    position about the principal point stays in the box."""
    W, H, f = 33, 25, 20.0
    Da, Db = 1.25, 1.0
    phi = 0.3
    theta = np.zeros((2, 6))
    theta[0, 5] = phi / 0.4                          # segment 0 = [0, 0.4]
    rho = np.stack([np.full((H, W), 1 / Da), np.full((H, W), 1 / Db)])
    win = geo_window(W, H, f, [0.0, 0.4, 1.0], rho, theta)
    g = oracle.geo(win)
    xs, ys = np.meshgrid(np.arange(W) - (W - 1) / 2, np.arange(H) - (H - 1) / 2)
    c, s = np.cos(phi), np.sin(phi)
    X, Y = c * xs - s * ys + (W - 1) / 2, s * xs + c * ys + (H - 1) / 2
    n = ((X >= 0) & (X <= W - 1) & (Y >= 0) & (Y <= H - 1)).sum()
    assert g["pairs"][0, 1] == n and n < W * H
    assert abs(g["loss"] - abs(Da - Db) / (Da + Db)) < 1e-13


# ---------------------------------------------------------------------------
# scipy reference.  Catches: the wrong pose convention (R (X + t) instead of
# R X + t), the segment length not applied (or applied to the wrong set), the
# wrong pair (f, f+1), depth interpolated as inverse depth, a wrong mean.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("refs", [[0.0, 0.5, 1.0], [0.1, 0.35, 0.8], [0.0, 0.2, 0.3, 0.6, 1.0]])
def test_matches_scipy_reference(refs):
    rng = np.random.default_rng(7 + len(refs))
    W, H = 37, 29
    F = len(knots_of(refs)) - 1
    rho = smooth_rho(rng, F, W, H)
    theta = rng.normal(0, 0.3, (F, 6))
    win = geo_window(W, H, 28.0, refs, rho, theta, cx=17.25, cy=14.625)   # FP32-exact
    g = oracle.geo(win)
    want, pairs = scipy_geo(win)
    assert np.all(pairs[:, 1] > 0.3 * W * H) and np.all(pairs[:, 1] < W * H)
    np.testing.assert_allclose(g["pairs"][:, 1], pairs[:, 1])
    np.testing.assert_allclose(g["pairs"][:, 0], pairs[:, 0], rtol=1e-12)
    assert abs(g["loss"] - want) < 1e-12 * want


def test_depth_scale_invariance():
    """Depth is known up to scale (Eq. 2's ~): scaling every depth and the
    translation by k leaves L_geo unchanged.  Catches a translation not
    expressed in the depth's units."""
    rng = np.random.default_rng(3)
    W, H = 31, 23
    refs = [0.0, 0.3, 0.7, 1.0]
    rho = smooth_rho(rng, 3, W, H)
    theta = rng.normal(0, 0.5, (3, 6))
    a = oracle.geo(geo_window(W, H, 22.0, refs, rho, theta))["loss"]
    k = 3.7
    th2 = theta.copy()
    th2[:, :3] *= k
    b = oracle.geo(geo_window(W, H, 22.0, refs, rho / k, th2))["loss"]
    assert a > 0.01 and abs(a - b) < 1e-12 * a


def test_invalid_depths_leave_v_and_one_set_has_no_pair():
    """Catches: non-positive inverse depth entering the mean (division by zero
    or negative depth), a loss from a window with a single flow set."""
    rng = np.random.default_rng(5)
    W, H = 24, 18
    rho = smooth_rho(rng, 2, W, H)
    theta = np.zeros((2, 6))
    base = oracle.geo(geo_window(W, H, 20.0, [0.0, 0.5, 1.0], rho, theta))
    assert base["pairs"][0, 1] == W * H
    r2 = rho.copy()
    r2[0, 3:6, 4:9] = 0.0                           # 15 source pixels without depth
    # a target pixel without depth: the four source pixels (zero motion maps x
    # to x) whose taps include it leave V
    r2[1, 10, 10] = -1.0
    g = oracle.geo(geo_window(W, H, 20.0, [0.0, 0.5, 1.0], r2, theta), grad=True)
    assert g["pairs"][0, 1] == W * H - 15 - 4
    assert np.isfinite(g["loss"]) and np.all(np.isfinite(g["drho"]))
    one = geo_window(W, H, 20.0, [0.0, 1.0], rho[0], theta[0])
    g1 = oracle.geo(one, grad=True)
    assert g1["loss"] == 0.0 and not g1["drho"].any() and not g1["dtheta"].any()


# ---------------------------------------------------------------------------
# Finite differences.  Catches: a wrong adjoint of the projection, of the
# rotation (right Jacobian), of the interpolation, of the segment scaling, a
# gradient sent to the wrong set.
# ---------------------------------------------------------------------------

def _fd_case(seed, refs, W=18, H=14):
    F = len(knots_of(refs)) - 1
    for s in range(seed, seed + 200):
        rng = np.random.default_rng(s)
        rho = smooth_rho(rng, F, W, H)
        theta = rng.normal(0, 0.3, (F, 6))
        win = geo_window(W, H, 15.0, refs, rho, theta)
        good = True
        for f in range(F - 1):
            z, xp, yp, ok = _project(win, f)
            fin = np.isfinite(xp) & np.isfinite(yp) & (z > 0)
            mx = np.minimum(np.abs(xp[fin]), np.abs(xp[fin] - (W - 1)))
            my = np.minimum(np.abs(yp[fin]), np.abs(yp[fin] - (H - 1)))
            frac = np.minimum(np.abs(xp[ok] - np.rint(xp[ok])), np.abs(yp[ok] - np.rint(yp[ok])))
            if mx.min() < 1e-4 or my.min() < 1e-4 or frac.min() < 1e-4 or ok.sum() < W * H // 2:
                good = False
        if good:
            return win
    raise RuntimeError("no smooth case found")


@pytest.mark.parametrize("refs", [[0.0, 0.5, 1.0], [0.2, 0.45, 0.9]])
def test_geo_gradient_matches_central_differences(refs):
    win = _fd_case(40 + len(refs), refs)
    F = win.rho.shape[0]
    g = oracle.geo(win, grad=True, grad_loss=1.7)
    L = lambda **kw: 1.7 * oracle.geo(win, **kw)["loss"]
    h = 1e-6
    fd_th = np.zeros_like(win.theta)
    for s in range(F):
        for k in range(6):
            tp = win.theta.copy(); tp[s, k] += h
            tm = win.theta.copy(); tm[s, k] -= h
            fd_th[s, k] = (L(theta=tp) - L(theta=tm)) / (2 * h)
    assert not fd_th[F - 1].any()                    # the last set's pose is in no pair
    sc = np.abs(fd_th).max()
    assert sc > 1e-4
    np.testing.assert_allclose(g["dtheta"], fd_th, atol=1e-6 * sc)
    fd_r = np.zeros_like(win.rho)
    for s in range(F):
        for j in range(win.height):
            for i in range(win.width):
                rp = win.rho.copy(); rp[s, j, i] += h
                rm = win.rho.copy(); rm[s, j, i] -= h
                fd_r[s, j, i] = (L(rho=rp) - L(rho=rm)) / (2 * h)
    sc = np.abs(fd_r).max()
    assert sc > 1e-5
    np.testing.assert_allclose(g["drho"], fd_r, atol=1e-6 * sc)


def test_full_loss_is_cm_plus_weighted_geo():
    """Eq. 4 with the paper's lambda = 0.05."""
    import eventgen
    win = eventgen.make_window("c6", 1)
    L = oracle.full_loss(win)
    assert oracle.LAMBDA_GEO == 0.05
    assert abs(L - (oracle.loss(win) + 0.05 * oracle.geo(win)["loss"])) < 1e-15


def test_rsat_is_one_without_motion_and_a_loss_ratio():
    """RSAT = L(motion) / L(no motion): exactly 1 at zero motion.  Catches an
    RSAT computed against the wrong reference loss."""
    import eventgen
    win = eventgen.edge_window(4, "64x64", 3000, refs=[0.0, 0.5, 1.0], n_segments=10)
    assert oracle.rsat(win, theta=np.zeros(6)) == 1.0
    r = oracle.rsat(win)
    assert r == oracle.loss(win) / oracle.loss(win, theta=np.zeros(6)) and r != 1.0

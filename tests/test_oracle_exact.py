"""Pins for the oracle's exact-reprojection flow (Eq. 2 without the first-order
expansion): rotation by exponential coordinates (Rodrigues), translation,
pinhole projection; the flow is the displacement over the window.

Each test states the mistake it is there to catch.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from tests.test_oracle_pins import mkwin


def _scipy_flow(W, H, K, rho, theta):
    """Reference: back-project with depth 1/rho, rotate with scipy's rotation
    vector, translate, project; flow = projection - pixel."""
    fx, fy, cx, cy = K
    Rm = Rotation.from_rotvec(np.asarray(theta[3:], np.float64)).as_matrix()
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    X0 = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)], -1) / rho[..., None]
    X1 = X0 @ Rm.T + np.asarray(theta[:3], np.float64)
    u = np.stack([fx * X1[..., 0] / X1[..., 2] + cx - xs, fy * X1[..., 1] / X1[..., 2] + cy - ys], -1)
    return u, X1[..., 2]


# ---------------------------------------------------------------------------
# Catches: a wrong Rodrigues formula (sign, missing quadratic term, broken
# small-angle series), translation scaled by depth instead of inverse depth,
# swapped axes or intrinsics in the projection.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1e-7, 4e-5, 1e-3, 0.3, 1.5])
def test_exact_flow_matches_scipy_reprojection(scale):
    rng = np.random.default_rng(21)
    W, H = 27, 19
    K = np.array([23.0, 31.0, 12.5, 8.25])
    rho = rng.uniform(0.4, 2.0, (H, W))
    for _ in range(4):
        theta = scale * rng.normal(0, 1, 6)
        theta[2] = abs(theta[2]) * 0.1          # keep points in front of the camera
        u = oracle.flow_field(W, H, K, rho, theta, model=1)
        ref, z = _scipy_flow(W, H, K, rho, theta)
        front = z > 0                            # large rotations turn some points away
        assert front.sum() > 20
        np.testing.assert_allclose(u[front], ref[front], rtol=1e-11,
                                   atol=1e-11 * (1 + np.abs(ref[front]).max()))
        assert not u[~front].any()


def test_exact_flow_roll_about_optical_axis_is_a_rotation():
    # w = (0, 0, phi), v = 0, fx = fy: pixels rotate about the principal point
    W, H, f = 21, 17, 30.0
    K = np.array([f, f, 10.0, 8.0])
    phi = 0.4
    u = oracle.flow_field(W, H, K, np.ones((H, W)), [0, 0, 0, 0, 0, phi], model=1)
    xs, ys = np.meshgrid(np.arange(W) - 10.0, np.arange(H) - 8.0)
    c, s = np.cos(phi), np.sin(phi)
    np.testing.assert_allclose(u[..., 0], c * xs - s * ys - xs, atol=1e-12)
    np.testing.assert_allclose(u[..., 1], s * xs + c * ys - ys, atol=1e-12)


def test_exact_and_first_order_agree_to_first_order():
    """Catches: a first-order model that is not the linearisation of the exact
    one (the difference must shrink 4x when the motion halves)."""
    rng = np.random.default_rng(22)
    W, H = 25, 21
    K = np.array([28.0, 28.0, 12.0, 10.0])
    rho = rng.uniform(0.5, 1.5, (H, W))
    theta = rng.normal(0, 1.0, 6)
    errs = []
    for sc in (0.02, 0.01):
        d = oracle.flow_field(W, H, K, rho, sc * theta, model=1) - \
            oracle.flow_field(W, H, K, rho, sc * theta, model=0)
        errs.append(np.abs(d).max())
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_points_behind_the_camera_have_zero_flow_and_no_gradient():
    """Catches: a missing guard (huge or sign-flipped flows from points behind
    the camera plane)."""
    W, H = 30, 24
    K = np.array([20.0, 20.0, 14.5, 11.5])
    rho = np.full((H, W), 1.0)
    rho[:, 15:] = 3.0                              # these points get pushed behind the camera
    theta = np.array([0.0, 0.0, -0.5, 0.0, 0.0, 0.0])
    u = oracle.flow_field(W, H, K, rho, theta, model=1)
    _, z = _scipy_flow(W, H, K, rho, theta)
    assert (z[:, 15:] < 0).all() and (z[:, :15] > 0).all()
    assert not u[:, 15:].any() and np.abs(u[:, :15]).max() > 0
    rng = np.random.default_rng(23)
    n = 300
    win = mkwin(W, H, 20.0, [0.0, 1.0], rng.uniform(0, 14, n), rng.uniform(0, 23, n),
                rng.random(n), np.ones(n), rho, theta).replace(flow_model=1)
    g = oracle.backward(win)
    assert not g["drho"][:, 16:].any()


# ---------------------------------------------------------------------------
# Finite differences of the whole loss with the exact flow.  Catches: a wrong
# adjoint of the projection (missing -p/pz^2 term), of the rotation (right
# Jacobian transposed, missing or wrong sign), of the translation.
# ---------------------------------------------------------------------------

def _fd_window(seed, refs, model=1, n=40, W=16, H=14, f=12.0, sets=1):
    for s in range(seed, seed + 300):
        rng = np.random.default_rng(s)
        x = rng.uniform(2, W - 3, n)
        y = rng.uniform(2, H - 3, n)
        t = rng.random(n)
        p = np.where(rng.random(n) < 0.5, 1, -1)
        xs, ys = np.meshgrid(np.arange(W), np.arange(H))
        rho = np.stack([0.7 + 0.5 * np.exp(-((xs - rng.uniform(0, W)) ** 2
                                               + (ys - rng.uniform(0, H)) ** 2) / 20.0)
                        for _ in range(sets)])
        theta = rng.normal(0, 0.25, (sets, 6))
        if sets == 1:
            rho, theta = rho[0], theta[0]
        win = mkwin(W, H, f, refs, x, y, t, p, rho, theta).replace(flow_model=model)
        res = oracle.forward(win, positions=True, valid=True)
        if res["valid"].sum() < n // 2:
            continue
        P = res["positions"][res["valid"]]
        frac = np.abs(P - np.rint(P))
        border = np.minimum(P, np.array([W - 1, H - 1]) - P)
        ev = np.stack([x, y], 1)
        if frac.min() > 1e-3 and border.min() > 1e-3 and np.abs(ev - np.rint(ev)).min() > 1e-3:
            return win
    raise RuntimeError("no smooth seed found")


@pytest.mark.parametrize("refs,sets", [([0.0, 0.4, 1.0], 1), ([1.0], 1), ([0.0, 0.5, 1.0], 2)])
def test_exact_flow_gradient_matches_central_differences(refs, sets):
    win = _fd_window(900 + len(refs) + sets, refs, sets=sets)
    g = oracle.backward(win)
    h = 1e-6
    L = lambda **kw: oracle.loss(win, **kw)
    th = np.atleast_2d(win.theta)
    gth = np.atleast_2d(g["dtheta"])
    grho = g["drho"].reshape((sets,) + win.rho.shape[-2:])
    for s in range(sets):
        fd = np.zeros(6)
        for k in range(6):
            tp = th.copy(); tp[s, k] += h
            tm = th.copy(); tm[s, k] -= h
            fd[k] = (L(theta=tp.reshape(win.theta.shape)) - L(theta=tm.reshape(win.theta.shape))) / (2 * h)
        scale = np.abs(fd).max()
        assert scale > 1e-5
        np.testing.assert_allclose(gth[s], fd, atol=1e-6 * scale)
        rho = win.rho.reshape((sets,) + win.rho.shape[-2:])
        fdr = np.zeros(rho.shape[1:])
        for j in range(rho.shape[1]):
            for i in range(rho.shape[2]):
                rp = rho.copy(); rp[s, j, i] += h
                rm = rho.copy(); rm[s, j, i] -= h
                fdr[j, i] = (L(rho=rp.reshape(win.rho.shape)) - L(rho=rm.reshape(win.rho.shape))) / (2 * h)
        scale = np.abs(fdr).max()
        assert scale > 1e-6
        np.testing.assert_allclose(grho[s], fdr, atol=1e-6 * scale)

"""Pins for the FP64 oracle: facts fixed by the paper and by mathematics, not by
the oracle's own formulas.

Each test names the passage it checks and the mistake it is there to catch.
The paper prints no worked numeric example, so the pins are closed forms,
invariants, special cases that reduce to a library routine, and finite
differences.
"""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from eventgen import Window


def mkwin(W, H, f, refs, x, y, t, p, rho, theta, cx=None, cy=None, fy=None, eps=1e-9):
    return Window("pin", W, H, f, f if fy is None else fy,
                  (W - 1) / 2.0 if cx is None else cx, (H - 1) / 2.0 if cy is None else cy,
                  np.asarray(refs, dtype=np.float64), np.asarray(x, dtype=np.float64),
                  np.asarray(y, dtype=np.float64), np.asarray(t, dtype=np.float64),
                  np.asarray(p, dtype=np.int8), np.asarray(rho, dtype=np.float64),
                  np.asarray(theta, dtype=np.float64), eps)


def tbar(r, t):
    return 1.0 - abs(r - t)


# ---------------------------------------------------------------------------
# Eq. 2: the flow is the time derivative of the exact rigid reprojection.
# Catches: any dropped term, wrong sign or swapped axis in the motion field.
# ---------------------------------------------------------------------------

def _project_exact(xpix, ypix, rho, K, theta, s):
    fx, fy, cx, cy = K
    X0 = np.array([(xpix - cx) / fx, (ypix - cy) / fy, 1.0]) / rho
    Rm = Rotation.from_rotvec(s * np.asarray(theta[3:], dtype=np.float64)).as_matrix()
    X = Rm @ X0 + s * np.asarray(theta[:3], dtype=np.float64)
    return np.array([fx * X[0] / X[2] + cx, fy * X[1] / X[2] + cy])


def test_flow_is_derivative_of_exact_reprojection():
    rng = np.random.default_rng(11)
    W, H = 23, 17
    K = np.array([19.0, 27.0, 10.25, 7.75])
    rho = rng.uniform(0.3, 2.0, (H, W))
    for trial in range(5):
        theta = rng.normal(0, 0.7, 6)
        u = oracle.flow_field(W, H, K, rho, theta)
        for (i, j) in [(0, 0), (22, 16), (5, 11), (17, 3)]:
            h = 1e-5
            d = (_project_exact(i, j, rho[j, i], K, theta, h)
                 - _project_exact(i, j, rho[j, i], K, theta, -h)) / (2 * h)
            np.testing.assert_allclose(u[j, i], d, rtol=1e-7, atol=1e-7 * np.abs(d).max())


def test_flow_error_against_exact_motion_is_second_order():
    rng = np.random.default_rng(12)
    W, H = 31, 29
    K = np.array([30.0, 30.0, 15.0, 14.0])
    rho = rng.uniform(0.5, 1.5, (H, W))
    theta = rng.normal(0, 1.0, 6)
    errs = []
    for scale in (0.02, 0.01):
        th = scale * theta
        u = oracle.flow_field(W, H, K, rho, th)
        i, j = 4, 22
        disp = _project_exact(i, j, rho[j, i], K, th, 1.0) - np.array([i, j])
        errs.append(np.linalg.norm(disp - u[j, i]))
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4, ratio


def test_flow_special_cases():
    W, H = 9, 7
    K = np.array([5.0, 5.0, 4.0, 3.0])
    rho = np.full((H, W), 0.8)
    # pure translation parallel to the image plane: uniform flow f * rho * v
    u = oracle.flow_field(W, H, K, rho, [0.3, -0.2, 0, 0, 0, 0])
    np.testing.assert_allclose(u[..., 0], 5.0 * 0.8 * 0.3, rtol=1e-15)
    np.testing.assert_allclose(u[..., 1], 5.0 * 0.8 * -0.2, rtol=1e-15)
    # pure forward motion: radial expansion from the principal point
    u = oracle.flow_field(W, H, K, rho, [0, 0, 0.5, 0, 0, 0])
    xs, ys = np.meshgrid(np.arange(W) - 4.0, np.arange(H) - 3.0)
    np.testing.assert_allclose(u[..., 0], -0.8 * 0.5 * xs, atol=1e-15)
    np.testing.assert_allclose(u[..., 1], -0.8 * 0.5 * ys, atol=1e-15)
    # rotation only: the flow does not depend on depth
    th = [0, 0, 0, 0.1, -0.2, 0.3]
    u1 = oracle.flow_field(W, H, K, rho, th)
    u2 = oracle.flow_field(W, H, K, 3.0 * rho, th)
    np.testing.assert_array_equal(u1, u2)


# ---------------------------------------------------------------------------
# Sec. 3.1 splatting: zero flow reproduces the raw per-polarity histogram.
# Catches: wrong tap indexing, wrong polarity channel, wrong tbar.
# ---------------------------------------------------------------------------

def test_zero_flow_gives_raw_histogram():
    rng = np.random.default_rng(3)
    W, H, n = 13, 9, 400
    refs = [0.0, 0.3, 1.0]
    x = rng.integers(0, W, n)
    y = rng.integers(0, H, n)
    t = np.sort(rng.random(n))
    p = np.where(rng.random(n) < 0.5, 1, -1)
    win = mkwin(W, H, 10.0, refs, x, y, t, p, rng.uniform(0.5, 1.5, (H, W)), np.zeros(6))
    res = oracle.forward(win, images=True, valid=True)
    assert res["valid"].all()
    img = res["images"]
    for r, ref in enumerate(refs):
        for pol, sgn in ((0, 1), (1, -1)):
            C = np.zeros((H, W))
            S = np.zeros((H, W))
            sel = p == sgn
            np.add.at(C, (y[sel], x[sel]), 1.0)
            np.add.at(S, (y[sel], x[sel]), 1.0 - np.abs(ref - t[sel]))
            np.testing.assert_array_equal(img[r, pol, 0], C)
            np.testing.assert_allclose(img[r, pol, 1], S, rtol=1e-13, atol=1e-13)
        assert res["nact"][r] == np.count_nonzero(
            np.bincount(y * W + x, minlength=W * H))


def test_single_event_fractional_position_images():
    # zero flow, real-valued position: the four bilinear weights, exactly
    win = mkwin(20, 30, 10.0, [0.0, 0.5, 1.0], [10.3], [20.6], [0.25], [1],
                np.ones((30, 20)), np.zeros(6))
    res = oracle.forward(win, images=True)
    img = res["images"]
    a, b = 0.3, 0.6
    expect = {(20, 10): (1 - a) * (1 - b), (20, 11): a * (1 - b), (21, 10): (1 - a) * b,
              (21, 11): a * b}
    for r, ref in enumerate([0.0, 0.5, 1.0]):
        C = img[r, 0, 0]
        assert np.count_nonzero(C) == 4 and np.count_nonzero(img[r, 1]) == 0
        for (yy, xx), wv in expect.items():
            assert C[yy, xx] == pytest.approx(wv, rel=1e-12)
            assert img[r, 0, 1][yy, xx] == pytest.approx(wv * tbar(ref, 0.25), rel=1e-12)


# ---------------------------------------------------------------------------
# Eq. 1: closed forms of the loss for one and two events.
# Catches: missing square, missing polarity split, normalising by events or by
# per-polarity pixels instead of active pixels, wrong tbar, wrong mean over refs.
# ---------------------------------------------------------------------------

REFS3 = [0.0, 0.5, 1.0]


def _static(x, y, t, p, refs=REFS3, W=40, H=30):
    return mkwin(W, H, 10.0, refs, x, y, t, p, np.ones((H, W)), np.zeros(6))


def test_loss_single_event():
    L = oracle.loss(_static([10.3], [20.6], [0.25], [1]))
    expect = np.mean([tbar(r, 0.25) ** 2 for r in REFS3])      # = 0.395833...
    assert L == pytest.approx(expect, rel=1e-7)
    # an event on an integer pixel activates one pixel, not four
    res = oracle.forward(_static([7.0], [3.0], [0.75], [-1]))
    assert list(res["nact"]) == [1.0, 1.0, 1.0]
    assert res["loss"] == pytest.approx(np.mean([tbar(r, 0.75) ** 2 for r in REFS3]), rel=1e-7)


def test_loss_two_events_same_and_opposite_polarity():
    t1, t2 = 0.1, 0.7
    same = oracle.loss(_static([10.3, 10.3], [20.6, 20.6], [t1, t2], [1, 1]))
    assert same == pytest.approx(np.mean([((tbar(r, t1) + tbar(r, t2)) / 2) ** 2 for r in REFS3]),
                                 rel=1e-7)
    opp = oracle.forward(_static([10.3, 10.3], [20.6, 20.6], [t1, t2], [1, -1]))
    assert list(opp["nact"]) == [4.0, 4.0, 4.0]
    assert opp["loss"] == pytest.approx(
        np.mean([tbar(r, t1) ** 2 + tbar(r, t2) ** 2 for r in REFS3]), rel=1e-7)
    apart = oracle.loss(_static([3.5, 30.25], [4.5, 20.75], [t1, t2], [1, 1]))
    assert apart == pytest.approx(
        np.mean([(tbar(r, t1) ** 2 + tbar(r, t2) ** 2) / 2 for r in REFS3]), rel=1e-7)


def test_empty_and_all_invalid_give_zero():
    assert oracle.loss(_static([], [], [], [])) == 0.0
    # t outside [0,1], a non-finite coordinate, a start off the sensor: all masked
    win = _static([5.0, np.nan, -0.5, 3.0], [5.0, 2.0, 1.0, 30.0], [1.5, 0.5, 0.5, 0.5],
                  [1, 1, 1, 1])
    res = oracle.forward(win, valid=True)
    assert res["loss"] == 0.0 and not res["valid"].any()
    g = oracle.backward(win)
    assert not g["drho"].any() and not g["dtheta"].any()


# ---------------------------------------------------------------------------
# Sec. 3.1 warp: constant flow moves events along straight lines, in the
# direction of time.  Catches: wrong sign of dt, forward/backward sweeps
# swapped, reference equal to t_k mishandled, masking per ref instead of global.
# ---------------------------------------------------------------------------

def _const_flow_window(x, y, t, p, refs, W=60, H=50, f=20.0, rho0=0.5, v=(1.2, -0.8)):
    theta = np.array([v[0], v[1], 0.0, 0.0, 0.0, 0.0])
    return mkwin(W, H, f, refs, x, y, t, p, np.full((H, W), rho0), theta), \
        np.array([f * rho0 * v[0], f * rho0 * v[1]])


def test_constant_flow_positions_and_mask():
    rng = np.random.default_rng(5)
    n = 300
    refs = [0.0, 0.25, 0.5, 1.0]
    x = rng.uniform(0, 59, n)
    y = rng.uniform(0, 49, n)
    t = rng.random(n)
    t[:4] = [0.0, 0.25, 1.0, 0.5]         # events exactly at reference times
    win, u = _const_flow_window(x, y, t, np.ones(n), refs)
    res = oracle.forward(win, valid=True, positions=True, images=True)
    expect_valid = np.ones(n, bool)
    for r, ref in enumerate(refs):
        px = x + (ref - t) * u[0]
        py = y + (ref - t) * u[1]
        expect_valid &= (px >= 0) & (px <= 59) & (py >= 0) & (py <= 49)
    np.testing.assert_array_equal(res["valid"], expect_valid)
    for r, ref in enumerate(refs):
        ok = res["valid"]
        np.testing.assert_allclose(res["positions"][ok, r, 0], (x + (ref - t) * u[0])[ok],
                                   atol=1e-12)
        np.testing.assert_allclose(res["positions"][ok, r, 1], (y + (ref - t) * u[1])[ok],
                                   atol=1e-12)
        # splatted mass equals the number of valid events (global mask)
        assert res["images"][r, :, 0].sum() == pytest.approx(ok.sum(), rel=1e-12)
    # the masked events change nothing
    keep = res["valid"]
    win2 = win.replace(x=x[keep], y=y[keep], t=t[keep], p=np.ones(keep.sum(), np.int8))
    assert oracle.loss(win2) == pytest.approx(res["loss"], rel=1e-14)


def test_constant_flow_collapse_is_the_minimum():
    # events of 40 scene points, each seen at 25 times along its straight path
    rng = np.random.default_rng(6)
    q = np.stack([rng.uniform(20, 40, 40), rng.uniform(15, 35, 40)], 1)
    pts = np.repeat(q, 25, axis=0)
    t = rng.random(pts.shape[0])
    win0, u = _const_flow_window(pts[:, 0], pts[:, 1], t, np.ones(t.size), [0.0, 0.5, 1.0])
    x = pts[:, 0] + t * u[0]
    y = pts[:, 1] + t * u[1]
    win = win0.replace(x=x, y=y)
    truth = win.theta.copy()
    L0 = oracle.loss(win)
    # at the truth every point collapses to one position per reference:
    # the loss is the mean over points of the squared mean tbar (points rarely share taps)
    res = oracle.forward(win, positions=True)
    for r, ref in enumerate([0.0, 0.5, 1.0]):
        np.testing.assert_allclose(res["positions"][:, r, 0], pts[:, 0] + ref * u[0], atol=1e-10)
    for dvx in (-0.1, -0.03, 0.03, 0.1):
        for dvy in (-0.1, 0.0, 0.1):
            th = truth.copy()
            th[0] += dvx
            th[1] += dvy
            assert oracle.loss(win, theta=th) > L0


# ---------------------------------------------------------------------------
# Sec. 3.1 flow concatenation: the flow is re-sampled at every reference time.
# For a linear flow field bilinear sampling is exact, so the positions follow
# the explicit Euler recursion between references.  Catches: warping linearly
# from t_k (no re-sampling), wrong step order, wrong rotation sign.
# ---------------------------------------------------------------------------

def test_iterative_warp_follows_euler_steps_in_linear_flow():
    W, H, f = 101, 81, 40.0
    refs = [0.0, 0.2, 0.45, 0.7, 1.0]
    cx, cy = 50.0, 40.0
    x = np.array([60.3, 40.7, 55.5])
    y = np.array([30.2, 47.9, 41.1])
    t = np.array([0.1, 0.6, 0.45])
    for theta, A in (([0, 0, 0.6, 0, 0, 0], -0.8 * 0.6 * np.eye(2)),              # zoom
                     ([0, 0, 0, 0, 0, 0.5], 0.5 * np.array([[0.0, -1.0], [1.0, 0.0]]))):  # roll
        win = mkwin(W, H, f, refs, x, y, t, [1, 1, 1], np.full((H, W), 0.8), theta, cx=cx, cy=cy)
        res = oracle.forward(win, positions=True, valid=True)
        assert res["valid"].all()
        for k in range(3):
            for direction in (+1, -1):
                P = np.array([x[k] - cx, y[k] - cy])
                tau = t[k]
                order = [r for r in range(5) if (refs[r] - t[k]) * direction > 0]
                order = order if direction > 0 else order[::-1]
                for r in order:
                    P = P + (refs[r] - tau) * (A @ P)
                    tau = refs[r]
                    got = res["positions"][k, r] - np.array([cx, cy])
                    np.testing.assert_allclose(got, P, atol=1e-11)
            r_eq = [r for r in range(5) if refs[r] == t[k]]
            for r in r_eq:
                np.testing.assert_array_equal(res["positions"][k, r], [x[k], y[k]])


# ---------------------------------------------------------------------------
# Invariances of the loss (the paper's augmentations: polarity flip,
# left-right flip, time reversal) and the depth-scale ambiguity of Eq. 2.
# ---------------------------------------------------------------------------

def _generic(seed=21, W=24, H=18, n=150, refs=(0.0, 0.25, 0.5, 1.0)):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, W, n).astype(np.float64)
    y = rng.integers(0, H, n).astype(np.float64)
    t = np.sort(rng.integers(0, 2 ** 20, n)) / 2.0 ** 20      # exact under t -> 1 - t
    p = np.where(rng.random(n) < 0.5, 1, -1)
    xs, ys = np.meshgrid(np.arange(W), np.arange(H))
    rho = 0.6 + 0.4 * np.exp(-((xs - 9) ** 2 + (ys - 8) ** 2) / 30.0)
    theta = rng.normal(0, 0.15, 6)
    return mkwin(W, H, 15.0, refs, x, y, t, p, rho, theta)


def test_polarity_swap_invariance():
    win = _generic()
    assert oracle.loss(win.replace(p=-win.p)) == pytest.approx(oracle.loss(win), rel=1e-14)


def test_time_reversal_invariance():
    win = _generic()
    rev = win.replace(t=1.0 - win.t, refs=np.sort(1.0 - win.refs), theta=-win.theta)
    assert oracle.loss(rev) == pytest.approx(oracle.loss(win), rel=1e-13)


def test_left_right_mirror_invariance():
    win = _generic()
    sgn = np.array([-1, 1, 1, 1, -1, -1.0])
    mir = win.replace(x=(win.width - 1) - win.x, rho=win.rho[:, ::-1].copy(),
                      theta=win.theta * sgn)
    assert oracle.loss(mir) == pytest.approx(oracle.loss(win), rel=1e-13)
    g = oracle.backward(win)
    gm = oracle.backward(mir)
    np.testing.assert_allclose(gm["drho"][:, ::-1], g["drho"], atol=1e-12 * np.abs(g["drho"]).max())
    np.testing.assert_allclose(gm["dtheta"] * sgn, g["dtheta"], atol=1e-12 * np.abs(g["dtheta"]).max())


def test_depth_scale_invariance_and_gradient_identity():
    win = _generic()
    c = 2.5
    scaled = win.replace(rho=win.rho * c, theta=np.concatenate([win.theta[:3] / c, win.theta[3:]]))
    assert oracle.loss(scaled) == pytest.approx(oracle.loss(win), rel=1e-13)
    g = oracle.backward(win)
    lhs = np.sum(win.rho * g["drho"])
    rhs = np.dot(win.theta[:3], g["dtheta"][:3])
    assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-14)
    assert abs(lhs) > 1e-6


# ---------------------------------------------------------------------------
# Sec. 3.3 analytic gradient vs FP64 central finite differences on tiny inputs.
# Catches: any error in the seeds, the reverse sweep, the Jacobian term, the
# tap distribution or the chain through Eq. 2.
# ---------------------------------------------------------------------------

def _fd_window(seed, refs, n=40, W=16, H=14, f=12.0, eps=1e-9):
    """Real-valued events, seeded; re-drawn until no visited position lies within
    1e-3 px of a tap boundary or the image border (the loss is smooth there)."""
    for s in range(seed, seed + 200):
        rng = np.random.default_rng(s)
        x = rng.uniform(2, W - 3, n)
        y = rng.uniform(2, H - 3, n)
        t = rng.random(n)
        p = np.where(rng.random(n) < 0.5, 1, -1)
        xs, ys = np.meshgrid(np.arange(W), np.arange(H))
        rho = 0.7 + 0.5 * np.exp(-((xs - rng.uniform(0, W)) ** 2 + (ys - rng.uniform(0, H)) ** 2)
                                 / 20.0)
        theta = rng.normal(0, 0.12, 6)
        win = mkwin(W, H, f, refs, x, y, t, p, rho, theta, eps=eps)
        res = oracle.forward(win, positions=True, valid=True)
        if res["valid"].sum() < n // 2:
            continue
        P = res["positions"][res["valid"]]
        frac = np.abs(P - np.rint(P))
        border = np.minimum(P, np.array([W - 1, H - 1]) - P)
        if frac.min() > 1e-3 and border.min() > 1e-3 and \
                np.abs(np.stack([x, y], 1) - np.rint(np.stack([x, y], 1))).min() > 1e-3:
            return win
    raise RuntimeError("no smooth seed found")


@pytest.mark.parametrize("refs", [[0.0, 0.4, 1.0], [1.0], [0.1, 0.3, 0.55, 0.6, 0.9]])
def test_gradient_matches_central_differences(refs):
    win = _fd_window(100 + len(refs), refs)
    g = oracle.backward(win, grad_loss=1.0)
    h = 1e-6

    def L(rho=None, theta=None):
        return oracle.loss(win, rho=rho, theta=theta)

    fd_th = np.zeros(6)
    for k in range(6):
        tp = win.theta.copy(); tp[k] += h
        tm = win.theta.copy(); tm[k] -= h
        fd_th[k] = (L(theta=tp) - L(theta=tm)) / (2 * h)
    scale_th = np.abs(fd_th).max()
    assert scale_th > 1e-4
    np.testing.assert_allclose(g["dtheta"], fd_th, atol=1e-6 * scale_th)

    fd_rho = np.zeros_like(win.rho)
    for j in range(win.height):
        for i in range(win.width):
            rp = win.rho.copy(); rp[j, i] += h
            rm = win.rho.copy(); rm[j, i] -= h
            fd_rho[j, i] = (L(rho=rp) - L(rho=rm)) / (2 * h)
    scale = np.abs(fd_rho).max()
    assert scale > 1e-5
    np.testing.assert_allclose(g["drho"], fd_rho, atol=1e-6 * scale)


def test_grad_loss_scales_linearly():
    win = _fd_window(300, [0.0, 0.5, 1.0])
    g1 = oracle.backward(win, grad_loss=1.0)
    g3 = oracle.backward(win, grad_loss=-3.0)
    np.testing.assert_allclose(g3["drho"], -3.0 * g1["drho"], rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(g3["dtheta"], -3.0 * g1["dtheta"], rtol=1e-13)


def test_rotation_only_has_no_depth_gradient():
    win = _generic()
    win = win.replace(theta=np.concatenate([np.zeros(3), win.theta[3:]]))
    g = oracle.backward(win)
    assert not g["drho"].any()
    assert np.abs(g["dtheta"]).max() > 0


def test_single_ref_depth_gradient_support_is_event_pixels():
    # one reference: one warp step from the (integer) event position, so the
    # flow is sampled only at event pixels with weight one
    rng = np.random.default_rng(8)
    W, H, n = 20, 16, 60
    x = rng.integers(0, W, n).astype(np.float64)
    y = rng.integers(0, H, n).astype(np.float64)
    t = rng.random(n) * 0.9
    win = mkwin(W, H, 10.0, [1.0], x, y, t, np.ones(n), np.full((H, W), 0.9),
                rng.normal(0, 0.1, 6))
    res = oracle.forward(win, valid=True)
    g = oracle.backward(win)
    support = np.zeros((H, W), bool)
    ok = res["valid"]
    support[y[ok].astype(int), x[ok].astype(int)] = True
    assert not g["drho"][~support].any()
    assert np.count_nonzero(g["drho"]) > 0


# ---------------------------------------------------------------------------
# Eq. 1's regulariser (Sec. 3.1): where eps sits.  The paper gives no value;
# the reading is eps in the per-pixel ratio S/(C+eps) and in the active-pixel
# normaliser N_r+eps.  At eps = 1e-9 a misplaced eps moves the loss by less
# than 1e-8 relative, so these pins take eps = 0.25 (loss) and 0.05 (gradient),
# where every placement gives a visibly different number.
# Catches: eps dropped from N_r, eps dropped from (or added outside) the
# ratio, (C+eps)^2 or (C+eps)^3 written as C^2 / C^3 in the adjoint seeds.
# ---------------------------------------------------------------------------

def _static_eps(x, y, t, p, eps, refs=REFS3, W=40, H=30):
    return mkwin(W, H, 10.0, refs, x, y, t, p, np.ones((H, W)), np.zeros(6), eps=eps)


def _bilinear_weights(X, Y):
    a, b = X - math.floor(X), Y - math.floor(Y)
    return np.array([(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b])


def test_eps_single_event_closed_form():
    eps = 0.25
    X, Y, tk = 10.3, 20.6, 0.25
    w = _bilinear_weights(X, Y)
    res = oracle.forward(_static_eps([X], [Y], [tk], [1], eps))
    assert list(res["nact"]) == [4.0, 4.0, 4.0]
    per_ref = []
    for r in REFS3:
        tb = tbar(r, tk)
        per_ref.append(np.sum((tb * w / (w + eps)) ** 2) / (4.0 + eps))
        # the numerator alone: sum over the four taps of (tbar w / (w + eps))^2
    np.testing.assert_allclose(res["num"], [np.sum((tbar(r, tk) * w / (w + eps)) ** 2)
                                            for r in REFS3], rtol=1e-13)
    assert res["loss"] == pytest.approx(np.mean(per_ref), rel=1e-13)
    # on an integer pixel: one active pixel, weight 1
    res = oracle.forward(_static_eps([7.0], [3.0], [0.75], [-1], eps))
    assert list(res["nact"]) == [1.0, 1.0, 1.0]
    expect = np.mean([(tbar(r, 0.75) / (1.0 + eps)) ** 2 / (1.0 + eps) for r in REFS3])
    assert res["loss"] == pytest.approx(expect, rel=1e-13)


def test_eps_two_coincident_events_closed_form():
    eps = 0.25
    X, Y, t1, t2 = 10.3, 20.6, 0.1, 0.7
    w = _bilinear_weights(X, Y)
    same = oracle.loss(_static_eps([X, X], [Y, Y], [t1, t2], [1, 1], eps))
    expect = np.mean([np.sum((w * (tbar(r, t1) + tbar(r, t2)) / (2 * w + eps)) ** 2) / (4 + eps)
                      for r in REFS3])
    assert same == pytest.approx(expect, rel=1e-13)
    opp = oracle.loss(_static_eps([X, X], [Y, Y], [t1, t2], [1, -1], eps))
    expect = np.mean([np.sum((tbar(r, t1) * w / (w + eps)) ** 2
                             + (tbar(r, t2) * w / (w + eps)) ** 2) / (4 + eps) for r in REFS3])
    assert opp == pytest.approx(expect, rel=1e-13)


def test_eps_moves_the_loss_as_the_reading_says():
    # the same window at eps = 1e-9 and 0.25: the loss follows the closed form
    # at both, and the two differ by far more than rounding
    X, Y, tk = 10.3, 20.6, 0.25
    w = _bilinear_weights(X, Y)
    for eps in (1e-9, 1e-3, 0.25, 2.0):
        e = float(np.float32(eps))       # the descriptor holds eps in FP32
        L = oracle.loss(_static_eps([X], [Y], [tk], [1], eps))
        expect = np.mean([np.sum((tbar(r, tk) * w / (w + e)) ** 2) / (4 + e) for r in REFS3])
        assert L == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("refs", [[0.0, 0.4, 1.0], [0.1, 0.3, 0.55, 0.6, 0.9]])
def test_eps_gradient_matches_central_differences(refs):
    # with a large eps the seeds' (C+eps)^2 and (C+eps)^3 differ from C^2, C^3
    # by ~10 % at the typical C of these windows
    win = _fd_window(500 + len(refs), refs, eps=0.05)
    g = oracle.backward(win, grad_loss=1.0)
    h = 1e-6

    def L(rho=None, theta=None):
        return oracle.loss(win, rho=rho, theta=theta)

    fd_th = np.zeros(6)
    for k in range(6):
        tp = win.theta.copy(); tp[k] += h
        tm = win.theta.copy(); tm[k] -= h
        fd_th[k] = (L(theta=tp) - L(theta=tm)) / (2 * h)
    scale_th = np.abs(fd_th).max()
    assert scale_th > 1e-4
    np.testing.assert_allclose(g["dtheta"], fd_th, atol=1e-6 * scale_th)

    fd_rho = np.zeros_like(win.rho)
    for j in range(win.height):
        for i in range(win.width):
            rp = win.rho.copy(); rp[j, i] += h
            rm = win.rho.copy(); rm[j, i] -= h
            fd_rho[j, i] = (L(rho=rp) - L(rho=rm)) / (2 * h)
    scale = np.abs(fd_rho).max()
    assert scale > 1e-5
    np.testing.assert_allclose(g["drho"], fd_rho, atol=1e-6 * scale)

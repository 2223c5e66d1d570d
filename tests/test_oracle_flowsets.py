"""Pins for the oracle's flow sets: one flow per segment between consecutive
knots {0, 1} U refs, each from its own inverse depth and ego-motion (Sec. 3.1:
flows of consecutive slices are concatenated, Delta x_k = sum_i (Delta t_i u_i)).

Each test states the mistake it is there to catch.
"""

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import mkwin


def knots_of(refs):
    k = list(refs)
    if k[0] > 0.0:
        k = [0.0] + k
    if k[-1] < 1.0:
        k = k + [1.0]
    return np.asarray(k)


def _sets(win, F):
    return win.replace(rho=np.repeat(win.rho[None], F, axis=0),
                       theta=np.repeat(win.theta[None], F, axis=0))


def _generic(seed, refs, n=200, W=26, H=20, f=15.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, W - 1, n)
    y = rng.uniform(0, H - 1, n)
    t = rng.random(n)
    t[:3] = [refs[0], refs[-1], refs[len(refs) // 2]]     # events on knots too
    p = np.where(rng.random(n) < 0.5, 1, -1)
    xs, ys = np.meshgrid(np.arange(W), np.arange(H))
    rho = 0.6 + 0.6 * np.exp(-((xs - W / 3) ** 2 + (ys - H / 2) ** 2) / 30.0)
    theta = rng.normal(0, 0.25, 6)
    return mkwin(W, H, f, refs, x, y, t, p, rho, theta)


# ---------------------------------------------------------------------------
# Identical flow sets reduce to the single flow.  Catches: a set index that
# picks the wrong array, gradients sent to the wrong set or double-counted.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("refs", [[0.0, 0.25, 0.5, 1.0], [0.2, 0.6], [0.0, 0.7], [0.35]])
def test_identical_sets_equal_single_flow(refs):
    win = _generic(3, refs)
    F = len(knots_of(refs)) - 1
    one = oracle.forward(win, images=True)
    many = oracle.forward(_sets(win, F), images=True)
    assert many["loss"] == one["loss"]
    np.testing.assert_array_equal(many["images"], one["images"])
    g1 = oracle.backward(win)
    gF = oracle.backward(_sets(win, F))
    assert gF["drho"].shape == (F, win.height, win.width) and gF["dtheta"].shape == (F, 6)
    np.testing.assert_allclose(gF["drho"].sum(0), g1["drho"], rtol=0,
                               atol=1e-12 * np.abs(g1["drho"]).max())
    np.testing.assert_allclose(gF["dtheta"].sum(0), g1["dtheta"], rtol=0,
                               atol=1e-12 * np.abs(g1["dtheta"]).max())


# ---------------------------------------------------------------------------
# Piecewise-constant flow in time: with a uniform flow per segment the warped
# position is x_k plus the integral of the flow from t_k to the reference time,
# i.e. sum_i Delta t_i u_i over the segments crossed.  Catches: the wrong
# segment for a forward or backward step, for steps starting exactly on a knot,
# or for the outer segments [0, first ref] and [last ref, 1].
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("refs", [[0.0, 0.25, 0.5, 1.0], [0.2, 0.6], [0.1, 0.45, 0.5, 0.9]])
def test_piecewise_constant_flow_positions(refs):
    rng = np.random.default_rng(8)
    W, H, f, rho0 = 200, 160, 20.0, 0.5
    K = knots_of(refs)
    F = len(K) - 1
    v = rng.uniform(-1.5, 1.5, (F, 2))
    theta = np.zeros((F, 6))
    theta[:, :2] = v
    u = f * rho0 * v                                 # uniform flow of each segment
    n = 400
    x = rng.uniform(60, 140, n)
    y = rng.uniform(50, 110, n)
    t = rng.random(n)
    t[:len(K)] = K                                   # events exactly on every knot
    win = mkwin(W, H, f, refs, x, y, t, np.ones(n), np.full((F, H, W), rho0), theta)
    res = oracle.forward(win, valid=True, positions=True)
    assert res["valid"].all()

    def integral(a, b):
        """Integral of the piecewise-constant flow from time a to time b."""
        lo, hi, sgn = (a, b, 1.0) if b >= a else (b, a, -1.0)
        acc = np.zeros(2)
        for s in range(F):
            d = min(hi, K[s + 1]) - max(lo, K[s])
            if d > 0:
                acc += d * u[s]
        return sgn * acc

    for k in range(n):
        for r, ref in enumerate(refs):
            want = np.array([x[k], y[k]]) + integral(t[k], ref)
            np.testing.assert_allclose(res["positions"][k, r], want, rtol=0, atol=1e-11)


# ---------------------------------------------------------------------------
# A segment no event step crosses has no influence and no gradient.
# Catches: gradients accumulated into a set that the forward never sampled.
# ---------------------------------------------------------------------------

def test_unused_set_has_no_influence_and_no_gradient():
    win = _generic(4, [0.5, 1.0])
    win = win.replace(t=0.5 + 0.5 * np.asarray(win.t))          # all events in [0.5, 1]
    rng = np.random.default_rng(1)
    rho = np.stack([win.rho * 1.7, win.rho])
    theta = np.stack([rng.normal(0, 0.4, 6), win.theta])
    wF = win.replace(rho=rho, theta=theta)
    base = oracle.loss(wF)
    w2 = wF.replace(rho=np.stack([win.rho * 0.3, win.rho]),
                    theta=np.stack([rng.normal(0, 0.4, 6), win.theta]))
    assert oracle.loss(w2) == base
    assert oracle.loss(win) == base                 # set 1 alone is the single flow
    g = oracle.backward(wF)
    assert not g["drho"][0].any() and not g["dtheta"][0].any()
    assert np.abs(g["dtheta"][1]).max() > 0


# ---------------------------------------------------------------------------
# Finite differences through every flow set.  Catches: a dropped or misrouted
# adjoint term between segments (the Jacobian of a later step taken with the
# wrong set's flow), a wrong chain through Eq. 2 for one set.
# ---------------------------------------------------------------------------

def _fd_sets_window(seed, refs, n=40, W=16, H=14, f=12.0):
    F = len(knots_of(refs)) - 1
    for s in range(seed, seed + 300):
        rng = np.random.default_rng(s)
        x = rng.uniform(2, W - 3, n)
        y = rng.uniform(2, H - 3, n)
        t = rng.random(n)
        p = np.where(rng.random(n) < 0.5, 1, -1)
        xs, ys = np.meshgrid(np.arange(W), np.arange(H))
        rho = np.stack([0.7 + 0.5 * np.exp(-((xs - rng.uniform(0, W)) ** 2
                                               + (ys - rng.uniform(0, H)) ** 2) / 20.0)
                        for _ in range(F)])
        theta = rng.normal(0, 0.12, (F, 6))
        win = mkwin(W, H, f, refs, x, y, t, p, rho, theta)
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


@pytest.mark.parametrize("refs", [[0.0, 0.5, 1.0], [0.15, 0.4, 0.8]])
def test_flow_set_gradients_match_central_differences(refs):
    win = _fd_sets_window(500 + len(refs), refs)
    F = win.rho.shape[0]
    g = oracle.backward(win)
    h = 1e-6
    L = lambda **kw: oracle.loss(win, **kw)
    for s in range(F):
        fd_th = np.zeros(6)
        for k in range(6):
            tp = win.theta.copy(); tp[s, k] += h
            tm = win.theta.copy(); tm[s, k] -= h
            fd_th[k] = (L(theta=tp) - L(theta=tm)) / (2 * h)
        scale = np.abs(fd_th).max()
        assert scale > 1e-5, s
        np.testing.assert_allclose(g["dtheta"][s], fd_th, atol=1e-6 * scale)
        fd_rho = np.zeros(win.rho.shape[1:])
        for j in range(win.height):
            for i in range(win.width):
                rp = win.rho.copy(); rp[s, j, i] += h
                rm = win.rho.copy(); rm[s, j, i] -= h
                fd_rho[j, i] = (L(rho=rp) - L(rho=rm)) / (2 * h)
        scale = np.abs(fd_rho).max()
        assert scale > 1e-6, s
        np.testing.assert_allclose(g["drho"][s], fd_rho, atol=1e-6 * scale)


def test_flow_set_count_must_match_segments():
    win = _generic(5, [0.0, 1.0])
    with pytest.raises(ValueError):
        oracle.forward(_sets(win, 2))
    win = _generic(5, [0.2, 0.6])                   # knots 0, .2, .6, 1: three segments
    with pytest.raises(ValueError):
        oracle.forward(_sets(win, 2))
    oracle.forward(_sets(win, 3))

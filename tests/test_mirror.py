"""The canonical-order mirror of the deterministic mode computes the same loss
and gradient as the FP64 oracle (within the parity tolerance): it only fixes
the order of the additions, not what is added."""

import numpy as np
import pytest

import eventgen
import oracle
from tests.helpers import assert_grads_close, assert_loss_close


@pytest.mark.parametrize("case", ["c1", "edge3", "edge8", "ragged", "c1/sub", "edge3/sub",
                                  "edge3 eps=0.25", "c1/sub eps=1e-3"])
def test_mirror_agrees_with_oracle(case):
    if case == "c1":
        win = eventgen.make_window("c1")
    elif case == "c1/sub":
        win = eventgen.make_window("c1", subpixel=True)
    elif case == "edge3/sub":
        win = eventgen.edge_window(31, "346x260", 6000, refs=[0.0, 0.5, 1.0], n_segments=20,
                                   subpixel=True)
    elif case == "edge3 eps=0.25":
        win = eventgen.edge_window(31, "346x260", 6000, refs=[0.0, 0.5, 1.0],
                                   n_segments=20).replace(eps=0.25)
    elif case == "c1/sub eps=1e-3":
        win = eventgen.make_window("c1", subpixel=True).replace(eps=1e-3)
    elif case == "edge3":
        win = eventgen.edge_window(31, "346x260", 6000, refs=[0.0, 0.5, 1.0], n_segments=20)
    elif case == "edge8":
        win = eventgen.edge_window(32, "346x260", 3000, refs=list(eventgen.refs_even(8)),
                                   n_segments=10, motion_sigma=0.3)
    else:
        win = eventgen.edge_window(33, "346x260", 130, refs=[0.2, 0.7], n_segments=3)
    m = oracle.mirror_forward(win)
    o = oracle.forward(win, valid=True)
    assert m["n_valid"] == int(o["valid"].sum())
    np.testing.assert_array_equal(m["nact"], o["nact"])
    assert_loss_close(float(m["loss64"]), o["loss"], rtol=1e-12, what=case)
    mb = oracle.mirror_backward(win, grad_loss=1.5)
    ob = oracle.backward(win, grad_loss=1.5)
    assert_grads_close(mb["drho"], mb["dtheta"], ob["drho"], ob["dtheta"], rtol=1e-5, what=case)


def test_mirror_empty_window():
    win = eventgen.make_window("c1")
    e = np.zeros(0, np.float32)
    win = win.replace(x=e, y=e, t=e, p=np.zeros(0, np.int8))
    assert oracle.mirror_forward(win)["loss"] == 0.0
    mb = oracle.mirror_backward(win)
    assert not mb["drho"].any() and not mb["dtheta"].any()


@pytest.mark.parametrize("refs", [[0.0, 0.25, 0.5, 0.75, 1.0], [0.15, 0.5, 0.85]])
def test_mirror_agrees_with_oracle_flow_sets(refs):
    """One flow per segment: the mirror routes steps and gradients to the same
    sets as the oracle."""
    win = eventgen.edge_window(34, "346x260", 4000, refs=refs, n_segments=12, motion_sigma=0.3)
    win = eventgen.with_flow_sets(win, 35)
    F = win.rho.shape[0]
    assert F == len(eventgen.knots_of(refs)) - 1
    m = oracle.mirror_forward(win)
    o = oracle.forward(win, valid=True)
    assert m["n_valid"] == int(o["valid"].sum())
    np.testing.assert_array_equal(m["nact"], o["nact"])
    assert_loss_close(float(m["loss64"]), o["loss"], rtol=1e-12, what="sets")
    mb = oracle.mirror_backward(win, grad_loss=0.7)
    ob = oracle.backward(win, grad_loss=0.7)
    assert mb["drho"].shape == (F, win.height, win.width) and mb["dtheta"].shape == (F, 6)
    for f in range(F):
        assert_grads_close(mb["drho"][f], mb["dtheta"][f], ob["drho"][f], ob["dtheta"][f],
                           rtol=1e-5, what=f"set {f}")


def test_c6_window_shape():
    win = eventgen.make_window("c6", 3)
    assert win.rho.shape == (10, win.height, win.width) and win.theta.shape == (10, 6)
    assert len(win.refs) == 11 and 10_000 <= win.n <= 100_000


@pytest.mark.parametrize("sets", [False, True])
def test_mirror_agrees_with_oracle_exact_flow(sets):
    """Exact reprojection (Eq. 2 without the first-order expansion): the
    mirror's rotation series, reprojection and chain agree with the oracle's
    Rodrigues formula and adjoint."""
    refs = [0.0, 0.3, 0.6, 1.0] if sets else [0.1, 0.5, 0.9]
    win = eventgen.edge_window(36, "346x260", 3000, refs=refs, n_segments=12, motion_sigma=0.3)
    if sets:
        win = eventgen.with_flow_sets(win, 37)
    win = win.replace(flow_model=1)
    m = oracle.mirror_forward(win)
    o = oracle.forward(win, valid=True)
    assert m["n_valid"] == int(o["valid"].sum()) and m["n_valid"] > 1000
    np.testing.assert_array_equal(m["nact"], o["nact"])
    assert_loss_close(float(m["loss64"]), o["loss"], rtol=1e-12, what="exact")
    # the first-order loss differs: the model switch is live
    assert abs(oracle.loss(win.replace(flow_model=0)) - o["loss"]) > 1e-6 * abs(o["loss"])
    mb = oracle.mirror_backward(win, grad_loss=1.3)
    ob = oracle.backward(win, grad_loss=1.3)
    F = win.rho.shape[0] if win.rho.ndim == 3 else 1
    drm, dtm = mb["drho"].reshape(F, -1), mb["dtheta"].reshape(F, 6)
    dro, dto = ob["drho"].reshape(F, -1), ob["dtheta"].reshape(F, 6)
    for f in range(F):
        assert_grads_close(drm[f], dtm[f], dro[f], dto[f], rtol=1e-5, what=f"exact set {f}")

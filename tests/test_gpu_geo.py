"""GPU: geometry-consistency loss between consecutive flow sets (Eq. 3) and
the full loss L = L_CM + lambda L_geo (Eq. 4), through the C ABI, against the
FP64 oracle."""

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import assert_grads_close, assert_loss_close, to_device
from tests.test_gpu_batch import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


def sets_window(seed, n, refs, sensor="346x260"):
    w = eventgen.edge_window(seed, sensor, n, refs=refs, n_segments=20, motion_sigma=0.3,
                             name=f"geo{seed}")
    return eventgen.with_flow_sets(w, seed + 1)


def run_geo(cm, win, mode=0, lam=1.0):
    """L_geo and lam * its gradient alone (gradient buffers start at zero)."""
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=mode)
    print(f"[gpu] geo {win.name} F={desc.F} mode={mode}", flush=True)
    lg, _, st = cm.geo_forward(desc, d["rho"], d["ego"], lam)
    g_rho = torch.zeros_like(d["rho"])
    g_ego = torch.zeros_like(d["ego"])
    cm.geo_backward(desc, d["rho"], d["ego"], st, torch.ones(1, device="cuda:0"), g_rho, g_ego,
                    lam)
    torch.cuda.synchronize()
    return float(lg.item()), g_rho.cpu().numpy(), g_ego.cpu().numpy()


def check_geo(win, lg, g_rho, g_ego, what, lam=1.0):
    o = oracle.geo(win, grad=True, grad_loss=lam)
    assert o["loss"] > 1e-3
    assert_loss_close(lg, o["loss"], what=what)
    F = win.rho.shape[0]
    g_rho = np.asarray(g_rho, np.float64).reshape(F, -1)
    g_ego = np.asarray(g_ego, np.float64).reshape(F, 6)
    o_rho = o["drho"].reshape(F, -1)
    for f in range(F):
        if f < F - 1:
            assert_grads_close(g_rho[f], g_ego[f], o_rho[f], o["dtheta"][f], what=f"{what} set {f}")
        else:   # the last set has no pose in any pair
            assert not g_ego[f].any()
            assert np.linalg.norm(g_rho[f] - o_rho[f]) <= 1e-4 * np.linalg.norm(o_rho[f])


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("refs", [[0.0, 0.5, 1.0], [0.15, 0.4, 0.8], list(np.linspace(0, 1, 11))])
def test_geo_matches_oracle(cm, refs, mode):
    win = sets_window(900 + len(refs), 2000, refs)
    check_geo(win, *run_geo(cm, win, mode), what=f"geo R={len(refs)} mode={mode}")


def test_geo_c6_window_and_lambda(cm):
    win = eventgen.make_window("c6", 2)
    lg, g_rho, g_ego = run_geo(cm, win, lam=0.05)
    check_geo(win, lg, g_rho, g_ego, what="c6 geo", lam=0.05)


def test_geo_zero_motion_equal_depths_is_exactly_zero(cm):
    """Zero motion maps every pixel onto itself (no rounding): L_geo = 0 and
    a zero gradient when consecutive depths are equal."""
    win = sets_window(910, 1000, [0.0, 0.5, 1.0])
    rho = np.repeat(np.asarray(win.rho[:1]), 2, 0)
    win = win.replace(rho=rho, theta=np.zeros((2, 6), np.float32))
    lg, g_rho, g_ego = run_geo(cm, win)
    assert lg == 0.0 and not g_rho.any() and not g_ego.any()
    assert oracle.geo(win)["pairs"][0, 1] == win.width * win.height


def test_geo_invalid_depths(cm):
    """Non-positive inverse depths leave V on the GPU as in the oracle."""
    win = sets_window(911, 1000, [0.0, 0.5, 1.0])
    rho = np.array(win.rho, np.float32)
    rho[0, 40:60, 100:180] = 0.0
    rho[1, 100:104, 10:300] = -1.0
    win = win.replace(rho=rho)
    lg, g_rho, g_ego = run_geo(cm, win)
    assert np.all(np.isfinite(g_rho)) and np.all(np.isfinite(g_ego))
    check_geo(win, lg, g_rho, g_ego, what="invalid depths")


def test_geo_deterministic_bitwise(cm):
    win = eventgen.make_window("c6", 3)
    a = run_geo(cm, win, mode=cm.CM_MODE_DETERMINISTIC)
    b = run_geo(cm, win, mode=cm.CM_MODE_DETERMINISTIC)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_geo_state_bytes_and_bad_args(cm):
    win = sets_window(912, 100, [0.0, 0.5, 1.0])
    desc = cm.WindowDesc.from_window(win)
    assert cm.geo_state_bytes(desc) > 0
    d = to_device(win)
    with pytest.raises(cm.CMError):
        cm.geo_forward(desc, d["rho"], d["ego"], float("nan"))


@pytest.mark.parametrize("mode", [0, 1])
def test_full_loss_autograd_matches_oracle(cm, mode):
    win = sets_window(920, 20000, [0.0, 0.3, 0.6, 1.0])
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=mode)
    rho = d["rho"].clone().requires_grad_(True)
    ego = d["ego"].clone().requires_grad_(True)
    L = cm.full_loss(d["x"], d["y"], d["t"], d["p"], rho, ego, desc)
    L.backward()
    assert_loss_close(L.item(), oracle.full_loss(win), what="full loss")
    o = oracle.full_backward(win)
    F = win.rho.shape[0]
    gr = rho.grad.cpu().numpy().reshape(F, -1).astype(np.float64)
    ge = ego.grad.cpu().numpy().reshape(F, 6).astype(np.float64)
    for f in range(F):
        assert_grads_close(gr[f], ge[f], o["drho"][f].ravel(), o["dtheta"][f], what=f"full set {f}")


def test_full_loss_batch(cm):
    """A batch mixing flow-set windows and a one-flow window (L_geo = 0): the
    per-window full losses and gradients match the oracle."""
    wins = [eventgen.make_window("c6", 4), sets_window(930, 5000, [0.2, 0.6]),
            eventgen.edge_window(931, "346x260", 3000, refs=[0.0, 0.5, 1.0], n_segments=20),
            sets_window(932, 3000, [0.0, 0.5, 1.0], sensor="640x480")]
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    batch = cm.Batch(descs, [w.n for w in wins])
    d = pack(wins)
    rho = d["rho"].clone().requires_grad_(True)
    ego = d["ego"].clone().requires_grad_(True)
    L = cm.BatchFullLoss.apply(d["x"], d["y"], d["t"], d["p"], rho, ego, batch, 0.05)
    L.sum().backward()
    L = L.detach().cpu().numpy()
    gr = rho.grad.cpu().numpy()
    ge = ego.grad.cpu().numpy()
    for w, win in enumerate(wins):
        assert_loss_close(float(L[w]), oracle.full_loss(win), what=f"batch full {w}")
        o = oracle.full_backward(win)
        F = 1 if np.ndim(win.rho) == 2 else win.rho.shape[0]
        pr = gr[batch.pixel_offsets[w]:batch.pixel_offsets[w + 1]].reshape(F, -1)
        pe = ge[6 * batch.set_offsets[w]:6 * batch.set_offsets[w + 1]].reshape(F, 6)
        o_r, o_e = o["drho"].reshape(F, -1), o["dtheta"].reshape(F, 6)
        for f in range(F):
            assert_grads_close(pr[f], pe[f], o_r[f], o_e[f], what=f"batch full {w} set {f}")
    assert oracle.geo(wins[2])["loss"] == 0.0

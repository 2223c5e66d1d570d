"""GPU: the exact-reprojection flow (Eq. 2 without the first-order expansion:
back-projection with depth 1/rho, rigid motion by Rodrigues' rotation and
translation, projection), through the C ABI, against the FP64 oracle and, in
the deterministic mode, the canonical-order mirror bit for bit."""

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import assert_grads_close, assert_loss_close, to_device
from tests.test_gpu_batch import pack
from tests.test_gpu_flowsets import check_oracle, run_single

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


def exact_window(seed, n, refs, sets=False, sigma=0.25, sensor="346x260"):
    w = eventgen.edge_window(seed, sensor, n, refs=refs, n_segments=20, motion_sigma=sigma,
                             name=f"ex{seed}")
    if sets:
        w = eventgen.with_flow_sets(w, seed + 1)
    return w.replace(flow_model=1)


def check(win, loss, g_rho, g_ego, what):
    if np.ndim(win.rho) == 3:
        check_oracle(win, loss, g_rho, g_ego, what)
        return
    o = oracle.forward(win)
    assert_loss_close(float(loss[0]), o["loss"], what=what)
    ob = oracle.backward(win)
    assert_grads_close(g_rho, g_ego, ob["drho"], ob["dtheta"], what=what)


@pytest.mark.parametrize("path", ["direct", "tiled"])
@pytest.mark.parametrize("refs,n,sets", [([0.0, 0.5, 1.0], 3000, False),
                                         ([0.2, 0.6], 257, False),
                                         (list(np.linspace(0, 1, 8)), 30000, False),
                                         ([0.0, 0.5, 1.0], 5000, True),
                                         ([0.1, 0.3, 0.31, 0.9], 20000, True)])
def test_exact_flow_matches_oracle(cm, path, refs, n, sets):
    cm.set_path(0, cm.CM_PATH_DIRECT if path == "direct" else cm.CM_PATH_TILED)
    try:
        win = exact_window(800 + n % 89, n, refs, sets)
        check(win, *run_single(cm, win), what=f"exact {path} R={len(refs)} sets={sets}")
    finally:
        cm.set_path(0, cm.CM_PATH_AUTO)


def test_exact_flow_differs_from_first_order(cm):
    """The descriptor's flow model reaches the kernels: the two models give
    different losses on a window with large motion."""
    win = exact_window(810, 20000, [0.0, 0.5, 1.0])
    le = run_single(cm, win)[0][0]
    l1 = run_single(cm, win.replace(flow_model=0))[0][0]
    assert abs(le - oracle.loss(win)) <= 1e-5 * abs(oracle.loss(win))
    assert abs(l1 - oracle.loss(win.replace(flow_model=0))) <= 1e-5 * abs(l1)
    assert abs(le - l1) > 1e-4 * abs(l1)


def test_points_behind_the_camera(cm):
    """A forward motion that pushes near points behind the camera plane: those
    pixels have zero flow and zero d rho on the GPU as in the oracle."""
    base = eventgen.edge_window(811, "346x260", 20000, refs=[0.0, 0.5, 1.0], n_segments=20)
    rho = np.asarray(base.rho, np.float64).copy()
    rho[:, 200:] = 4.0                                  # near points on the right
    theta = np.array([0.0, 0.0, -0.3, 0.0, 0.0, 0.0])   # p_z = 1 - 0.3 rho
    win = base.replace(rho=rho.astype(np.float32), theta=theta.astype(np.float32), flow_model=1)
    for path in (cm.CM_PATH_DIRECT, cm.CM_PATH_TILED):
        cm.set_path(0, path)
        try:
            loss, g_rho, g_ego = run_single(cm, win)
        finally:
            cm.set_path(0, cm.CM_PATH_AUTO)
        check(win, loss, g_rho, g_ego, what=f"behind path={path}")
        assert not g_rho.reshape(win.height, win.width)[:, 201:].any()


@pytest.mark.parametrize("sets", [False, True])
def test_exact_deterministic_matches_mirror_bitwise(cm, sets):
    refs = [0.0, 0.3, 0.6, 1.0] if sets else [0.1, 0.5, 0.9]
    win = exact_window(820 + sets, 30000, refs, sets)
    a = run_single(cm, win, mode=cm.CM_MODE_DETERMINISTIC)
    b = run_single(cm, win, mode=cm.CM_MODE_DETERMINISTIC)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    m = oracle.mirror_forward(win)
    assert a[0][0] == m["loss"]
    mb = oracle.mirror_backward(win)
    assert np.array_equal(a[1].reshape(mb["drho"].shape), mb["drho"])
    assert np.array_equal(a[2].reshape(mb["dtheta"].shape), mb["dtheta"])


def test_exact_batch(cm):
    """A batch of exact-flow windows (one and several flow sets): each window
    matches the oracle; a batch that mixes flow models is rejected."""
    wins = [exact_window(830, 5000, [0.0, 0.5, 1.0]),
            exact_window(831, 40000, list(np.linspace(0, 1, 6)), sets=True),
            exact_window(832, 900, [0.3, 0.6], sensor="640x480")]
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    batch = cm.Batch(descs, [w.n for w in wins])
    d = pack(wins)
    print(f"[gpu] exact batch sets={batch.set_offsets[-1]}", flush=True)
    loss, state = batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                                  torch.ones(batch.n, device="cuda:0"))
    torch.cuda.synchronize()
    loss, g_rho, g_ego = loss.cpu().numpy(), g_rho.cpu().numpy(), g_ego.cpu().numpy()
    for w, win in enumerate(wins):
        pr = g_rho[batch.pixel_offsets[w]:batch.pixel_offsets[w + 1]]
        pe = g_ego[6 * batch.set_offsets[w]:6 * batch.set_offsets[w + 1]]
        check(win, loss[w:w + 1], pr, pe, what=f"batch {win.name}")
    mixed = descs[:1] + [cm.WindowDesc.from_window(wins[2].replace(flow_model=0))]
    with pytest.raises(cm.CMError):
        cm.Batch(mixed, [wins[0].n, wins[2].n])


def test_exact_autograd(cm):
    win = exact_window(840, 10000, [0.0, 0.5, 1.0], sets=True)
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win)
    assert desc.flow_model == cm.CM_FLOW_EXACT
    rho = d["rho"].clone().requires_grad_(True)
    ego = d["ego"].clone().requires_grad_(True)
    L = cm.cm_loss(d["x"], d["y"], d["t"], d["p"], rho, ego, desc)
    L.backward()
    check(win, np.array([L.item()]), rho.grad.cpu().numpy(), ego.grad.cpu().numpy(),
          what="exact autograd")

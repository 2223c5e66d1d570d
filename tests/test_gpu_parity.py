"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: loss within 1e-5 relative; d rho within 1e-4 relative in L2 norm
(and 1e-3 of the largest entry elementwise); d theta within 1e-4 of its largest
component; event counts and active-pixel counts exact.
"""

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import assert_grads_close, assert_loss_close, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["direct", "tiled"])
def cm(request):
    """The binding, with the handle's kernel path forced to each of the two."""
    import paper_2412_06359_amd as cm
    cm.load()                       # raises if the HIP library is missing
    assert torch.cuda.is_available()
    cm.set_path(0, cm.CM_PATH_DIRECT if request.param == "direct" else cm.CM_PATH_TILED)
    print(f"[gpu] path={request.param}", flush=True)
    yield cm
    cm.set_path(0, cm.CM_PATH_AUTO)


def run_gpu(cm, win, grad=True, grad_out=1.0):
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win)
    print(f"[gpu] {win.name} {win.width}x{win.height} n={win.n} R={len(win.refs)}", flush=True)
    rho = d["rho"].clone().requires_grad_(grad)
    ego = d["ego"].clone().requires_grad_(grad)
    L = cm.cm_loss(d["x"], d["y"], d["t"], d["p"], rho, ego, desc)
    out = dict(loss=float(L.item()))
    if grad:
        (L * grad_out).backward()
        out["drho"] = rho.grad.double().cpu().numpy()
        out["dtheta"] = ego.grad.double().cpu().numpy()
    return out


def check_window(cm, win, grad=True, what=""):
    g = run_gpu(cm, win, grad)
    o = oracle.forward(win, valid=True)
    assert_loss_close(g["loss"], o["loss"], what=what)
    if grad:
        ob = oracle.backward(win)
        assert_grads_close(g["drho"], g["dtheta"], ob["drho"], ob["dtheta"], what=what)
    return g, o


def test_c1_forward_and_sums(cm):
    win = eventgen.make_window("c1")
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win)
    loss, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    diag = cm.diagnostics(desc, state)
    o = oracle.forward(win, valid=True)
    assert_loss_close(float(loss.item()), o["loss"], what="c1")
    assert diag["n_valid"] == int(o["valid"].sum())
    assert diag["nact"] == list(o["nact"])
    np.testing.assert_allclose(diag["num"], o["num"], rtol=1e-5)
    assert abs(diag["loss"] - o["loss"]) <= 1e-5 * o["loss"]


def test_c1_backward(cm):
    check_window(cm, eventgen.make_window("c1"), what="c1")


def test_c2_full_fwd_bwd(cm):
    check_window(cm, eventgen.make_window("c2"), what="c2")


@pytest.mark.parametrize("refs", [[1.0], [0.0, 1.0], [0.0, 0.5, 1.0], [0.05, 0.3, 0.31, 0.9],
                                  list(eventgen.refs_even(8)), list(eventgen.refs_even(16))])
@pytest.mark.parametrize("n", [1, 255, 257, 5000])
def test_ref_counts_and_ragged_sizes(cm, refs, n):
    win = eventgen.edge_window(77 + n, "346x260", max(n, 1), refs=refs, n_segments=12,
                               motion_sigma=0.3, name=f"r{len(refs)}n{n}")
    check_window(cm, win, what=win.name)


def test_c3_windows_full_size(cm):
    for i in (0, 5, 17):
        check_window(cm, eventgen.make_window("c3", i), what=f"c3[{i}]")


def test_c5_full_size(cm):
    win = eventgen.make_window("c5")
    check_window(cm, win, what="c5")


def test_zero_flow_matches_histogram_loss(cm):
    win = eventgen.make_window("c1").replace(theta=np.zeros(6, np.float32))
    g, o = check_window(cm, win, grad=True, what="zero flow")
    assert o["valid"].all()


def test_empty_window(cm):
    win = eventgen.make_window("c1")
    e = np.zeros(0, np.float32)
    win = win.replace(x=e, y=e, t=e, p=np.zeros(0, np.int8))
    g = run_gpu(cm, win)
    assert g["loss"] == 0.0
    assert not g["drho"].any() and not g["dtheta"].any()


def test_masked_and_malformed_events(cm):
    win = eventgen.make_window("c1")
    x = win.x.copy(); y = win.y.copy(); t = win.t.copy()
    x[::7] = np.nan               # non-finite coordinate
    t[1::11] = 1.5                # timestamp outside [0, 1]
    y[2::13] = -1.0               # start off the image
    x[3::17] = win.width - 1      # on the border (valid start)
    t[4::19] = 1.0                # exactly on the reference time
    win = win.replace(x=x, y=y, t=t)
    check_window(cm, win, what="malformed")


def test_all_events_masked(cm):
    win = eventgen.make_window("c1")
    win = win.replace(t=np.full(win.n, 2.0, np.float32))
    g = run_gpu(cm, win)
    assert g["loss"] == 0.0 and not g["drho"].any() and not g["dtheta"].any()


def test_grad_output_scaling(cm):
    win = eventgen.make_window("c1")
    g1 = run_gpu(cm, win, grad_out=1.0)
    g2 = run_gpu(cm, win, grad_out=-2.5)
    np.testing.assert_allclose(g2["dtheta"], -2.5 * g1["dtheta"], rtol=1e-5,
                               atol=1e-6 * np.abs(g1["dtheta"]).max())
    assert np.linalg.norm(g2["drho"] + 2.5 * g1["drho"]) <= 1e-5 * np.linalg.norm(2.5 * g1["drho"])


def test_repeat_runs_agree(cm):
    win = eventgen.make_window("c2")
    a = run_gpu(cm, win, grad=False)["loss"]
    b = run_gpu(cm, win, grad=False)["loss"]
    assert abs(a - b) <= 1e-6 * abs(a)


def test_invalid_args_raise(cm):
    win = eventgen.make_window("c1")
    d = to_device(win)
    bad = cm.WindowDesc.from_window(win)
    bad.refs[0], bad.refs[1] = 0.5, 0.5
    bad.n_refs = 2
    with pytest.raises(cm.CMError):
        cm.forward(bad, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])


def test_path_pairing_between_forward_and_backward():
    """A tiled forward followed by a direct backward gives the oracle's
    gradients (the images are shared); a direct forward followed by a tiled
    backward has no source records and must return NaN, not plausible values."""
    import paper_2412_06359_amd as cm
    cm.load()
    win = eventgen.make_window("c2")
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win)
    gl = torch.ones(1, device="cuda:0")
    ob = oracle.backward(win)
    try:
        print("[gpu] tiled forward, direct backward", flush=True)
        cm.set_path(0, cm.CM_PATH_TILED)
        _, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
        cm.set_path(0, cm.CM_PATH_DIRECT)
        g_rho, g_ego = cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"],
                                   state, gl)
        assert_grads_close(g_rho.double().cpu().numpy(), g_ego.double().cpu().numpy(),
                           ob["drho"], ob["dtheta"], what="tiled fwd / direct bwd")
        print("[gpu] direct forward, tiled backward", flush=True)
        _, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
        cm.set_path(0, cm.CM_PATH_TILED)
        g_rho, g_ego = cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"],
                                   state, gl)
        assert torch.isnan(g_ego).all()
    finally:
        cm.set_path(0, cm.CM_PATH_AUTO)

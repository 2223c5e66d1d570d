"""GPU: deterministic mode.  Within tolerance of the oracle, bit-identical from
run to run, and bit-identical between a window alone and inside a batch."""

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import assert_grads_close, assert_loss_close, to_device
from tests.test_gpu_batch import mixed_windows, pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


def run_det(cm, win):
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=cm.CM_MODE_DETERMINISTIC)
    print(f"[gpu] det {win.name} n={win.n} R={len(win.refs)}", flush=True)
    loss, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                               torch.ones(1, device="cuda:0"))
    torch.cuda.synchronize()
    return loss.cpu().numpy(), g_rho.cpu().numpy(), g_ego.cpu().numpy()


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_deterministic_matches_oracle_and_repeats_bitwise(cm, name):
    win = eventgen.make_window(name)
    a = run_det(cm, win)
    b = run_det(cm, win)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    o = oracle.forward(win)
    assert_loss_close(float(a[0][0]), o["loss"], what=name)
    ob = oracle.backward(win)
    assert_grads_close(a[1], a[2], ob["drho"], ob["dtheta"], what=name)


def test_deterministic_c5_full_size(cm):
    win = eventgen.make_window("c5")
    a = run_det(cm, win)
    b = run_det(cm, win)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    o = oracle.forward(win)
    assert_loss_close(float(a[0][0]), o["loss"], what="c5 det")
    ob = oracle.backward(win)
    assert_grads_close(a[1], a[2], ob["drho"], ob["dtheta"], what="c5 det")


def test_deterministic_batch_equals_alone_bitwise(cm):
    wins = mixed_windows()
    descs = [cm.WindowDesc.from_window(w, mode=cm.CM_MODE_DETERMINISTIC) for w in wins]
    batch = cm.Batch(descs, [w.n for w in wins])
    d = pack(wins)
    loss, state = batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                                  torch.ones(batch.n, device="cuda:0"))
    loss = loss.cpu().numpy()
    g_rho = g_rho.cpu().numpy()
    g_ego = g_ego.cpu().numpy().reshape(-1, 6)
    for w, win in enumerate(wins):
        l1, r1, e1 = run_det(cm, win)
        assert loss[w] == l1[0], (w, loss[w], l1[0])
        a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
        assert np.array_equal(g_rho[a:b], r1.ravel()), w
        assert np.array_equal(g_ego[w], e1), w


def test_deterministic_ragged_and_edge_cases(cm):
    for n in (1, 63, 64, 65, 1000):
        win = eventgen.edge_window(900 + n, "346x260", n, refs=[0.0, 0.3, 1.0], n_segments=5,
                                   name=f"det{n}")
        a = run_det(cm, win)
        o = oracle.forward(win)
        assert_loss_close(float(a[0][0]), o["loss"], what=win.name)
        ob = oracle.backward(win)
        assert_grads_close(a[1], a[2], ob["drho"], ob["dtheta"], what=win.name)


def _mirror_cases():
    wins = [eventgen.make_window("c1"), eventgen.make_window("c2"), eventgen.make_window("c3", 5)]
    for n in (1, 65, 1000):
        wins.append(eventgen.edge_window(950 + n, "346x260", n, refs=[0.0, 0.3, 1.0],
                                         n_segments=5, name=f"m{n}"))
    w = eventgen.make_window("c1")
    t = w.t.copy()
    x = w.x.copy()
    t[::9] = 1.0
    x[::13] = np.nan
    wins.append(w.replace(t=t, x=x, name="c1-malformed"))
    return wins


@pytest.mark.parametrize("idx", range(7))
def test_deterministic_bitwise_equals_canonical_mirror(cm, idx):
    win = _mirror_cases()[idx]
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=cm.CM_MODE_DETERMINISTIC)
    print(f"[gpu] mirror {win.name} n={win.n}", flush=True)
    loss, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                               torch.full((1,), 0.75, device="cuda:0"))
    diag = cm.diagnostics(desc, state)
    m = oracle.mirror_forward(win)
    mb = oracle.mirror_backward(win, grad_loss=0.75)
    assert float(loss.item()) == float(m["loss"])
    assert diag["loss"] == m["loss64"]
    assert diag["n_valid"] == m["n_valid"]
    assert diag["num"] == list(m["num"]) and diag["nact"] == list(m["nact"])
    assert np.array_equal(g_rho.cpu().numpy().reshape(win.height, win.width), mb["drho"])
    assert np.array_equal(g_ego.cpu().numpy(), mb["dtheta"])


def test_deterministic_c5_bitwise_equals_canonical_mirror(cm):
    win = eventgen.make_window("c5")
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=cm.CM_MODE_DETERMINISTIC)
    loss, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                               torch.ones(1, device="cuda:0"))
    m = oracle.mirror_forward(win)
    mb = oracle.mirror_backward(win)
    assert float(loss.item()) == float(m["loss"])
    assert np.array_equal(g_rho.cpu().numpy().reshape(win.height, win.width), mb["drho"])
    assert np.array_equal(g_ego.cpu().numpy(), mb["dtheta"])

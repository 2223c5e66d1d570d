"""GPU: the continuous-batching server.  Each result equals the window's
result alone (bitwise in deterministic mode, within tolerance otherwise), the
admitted footprint never exceeds the budget, oversize windows are refused."""

import time

import numpy as np
import pytest
import torch

import eventgen
from tests.helpers import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


def windows(k=14):
    out = []
    for i in range(k):
        sensor = "346x260" if i % 2 == 0 else "640x480"
        n = [3000, 40000, 900, 120000, 15000, 70000, 5000][i % 7]
        out.append(eventgen.stream_window(sensor, n, 5000 + i))
    return out


def alone(cm, win, mode):
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=mode)
    loss, state = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                               torch.ones(1, device="cuda:0"))
    torch.cuda.synchronize()
    return float(loss.item()), g_rho.cpu().numpy(), g_ego.cpu().numpy()


def serve_all(cm, wins, mode, budget, gap_s=0.002):
    from paper_2412_06359_amd.serve import Server
    srv = Server(budget_bytes=budget, mode=mode)
    futs = []
    for w in wins:
        futs.append(srv.submit(w))
        time.sleep(gap_s)
    res = [f.result(timeout=120) for f in futs]
    srv.drain()
    st = srv.stats()
    srv.close()
    return res, st


def test_served_equals_alone_bitwise_deterministic(cm):
    wins = windows()
    print(f"[gpu] serving {len(wins)} windows, deterministic", flush=True)
    res, st = serve_all(cm, wins, cm.CM_MODE_DETERMINISTIC, budget=8 << 30)
    assert st["windows"] == len(wins) and st["batches"] >= 2
    cm.set_path(0, cm.CM_PATH_AUTO)
    for w, r in zip(wins, res):
        l1, g1, e1 = alone(cm, w, cm.CM_MODE_DETERMINISTIC)
        assert r["loss"] == l1
        assert np.array_equal(r["grad_inv_depth"].cpu().numpy().ravel(), g1.ravel())
        assert np.array_equal(r["grad_ego"].cpu().numpy(), e1)


def test_served_equals_alone_atomic(cm):
    wins = windows()
    res, st = serve_all(cm, wins, cm.CM_MODE_ATOMIC, budget=8 << 30, gap_s=0.0)
    for w, r in zip(wins, res):
        l1, g1, e1 = alone(cm, w, cm.CM_MODE_ATOMIC)
        assert abs(r["loss"] - l1) <= 1e-6 * abs(l1)
        g = r["grad_inv_depth"].cpu().numpy().ravel()
        assert np.linalg.norm(g - g1.ravel()) <= 1e-5 * np.linalg.norm(g1)
        np.testing.assert_allclose(r["grad_ego"].cpu().numpy(), e1, rtol=1e-5,
                                   atol=1e-6 * np.abs(e1).max())


def test_budget_is_respected_and_oversize_refused(cm):
    from paper_2412_06359_amd.serve import window_footprint
    wins = windows(10)
    fps = [window_footprint(cm.WindowDesc.from_window(w), w.n) for w in wins]
    budget = 2 * max(fps) + 1
    res, st = serve_all(cm, wins, cm.CM_MODE_ATOMIC, budget=budget, gap_s=0.0)
    assert st["windows"] == len(wins)
    assert 0 < st["max_used_bytes"] <= budget
    assert st["batches"] >= 3
    from paper_2412_06359_amd.serve import Server
    srv = Server(budget_bytes=max(fps) // 2)
    big = wins[int(np.argmax(fps))]
    with pytest.raises(cm.CMError) as ei:
        srv.submit(big).result(timeout=10)
    assert ei.value.status == -5
    srv.close()

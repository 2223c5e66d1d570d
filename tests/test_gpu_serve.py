"""GPU: the continuous-batching server.  Each result equals the window's
result alone (bitwise in deterministic mode, within tolerance otherwise), the
admitted footprint never exceeds the budget, oversize windows are refused."""

import threading
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


def test_budget_bounds_device_memory_and_oversize_refused(cm):
    """The budget bounds real device memory: torch's peak allocation while
    serving (slot workspaces, gradients in flight, results held) stays within
    it, with the client holding every result until the end."""
    from paper_2412_06359_amd.serve import Server, window_footprint
    wins = windows(10)
    fps = [window_footprint(cm.WindowDesc.from_window(w), w.n) for w in wins]
    # room for the largest window and half of it again: the windows cannot
    # all share a batch, so the budget has to split them
    budget = max(fps) + max(fps) // 2 + 1
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    res, st = serve_all(cm, wins, cm.CM_MODE_ATOMIC, budget=budget, gap_s=0.0)
    assert st["windows"] == len(wins)
    assert 0 < st["max_used_bytes"] <= budget
    assert 0 < st["peak_allocated_bytes"] <= budget, (st["peak_allocated_bytes"], budget)
    assert torch.cuda.max_memory_allocated() - base <= budget
    assert st["batches"] >= max(3, -(-sum(fps) // budget))
    assert st["windows_per_batch"] == len(wins) / st["batches"]
    srv = Server(budget_bytes=max(fps) // 2)
    big = wins[int(np.argmax(fps))]
    with pytest.raises(cm.CMError) as ei:
        srv.submit(big).result(timeout=10)
    assert ei.value.status == -5
    srv.close()


def test_held_results_exhaust_the_budget_without_hanging(cm):
    """Results the client keeps count against the budget; when they fill it
    and nothing is in flight, the next window fails with CM_ERR_BUDGET instead
    of waiting forever."""
    from paper_2412_06359_amd.serve import Server, window_footprint
    big = eventgen.stream_window("640x480", 20000, 5100)
    fp = window_footprint(cm.WindowDesc.from_window(big), big.n)
    srv = Server(budget_bytes=fp + (1 << 20), n_streams=1)
    held = [srv.submit(big).result(timeout=60)]
    # one result held (1.2 MB of gradients) plus the idle workspace: a second
    # window of the same size cannot fit once the workspace is reclaimed
    held.append(torch.empty(fp, dtype=torch.uint8, device="cuda:0"))   # the client's own use
    with pytest.raises(cm.CMError) as ei:
        srv.submit(big).result(timeout=60)
    assert ei.value.status == -5
    del held
    torch.cuda.synchronize()
    ok = srv.submit(big).result(timeout=60)          # memory freed: served again
    assert np.isfinite(ok["loss"])
    srv.close()


def test_launch_failure_while_a_batch_is_in_flight(cm):
    """A launch error (raised from the host) fails only its own batch: the
    batch already in flight completes, and later requests are served."""
    from paper_2412_06359_amd.serve import Server
    wins = windows(3)
    srv = Server(budget_bytes=8 << 30, n_streams=2, max_batch=1)
    real = srv._launch
    calls = {"n": 0}

    def flaky(*a, **k):
        calls["n"] += 1
        if calls["n"] == 2:
            raise RuntimeError("injected launch failure")
        return real(*a, **k)
    srv._launch = flaky
    futs = [srv.submit(w) for w in wins]
    r0 = futs[0].result(timeout=60)
    with pytest.raises(RuntimeError, match="injected"):
        futs[1].result(timeout=60)
    r2 = futs[2].result(timeout=60)
    assert np.isfinite(r0["loss"]) and np.isfinite(r2["loss"])
    srv.close()


def test_scheduler_failure_fails_queued_and_in_flight(cm):
    """If the scheduler itself fails (raised from the host while a batch is in
    flight and others are queued), every unresolved request fails with that
    error (none is left pending) and later submissions raise."""
    from paper_2412_06359_amd.serve import Server
    wins = windows(6)
    srv = Server(budget_bytes=8 << 30, n_streams=1, max_batch=1)
    real_retire, real_admit = srv._retire, srv._admit
    go = threading.Event()

    def broken():
        if any(b is not None for b in srv._busy):
            raise RuntimeError("injected scheduler failure")
        return real_retire()

    def gated():
        go.wait(30)                 # admit nothing until every request is queued
        return real_admit()
    srv._retire, srv._admit = broken, gated
    futs = [srv.submit(w) for w in wins]
    go.set()
    for f in futs:
        with pytest.raises(RuntimeError, match="injected"):
            f.result(timeout=60)
    with pytest.raises(RuntimeError):
        srv.submit(wins[0])
    torch.cuda.synchronize()


def test_close_finishes_in_flight_and_queued(cm):
    from paper_2412_06359_amd.serve import Server
    wins = windows(8)
    srv = Server(budget_bytes=8 << 30, n_streams=2, max_batch=2)
    futs = [srv.submit(w) for w in wins]
    srv.close()
    assert all(f.done() for f in futs)
    assert all(np.isfinite(f.result()["loss"]) for f in futs)
    with pytest.raises(RuntimeError):
        srv.submit(wins[0])

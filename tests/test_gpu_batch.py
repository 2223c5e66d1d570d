"""GPU: batched windows (one launch sequence over a flat event buffer) against
the oracle per window, against single-window calls, and under hipGraph replay."""

import concurrent.futures as cf

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import assert_grads_close, assert_loss_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


def mixed_windows():
    """Uneven sizes, two sensors, 1-8 references, an empty and a one-event window."""
    wins = []
    for i, (sensor, n, refs) in enumerate([
            ("346x260", 5000, [0.0, 1.0]), ("640x480", 30000, [0.0, 0.5, 1.0]),
            ("346x260", 1, [0.0, 1.0]), ("346x260", 0, [0.0, 1.0]),
            ("346x260", 120000, [0.0, 1.0]), ("640x480", 777, list(eventgen.refs_even(8))),
            ("346x260", 20000, [1.0]), ("346x260", 60000, [0.0, 1.0])]):
        w = eventgen.edge_window(600 + i, sensor, max(n, 1), refs=refs, n_segments=30,
                                 name=f"b{i}")
        if n == 0:
            e = np.zeros(0, np.float32)
            w = w.replace(x=e, y=e, t=e, p=np.zeros(0, np.int8))
        wins.append(w)
    return wins


def pack(wins, dev="cuda:0"):
    f = lambda arrs: torch.from_numpy(np.ascontiguousarray(np.concatenate(
        [np.asarray(a, np.float32).ravel() for a in arrs]))).to(dev)
    return dict(x=f([w.x for w in wins]), y=f([w.y for w in wins]), t=f([w.t for w in wins]),
                p=torch.from_numpy(np.concatenate([np.asarray(w.p, np.int8) for w in wins])).to(dev),
                rho=f([w.rho for w in wins]), ego=f([w.theta for w in wins]))


def make_batch(cm, wins, graph=False):
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    return cm.Batch(descs, [w.n for w in wins], graph=graph)


def run_batch(cm, batch, d, grad_out=None):
    n = batch.n
    loss, state = batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    gl = torch.ones(n, device="cuda:0") if grad_out is None else grad_out
    g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state, gl)
    torch.cuda.synchronize()
    return (loss.double().cpu().numpy(), g_rho.double().cpu().numpy(),
            g_ego.double().cpu().numpy().reshape(n, 6), batch.diagnostics(state))


def test_batch_matches_oracle_per_window(cm):
    wins = mixed_windows()
    batch = make_batch(cm, wins)
    print(f"[gpu] batch of {batch.n} windows, {batch.event_offsets[-1]} events", flush=True)
    loss, g_rho, g_ego, diag = run_batch(cm, batch, pack(wins))
    for w, win in enumerate(wins):
        o = oracle.forward(win, valid=True)
        assert_loss_close(loss[w], o["loss"], what=win.name)
        assert diag[w][1] == int(o["valid"].sum())
        ob = oracle.backward(win)
        a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
        assert_grads_close(g_rho[a:b], g_ego[w], ob["drho"].ravel(), ob["dtheta"], what=win.name)


def test_batch_of_many_bins_matches_oracle(cm):
    """A batch with more forward bins than the scan's one-pass limit (20 windows of
    1280x720 with 8 references: 147,200 bins, 18 chunks of 8192), so that the scan
    takes per-chunk totals first; every window's loss and the last windows'
    gradients against the oracle (a wrong chunk prefix misplaces every later
    window's records)."""
    refs = list(eventgen.refs_even(8))
    wins = [eventgen.edge_window(900 + i, "1280x720", 3000, refs=refs, n_segments=20,
                                 name=f"m{i}") for i in range(20)]
    batch = make_batch(cm, wins)
    print(f"[gpu] batch of {batch.n} windows, {batch.event_offsets[-1]} events, 8 refs",
          flush=True)
    loss, g_rho, g_ego, diag = run_batch(cm, batch, pack(wins))
    for w, win in enumerate(wins):
        o = oracle.forward(win, valid=True)
        assert_loss_close(loss[w], o["loss"], what=win.name)
        assert diag[w][1] == int(o["valid"].sum())
    for w in (0, 10, 19):
        ob = oracle.backward(wins[w])
        a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
        assert_grads_close(g_rho[a:b], g_ego[w], ob["drho"].ravel(), ob["dtheta"],
                           what=wins[w].name)


def _masked(win):
    """Every event's time outside [0, 1]: every event masked (Sec. 3.1's validity)."""
    return win.replace(t=np.full(win.n, 2.0, np.float32))


@pytest.mark.parametrize("refs", [[0.0, 1.0], [0.0, 0.5, 1.0]], ids=["at_events", "three_refs"])
def test_batch_with_masked_windows(cm, refs):
    """Windows whose events are all masked, in a batch with ordinary ones (their bins
    stay empty and no source record names them) and in a batch of nothing else (no
    occupied bin at all: the splat's list and the backward's are empty).  A masked
    window has loss 0 and zero gradients, as in the oracle; the others match the
    oracle.  Both backward paths: sampled at the events (refs {0, 1}) and binned."""
    mk = lambda i, n: eventgen.edge_window(700 + i, "346x260", n, refs=refs, n_segments=30,
                                           name=f"k{i}")
    wins = [mk(0, 20000), _masked(mk(1, 8000)), mk(2, 5000), mk(3, 1), _masked(mk(4, 300))]
    fwd, bwd = {}, {}
    for group in (wins, [_masked(mk(5, 4000)), _masked(mk(6, 1)), _masked(mk(7, 9000))]):
        for graph in (False, True):
            batch = make_batch(cm, group, graph=graph)
            print(f"[gpu] masked windows: {batch.n} windows, refs {refs}, graph {graph}",
                  flush=True)
            d = pack(group)
            for _ in range(2 if graph else 1):     # (a replay after the capture)
                loss, g_rho, g_ego, diag = run_batch(cm, batch, d)
            for w, win in enumerate(group):
                a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
                if win.name not in fwd:
                    fwd[win.name] = oracle.forward(win, valid=True)
                o = fwd[win.name]
                if not o["valid"].any():
                    assert loss[w] == 0.0 and diag[w][1] == 0, win.name
                    assert not g_rho[a:b].any() and not g_ego[w].any(), win.name
                    continue
                assert_loss_close(loss[w], o["loss"], what=win.name)
                assert diag[w][1] == int(o["valid"].sum())
                if win.name not in bwd:
                    bwd[win.name] = oracle.backward(win)
                ob = bwd[win.name]
                assert_grads_close(g_rho[a:b], g_ego[w], ob["drho"].ravel(), ob["dtheta"],
                                   what=win.name)


def test_batch_equals_single_window_calls(cm):
    wins = mixed_windows()
    batch = make_batch(cm, wins)
    loss, g_rho, g_ego, _ = run_batch(cm, batch, pack(wins))
    cm.set_path(0, cm.CM_PATH_TILED)
    try:
        for w, win in enumerate(wins):
            d = pack([win])
            desc = cm.WindowDesc.from_window(win)
            rho = d["rho"].clone().requires_grad_(True)
            ego = d["ego"].clone().requires_grad_(True)
            L = cm.cm_loss(d["x"], d["y"], d["t"], d["p"], rho, ego, desc)
            L.backward()
            assert abs(float(L.item()) - loss[w]) <= 1e-6 * abs(loss[w]) + 1e-12
            a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
            ref = rho.grad.double().cpu().numpy()
            assert np.linalg.norm(g_rho[a:b] - ref) <= 1e-5 * np.linalg.norm(ref) + 1e-30
            np.testing.assert_allclose(g_ego[w], ego.grad.double().cpu().numpy(), rtol=1e-5,
                                       atol=1e-6 * np.abs(g_ego[w]).max() + 1e-30)
    finally:
        cm.set_path(0, cm.CM_PATH_AUTO)


def test_batch_graph_replays_match_eager(cm):
    wins = mixed_windows()
    d = pack(wins)
    eager = make_batch(cm, wins, graph=False)
    ref = run_batch(cm, eager, d)
    graphed = make_batch(cm, wins, graph=True)
    state = graphed.new_state()
    loss = torch.empty(graphed.n, device="cuda:0")
    g_rho = torch.empty_like(d["rho"])
    g_ego = torch.empty_like(d["ego"])
    gl = torch.ones(graphed.n, device="cuda:0")
    for rep in range(4):
        graphed.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state=state, loss=loss)
        graphed.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state, gl,
                         grad_rho=g_rho, grad_ego=g_ego)
        torch.cuda.synchronize()
        # eager work of the program between replays
        junk = torch.randn(1 << 20, device="cuda:0").sum().item()
        assert np.isfinite(junk)
        l = loss.double().cpu().numpy()
        np.testing.assert_allclose(l, ref[0], rtol=1e-6, atol=1e-12)
        gr = g_rho.double().cpu().numpy()
        assert np.linalg.norm(gr - ref[1]) <= 1e-5 * np.linalg.norm(ref[1])
        np.testing.assert_allclose(g_ego.double().cpu().numpy().reshape(-1, 6), ref[2],
                                   rtol=1e-5, atol=1e-6 * np.abs(ref[2]).max())


def test_batch_autograd_and_grad_scaling(cm):
    wins = mixed_windows()[:3]
    batch = make_batch(cm, wins)
    d = pack(wins)
    rho = d["rho"].clone().requires_grad_(True)
    ego = d["ego"].clone().requires_grad_(True)
    losses = cm.BatchCMLoss.apply(d["x"], d["y"], d["t"], d["p"], rho, ego, batch)
    weights = torch.tensor([1.0, -2.0, 0.5], device="cuda:0")
    (losses * weights).sum().backward()
    for w, win in enumerate(wins):
        ob = oracle.backward(win, grad_loss=float(weights[w]))
        a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
        assert_grads_close(rho.grad.double().cpu().numpy()[a:b],
                           ego.grad.double().cpu().numpy()[6 * w:6 * w + 6],
                           ob["drho"].ravel(), ob["dtheta"], what=win.name)


def test_c3_batch_full_size(cm):
    """All 64 windows of the batched workload, each against the oracle (the
    oracle calls run in a thread pool; ctypes releases the GIL)."""
    wins = eventgen.make_batch("c3", 64)
    batch = make_batch(cm, wins, graph=True)
    print(f"[gpu] c3 batch {batch.event_offsets[-1]} events", flush=True)
    loss, g_rho, g_ego, diag = run_batch(cm, batch, pack(wins))
    with cf.ThreadPoolExecutor(8) as ex:
        ref = list(ex.map(lambda w: (oracle.forward(w, valid=True), oracle.backward(w)), wins))
    for w, (o, ob) in enumerate(ref):
        assert_loss_close(loss[w], o["loss"], what=f"c3[{w}]")
        assert diag[w][1] == int(o["valid"].sum()), w
        a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
        assert_grads_close(g_rho[a:b], g_ego[w], ob["drho"].ravel(), ob["dtheta"],
                           what=f"c3[{w}]")


@pytest.fixture(scope="module")
def c3_reference():
    """The 64 c3 windows and the oracle's loss and gradients for each (computed once)."""
    wins = eventgen.make_batch("c3", 64)
    with cf.ThreadPoolExecutor(8) as ex:
        ref = list(ex.map(lambda w: (oracle.forward(w, valid=True), oracle.backward(w)), wins))
    return wins, ref


@pytest.mark.parametrize("tuning", [(8192, 512, 32, 32), (4096, 256, 32, 32),
                                    (16384, 512, 64, 32), (8192, 512, 16, 16)])
def test_c3_batch_full_size_tunings(cm, c3_reference, tuning):
    """All 64 c3 windows at the launch shapes the autotuner chooses between (the first
    is the one the bench times), graph replay, each against the oracle."""
    wins, ref = c3_reference
    eb, tt, tw, th = tuning
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    batch = cm.Batch(descs, [w.n for w in wins], graph=True,
                     tuning=dict(event_blocks=eb, tile_threads=tt, tile_w=tw, tile_h=th))
    print(f"[gpu] c3 batch at tuning {tuning}", flush=True)
    loss, g_rho, g_ego, diag = run_batch(cm, batch, pack(wins))
    for w, (o, ob) in enumerate(ref):
        assert_loss_close(loss[w], o["loss"], what=f"c3[{w}] {tuning}")
        assert diag[w][1] == int(o["valid"].sum()), w
        a, b = batch.pixel_offsets[w], batch.pixel_offsets[w + 1]
        assert_grads_close(g_rho[a:b], g_ego[w], ob["drho"].ravel(), ob["dtheta"],
                           what=f"c3[{w}] {tuning}")


def test_c6_batch_full_size(cm):
    """All 64 c6 windows (10 flow sets, references at the 11 slice edges) at the launch
    shape the bench times for them (64x32 tiles, 16384 event blocks), each flow set's
    gradients against the oracle."""
    wins = eventgen.make_batch("c6", 64)
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    batch = cm.Batch(descs, [w.n for w in wins], graph=True,
                     tuning=dict(event_blocks=16384, tile_threads=512, tile_w=64, tile_h=32))
    d = pack(wins)
    print(f"[gpu] c6 batch {batch.event_offsets[-1]} events, {batch.set_offsets[-1]} sets",
          flush=True)
    loss, state = batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                                  torch.ones(batch.n, device="cuda:0"))
    torch.cuda.synchronize()
    loss = loss.double().cpu().numpy()
    g_rho = g_rho.double().cpu().numpy()
    g_ego = g_ego.double().cpu().numpy()
    with cf.ThreadPoolExecutor(8) as ex:
        ref = list(ex.map(lambda w: (oracle.forward(w), oracle.backward(w)), wins))
    for w, (win, (o, ob)) in enumerate(zip(wins, ref)):
        assert_loss_close(loss[w], o["loss"], what=f"c6[{w}]")
        F = win.rho.shape[0]
        pr = g_rho[batch.pixel_offsets[w]:batch.pixel_offsets[w + 1]].reshape(F, win.height,
                                                                               win.width)
        pe = g_ego[6 * batch.set_offsets[w]:6 * batch.set_offsets[w + 1]].reshape(F, 6)
        for f in range(F):
            assert_grads_close(pr[f], pe[f], ob["drho"][f], ob["dtheta"][f],
                               what=f"c6[{w}] set {f}")


@pytest.mark.parametrize("case", ["c1", "edges_R3"])
def test_reused_state_zero_flow_reads_no_stale_pixels(cm, case):
    """The tiled splat stores only the image pixels some tap reached.  With
    zero motion every warped position stays on its pixel centre, where taps
    1-3 have zero weight but a non-zero weight derivative, so the backward
    reads those pixels: they must be stored too (a zero), not left holding a
    previous window's values.  One state serves a moving window first, then
    the same events without motion; the second run must give the oracle's
    loss and gradients."""
    if case == "c1":
        moving = eventgen.make_window("c1")
    else:
        moving = eventgen.edge_window(951, "346x260", 20000, refs=[0.0, 0.5, 1.0],
                                      n_segments=20, name="stale")
    still = moving.replace(theta=np.zeros_like(moving.theta))
    batch = make_batch(cm, [moving])
    state = batch.new_state()
    gl = torch.ones(1, device="cuda:0")
    for win in (moving, still):
        print(f"[gpu] stale-pixel check {case} theta={np.asarray(win.theta)[:3]}", flush=True)
        d = pack([win])
        loss, _ = batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state=state)
        g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                                      gl)
    torch.cuda.synchronize()
    o = oracle.forward(still)
    assert_loss_close(float(loss.item()), o["loss"], what=f"{case} zero flow, reused state")
    ob = oracle.backward(still)
    assert np.abs(ob["dtheta"]).max() > 0.0
    assert_grads_close(g_rho.double().cpu().numpy(), g_ego.double().cpu().numpy(), ob["drho"],
                       ob["dtheta"], what=f"{case} zero flow, reused state")

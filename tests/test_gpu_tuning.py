"""GPU: launch tuning (cm_set_tuning) and the autotuner.  Every tuning gives
the same per-window losses and gradients within the parity tolerances."""

import numpy as np
import pytest
import torch

import oracle
from tests.helpers import assert_grads_close, assert_loss_close
from tests.test_gpu_batch import mixed_windows, pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    yield cm
    cm.set_tuning(0)                      # back to the defaults


def test_set_tuning_validates(cm):
    t0 = cm.get_tuning(0)
    assert t0 == dict(event_blocks=4096, tile_threads=512, tiled_min_records=1 << 17,
                      tile_w=32, tile_h=32)
    for bad in (dict(event_blocks=100), dict(event_blocks=1 << 20), dict(tile_threads=384),
                dict(tiled_min_records=-5), dict(tile_w=48), dict(tile_w=16, tile_h=32),
                dict(tile_w=128, tile_h=32)):
        with pytest.raises(cm.CMError):
            cm.set_tuning(0, **bad)
        assert cm.get_tuning(0) == t0      # unchanged on error
    assert cm.set_tuning(0, event_blocks=1024, tile_threads=256)["tile_threads"] == 256
    cm.set_tuning(0)
    assert cm.get_tuning(0) == t0


def run_batch(cm, wins, tuning):
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    batch = cm.Batch(descs, [w.n for w in wins], tuning=tuning)
    print(f"[gpu] tuned batch {batch.tuning}", flush=True)
    d = pack(wins)
    loss, state = batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state,
                                  torch.ones(batch.n, device="cuda:0"))
    torch.cuda.synchronize()
    return batch, loss.cpu().numpy(), g_rho.cpu().numpy(), g_ego.cpu().numpy()


@pytest.mark.parametrize("tuning", [dict(event_blocks=256, tile_threads=256),
                                    dict(event_blocks=16384, tile_threads=512),
                                    dict(event_blocks=1024, tile_threads=512),
                                    dict(event_blocks=4096, tile_threads=256, tile_w=64, tile_h=32),
                                    dict(event_blocks=2048, tile_threads=512, tile_w=32, tile_h=16),
                                    dict(event_blocks=8192, tile_threads=256, tile_w=16, tile_h=16)])
def test_tuned_batches_match_oracle(cm, tuning):
    wins = mixed_windows()
    batch, loss, g_rho, g_ego = run_batch(cm, wins, tuning)
    assert batch.tuning["event_blocks"] == tuning["event_blocks"]
    assert batch.tuning["tile_w"] == tuning.get("tile_w", 32)
    assert cm.get_tuning(0)["event_blocks"] == 4096        # the handle's own is restored
    for w, win in enumerate(wins):
        o = oracle.forward(win)
        assert_loss_close(float(loss[w]), o["loss"], what=f"{tuning} {win.name}")
        ob = oracle.backward(win)
        pr = g_rho[batch.pixel_offsets[w]:batch.pixel_offsets[w + 1]]
        pe = g_ego[6 * batch.set_offsets[w]:6 * batch.set_offsets[w + 1]]
        assert_grads_close(pr, pe, ob["drho"].ravel(), ob["dtheta"], what=f"{tuning} {win.name}")


def test_autotuner_times_candidates_and_caches(cm, tmp_path):
    from paper_2412_06359_amd import autotune
    wins = mixed_windows()[:6]
    descs = [cm.WindowDesc.from_window(w) for w in wins]
    counts = [w.n for w in wins]
    cands = [dict(event_blocks=1024, tile_threads=256), dict(event_blocks=4096, tile_threads=512)]
    log = []
    path = str(tmp_path / "tune.json")
    best = autotune.tune(descs, counts, pack(wins), candidates=cands, steps=2, warmup=1,
                         cache_path=path, log=log)
    print(f"[gpu] autotune {log} -> {best}", flush=True)
    full = [autotune._tuning(c) for c in cands]            # every field, tile size included
    assert best in full and len(log) == 2 and all(ms > 0 for _, ms in log)
    assert best == autotune._tuning(min(log, key=lambda r: r[1])[0])
    assert autotune.tune(descs, counts, cache_path=path) == best      # cached


@pytest.mark.parametrize("tile", [(64, 32), (32, 16), (16, 16)])
def test_tuned_event_sampled_batches_match_oracle(cm, tile):
    """Windows whose backward samples the flow at the events only (references
    {0, 1} or a single one: source records binned by the event's tiles) at each
    tile size, a position on the last column / row of a tile included."""
    import eventgen
    wins = [eventgen.edge_window(700 + i, sensor, n, refs=refs, n_segments=30, name=f"e{i}")
            for i, (sensor, n, refs) in enumerate([("346x260", 40000, [0.0, 1.0]),
                                                   ("640x480", 25000, [0.0, 1.0]),
                                                   ("346x260", 9000, [1.0]),
                                                   ("346x260", 3000, [0.0, 1.0])])]
    wins.append(eventgen.make_window("c1", subpixel=True).replace(refs=[0.0, 1.0]))
    tuning = dict(event_blocks=2048, tile_threads=256, tile_w=tile[0], tile_h=tile[1])
    batch, loss, g_rho, g_ego = run_batch(cm, wins, tuning)
    for w, win in enumerate(wins):
        o = oracle.forward(win)
        assert_loss_close(float(loss[w]), o["loss"], what=f"{tile} {win.name}")
        ob = oracle.backward(win)
        pr = g_rho[batch.pixel_offsets[w]:batch.pixel_offsets[w + 1]]
        pe = g_ego[6 * batch.set_offsets[w]:6 * batch.set_offsets[w + 1]]
        assert_grads_close(pr, pe, ob["drho"].ravel(), ob["dtheta"], what=f"{tile} {win.name}")


def test_crossover_tuning(cm):
    """The direct / tiled crossover search: a threshold from the measured
    windows, set on the handle with the rest of the tuning kept."""
    import eventgen
    from paper_2412_06359_amd import autotune
    cm.set_tuning(0, event_blocks=2048)
    wins = [eventgen.edge_window(800 + i, "346x260", n, refs=[0.0, 1.0], n_segments=30,
                                 name=f"x{i}") for i, n in enumerate([500, 5000, 60000])]
    log = []
    try:
        cross = autotune.tune_crossover(wins, steps=2, warmup=1, log=log)
        print(f"[gpu] crossover {cross} from {log}", flush=True)
        recs = [r["records"] for r in log]
        assert len(log) == 3 and recs == sorted(recs)
        assert 1 <= cross <= recs[-1] + 1
        t = cm.get_tuning(0)
        assert t["tiled_min_records"] == cross and t["event_blocks"] == 2048
        assert cm.get_path(0) == cm.CM_PATH_AUTO          # the path is restored
    finally:
        cm.set_tuning(0)

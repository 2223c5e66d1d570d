"""GPU: RSAT (loss at the motion over loss without motion) and the online
fitting loop on the full loss (Eq. 4), through the library."""

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import to_device
from tests.test_gpu_batch import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rsat_matches_oracle(cm, seed):
    win = eventgen.edge_window(seed, "346x260", 20000, refs=[0.0, 0.5, 1.0], n_segments=20,
                               motion_sigma=0.3)
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win)
    r, l, l0 = cm.rsat(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    want = oracle.rsat(win)
    assert abs(r.item() - want) <= 2e-5 * want, (r.item(), want)


def test_rsat_of_zero_motion_is_one(cm):
    win = eventgen.bins_window(3)
    win = win.replace(theta=np.zeros_like(win.theta))
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win, mode=cm.CM_MODE_DETERMINISTIC)
    r, _, _ = cm.rsat(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    assert r.item() == 1.0
    assert oracle.rsat(win) == 1.0


def test_batch_rsat(cm):
    wins = [eventgen.bins_window(i) for i in range(3)] + \
        [eventgen.edge_window(9, "346x260", 5000, refs=[0.0, 1.0], n_segments=20)]
    batch = cm.Batch([cm.WindowDesc.from_window(w) for w in wins], [w.n for w in wins])
    d = pack(wins)
    r, _, _ = batch.rsat(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
    r = r.cpu().numpy()
    for w, win in enumerate(wins):
        want = oracle.rsat(win)
        assert abs(r[w] - want) <= 2e-5 * want, (w, r[w], want)


def test_online_tracking_lowers_loss_and_rsat(cm):
    """Online ego-motion fitting on a stream with drifting motion, starting
    from a perturbed estimate: every window's loss falls and RSAT falls on
    average over the windows."""
    from paper_2412_06359_amd.online import fit_stream
    wins = eventgen.motion_stream(1, 3)
    rng = np.random.default_rng(1)
    init = np.asarray(wins[0].theta, np.float64) + rng.normal(0.0, 0.05, 6)
    recs = fit_stream(wins, init, steps=40)
    for rec in recs:
        print(f"[gpu] online {rec}", flush=True)
        assert np.isfinite(rec["loss_end"]) and np.isfinite(rec["rsat_end"])
        assert rec["loss_end"] < rec["loss_start"]
    assert np.mean([r["rsat_end"] - r["rsat_start"] for r in recs]) < 0.0


def test_online_fit_with_depth_runs(cm):
    """Depth and ego-motion fitted together through exp(log rho): finite
    values and a loss that does not grow over the steps."""
    from paper_2412_06359_amd.online import fit_stream
    wins = eventgen.motion_stream(2, 1)
    init = np.asarray(wins[0].theta, np.float64) * 1.1
    rec = fit_stream(wins, init, steps=20, fit_depth=True)[0]
    print(f"[gpu] online depth {rec}", flush=True)
    assert np.isfinite(rec["loss_end"]) and rec["loss_end"] <= rec["loss_start"] * 1.01

"""GPU: cm_loss_forward_noalloc, the forward that allocates nothing (its whole
state lives in the library's per-device scratch array), against the existing
cm_loss_forward (state in a caller buffer) on the same windows.

Two no-alloc calls run back to back, the second on a smaller window, so the
second starts from the first's leftovers in the shared scratch.  Deterministic
mode: bit-identical to cm_loss_forward.  Atomic mode: within the loss
tolerance of cm_loss_forward and of the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import eventgen
import oracle
from tests.helpers import assert_loss_close, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import paper_2412_06359_amd as cm
    cm.load()
    assert torch.cuda.is_available()
    return cm


def _windows():
    big = eventgen.make_window("c2")                       # 640x480, 3 refs, 100k events
    small = eventgen.make_window("c1", subpixel=True)      # 64x64, 1 ref, 2k events
    return big, small


@pytest.mark.parametrize("path,mode", [("auto", 0), ("direct", 0), ("tiled", 0), ("auto", 1)])
def test_noalloc_forward_equals_forward_two_calls(cm, path, mode):
    cm.set_path(0, {"auto": cm.CM_PATH_AUTO, "direct": cm.CM_PATH_DIRECT,
                    "tiled": cm.CM_PATH_TILED}[path])
    try:
        wins = _windows()
        descs = [cm.WindowDesc.from_window(w, mode=mode) for w in wins]
        devs = [to_device(w) for w in wins]
        for w, desc in zip(wins, descs):
            assert cm.state_bytes(desc, w.n) <= cm.NOALLOC_MAX_STATE_BYTES
        print(f"[gpu] no-alloc path={path} mode={mode}: reference forwards", flush=True)
        ref = []
        for desc, d in zip(descs, devs):
            loss, _ = cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
            ref.append(loss)
        outs = [torch.full((1,), float("nan"), device="cuda:0") for _ in wins]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        print(f"[gpu] no-alloc path={path} mode={mode}: two calls, big then small", flush=True)
        for desc, d, out in zip(descs, devs, outs):
            cm.forward_noalloc(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free0 - free1 < (1 << 20), (free0, free1)
        for w, r, out in zip(wins, ref, outs):
            got, want = float(out.item()), float(r.item())
            if mode == 1:
                assert got == want, (w.name, got, want)
            else:
                assert_loss_close(got, want, rtol=1e-6, what=f"{w.name} vs cm_loss_forward")
            assert_loss_close(got, oracle.loss(w), what=f"{w.name} vs oracle")
    finally:
        cm.set_path(0, cm.CM_PATH_AUTO)


def test_noalloc_rejects_oversized_state(cm):
    """A state beyond the scratch array is refused on the host (CM_ERR_BUDGET)
    and nothing is written."""
    desc = cm.WindowDesc.make(1280, 720, 600.0, 600.0, 639.5, 359.5,
                              list(eventgen.refs_even(8)))
    assert cm.state_bytes(desc, 0) > cm.NOALLOC_MAX_STATE_BYTES
    e = torch.zeros(0, device="cuda:0")
    p = torch.zeros(0, dtype=torch.int8, device="cuda:0")
    rho = torch.ones(720 * 1280, device="cuda:0")
    ego = torch.zeros(6, device="cuda:0")
    out = torch.full((1,), 7.0, device="cuda:0")
    with pytest.raises(cm.CMError) as ei:
        cm.forward_noalloc(desc, e, e, e, p, rho, ego, out)
    assert ei.value.status == -5
    assert float(out.item()) == 7.0


def test_noalloc_empty_window(cm):
    win = eventgen.make_window("c1")
    d = to_device(win)
    desc = cm.WindowDesc.from_window(win)
    e = torch.zeros(0, device="cuda:0")
    out = torch.full((1,), float("nan"), device="cuda:0")
    cm.forward_noalloc(desc, e, e, e, torch.zeros(0, dtype=torch.int8, device="cuda:0"),
                       d["rho"], d["ego"], out)
    assert float(out.item()) == 0.0

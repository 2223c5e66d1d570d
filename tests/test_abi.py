"""CPU checks of the C ABI: the library builds, loads, exports every symbol the
header declares, and rejects invalid arguments on the host (no GPU needed)."""

import ctypes
import os
import re

import pytest

import paper_2412_06359_amd as cm
from paper_2412_06359_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmloss.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return cm.load()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "cm_loss_forward" in names and "cm_loss_backward" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in binding._STATUS.items():
        assert lib.cm_status_string(code).decode() == name


def _desc(**kw):
    base = dict(width=64, height=48, fx=50.0, fy=50.0, cx=31.5, cy=23.5, refs=[0.0, 0.5, 1.0])
    base.update(kw)
    return cm.WindowDesc.make(**base)


def test_state_bytes_formula(lib):
    d = _desc()
    n = cm.state_bytes(d, 0)
    assert n >= 32 * 3 * 64 * 48
    assert n - 32 * 3 * 64 * 48 < 1 << 20
    # the tiled path's workspace grows with the event count: in the atomic
    # mode up to four 32-byte record slots per position (one per tile its taps
    # reach) plus a source record per event; one slot per position in the
    # deterministic mode
    big = cm.state_bytes(d, 1_000_000)
    assert big > n + 4 * 32 * 3 * 1_000_000
    assert big < n + (4 * 32 * 3 + 32) * 1_000_000 + (64 << 20)
    dd = _desc(mode=cm.CM_MODE_DETERMINISTIC)
    nd = cm.state_bytes(dd, 0)
    bigd = cm.state_bytes(dd, 1_000_000)
    assert bigd > nd + 32 * 3 * 1_000_000
    assert bigd < nd + (32 * 3 + 32) * 1_000_000 + (64 << 20)


@pytest.mark.parametrize("bad", [
    dict(width=0), dict(height=-3), dict(fx=0.0), dict(fy=-1.0), dict(fx=float("nan")),
    dict(refs=[0.5, 0.5]), dict(refs=[0.7, 0.2]), dict(refs=[-0.1, 1.0]), dict(refs=[0.0, 1.5]),
    dict(mode=7), dict(eps=0.0), dict(eps=float("inf")), dict(flow_model=2),
    dict(flow_model=-1),
])
def test_invalid_descriptors_rejected(lib, bad):
    d = _desc(**bad)
    assert lib.cm_state_bytes(ctypes.byref(d), 0) == 0
    # a null handle or invalid descriptor returns CM_ERR_INVALID_ARG before any HIP call
    st = lib.cm_loss_forward(None, ctypes.byref(d), None, None, None, None, 0, None, None, None,
                             None, None)
    assert st == -1


def test_too_many_refs_rejected(lib):
    d = _desc()
    d.n_refs = 17
    assert lib.cm_state_bytes(ctypes.byref(d), 0) == 0
    d.n_refs = 0
    assert lib.cm_state_bytes(ctypes.byref(d), 0) == 0
    assert lib.cm_state_bytes(ctypes.byref(_desc()), -1) == 0


def test_null_arguments_rejected(lib):
    d = _desc()
    assert lib.cm_create(None, 0) == -1
    fake = ctypes.c_void_p(1)
    # n_events > 0 with null event pointers
    st = lib.cm_loss_forward(fake, ctypes.byref(d), None, None, None, None, 10, None, None, None,
                             None, None)
    assert st == -1
    st = lib.cm_loss_backward(fake, ctypes.byref(d), None, None, None, None, 0, None, None, None,
                              None, None, None, None)
    assert st == -1
    assert lib.cm_destroy(None) == 0
    assert lib.cm_set_path(None, 0) == -1
    assert lib.cm_set_path(fake, 3) == -1


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libcmloss.so")
    with pytest.raises(RuntimeError, match="missing"):
        binding.load()


@pytest.mark.parametrize("refs,F,ok", [
    ([0.0, 0.5, 1.0], 0, True), ([0.0, 0.5, 1.0], 1, True), ([0.0, 0.5, 1.0], 2, True),
    ([0.0, 0.5, 1.0], 3, False), ([0.0, 0.5, 1.0], -1, False),
    ([0.2, 0.6], 3, True), ([0.2, 0.6], 2, False), ([1.0], 1, True), ([1.0], 2, False),
    ([0.5], 2, True), ([0.0, 1.0], 1, True), ([0.0, 1.0], 2, False),
])
def test_flow_set_count_validated(lib, refs, F, ok):
    """n_flows must be 1 (or 0) or the number of segments between consecutive
    knots {0, 1} U refs."""
    d = _desc(refs=refs)
    d.n_flows = F
    assert (lib.cm_state_bytes(ctypes.byref(d), 100) > 0) == ok


def test_flow_sets_enlarge_only_the_scratch(lib):
    d1 = _desc(refs=[0.0, 0.25, 0.5, 0.75, 1.0])
    d4 = _desc(refs=[0.0, 0.25, 0.5, 0.75, 1.0])
    d4.n_flows = 4
    b1, b4 = cm.state_bytes(d1, 0), cm.state_bytes(d4, 0)
    assert b4 >= b1 and b4 - b1 < 2 << 20


def test_descriptor_layout_matches_header():
    """The ctypes mirror of cm_window_desc has the C layout: fields in header
    order, 4-byte members, flow_model last."""
    names = [f[0] for f in cm.WindowDesc._fields_]
    assert names[-2:] == ["n_flows", "flow_model"]
    assert ctypes.sizeof(cm.WindowDesc) == 4 * (2 + 4 + 1 + 16 + 1 + 1 + 1 + 1)
    assert cm.WindowDesc.flow_model.offset == ctypes.sizeof(cm.WindowDesc) - 4

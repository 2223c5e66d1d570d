"""ctypes binding of libcmloss.so (include/cmloss.h) for torch tensors.

Argument marshalling only: every step of the loss and its gradient runs in
the library's HIP kernels.  PyTorch supplies device memory and the stream.
There is no fallback: if the library is missing, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcmloss.so")

CM_MAX_REFS = 16
CM_MODE_ATOMIC = 0
CM_MODE_DETERMINISTIC = 1
CM_FLOW_FIRST_ORDER = 0
CM_FLOW_EXACT = 1

_STATUS = {0: "CM_OK", -1: "CM_ERR_INVALID_ARG", -2: "CM_ERR_OOM", -3: "CM_ERR_HIP",
           -4: "CM_ERR_UNSUPPORTED", -5: "CM_ERR_BUDGET"}


class CMError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_STATUS.get(status, status)}")
        self.status = status


class WindowDesc(ctypes.Structure):
    """cm_window_desc: sensor, intrinsics, reference times, mode, eps, flow sets."""

    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("n_refs", ctypes.c_int32), ("refs", ctypes.c_float * CM_MAX_REFS),
                ("mode", ctypes.c_int32), ("eps", ctypes.c_float), ("n_flows", ctypes.c_int32),
                ("flow_model", ctypes.c_int32)]

    @classmethod
    def make(cls, width: int, height: int, fx: float, fy: float, cx: float, cy: float,
             refs: Sequence[float], mode: int = CM_MODE_ATOMIC, eps: float = 1e-9,
             n_flows: int = 1, flow_model: int = CM_FLOW_FIRST_ORDER) -> "WindowDesc":
        refs = [float(r) for r in refs]
        if not 1 <= len(refs) <= CM_MAX_REFS:
            raise ValueError(f"need 1..{CM_MAX_REFS} reference times, got {len(refs)}")
        d = cls()
        d.width, d.height = int(width), int(height)
        d.fx, d.fy, d.cx, d.cy = fx, fy, cx, cy
        d.n_refs = len(refs)
        for i, r in enumerate(refs):
            d.refs[i] = r
        d.mode = int(mode)
        d.eps = eps
        d.n_flows = int(n_flows)
        d.flow_model = int(flow_model)
        return d

    @classmethod
    def from_window(cls, win, mode: int = CM_MODE_ATOMIC) -> "WindowDesc":
        """From an object with width, height, fx, fy, cx, cy, refs, eps, rho
        ([H, W] for one flow, [F, H, W] for F flow sets) and optionally
        flow_model (0 first order, 1 exact)."""
        rho = getattr(win, "rho", None)
        F = 1 if rho is None or len(getattr(rho, "shape", ())) != 3 else int(rho.shape[0])
        return cls.make(win.width, win.height, win.fx, win.fy, win.cx, win.cy, list(win.refs),
                        mode, getattr(win, "eps", 1e-9), F,
                        int(getattr(win, "flow_model", CM_FLOW_FIRST_ORDER)))

    @property
    def R(self) -> int:
        return int(self.n_refs)

    @property
    def F(self) -> int:
        """Flow sets (inverse-depth images and ego-motion vectors)."""
        return max(1, int(self.n_flows))


class Tuning(ctypes.Structure):
    """cm_tuning: launch shape of batch plans (atomic mode) and the direct /
    tiled crossover of single windows; zero fields keep the defaults."""

    _fields_ = [("event_blocks", ctypes.c_int32), ("tile_threads", ctypes.c_int32),
                ("tiled_min_records", ctypes.c_int64), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return dict(event_blocks=int(self.event_blocks), tile_threads=int(self.tile_threads),
                    tiled_min_records=int(self.tiled_min_records), tile_w=int(self.tile_w),
                    tile_h=int(self.tile_h))


_lib = None
_lib_lock = threading.Lock()
_tuning_lock = threading.Lock()


def load() -> ctypes.CDLL:
    """Load libcmloss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2412_06359_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        D = ctypes.POINTER(WindowDesc)
        i64 = ctypes.c_int64
        lib.cm_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.cm_create.restype = ctypes.c_int
        lib.cm_destroy.argtypes = [P]
        lib.cm_destroy.restype = ctypes.c_int
        lib.cm_status_string.argtypes = [ctypes.c_int]
        lib.cm_status_string.restype = ctypes.c_char_p
        lib.cm_state_bytes.argtypes = [D, i64]
        lib.cm_state_bytes.restype = ctypes.c_size_t
        lib.cm_set_path.argtypes = [P, ctypes.c_int]
        lib.cm_set_path.restype = ctypes.c_int
        lib.cm_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        lib.cm_set_tuning.restype = ctypes.c_int
        lib.cm_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        lib.cm_get_tuning.restype = ctypes.c_int
        lib.cm_loss_forward.argtypes = [P, D, P, P, P, P, i64, P, P, P, P, P]
        lib.cm_loss_forward.restype = ctypes.c_int
        lib.cm_loss_backward.argtypes = [P, D, P, P, P, P, i64, P, P, P, P, P, P, P]
        lib.cm_loss_backward.restype = ctypes.c_int
        lib.cm_loss_forward_noalloc.argtypes = [P, D, P, P, P, P, i64, P, P, P, P]
        lib.cm_loss_forward_noalloc.restype = ctypes.c_int
        lib.cm_state_diagnostics.argtypes = [D, P, P, P]
        lib.cm_state_diagnostics.restype = ctypes.c_int
        lib.cm_batch_create.argtypes = [P, ctypes.c_int32, P, P, ctypes.POINTER(P)]
        lib.cm_batch_create.restype = ctypes.c_int
        lib.cm_batch_destroy.argtypes = [P]
        lib.cm_batch_destroy.restype = ctypes.c_int
        lib.cm_batch_state_bytes.argtypes = [P]
        lib.cm_batch_state_bytes.restype = ctypes.c_size_t
        lib.cm_batch_offsets.argtypes = [P, P, P]
        lib.cm_batch_offsets.restype = ctypes.c_int
        lib.cm_batch_flow_offsets.argtypes = [P, P]
        lib.cm_batch_flow_offsets.restype = ctypes.c_int
        lib.cm_batch_set_graph.argtypes = [P, ctypes.c_int]
        lib.cm_batch_set_graph.restype = ctypes.c_int
        lib.cm_loss_forward_batched.argtypes = [P, P, P, P, P, P, P, P, P, P]
        lib.cm_loss_forward_batched.restype = ctypes.c_int
        lib.cm_loss_backward_batched.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P]
        lib.cm_loss_backward_batched.restype = ctypes.c_int
        lib.cm_batch_diagnostics.argtypes = [P, P, P, P]
        lib.cm_batch_diagnostics.restype = ctypes.c_int
        lib.cm_batch_occupied_image_bytes.argtypes = [P, P, P, P]
        lib.cm_batch_occupied_image_bytes.restype = ctypes.c_int
        lib.cm_batch_active_pixels.argtypes = [P, P, P, P]
        lib.cm_batch_active_pixels.restype = ctypes.c_int
        f32 = ctypes.c_float
        lib.cm_geo_state_bytes.argtypes = [D]
        lib.cm_geo_state_bytes.restype = ctypes.c_size_t
        lib.cm_geo_forward.argtypes = [P, D, P, P, f32, P, P, P, P, P]
        lib.cm_geo_forward.restype = ctypes.c_int
        lib.cm_geo_backward.argtypes = [P, D, P, P, f32, P, P, P, P, P]
        lib.cm_geo_backward.restype = ctypes.c_int
        lib.cm_batch_geo_state_bytes.argtypes = [P]
        lib.cm_batch_geo_state_bytes.restype = ctypes.c_size_t
        lib.cm_geo_forward_batched.argtypes = [P, P, P, f32, P, P, P, P, P]
        lib.cm_geo_forward_batched.restype = ctypes.c_int
        lib.cm_geo_backward_batched.argtypes = [P, P, P, f32, P, P, P, P, P]
        lib.cm_geo_backward_batched.restype = ctypes.c_int
        lib.cm_profile_enable.argtypes = [P, ctypes.c_int]
        lib.cm_profile_enable.restype = ctypes.c_int
        lib.cm_profile_read.argtypes = [P, P, P]
        lib.cm_profile_read.restype = ctypes.c_int
        _lib = lib
        return lib


def _check(status: int, what: str):
    if status != 0:
        raise CMError(status, what)


_handles = {}


def handle(device: int) -> ctypes.c_void_p:
    """The library handle of a device (created once per process)."""
    h = _handles.get(device)
    if h is None:
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.cm_create(ctypes.byref(h), device), "cm_create")
        _handles[device] = h
    return h


CM_PATH_AUTO, CM_PATH_DIRECT, CM_PATH_TILED = 0, 1, 2


def state_bytes(desc: WindowDesc, n_events: int) -> int:
    n = load().cm_state_bytes(ctypes.byref(desc), int(n_events))
    if n == 0:
        raise CMError(-1, "cm_state_bytes (invalid descriptor)")
    return int(n)


_path_of: dict = {}


def set_path(device: int, path: int):
    """Kernel path of this device's handle: CM_PATH_AUTO, _DIRECT or _TILED."""
    _check(load().cm_set_path(handle(device), int(path)), "cm_set_path")
    _path_of[device] = int(path)


def get_path(device: int = 0) -> int:
    """The path set_path last gave this device's handle (CM_PATH_AUTO before
    any call)."""
    return _path_of.get(device, CM_PATH_AUTO)


def get_tuning(device: int = 0) -> dict:
    t = Tuning()
    _check(load().cm_get_tuning(handle(device), ctypes.byref(t)), "cm_get_tuning")
    return t.as_dict()


def set_tuning(device: int = 0, event_blocks: int = 0, tile_threads: int = 0,
               tiled_min_records: int = 0, tile_w: int = 0, tile_h: int = 0) -> dict:
    """cm_set_tuning on this device's handle (0 keeps a field's default);
    returns the tuning now in effect."""
    t = Tuning(int(event_blocks), int(tile_threads), int(tiled_min_records), int(tile_w),
               int(tile_h))
    _check(load().cm_set_tuning(handle(device), ctypes.byref(t)), "cm_set_tuning")
    return get_tuning(device)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_events(x, y, t, p):
    n = x.numel()
    for name, a, dt in (("x", x, torch.float32), ("y", y, torch.float32), ("t", t, torch.float32),
                        ("p", p, torch.int8)):
        if a.dtype != dt or a.dim() != 1 or a.numel() != n or not a.is_contiguous():
            raise ValueError(f"event array {name}: need contiguous 1-D {dt} of length {n}")
        if not a.is_cuda:
            raise ValueError(f"event array {name} must be on a GPU")
    return n


def _check_params(desc, rho, ego):
    F = desc.F
    if rho.dtype != torch.float32 or rho.numel() != F * desc.width * desc.height or \
            not rho.is_contiguous() or not rho.is_cuda:
        raise ValueError(f"inv_depth: need contiguous float32 GPU tensor of "
                         f"{F}x{desc.height}x{desc.width} elements")
    if ego.dtype != torch.float32 or ego.numel() != 6 * F or not ego.is_contiguous() or \
            not ego.is_cuda:
        raise ValueError(f"ego: need contiguous float32 GPU tensor of {6 * F} elements")


def forward(desc: WindowDesc, x, y, t, p, rho, ego, state: Optional[torch.Tensor] = None,
            loss: Optional[torch.Tensor] = None):
    """cm_loss_forward on torch's current stream.  Returns (loss [1], state)."""
    n = _check_events(x, y, t, p)
    _check_params(desc, rho, ego)
    dev = rho.device
    nbytes = state_bytes(desc, n)
    if state is None:
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    elif state.numel() * state.element_size() < nbytes or not state.is_contiguous():
        raise ValueError(f"state: need {nbytes} contiguous bytes")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    lib = load()
    st = lib.cm_loss_forward(handle(dev.index), ctypes.byref(desc), _ptr(x), _ptr(y), _ptr(t),
                             _ptr(p), n, _ptr(rho), _ptr(ego), _ptr(loss), _ptr(state),
                             _stream(dev))
    _check(st, "cm_loss_forward")
    return loss, state


NOALLOC_MAX_STATE_BYTES = 128 * 1024 * 1024    # CM_NOALLOC_MAX_STATE_BYTES


def forward_noalloc(desc: WindowDesc, x, y, t, p, rho, ego, loss: torch.Tensor):
    """cm_loss_forward_noalloc on torch's current stream: the loss into `loss`
    (a float32 [1] GPU tensor the caller owns), with the window's state in the
    library's own per-device scratch (no allocation; no backward can follow;
    calls on one device must not overlap).  Raises CMError (CM_ERR_BUDGET) if
    the window's state exceeds NOALLOC_MAX_STATE_BYTES."""
    n = _check_events(x, y, t, p)
    _check_params(desc, rho, ego)
    if loss.dtype != torch.float32 or loss.numel() < 1 or not loss.is_cuda:
        raise ValueError("loss: need a float32 GPU tensor of at least 1 element")
    dev = rho.device
    lib = load()
    st = lib.cm_loss_forward_noalloc(handle(dev.index), ctypes.byref(desc), _ptr(x), _ptr(y),
                                     _ptr(t), _ptr(p), n, _ptr(rho), _ptr(ego), _ptr(loss),
                                     _stream(dev))
    _check(st, "cm_loss_forward_noalloc")
    return loss


def backward(desc: WindowDesc, x, y, t, p, rho, ego, state, grad_loss,
             grad_rho: Optional[torch.Tensor] = None, grad_ego: Optional[torch.Tensor] = None):
    """cm_loss_backward on torch's current stream.  Returns (grad_rho, grad_ego)."""
    n = _check_events(x, y, t, p)
    _check_params(desc, rho, ego)
    dev = rho.device
    if state.numel() * state.element_size() < state_bytes(desc, n):
        raise ValueError("state buffer too small")
    gl = grad_loss.reshape(1).to(device=dev, dtype=torch.float32).contiguous()
    if grad_rho is None:
        grad_rho = torch.empty_like(rho)
    if grad_ego is None:
        grad_ego = torch.empty_like(ego)
    lib = load()
    st = lib.cm_loss_backward(handle(dev.index), ctypes.byref(desc), _ptr(x), _ptr(y), _ptr(t),
                              _ptr(p), n, _ptr(rho), _ptr(ego), _ptr(state), _ptr(gl),
                              _ptr(grad_rho), _ptr(grad_ego), _stream(dev))
    _check(st, "cm_loss_backward")
    return grad_rho, grad_ego


LAMBDA_GEO = 0.05       # weight of L_geo in the full loss (the paper's training value)


def geo_state_bytes(desc: WindowDesc) -> int:
    n = load().cm_geo_state_bytes(ctypes.byref(desc))
    if n == 0:
        raise CMError(-1, "cm_geo_state_bytes (invalid descriptor)")
    return int(n)


def geo_forward(desc: WindowDesc, rho, ego, lam: float = LAMBDA_GEO, loss_cm=None, state=None):
    """cm_geo_forward on torch's current stream.  Returns (loss_geo [1],
    loss_total [1] = loss_cm + lam * loss_geo (None without loss_cm), state)."""
    _check_params(desc, rho, ego)
    dev = rho.device
    nbytes = geo_state_bytes(desc)
    if state is None:
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    elif state.numel() * state.element_size() < nbytes or not state.is_contiguous():
        raise ValueError(f"geo state: need {nbytes} contiguous bytes")
    loss_geo = torch.empty(1, dtype=torch.float32, device=dev)
    total = None if loss_cm is None else torch.empty(1, dtype=torch.float32, device=dev)
    st = load().cm_geo_forward(handle(dev.index), ctypes.byref(desc), _ptr(rho), _ptr(ego),
                               float(lam), _ptr(loss_cm), _ptr(loss_geo), _ptr(total),
                               _ptr(state), _stream(dev))
    _check(st, "cm_geo_forward")
    return loss_geo, total, state


def geo_backward(desc: WindowDesc, rho, ego, state, grad_loss, grad_rho, grad_ego,
                 lam: float = LAMBDA_GEO):
    """cm_geo_backward: adds grad_loss * lam * dL_geo/d(rho, ego) into grad_rho
    and grad_ego (in place)."""
    _check_params(desc, rho, ego)
    dev = rho.device
    if state.numel() * state.element_size() < geo_state_bytes(desc):
        raise ValueError("geo state buffer too small")
    gl = grad_loss.reshape(1).to(device=dev, dtype=torch.float32).contiguous()
    for name, g, ref in (("grad_rho", grad_rho, rho), ("grad_ego", grad_ego, ego)):
        if g.dtype != torch.float32 or g.numel() != ref.numel() or not g.is_contiguous():
            raise ValueError(f"{name}: need contiguous float32 of {ref.numel()} elements")
    st = load().cm_geo_backward(handle(dev.index), ctypes.byref(desc), _ptr(rho), _ptr(ego),
                                float(lam), _ptr(state), _ptr(gl), _ptr(grad_rho),
                                _ptr(grad_ego), _stream(dev))
    _check(st, "cm_geo_backward")
    return grad_rho, grad_ego


def rsat(desc: WindowDesc, x, y, t, p, rho, ego):
    """RSAT, the paper's deblurring metric (ratio of squared average
    timestamps, after Hagenaars et al.): the CM loss at `ego` over the CM loss
    at zero motion, two library forwards.  Returns (rsat, loss, loss_zero),
    0-d device tensors."""
    loss, _ = forward(desc, x, y, t, p, rho, ego)
    loss0, _ = forward(desc, x, y, t, p, rho, torch.zeros_like(ego))
    return (loss / loss0).reshape(()), loss.reshape(()), loss0.reshape(())


def diagnostics(desc: WindowDesc, state: torch.Tensor) -> dict:
    """Per-window sums of the last forward (synchronises the stream)."""
    R = desc.R
    out = (ctypes.c_double * (2 + 2 * R))()
    st = load().cm_state_diagnostics(ctypes.byref(desc), _ptr(state), out, _stream(state.device))
    _check(st, "cm_state_diagnostics")
    vals = list(out)
    return dict(loss=vals[0], n_valid=int(vals[1]), num=vals[2:2 + R], nact=vals[2 + R:])


class Batch:
    """A plan for many windows in one launch sequence (cm_batch).

    Events of all windows are packed in flat arrays (window w at
    event_offsets[w]:event_offsets[w+1]), inverse depth and its gradient at
    pixel_offsets (F images per window); ego / grad ego hold 6 floats per flow
    set, window w's at 6 * set_offsets[w]; loss / grad_loss are [n]."""

    def __init__(self, descs: Sequence[WindowDesc], n_events: Sequence[int], device: int = 0,
                 graph: bool = False, tuning: Optional[dict] = None):
        """tuning: dict(event_blocks=, tile_threads=, tile_w=, tile_h=) for this
        plan (atomic mode), e.g. from autotune.tune; absent fields take the
        defaults; None takes the handle's current tuning."""
        lib = load()
        n = len(descs)
        self.device = device
        self.descs = list(descs)
        arr = (WindowDesc * n)(*descs)
        cnt = (ctypes.c_int64 * n)(*[int(v) for v in n_events])
        self._b = ctypes.c_void_p()
        h = handle(device)
        with _tuning_lock:
            prev = Tuning()
            _check(lib.cm_get_tuning(h, ctypes.byref(prev)), "cm_get_tuning")
            if tuning is not None:
                t = Tuning(int(tuning.get("event_blocks", 0)), int(tuning.get("tile_threads", 0)),
                           int(prev.tiled_min_records), int(tuning.get("tile_w", 0)),
                           int(tuning.get("tile_h", 0)))
                _check(lib.cm_set_tuning(h, ctypes.byref(t)), "cm_set_tuning")
            try:
                st = lib.cm_batch_create(h, n, arr, cnt, ctypes.byref(self._b))
                self.tuning = get_tuning(device)
            finally:
                if tuning is not None:
                    lib.cm_set_tuning(h, ctypes.byref(prev))
        _check(st, "cm_batch_create")
        self.n = n
        self.state_bytes = int(lib.cm_batch_state_bytes(self._b))
        ev = (ctypes.c_int64 * (n + 1))()
        px = (ctypes.c_int64 * (n + 1))()
        _check(lib.cm_batch_offsets(self._b, ev, px), "cm_batch_offsets")
        so = (ctypes.c_int64 * (n + 1))()
        _check(lib.cm_batch_flow_offsets(self._b, so), "cm_batch_flow_offsets")
        self.event_offsets = list(ev)
        self.pixel_offsets = list(px)
        self.set_offsets = list(so)
        self.set_graph(graph)

    def set_graph(self, enable: bool):
        _check(load().cm_batch_set_graph(self._b, int(enable)), "cm_batch_set_graph")

    def close(self):
        if self._b:
            load().cm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self) -> torch.Tensor:
        return torch.empty(self.state_bytes, dtype=torch.uint8, device=f"cuda:{self.device}")

    def _check_flat(self, x, y, t, p, rho, ego):
        n = _check_events(x, y, t, p)
        if n != self.event_offsets[-1]:
            raise ValueError(f"batch has {self.event_offsets[-1]} events, got {n}")
        if rho.dtype != torch.float32 or rho.numel() != self.pixel_offsets[-1] or \
                not rho.is_contiguous() or not rho.is_cuda:
            raise ValueError(f"inv_depth: need {self.pixel_offsets[-1]} contiguous float32 values")
        ne = 6 * self.set_offsets[-1]
        if ego.dtype != torch.float32 or ego.numel() != ne or not ego.is_contiguous():
            raise ValueError(f"ego: need {ne} contiguous float32 values")

    def forward(self, x, y, t, p, rho, ego, state=None, loss=None):
        self._check_flat(x, y, t, p, rho, ego)
        dev = rho.device
        state = self.new_state() if state is None else state
        if state.numel() * state.element_size() < self.state_bytes:
            raise ValueError("state buffer too small")
        loss = torch.empty(self.n, dtype=torch.float32, device=dev) if loss is None else loss
        st = load().cm_loss_forward_batched(self._b, _ptr(x), _ptr(y), _ptr(t), _ptr(p),
                                            _ptr(rho), _ptr(ego), _ptr(loss), _ptr(state),
                                            _stream(dev))
        _check(st, "cm_loss_forward_batched")
        return loss, state

    def backward(self, x, y, t, p, rho, ego, state, grad_loss, grad_rho=None, grad_ego=None):
        self._check_flat(x, y, t, p, rho, ego)
        dev = rho.device
        gl = grad_loss.reshape(self.n).to(device=dev, dtype=torch.float32).contiguous()
        grad_rho = torch.empty_like(rho) if grad_rho is None else grad_rho
        grad_ego = torch.empty_like(ego) if grad_ego is None else grad_ego
        st = load().cm_loss_backward_batched(self._b, _ptr(x), _ptr(y), _ptr(t), _ptr(p),
                                             _ptr(rho), _ptr(ego), _ptr(state), _ptr(gl),
                                             _ptr(grad_rho), _ptr(grad_ego), _stream(dev))
        _check(st, "cm_loss_backward_batched")
        return grad_rho, grad_ego

    def geo_state_bytes(self) -> int:
        return int(load().cm_batch_geo_state_bytes(self._b))

    def geo_forward(self, rho, ego, lam: float = LAMBDA_GEO, loss_cm=None, state=None):
        """cm_geo_forward_batched: (loss_geo [n], loss_total [n] or None, state)."""
        dev = rho.device
        ne = 6 * self.set_offsets[-1]
        if rho.dtype != torch.float32 or rho.numel() != self.pixel_offsets[-1] or \
                not rho.is_contiguous() or ego.dtype != torch.float32 or ego.numel() != ne or \
                not ego.is_contiguous():
            raise ValueError("inv_depth / ego do not match the batch")
        nbytes = self.geo_state_bytes()
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev) if state is None else state
        if state.numel() * state.element_size() < nbytes:
            raise ValueError("geo state buffer too small")
        loss_geo = torch.empty(self.n, dtype=torch.float32, device=dev)
        total = None if loss_cm is None else torch.empty(self.n, dtype=torch.float32, device=dev)
        st = load().cm_geo_forward_batched(self._b, _ptr(rho), _ptr(ego), float(lam),
                                           _ptr(loss_cm), _ptr(loss_geo), _ptr(total),
                                           _ptr(state), _stream(dev))
        _check(st, "cm_geo_forward_batched")
        return loss_geo, total, state

    def geo_backward(self, rho, ego, state, grad_loss, grad_rho, grad_ego,
                     lam: float = LAMBDA_GEO):
        """cm_geo_backward_batched: adds the L_geo gradient into grad_rho / grad_ego."""
        dev = rho.device
        gl = grad_loss.reshape(self.n).to(device=dev, dtype=torch.float32).contiguous()
        if grad_rho.numel() != rho.numel() or grad_ego.numel() != ego.numel():
            raise ValueError("gradient buffers do not match the batch")
        st = load().cm_geo_backward_batched(self._b, _ptr(rho), _ptr(ego), float(lam),
                                            _ptr(state), _ptr(gl), _ptr(grad_rho),
                                            _ptr(grad_ego), _stream(dev))
        _check(st, "cm_geo_backward_batched")
        return grad_rho, grad_ego

    def rsat(self, x, y, t, p, rho, ego):
        """Per-window RSAT: (rsat [n], loss [n], loss at zero motion [n])."""
        loss, _ = self.forward(x, y, t, p, rho, ego)
        loss0, _ = self.forward(x, y, t, p, rho, torch.zeros_like(ego))
        return loss / loss0, loss, loss0

    def occupied_image_bytes(self, state) -> list:
        """Per window, splat-image bytes of its occupied tiles after the last
        forward (call before the backward; synchronises)."""
        out = (ctypes.c_double * self.n)()
        st = load().cm_batch_occupied_image_bytes(self._b, _ptr(state), out,
                                                  _stream(state.device))
        _check(st, "cm_batch_occupied_image_bytes")
        return list(out)

    def active_pixels(self, state) -> list:
        """Per window, [N_r for r < R] of the last forward (synchronises)."""
        out = (ctypes.c_double * (CM_MAX_REFS * self.n))()
        st = load().cm_batch_active_pixels(self._b, _ptr(state), out, _stream(state.device))
        _check(st, "cm_batch_active_pixels")
        return [[out[CM_MAX_REFS * w + r] for r in range(self.descs[w].R)]
                for w in range(self.n)]

    def diagnostics(self, state) -> list:
        out = (ctypes.c_double * (2 * self.n))()
        st = load().cm_batch_diagnostics(self._b, _ptr(state), out, _stream(state.device))
        _check(st, "cm_batch_diagnostics")
        return [(out[2 * w], int(out[2 * w + 1])) for w in range(self.n)]


class BatchCMLoss(torch.autograd.Function):
    """Per-window CM losses of a batch; differentiable in inv_depth and ego."""

    @staticmethod
    def forward(ctx, x, y, t, p, rho, ego, batch):
        rho_c = rho.detach().contiguous()
        ego_c = ego.detach().contiguous()
        loss, state = batch.forward(x, y, t, p, rho_c, ego_c)
        ctx.batch = batch
        ctx.save_for_backward(x, y, t, p, rho_c, ego_c, state)
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        x, y, t, p, rho, ego, state = ctx.saved_tensors
        g_rho, g_ego = ctx.batch.backward(x, y, t, p, rho, ego, state, grad_out.contiguous())
        return None, None, None, None, g_rho.reshape(rho.shape), g_ego.reshape(ego.shape), None


class BatchFullLoss(torch.autograd.Function):
    """Per-window full losses L = L_CM + lam L_geo (Eq. 4) of a batch;
    differentiable in inv_depth and ego."""

    @staticmethod
    def forward(ctx, x, y, t, p, rho, ego, batch, lam):
        rho_c = rho.detach().contiguous()
        ego_c = ego.detach().contiguous()
        loss_cm, state = batch.forward(x, y, t, p, rho_c, ego_c)
        _, total, gstate = batch.geo_forward(rho_c, ego_c, lam, loss_cm)
        ctx.batch, ctx.lam = batch, lam
        ctx.save_for_backward(x, y, t, p, rho_c, ego_c, state, gstate)
        return total

    @staticmethod
    def backward(ctx, grad_out):
        x, y, t, p, rho, ego, state, gstate = ctx.saved_tensors
        g = grad_out.contiguous()
        g_rho, g_ego = ctx.batch.backward(x, y, t, p, rho, ego, state, g)
        ctx.batch.geo_backward(rho, ego, gstate, g, g_rho, g_ego, ctx.lam)
        return (None, None, None, None, g_rho.reshape(rho.shape), g_ego.reshape(ego.shape), None,
                None)


PHASES = ("zero", "splat", "reduce", "finalize", "grad_zero", "adjoint", "grad_finalize",
          "count", "scan", "scatter", "grad_count", "grad_scan", "grad_tile")


def profile_enable(device: int, enable: bool = True):
    """Record HIP events around every kernel launched through this device's handle."""
    _check(load().cm_profile_enable(handle(device), int(enable)), "cm_profile_enable")


def profile_read(device: int) -> dict:
    """{phase: (total_ms, launches)} since the last read (waits for the events)."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(load().cm_profile_read(handle(device), ms, cnt), "cm_profile_read")
    return {PHASES[i]: (ms[i], int(cnt[i])) for i in range(n)}


class CMLoss(torch.autograd.Function):
    """Contrast-maximization loss of one window; differentiable in inv_depth and ego.

    forward(x, y, t, p, inv_depth, ego, desc) -> 0-d loss tensor
    backward -> (None, None, None, None, d inv_depth, d ego, None), computed by
    the library's adjoint kernels (the warp is recomputed, not stored).
    """

    @staticmethod
    def forward(ctx, x, y, t, p, rho, ego, desc):
        rho_c = rho.detach().contiguous()
        ego_c = ego.detach().contiguous()
        loss, state = forward(desc, x, y, t, p, rho_c, ego_c)
        ctx.desc = desc
        ctx.save_for_backward(x, y, t, p, rho_c, ego_c, state)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        x, y, t, p, rho, ego, state = ctx.saved_tensors
        g_rho, g_ego = backward(ctx.desc, x, y, t, p, rho, ego, state, grad_out)
        return None, None, None, None, g_rho.reshape(rho.shape), g_ego.reshape(ego.shape), None


def cm_loss(x, y, t, p, inv_depth, ego, desc: WindowDesc) -> torch.Tensor:
    """Differentiable CM loss (see CMLoss)."""
    return CMLoss.apply(x, y, t, p, inv_depth, ego, desc)


class FullLoss(torch.autograd.Function):
    """Full loss of one window, L = L_CM + lam L_geo (Eq. 4); differentiable
    in inv_depth and ego (both terms' gradients come from the library)."""

    @staticmethod
    def forward(ctx, x, y, t, p, rho, ego, desc, lam):
        rho_c = rho.detach().contiguous()
        ego_c = ego.detach().contiguous()
        loss_cm, state = forward(desc, x, y, t, p, rho_c, ego_c)
        _, total, gstate = geo_forward(desc, rho_c, ego_c, lam, loss_cm)
        ctx.desc, ctx.lam = desc, lam
        ctx.save_for_backward(x, y, t, p, rho_c, ego_c, state, gstate)
        return total.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        x, y, t, p, rho, ego, state, gstate = ctx.saved_tensors
        g_rho, g_ego = backward(ctx.desc, x, y, t, p, rho, ego, state, grad_out)
        geo_backward(ctx.desc, rho, ego, gstate, grad_out, g_rho, g_ego, ctx.lam)
        return (None, None, None, None, g_rho.reshape(rho.shape), g_ego.reshape(ego.shape), None,
                None)


def full_loss(x, y, t, p, inv_depth, ego, desc: WindowDesc, lam: float = LAMBDA_GEO):
    """Differentiable L = L_CM + lam L_geo of one window (see FullLoss)."""
    return FullLoss.apply(x, y, t, p, inv_depth, ego, desc, lam)

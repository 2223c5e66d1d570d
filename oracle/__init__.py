"""FP64 CPU oracle for the contrast-maximization loss and its gradient.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.  The arithmetic lives
in ``cm_oracle.c`` (plain C, FP64, no code shared with the GPU library); this
module builds and loads it and marshals numpy arrays.

Paper: Sec. 3.1 (iterative warp, Eq. 1, bilinear splatting, active-pixel
normalisation and out-of-image masking), Sec. 3.2 (Eq. 2, flow from depth and
ego-motion), Sec. 3.3 (per-event forward, analytic backward).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcm_oracle.so")
_lib = None

# -O2, no fast-math, no FMA contraction: every FP64 operation is the one written.
GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build() -> str:
    """Compile the oracle library in place (always recompiles)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc"] + GCC_FLAGS + [_SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.cmo_flow_field.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P]
    lib.cmo_flow_field.restype = ctypes.c_int
    lib.cmo_forward.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P,
                                P, P, P]
    lib.cmo_forward.restype = ctypes.c_int
    lib.cmo_backward.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P,
                                 ctypes.c_double, P, P, P]
    lib.cmo_backward.restype = ctypes.c_int
    lib.cmo_geo.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P,
                            ctypes.c_double, P, P, P, P]
    lib.cmo_geo.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    """Widen to FP64 (exact for FP32 data)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _window_args(win, rho=None, theta=None):
    """The window's arrays as the oracle takes them.  FP32 fields (the form the
    GPU library reads) widen exactly; FP64 arrays pass through unchanged so
    that finite-difference tests can perturb below FP32 resolution.  rho is
    [H, W] with theta [6] (one flow), or [F, H, W] with theta [F, 6] (one flow
    per segment between consecutive knots {0, 1} U refs)."""
    rho = _f64(win.rho if rho is None else rho)
    theta = _f64(win.theta if theta is None else theta)
    K = _f64([_as_f(win.fx), _as_f(win.fy), _as_f(win.cx), _as_f(win.cy)])
    refs = _f64(win.refs)
    x, y, t = _f64(win.x), _f64(win.y), _f64(win.t)
    p = np.ascontiguousarray(np.asarray(win.p, dtype=np.int8))
    return K, refs, x, y, t, p, rho, theta


def _as_f(v):
    """Scalars of the window descriptor are FP32 on the GPU side."""
    return float(np.float32(v)) if not isinstance(v, np.float64) else float(v)


def _eps(win):
    return ctypes.c_double(_as_f(win.eps))


def flow_field(width, height, K, rho, theta, model: int = 0) -> np.ndarray:
    """Eq. 2: flow [H, W, 2] in px per window (model 0: first order, 1: exact
    reprojection)."""
    lib = _load()
    K = _f64(K)
    rho = _f64(rho)
    theta = _f64(theta)
    u = np.empty((height, width, 2), dtype=np.float64)
    st = lib.cmo_flow_field(width, height, _ptr(K), _ptr(rho), _ptr(theta), int(model), _ptr(u))
    if st != 0:
        raise ValueError(f"cmo_flow_field failed ({st})")
    return u


def n_flows(rho) -> int:
    """Number of flow sets an inverse-depth array holds ([H, W] -> 1)."""
    return 1 if np.ndim(rho) == 2 else int(np.shape(rho)[0])


def forward(win, rho=None, theta=None, images=False, valid=False, positions=False) -> dict:
    """Loss and per-reference terms of Eq. 1 for one window.

    Returns dict(loss, num[R], nact[R]) and optionally
    images [R, 2 pol, 2 (C,S), H, W], valid [n] bool, positions [n, R, 2]."""
    lib = _load()
    K, refs, x, y, t, p, rho, theta = _window_args(win, rho, theta)
    F = n_flows(rho)
    R = refs.shape[0]
    n = x.shape[0]
    out = np.zeros(1 + 2 * R, dtype=np.float64)
    img = np.zeros((R, 2, 2, win.height, win.width), dtype=np.float64) if images else None
    val = np.zeros(n, dtype=np.uint8) if valid else None
    pos = np.zeros((n, R, 2), dtype=np.float64) if positions else None
    st = lib.cmo_forward(win.width, win.height, _ptr(K), R, _ptr(refs), _eps(win), F,
                         _flow_model(win), n, _ptr(x), _ptr(y), _ptr(t), _ptr(p), _ptr(rho), _ptr(theta), _ptr(out),
                         _ptr(img), _ptr(val), _ptr(pos))
    if st != 0:
        raise ValueError(f"cmo_forward failed ({st})")
    res = dict(loss=float(out[0]), num=out[1:1 + R].copy(), nact=out[1 + R:].copy())
    if images:
        res["images"] = img
    if valid:
        res["valid"] = val.astype(bool)
    if positions:
        res["positions"] = pos
    return res


def loss(win, rho=None, theta=None) -> float:
    return forward(win, rho, theta)["loss"]


def backward(win, rho=None, theta=None, grad_loss: float = 1.0, flow_grad=False) -> dict:
    """Gradient of the loss: dict(drho, dtheta) (+ dflow) shaped like the flow
    sets: [H, W], [6], [H, W, 2] for one flow; [F, H, W], [F, 6], [F, H, W, 2]
    for F."""
    lib = _load()
    K, refs, x, y, t, p, rho, theta = _window_args(win, rho, theta)
    R = refs.shape[0]
    n = x.shape[0]
    F = n_flows(rho)
    lead = () if rho.ndim == 2 else (F,)
    drho = np.zeros(lead + (win.height, win.width), dtype=np.float64)
    dth = np.zeros(lead + (6,), dtype=np.float64)
    dflow = np.zeros(lead + (win.height, win.width, 2), dtype=np.float64) if flow_grad else None
    st = lib.cmo_backward(win.width, win.height, _ptr(K), R, _ptr(refs), _eps(win), F,
                          _flow_model(win), n, _ptr(x), _ptr(y), _ptr(t), _ptr(p), _ptr(rho), _ptr(theta),
                          ctypes.c_double(grad_loss), _ptr(drho), _ptr(dth), _ptr(dflow))
    if st != 0:
        raise ValueError(f"cmo_backward failed ({st})")
    res = dict(drho=drho, dtheta=dth)
    if flow_grad:
        res["dflow"] = dflow
    return res


# ---------------------------------------------------------------------------
# Geometry consistency (Eq. 3) and the full loss (Eq. 4)
# ---------------------------------------------------------------------------

LAMBDA_GEO = 0.05       # weight of L_geo in the paper's training set-up


def geo(win, rho=None, theta=None, grad=False, grad_loss: float = 1.0) -> dict:
    """L_geo (Eq. 3) of a window's consecutive flow sets: dict(loss,
    pairs [F-1, 2] = per-pair (mean over V, |V|)) and, with grad, drho and
    dtheta shaped like the flow sets (grad_loss * dL_geo/d(.)).  A window with
    one flow set has L_geo = 0."""
    lib = _load()
    rho = _f64(win.rho if rho is None else rho)
    theta = _f64(win.theta if theta is None else theta)
    K = _f64([_as_f(win.fx), _as_f(win.fy), _as_f(win.cx), _as_f(win.cy)])
    refs = _f64(win.refs)
    F = n_flows(rho)
    out = np.zeros(1, np.float64)
    pairs = np.zeros((max(F - 1, 0), 2), np.float64)
    drho = np.zeros(rho.shape, np.float64) if grad else None
    dth = np.zeros(theta.shape, np.float64) if grad else None
    st = lib.cmo_geo(win.width, win.height, _ptr(K), refs.shape[0], _ptr(refs), F, _ptr(rho),
                     _ptr(theta), ctypes.c_double(grad_loss), _ptr(out),
                     _ptr(pairs) if F > 1 else None, _ptr(drho), _ptr(dth))
    if st != 0:
        raise ValueError(f"cmo_geo failed ({st})")
    res = dict(loss=float(out[0]), pairs=pairs)
    if grad:
        res["drho"], res["dtheta"] = drho, dth
    return res


def rsat(win, rho=None, theta=None) -> float:
    """RSAT (ratio of squared average timestamps, the paper's deblurring
    metric after Hagenaars et al.): the loss of Eq. 1 at the window's motion
    over the loss with zero motion (no warp).  Below 1: the warp sharpens."""
    th = _f64(win.theta if theta is None else theta)
    return loss(win, rho, th) / loss(win, rho, np.zeros_like(th))


def full_loss(win, lam: float = LAMBDA_GEO, rho=None, theta=None) -> float:
    """Eq. 4: L = L_CM + lambda L_geo."""
    return loss(win, rho, theta) + lam * geo(win, rho, theta)["loss"]


def full_backward(win, lam: float = LAMBDA_GEO, grad_loss: float = 1.0) -> dict:
    """Gradient of Eq. 4: the CM gradient plus lambda times the L_geo one."""
    b = backward(win, grad_loss=grad_loss)
    g = geo(win, grad=True, grad_loss=grad_loss)
    return dict(drho=b["drho"] + lam * g["drho"], dtheta=b["dtheta"] + lam * g["dtheta"])


# ---------------------------------------------------------------------------
# Canonical-order mirror of the deterministic mode (cm_mirror.c)
# ---------------------------------------------------------------------------

_MIRROR_SRC = os.path.join(_HERE, "cm_mirror.c")
_MIRROR_PATH = os.path.join(_HERE, "libcm_mirror.so")
_mirror = None


def build_mirror() -> str:
    tmp = _MIRROR_PATH + ".tmp"
    subprocess.run(["gcc"] + GCC_FLAGS + [_MIRROR_SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, _MIRROR_PATH)
    return _MIRROR_PATH


def _flow_model(win) -> int:
    """0: first-order flow (motion field), 1: exact reprojection."""
    m = int(getattr(win, "flow_model", 0))
    if m not in (0, 1):
        raise ValueError(f"flow_model must be 0 or 1, got {m}")
    return m


def _load_mirror():
    global _mirror
    if _mirror is None:
        if not os.path.exists(_MIRROR_PATH):
            build_mirror()
        lib = ctypes.CDLL(_MIRROR_PATH)
        P = ctypes.c_void_p
        lib.cmm_forward.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_float,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P,
                                    P, P]
        lib.cmm_forward.restype = ctypes.c_int
        lib.cmm_backward.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P,
                                     ctypes.c_float, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                     P, P, P, P, P, P, ctypes.c_float, P, P]
        lib.cmm_backward.restype = ctypes.c_int
        _mirror = lib
    return _mirror


def _mirror_args(win):
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return (f([win.fx, win.fy, win.cx, win.cy]), f(win.refs), f(win.x), f(win.y), f(win.t),
            np.ascontiguousarray(np.asarray(win.p, dtype=np.int8)), f(win.rho), f(win.theta))


def mirror_forward(win) -> dict:
    """Deterministic-mode forward in its canonical order: dict(loss (float32),
    loss64, n_valid, num [R], nact [R])."""
    lib = _load_mirror()
    K, refs, x, y, t, p, rho, th = _mirror_args(win)
    R = refs.shape[0]
    loss = np.zeros(1, np.float32)
    hdr = np.zeros(2 + 2 * R, np.float64)
    st = lib.cmm_forward(win.width, win.height, _ptr(K), R, _ptr(refs), float(np.float32(win.eps)),
                         n_flows(rho), _flow_model(win), x.shape[0], _ptr(x), _ptr(y), _ptr(t), _ptr(p), _ptr(rho), _ptr(th),
                         _ptr(loss), _ptr(hdr))
    if st != 0:
        raise ValueError(f"cmm_forward failed ({st})")
    return dict(loss=loss[0], loss64=hdr[0], n_valid=int(hdr[1]), num=hdr[2:2 + R],
                nact=hdr[2 + R:])


def mirror_backward(win, grad_loss: float = 1.0) -> dict:
    """Deterministic-mode backward in its canonical order: dict(drho float32
    [H, W] or [F, H, W], dtheta float32 [6] or [F, 6])."""
    lib = _load_mirror()
    K, refs, x, y, t, p, rho, th = _mirror_args(win)
    R = refs.shape[0]
    F = n_flows(rho)
    lead = () if rho.ndim == 2 else (F,)
    drho = np.zeros(lead + (win.height, win.width), np.float32)
    dth = np.zeros(lead + (6,), np.float32)
    st = lib.cmm_backward(win.width, win.height, _ptr(K), R, _ptr(refs),
                          float(np.float32(win.eps)), F, _flow_model(win), x.shape[0], _ptr(x), _ptr(y), _ptr(t),
                          _ptr(p), _ptr(rho), _ptr(th), float(np.float32(grad_loss)), _ptr(drho),
                          _ptr(dth))
    if st != 0:
        raise ValueError(f"cmm_backward failed ({st})")
    return dict(drho=drho, dtheta=dth)

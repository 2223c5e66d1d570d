"""Shared helpers for the GPU tests: move a window to the device, compare with
the oracle within the tolerances the design fixes."""

import numpy as np
import torch

LOSS_RTOL = 1e-5          # relative, on the loss
GRAD_RTOL = 1e-4          # relative, on gradient norms


def to_device(win, device="cuda:0"):
    f = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).to(device)
    return dict(x=f(win.x), y=f(win.y), t=f(win.t),
                p=torch.from_numpy(np.ascontiguousarray(np.asarray(win.p, dtype=np.int8))).to(device),
                rho=f(win.rho).reshape(np.shape(win.rho)), ego=f(win.theta))


def assert_loss_close(got, want, rtol=LOSS_RTOL, what=""):
    assert abs(got - want) <= rtol * abs(want) + 1e-12, \
        f"{what} loss {got!r} vs oracle {want!r} (rel {abs(got - want) / max(abs(want), 1e-300):.3g})"


def assert_grads_close(g_rho, g_th, o_rho, o_th, rtol=GRAD_RTOL, what=""):
    """d rho: ||diff||_2 <= rtol ||g||_2 and max|diff| <= 10 rtol ||g||_inf;
    d theta: |diff_i| <= rtol ||g_theta||_inf."""
    g_rho = np.asarray(g_rho, dtype=np.float64).reshape(o_rho.shape)
    g_th = np.asarray(g_th, dtype=np.float64)
    d = g_rho - o_rho
    n2 = np.linalg.norm(o_rho)
    ninf = np.abs(o_rho).max() if o_rho.size else 0.0
    assert np.linalg.norm(d) <= rtol * n2 + 1e-30, \
        f"{what} d rho: rel L2 err {np.linalg.norm(d) / max(n2, 1e-300):.3g}"
    assert np.abs(d).max() <= 10 * rtol * ninf + 1e-30, \
        f"{what} d rho: max err {np.abs(d).max():.3g} vs ||g||inf {ninf:.3g}"
    tinf = np.abs(o_th).max()
    assert np.all(np.abs(g_th - o_th) <= rtol * tinf + 1e-30), \
        f"{what} d theta {g_th} vs oracle {o_th}"

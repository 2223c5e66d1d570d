"""Seeded synthetic event windows shaped like the paper's CM workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
holds randomness and a scene simulator only; it contains none of the
contrast-maximization arithmetic (no motion-field formula, no bilinear
sampling, no warp, splat or loss).  Events are produced by simulating a
camera that moves rigidly through a static scene: back-projected edge points
are moved with the exact rigid motion X(t) = exp(t [w]x) X0 + t v and
re-projected with the pinhole model.  The method under test models the same
motion with the first-order motion field, so at the generating parameters the
events line up to first order, which is what gives the image of warped events
its sharp edges (the situation the paper's Sec. 3.1 describes).

Workloads (sizes from the paper's datasets: 1k-10k events per bin, 10 bins per
window, up to 100k per bin on DSEC; see the paper's Sec. 3.3 and the
supplement's training details):

  c1  64x64, f=50, 2,000 uniform random events, 1 reference time {1}
  c2  640x480, f=300, 100k edge-map events (50 segments), refs {0, 1/2, 1}
  c3  64 windows at 346x260, f=200, log-uniform 5k..200k events, refs {0, 1}
  c4  Poisson stream, 346x260 (f=200) or 640x480 (f=300), 1k..500k events, refs {0, 1}
  c5  1280x720, f=600, 2M events (400 segments), 8 refs evenly spaced in [0, 1]
  c6  64 windows at 346x260, f=200, 10 bins of 1k..10k events each (log-uniform),
      refs at the 11 bin edges, one inverse depth and ego-motion per bin (the
      paper's training setting: flows of consecutive slices concatenated)

Seeds: numpy PCG64 with seed = 1000 * config_number + window_index.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

EPS_DEFAULT = 1e-9


@dataclasses.dataclass
class Window:
    """One CM window: sensor, intrinsics, reference times, events, rho, theta.

    x, y, t are float32 arrays of length n, p is int8 (+1 / -1).  rho is the
    per-pixel inverse depth, float32 [H, W] (row-major, row y, column x), or
    [F, H, W] for F flow sets.  theta is float32 [6] = (v_x, v_y, v_z, w_x,
    w_y, w_z), or [F, 6].  flow_model: 0 for the first-order motion field of
    Eq. 2, 1 for exact reprojection.
    """

    name: str
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    refs: np.ndarray
    x: np.ndarray
    y: np.ndarray
    t: np.ndarray
    p: np.ndarray
    rho: np.ndarray
    theta: np.ndarray
    eps: float = EPS_DEFAULT
    flow_model: int = 0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def intrinsics(self) -> np.ndarray:
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)

    def replace(self, **kw) -> "Window":
        return dataclasses.replace(self, **kw)

    def subsample(self, n: int, seed: int = 0) -> "Window":
        """A window with a random subset of n events (time order kept)."""
        n = min(n, self.n)
        rng = np.random.default_rng(seed)
        idx = np.sort(rng.choice(self.n, size=n, replace=False))
        return self.replace(x=self.x[idx].copy(), y=self.y[idx].copy(),
                            t=self.t[idx].copy(), p=self.p[idx].copy())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# Inverse-depth maps
# ----------------------------------------------------------------------------

class _GaussianBumps:
    """rho(x, y) = base + amp * sum_i exp(-|x - mu_i|^2 / (2 sigma^2)), optionally
    min-max normalised over the pixel grid and mapped to [lo, hi]."""

    def __init__(self, mus, sigma, base=0.0, amp=1.0, norm_range=None, grid=None):
        self.mus = np.asarray(mus, dtype=np.float64)
        self.sigma = float(sigma)
        self.base = base
        self.amp = amp
        self.norm_range = norm_range
        self.gmin = self.gmax = None
        if norm_range is not None:
            W, H = grid
            g = self._raw(*np.meshgrid(np.arange(W, dtype=np.float64),
                                       np.arange(H, dtype=np.float64)))
            self.gmin, self.gmax = float(g.min()), float(g.max())

    def _raw(self, xs, ys):
        g = np.zeros(np.broadcast(xs, ys).shape, dtype=np.float64)
        for mx, my in self.mus:
            g += np.exp(-((xs - mx) ** 2 + (ys - my) ** 2) / (2.0 * self.sigma ** 2))
        return g

    def __call__(self, xs, ys):
        g = self._raw(xs, ys)
        if self.norm_range is None:
            return self.base + self.amp * g
        lo, hi = self.norm_range
        n = np.clip((g - self.gmin) / max(self.gmax - self.gmin, 1e-300), 0.0, 1.0)
        return lo + (hi - lo) * n

    def grid(self, W, H) -> np.ndarray:
        xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
        return self(xs, ys).astype(np.float32)


# ----------------------------------------------------------------------------
# Scene simulation (exact rigid motion, pinhole projection)
# ----------------------------------------------------------------------------

def _rotate(points, phi):
    """Rotate 3-vectors `points` [n,3] by rotation vectors `phi` [n,3] (Rodrigues)."""
    ang = np.linalg.norm(phi, axis=1)
    small = ang < 1e-12
    safe = np.where(small, 1.0, ang)
    k = phi / safe[:, None]
    c = np.cos(ang)[:, None]
    s = np.sin(ang)[:, None]
    kx = np.cross(k, points)
    kd = np.sum(k * points, axis=1, keepdims=True)
    out = points * c + kx * s + k * kd * (1.0 - c)
    return np.where(small[:, None], points, out)


def _simulate_edge_events(rng, n_events, W, H, fx, fy, cx, cy, rho_fn, v, w, n_segments,
                          max_rounds=400, subpixel=False):
    """Events of a random edge map observed by a camera in constant rigid motion.

    Each event: t ~ U[0,1]; a segment picked with probability proportional to
    its length and a point q uniform on it (image at t = 0); q is back-projected
    at depth 1/rho(q), moved by the camera motion to time t, projected, rounded
    to the nearest pixel and kept if it lands on the sensor in front of the
    camera.  Polarity is the segment's contrast sign.  Sampling repeats until
    n_events are kept; the result is sorted by time.

    subpixel: keep the projected position real-valued (undistorted, rectified
    events, as the supplement's training data are) instead of rounding it to
    the pixel; see _subpixel_mix for the share placed on integers and borders.
    """
    A = np.stack([rng.uniform(0, W - 1, n_segments), rng.uniform(0, H - 1, n_segments)], 1)
    B = np.stack([rng.uniform(0, W - 1, n_segments), rng.uniform(0, H - 1, n_segments)], 1)
    sign = np.where(rng.random(n_segments) < 0.5, 1, -1).astype(np.int8)
    seglen = np.linalg.norm(B - A, axis=1) + 1e-9
    prob = seglen / seglen.sum()
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)

    xs, ys, ts, ps = [], [], [], []
    have = 0
    accept = 0.5
    for _ in range(max_rounds):
        need = n_events - have
        if need <= 0:
            break
        m = int(min(max(need / max(accept, 0.02) * 1.2 + 1024, 4096), 8_000_000))
        t = rng.random(m).astype(np.float32)
        seg = rng.choice(n_segments, size=m, p=prob)
        s = rng.random(m)
        q = A[seg] + s[:, None] * (B[seg] - A[seg])
        rho_q = rho_fn(q[:, 0], q[:, 1])
        depth = 1.0 / rho_q
        X0 = np.stack([(q[:, 0] - cx) / fx * depth, (q[:, 1] - cy) / fy * depth, depth], 1)
        tt = t.astype(np.float64)[:, None]
        Xt = _rotate(X0, tt * w[None, :]) + tt * v[None, :]
        front = Xt[:, 2] > 1e-3
        Z = np.where(front, Xt[:, 2], 1.0)
        px = fx * Xt[:, 0] / Z + cx
        py = fy * Xt[:, 1] / Z + cy
        if not subpixel:
            px = np.rint(px)
            py = np.rint(py)
        ok = front & (px >= 0) & (px <= W - 1) & (py >= 0) & (py <= H - 1)
        accept = 0.7 * accept + 0.3 * max(float(ok.mean()), 1e-4)
        idx = np.nonzero(ok)[0][:need]
        xs.append(px[idx].astype(np.float32))
        ys.append(py[idx].astype(np.float32))
        ts.append(t[idx])
        ps.append(sign[seg[idx]])
        have += idx.size
    if have < n_events:
        raise RuntimeError(f"edge-map simulation kept only {have}/{n_events} events")
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    t = np.concatenate(ts)
    p = np.concatenate(ps)
    if subpixel:
        x, y = _subpixel_mix(rng, x, y, W, H)
    order = np.argsort(t, kind="stable")
    return x[order], y[order], t[order], p[order]


SUBPIXEL_ON_INTEGER = 0.10      # share of real-valued events moved onto a pixel centre
SUBPIXEL_ON_BORDER = 0.02       # share moved onto the image border (one coordinate)
SUBPIXEL_ON_ROW = 0.05          # share with one coordinate on an integer, the other real


def _subpixel_mix(rng, x, y, W, H):
    """Real-valued event coordinates (float32, inside [0, W-1] x [0, H-1]) with
    the special positions of the bilinear kernel mixed in: a share exactly on
    pixel centres, a share with one integer coordinate, and a share exactly on
    the image border (x = 0, x = W-1, y = 0 or y = H-1), the rest as projected."""
    x = np.asarray(x, np.float32).copy()
    y = np.asarray(y, np.float32).copy()
    n = x.shape[0]
    u = rng.random(n)
    on_int = u < SUBPIXEL_ON_INTEGER
    x[on_int] = np.rint(x[on_int])
    y[on_int] = np.rint(y[on_int])
    on_row = (u >= SUBPIXEL_ON_INTEGER) & (u < SUBPIXEL_ON_INTEGER + SUBPIXEL_ON_ROW)
    which = rng.random(n) < 0.5
    x[on_row & which] = np.rint(x[on_row & which])
    y[on_row & ~which] = np.rint(y[on_row & ~which])
    lo = SUBPIXEL_ON_INTEGER + SUBPIXEL_ON_ROW
    on_border = (u >= lo) & (u < lo + SUBPIXEL_ON_BORDER)
    side = rng.integers(0, 4, n)
    x[on_border & (side == 0)] = 0.0
    x[on_border & (side == 1)] = np.float32(W - 1)
    y[on_border & (side == 2)] = 0.0
    y[on_border & (side == 3)] = np.float32(H - 1)
    np.clip(x, 0.0, np.float32(W - 1), out=x)
    np.clip(y, 0.0, np.float32(H - 1), out=y)
    return x, y


# ----------------------------------------------------------------------------
# Workload configurations
# ----------------------------------------------------------------------------

SENSORS = {
    "64x64": dict(width=64, height=64, f=50.0),
    "346x260": dict(width=346, height=260, f=200.0),
    "640x480": dict(width=640, height=480, f=300.0),
    "1280x720": dict(width=1280, height=720, f=600.0),
}


def refs_even(k: int) -> np.ndarray:
    """k reference times evenly spaced in [0, 1] (k >= 2), as float32."""
    return np.array([i / (k - 1) for i in range(k)], dtype=np.float32)


def uniform_window(seed: int, sensor: str = "64x64", n_events: int = 2000,
                   refs=(1.0,), motion_sigma: float = 0.3, name: str = "c1",
                   subpixel: bool = False) -> Window:
    """Config c1: integer-uniform x, y; t ~ U[0,1] sorted; fair-coin polarity;
    rho = 0.5 + sum of three Gaussian bumps (amplitude 0.5, sigma 8 px).
    subpixel: x, y uniform over the closed image box instead (real-valued,
    with the mix of integer and border positions of _subpixel_mix)."""
    s = SENSORS[sensor]
    W, H, f = s["width"], s["height"], s["f"]
    rng = _rng(seed)
    x = rng.integers(0, W, n_events).astype(np.float32)
    y = rng.integers(0, H, n_events).astype(np.float32)
    if subpixel:
        x, y = _subpixel_mix(rng, rng.uniform(0, W - 1, n_events),
                             rng.uniform(0, H - 1, n_events), W, H)
    t = np.sort(rng.random(n_events).astype(np.float32))
    p = np.where(rng.random(n_events) < 0.5, 1, -1).astype(np.int8)
    mus = np.stack([rng.uniform(0, W - 1, 3), rng.uniform(0, H - 1, 3)], 1)
    rho = _GaussianBumps(mus, 8.0, base=0.5, amp=0.5).grid(W, H)
    theta = rng.normal(0.0, motion_sigma, 6).astype(np.float32)
    return Window(name, W, H, f, f, (W - 1) / 2.0, (H - 1) / 2.0,
                  np.asarray(refs, dtype=np.float32), x, y, t, p, rho, theta)


def edge_window(seed: int, sensor: str, n_events: int, refs, n_segments: int = 50,
                motion_sigma: float = 0.5, name: str = "edge", subpixel: bool = False) -> Window:
    """Configs c2-c5: events of a moving random edge map.

    rho = 0.2 + 1.8 * (min-max normalised sum of 4 Gaussians, sigma = W/6);
    v, w ~ N(0, motion_sigma^2) per axis.  subpixel: real-valued event
    coordinates (see _simulate_edge_events).
    """
    s = SENSORS[sensor]
    W, H, f = s["width"], s["height"], s["f"]
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    rng = _rng(seed)
    mus = np.stack([rng.uniform(0, W - 1, 4), rng.uniform(0, H - 1, 4)], 1)
    rho_fn = _GaussianBumps(mus, W / 6.0, norm_range=(0.2, 2.0), grid=(W, H))
    rho = rho_fn.grid(W, H)
    theta = rng.normal(0.0, motion_sigma, 6).astype(np.float32)
    v = theta[:3].astype(np.float64)
    w = theta[3:].astype(np.float64)
    x, y, t, p = _simulate_edge_events(rng, n_events, W, H, f, f, cx, cy, rho_fn, v, w,
                                       n_segments, subpixel=subpixel)
    return Window(name, W, H, f, f, cx, cy, np.asarray(refs, dtype=np.float32),
                  x, y, t, p, rho, theta)


def motion_stream(seed: int, n_windows: int, sensor: str = "346x260", n_events: int = 20000,
                  refs=(0.0, 0.5, 1.0), motion_sigma: float = 0.3, drift: float = 0.03,
                  n_segments: int = 20) -> List[Window]:
    """Windows of one stream for online fitting: a fixed edge map and depth
    (drawn as in edge_window), camera motion theta_0 ~ N(0, motion_sigma^2)
    per axis drifting by N(0, drift^2) per axis from one window to the next.
    Each window observes the same edge map (same segments and event draws)
    under its own motion; theta of window k is its ground truth."""
    s = SENSORS[sensor]
    W, H, f = s["width"], s["height"], s["f"]
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    rng = _rng(seed)
    mus = np.stack([rng.uniform(0, W - 1, 4), rng.uniform(0, H - 1, 4)], 1)
    rho_fn = _GaussianBumps(mus, W / 6.0, norm_range=(0.2, 2.0), grid=(W, H))
    rho = rho_fn.grid(W, H)
    theta = rng.normal(0.0, motion_sigma, 6)
    out = []
    for k in range(n_windows):
        if k > 0:
            theta = theta + rng.normal(0.0, drift, 6)
        th = theta.astype(np.float32)
        x, y, t, p = _simulate_edge_events(_rng(seed + 77), n_events, W, H, f, f, cx, cy, rho_fn,
                                           th[:3].astype(np.float64), th[3:].astype(np.float64),
                                           n_segments)
        out.append(Window(f"stream{k}", W, H, f, f, cx, cy, np.asarray(refs, dtype=np.float32),
                          x, y, t, p, rho, th))
    return out


def knots_of(refs) -> np.ndarray:
    """Sorted knots {0, 1} U refs (refs sorted and in [0, 1])."""
    k = [float(r) for r in refs]
    if k[0] > 0.0:
        k = [0.0] + k
    if k[-1] < 1.0:
        k = k + [1.0]
    return np.asarray(k)


def with_flow_sets(win: Window, seed: int, jitter: float = 0.15) -> Window:
    """The window with one inverse depth and ego-motion per segment between
    consecutive knots {0, 1} U refs.  Each set is the window's own, perturbed:
    rho times a smooth positive field (1 + jitter * bump), theta plus
    N(0, jitter^2 |theta|_rms^2) per axis."""
    F = len(knots_of(win.refs)) - 1
    rng = _rng(seed)
    W, H = win.width, win.height
    rhos, thetas = [], []
    base_rho = np.asarray(win.rho, np.float64)
    base_th = np.asarray(win.theta, np.float64)
    scale = float(np.sqrt(np.mean(base_th ** 2))) or 1.0
    for _ in range(F):
        mus = np.stack([rng.uniform(0, W - 1, 2), rng.uniform(0, H - 1, 2)], 1)
        bump = _GaussianBumps(mus, W / 5.0, base=0.0, amp=1.0).grid(W, H)
        rhos.append(base_rho * (1.0 + jitter * (bump - 0.5)))
        thetas.append(base_th + rng.normal(0.0, jitter * scale, 6))
    return win.replace(rho=np.stack(rhos).astype(np.float32),
                       theta=np.stack(thetas).astype(np.float32))


def bins_window(index: int, n_bins: int = 10, sensor: str = "346x260",
                per_bin=(1e3, 1e4), subpixel: bool = False) -> Window:
    """Workload c6: an edge-map window of n_bins slices with log-uniform 1k..10k
    events per slice, references at the n_bins + 1 slice edges and one flow
    set per slice."""
    seed = 1000 * 6 + index
    counts = log_uniform_counts(_rng(seed + 500), n_bins, *per_bin)
    refs = np.linspace(0.0, 1.0, n_bins + 1)
    win = edge_window(seed, sensor, int(counts.sum()), refs=refs, n_segments=50, name="c6",
                      subpixel=subpixel)
    return with_flow_sets(win, seed + 700)


def log_uniform_counts(rng, n, lo, hi) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)


def make_window(config: str, index: int = 0, n_events: Optional[int] = None,
                subpixel: bool = False) -> Window:
    """The `index`-th window of workload `config` (c1, c2, c3, c5, c6).
    subpixel: the same workload with real-valued event coordinates (names
    get a "/sub" suffix)."""
    sfx = "/sub" if subpixel else ""
    if config == "c1":
        return uniform_window(1000 * 1 + index, n_events=n_events or 2000, subpixel=subpixel,
                              name="c1" + sfx)
    if config == "c2":
        return edge_window(1000 * 2 + index, "640x480", n_events or 100_000,
                           refs=[0.0, 0.5, 1.0], n_segments=50, name="c2" + sfx,
                           subpixel=subpixel)
    if config == "c3":
        counts = log_uniform_counts(_rng(1000 * 3 + 999), 64, 5e3, 2e5)
        n = n_events or int(counts[index % 64])
        return edge_window(1000 * 3 + index, "346x260", n, refs=[0.0, 1.0],
                           n_segments=50, name="c3" + sfx, subpixel=subpixel)
    if config == "c5":
        return edge_window(1000 * 5 + index, "1280x720", n_events or 2_000_000,
                           refs=refs_even(8), n_segments=400, name="c5" + sfx,
                           subpixel=subpixel)
    if config == "c6":
        return bins_window(index, subpixel=subpixel).replace(name="c6" + sfx)
    raise ValueError(f"unknown config {config!r}")


def make_batch(config: str = "c3", n_windows: int = 64, scale: float = 1.0,
               subpixel: bool = False) -> List[Window]:
    """Workload c3 (or c6): n_windows windows with log-uniform event counts
    (optionally scaled)."""
    if config == "c6":
        return [make_window("c6", i, subpixel=subpixel) for i in range(n_windows)]
    counts = log_uniform_counts(_rng(1000 * 3 + 999), 64, 5e3, 2e5)
    out = []
    for i in range(n_windows):
        n = max(1, int(round(counts[i % 64] * scale)))
        out.append(make_window(config, i, n_events=n, subpixel=subpixel))
    return out


def poisson_stream(rate_hz: float = 500.0, duration_s: float = 20.0, seed: int = 4000,
                   n_lo: float = 1e3, n_hi: float = 5e5):
    """Workload c4 arrival trace: (arrival_time_s, sensor, n_events) per window.

    Arrivals are a Poisson process; sensors are 50/50 346x260 / 640x480; event
    counts are log-uniform in [n_lo, n_hi]."""
    rng = _rng(seed)
    times = []
    tnow = 0.0
    while True:
        tnow += rng.exponential(1.0 / rate_hz)
        if tnow >= duration_s:
            break
        times.append(tnow)
    k = len(times)
    sensors = np.where(rng.random(k) < 0.5, "346x260", "640x480")
    counts = log_uniform_counts(rng, k, n_lo, n_hi)
    return [(times[i], str(sensors[i]), int(counts[i])) for i in range(k)]


def stream_window(sensor: str, n_events: int, seed: int) -> Window:
    """One window of the c4 stream (edge map, refs {0, 1})."""
    return edge_window(seed, sensor, n_events, refs=[0.0, 1.0], n_segments=50, name="c4")


def stream_pool(n_per_sensor: int = 2, n_events: int = 500_000, seed: int = 4100):
    """Base windows the c4 stream draws from: n_per_sensor edge-map windows of
    n_events events per sensor (346x260 and 640x480), refs {0, 1}."""
    pool = {}
    for s, sensor in enumerate(("346x260", "640x480")):
        pool[sensor] = [stream_window(sensor, n_events, seed + 10 * s + i)
                        for i in range(n_per_sensor)]
    return pool


def thin(win: Window, n: int, offset: int = 0) -> Window:
    """A window of about n events taken as every k-th event of `win` (time order
    kept, the time span unchanged): a cheap way to vary the event count."""
    k = max(1, win.n // max(n, 1))
    sl = slice(offset % k, None, k)
    return win.replace(x=win.x[sl][:n], y=win.y[sl][:n], t=win.t[sl][:n], p=win.p[sl][:n])

"""Online learning on an event stream (the paper's on-board fine-tuning,
Sec. 4): the camera's ego-motion -- and, optionally, inverse depth -- fitted
window after window by gradient descent on the full loss
L = L_CM + lambda L_geo (Eq. 4), with RSAT (the loss at the estimate over the
loss without motion) as the quality measure.

The paper fine-tunes a recurrent network whose outputs are these quantities;
here they are the parameters themselves (no network), so the loop exercises
exactly the loss and gradients the library computes.  The stream is seen once,
in order: each window starts from the previous window's estimate, the first
from an initial estimate (e.g. a pre-trained model's).  Zero motion is a poor
start: events sit on pixel centres, so the unwarped image of events is sharp
by construction and the loss jumps as soon as the events move.  Inverse depth
is kept positive as exp(log rho).

    python -m paper_2412_06359_amd.online --windows 8 --steps 30
"""

import argparse
import json
import sys

import numpy as np
import torch

from . import binding as cm


def fit_stream(windows, init_ego, steps: int = 30, lr_ego: float = 0.01,
               fit_depth: bool = False, lr_rho: float = 0.01, lam: float = cm.LAMBDA_GEO,
               device: int = 0, log=None):
    """Fits the windows in stream order.  Without fit_depth the windows'
    inverse depth is used as given.  Returns one record per window:
    dict(window, rsat_start, rsat_end, loss_start, loss_end, ego_err_start,
    ego_err_end) with ego_err the max-abs error against the window's theta."""
    dev = torch.device(f"cuda:{device}")
    records = []
    ego = torch.as_tensor(np.asarray(init_ego, np.float32), device=dev)
    log_rho = None
    for k, win in enumerate(windows):
        desc = cm.WindowDesc.from_window(win)
        f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(np.asarray(a, dt))).to(dev)
        x, y, t = f(win.x, np.float32), f(win.y, np.float32), f(win.t, np.float32)
        p = f(win.p, np.int8)
        rho_true = f(win.rho, np.float32)
        truth = f(win.theta, np.float32)
        if log_rho is None or log_rho.shape != rho_true.shape:
            log_rho = torch.zeros_like(rho_true)
        ego = ego.detach().clone().reshape(truth.shape).requires_grad_(True)
        params = [{"params": [ego], "lr": lr_ego}]
        if fit_depth:
            log_rho = log_rho.detach().clone().requires_grad_(True)
            params.append({"params": [log_rho], "lr": lr_rho})
        opt = torch.optim.Adam(params)
        rho_of = (lambda: torch.exp(log_rho)) if fit_depth else (lambda: rho_true)

        def evaluate():
            with torch.no_grad():
                r, l, _ = cm.rsat(desc, x, y, t, p, rho_of().contiguous(), ego.contiguous())
                err = (ego - truth).abs().max()
            return float(r), float(l), float(err)

        r0, l0, e0 = evaluate()
        for _ in range(steps):
            opt.zero_grad()
            L = cm.full_loss(x, y, t, p, rho_of(), ego, desc, lam)
            L.backward()
            opt.step()
        r1, l1, e1 = evaluate()
        rec = dict(window=k, events=int(win.n), rsat_start=r0, rsat_end=r1, loss_start=l0,
                   loss_end=l1, ego_err_start=e0, ego_err_end=e1,
                   rsat_true=float(cm.rsat(desc, x, y, t, p, rho_true, truth)[0]))
        records.append(rec)
        if log is not None:
            print(json.dumps(rec), file=log, flush=True)
    return records


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--windows", type=int, default=8)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--init-noise", type=float, default=0.05,
                    help="std of the first window's initial ego-motion error")
    ap.add_argument("--fit-depth", action="store_true")
    args = ap.parse_args(argv)
    import eventgen
    cm.load()
    wins = eventgen.motion_stream(args.seed, args.windows)
    rng = np.random.default_rng(args.seed)
    init = np.asarray(wins[0].theta, np.float64) + rng.normal(0.0, args.init_noise, 6)
    fit_stream(wins, init, steps=args.steps, fit_depth=args.fit_depth, log=sys.stdout)


if __name__ == "__main__":
    main()

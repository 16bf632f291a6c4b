"""Learned prescreen of slice proposals (an addition; the paper's sampler
evaluates every proposal exactly).

The network of ``Mlp`` (11 -> 256 -> 256 -> 256 -> 1, GELU) learns log L over
the unit cube from pairs the sampler has already produced: the recent dead
points and the live set of a nested-sampling run, plus the exactly evaluated
proposals of earlier batches.  Inputs are standardised by the mean and spread
of the current live set (the region where proposals land) and targets are
floored a fixed distance below log L*, so the net spends its capacity near the
constraint rather than on the far tail.  A candidate is evaluated exactly when
its prediction is within ``margin`` of log L* or when it is drawn for the
audit; the accept decision always uses the exact value.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import _lib
from .nested import BLOCKS, N_DIM


def library_injection(gw_context_cls, prob, theta, snr=None):
    """Add the library's own template of ``theta`` to ``prob.data``.

    With ``snr`` the distance is rescaled so that the network optimal SNR is
    ``snr``: on a zero-data context the undistorted log L is -<h|h>/2.
    Returns the injected parameter vector.
    """
    import torch
    th = np.array(theta, dtype=np.float64).reshape(1, 13)
    saved = prob.data
    prob.data = np.zeros_like(saved)
    with gw_context_cls(prob) as ctx:
        t = torch.from_numpy(th).cuda()
        if snr is not None:
            out = ctx.loglike(t, marg=_lib.GW_MARG_NONE, prec=_lib.GW_PREC_FP64)
            rho = math.sqrt(-2.0 * float(out[0].item()))
            th[0, 6] *= rho / snr
            t = torch.from_numpy(th).cuda()
        h = ctx.template(t)[0].cpu().numpy()
    prob.data = saved + h
    return th[0]


def block_cholesky(x_live, blocks=BLOCKS):
    out = []
    for b in blocks:
        cov = np.atleast_2d(np.cov(x_live[:, list(b)], rowvar=False)) + 1e-12 * np.eye(len(b))
        out.append(np.linalg.cholesky(cov))
    return out


def slice_candidates(x_live, n, seed, blocks=BLOCKS, w=1.0):
    """``n`` first-shrink slice proposals from live points, all inside the cube.

    A proposal moves a uniformly chosen live point along d = L_b u in a
    uniformly chosen block b (u uniform on the block's unit sphere, L_b the
    Cholesky factor of the live covariance) by t = w (v - r), v and r
    uniform: the first candidate of a bracket of width w at offset r.
    """
    rng = np.random.default_rng(seed)
    chols = block_cholesky(x_live, blocks)
    keep = []
    have = 0
    while have < n:
        m = 2 * (n - have) + 64
        s = rng.integers(len(x_live), size=m)
        bsel = rng.integers(len(blocks), size=m)
        t = w * (rng.uniform(size=m) - rng.uniform(size=m))
        x = x_live[s].copy()
        for bi, b in enumerate(blocks):
            rows = np.nonzero(bsel == bi)[0]
            if rows.size == 0:
                continue
            u = rng.normal(size=(rows.size, len(b)))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            d = u @ chols[bi].T
            x[np.ix_(rows, list(b))] += t[rows, None] * d
        ok = np.all((x >= 0.0) & (x <= 1.0), axis=1)
        keep.append(x[ok])
        have += int(ok.sum())
    return np.concatenate(keep)[:n]


@dataclass
class TrainResult:
    steps: int
    wall_s: float
    loss_first: float
    loss_last: float
    rmse_holdout: float
    n_train: int
    n_holdout: int


class Prescreen:
    """Owns an ``Mlp`` with its scaling, training loop and decision margin."""

    def __init__(self, ctx, seed: int = 7, floor_below: float = 20.0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.mlp = _lib.Mlp(ctx, seed=seed)
        self.seed = seed
        self.floor_below = float(floor_below)
        self.margin = None

    def fit_scaling(self, x_live, y_train):
        xm = x_live.mean(axis=0)
        xs = np.maximum(x_live.std(axis=0), 1e-6)
        self.y_mean = float(np.mean(y_train))
        self.y_std = float(max(np.std(y_train), 1e-6))
        self.mlp.set_scaling(xm, xs, self.y_mean, self.y_std)

    def train(self, x, y, x_live, logl_star, epochs=150, batch=256, lr=3e-3, holdout=0.1):
        """Adam on MSE over (x, max(y, log L* - floor_below)); returns TrainResult.

        x [n, 11] and y [n] are host arrays; a seeded ``holdout`` fraction is
        kept out of training for the RMSE used by ``set_margin``.
        """
        torch = self.torch
        rng = np.random.default_rng(self.seed)
        y = np.maximum(np.asarray(y, dtype=np.float64), logl_star - self.floor_below)
        perm = rng.permutation(len(x))
        n_hold = int(len(x) * holdout)
        hold, tr = perm[:n_hold], perm[n_hold:]
        self.fit_scaling(np.asarray(x_live), y[tr])
        dev = torch.device("cuda", self.ctx.device)
        xt = torch.from_numpy(np.ascontiguousarray(x[tr])).to(dev)
        yt = torch.from_numpy(np.ascontiguousarray(y[tr])).to(dev)
        self._hold = (torch.from_numpy(np.ascontiguousarray(x[hold])).to(dev), y[hold])
        n = len(tr)
        steps_per_epoch = max(1, n // batch)
        total = epochs * steps_per_epoch
        g = torch.Generator().manual_seed(self.seed)
        step = 0
        loss_first = loss_last = float("nan")
        t0 = time.perf_counter()
        for ep in range(epochs):
            order = torch.randperm(n, generator=g).to(dev)
            for j in range(steps_per_epoch):
                idx = order[j * batch:(j + 1) * batch]
                xb = xt.index_select(0, idx).contiguous()
                yb = yt.index_select(0, idx).contiguous()
                # cosine decay to 2 % of lr
                lr_t = lr * (0.02 + 0.98 * 0.5 * (1.0 + math.cos(math.pi * step / total)))
                want = step == 0 or step == total - 1
                loss = self.mlp.train_step(xb, yb, lr_t, want_loss=want)
                if step == 0:
                    loss_first = loss
                if want:
                    loss_last = loss
                step += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rmse = self.holdout_rmse(logl_star)
        return TrainResult(step, wall, loss_first, loss_last, rmse, n, n_hold)

    def predict(self, x, bf16=True):
        return self.mlp.forward(x, bf16=bf16)

    def holdout_rmse(self, logl_star, window=None):
        """RMSE of the BF16 predictions on held-out pairs (within ``window`` of
        log L* when given; the floor applies to both sides)."""
        xh, yh = self._hold
        if len(yh) == 0:
            return float("nan")
        p = self.predict(xh).cpu().numpy()
        p = np.maximum(p, logl_star - self.floor_below)
        sel = np.ones(len(yh), bool) if window is None else np.abs(yh - logl_star) < window
        if not sel.any():
            return float("nan")
        return float(np.sqrt(np.mean((p[sel] - yh[sel]) ** 2)))

    def set_margin(self, logl_star, k=3.0, window=10.0):
        r = self.holdout_rmse(logl_star, window)
        if not np.isfinite(r):
            r = self.holdout_rmse(logl_star)
        self.margin = k * r
        return self.margin

    def screen(self, x, logl_star, audit_frac=0.01, seed=None, like=_lib.GW_FULL, prec=_lib.GW_PREC_MIXED):
        """(log L or -inf, flags, predictions, number of exact evaluations)."""
        if self.margin is None:
            raise RuntimeError("Prescreen.screen: call set_margin first")
        return self.mlp.prescreen(x, logl_star, self.margin, audit_frac=audit_frac,
                                  seed=self.seed if seed is None else seed, use_mlp=True, like=like, prec=prec)

    def close(self):
        self.mlp.close()


def sampler_pairs(sampler, last_iters=None):
    """(x, log L) of the sampler's dead points (the last ``last_iters``
    iterations' worth when given) and its live set, as host arrays."""
    dx = np.array(sampler.dead_x).reshape(-1, N_DIM)
    dl = np.array(sampler.dead_logl)
    if last_iters is not None:
        keep = last_iters * sampler.k
        dx, dl = dx[-keep:], dl[-keep:]
    lx = sampler.x.cpu().numpy()
    ll = sampler.logl.cpu().numpy()
    return np.concatenate([dx, lx]), np.concatenate([dl, ll])

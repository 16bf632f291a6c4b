"""Slice-within-Gibbs nested sampling driven from the host.

Sec. II.B: m live points; every iteration deletes the k lowest-likelihood
points, raises log L* to the largest deleted value, accumulates their prior
volume into the evidence and replaces them by constrained draws.  Sec. II.C /
III.B: a replacement starts from a surviving live point and runs M Gibbs
sweeps over the parameter blocks, each block moved by one hit-and-run slice
step on the GPU along directions from the block covariance of the live
points.  By default a whole sweep is one ``slice_sweep`` call, in which each
chain moves on to its next block as soon as it has finished one; with
``async_sweep=False`` every block is a ``slice_step`` call of its own (all
chains finish the block before any starts the next).  Both give the same
chains bit for bit.  ``blocks=UNBLOCKED`` with ``sweeps=3 * 11`` is the
unblocked nested slice sampler that the sampler-configuration section runs as
a control (M d joint slice steps per iteration, M = 3).  With ``cache=True`` (full band) the sweep keeps each
chain's waveform and reuses it on the extrinsic blocks (Sec. III.B).  With
``marg=GW_MARG_PHASE_TIME`` the phase and coalescence time are marginalised
and d_L is sampled in place of t_c (the paper's GW170817 configuration).
With ``prescreen`` (an addition; see prescreen.py) every exactly evaluated
slice candidate is recorded (unit-cube point, log L) in a device ring buffer,
and from iteration ``start`` on a network trained on the recorded pairs and
the live set screens the candidates inside every sweep, retrained every
``every`` iterations.  The audit draws' false-negative count drives the margin:
whenever more than ``fn_target`` of the audited screened-out candidates since
the last change turn out inside, the margin grows by half.  An accepted point
always carries its exact log L.

The host keeps the FP64 evidence bookkeeping (the k deletions taken in order
with live counts m, m-1, ..., m-k+1), the start-point choice and the block
Cholesky factors; the live points and every likelihood stay on the device.
State can be written to an .npz checkpoint and resumed bit for bit.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import _lib

N_DIM = 11
# Slow blocks {Mc, q, Lambda1, Lambda2}, {chi1}, {chi2}, {iota};
# fast blocks {ra, dec}, {psi}, {t_c} (indices into the unit cube).
BLOCKS = ((0, 1, 4, 5), (2,), (3,), (6,), (7, 8), (9,), (10,))
UNBLOCKED = (tuple(range(N_DIM)),)


def _logsumexp(a):
    a = np.asarray(a, dtype=np.float64)
    if a.size == 0:
        return -math.inf
    m = np.max(a)
    if not np.isfinite(m):
        return float(m)
    return float(m + math.log(np.sum(np.exp(a - m))))


class NestedSampler:
    def __init__(self, ctx, n_live: int = 1000, n_delete: int = 125, seed: int = 6, dlogz: float = 0.1,
                 blocks=BLOCKS, like: int = _lib.GW_HET, prec: int = _lib.GW_PREC_MIXED, sweeps: int = 1,
                 w: float = 1.0, max_out: int = 10, max_shrink: int = 100, async_sweep: bool = True,
                 cache: bool = False, marg: int = _lib.GW_MARG_PHASE_DIST, prescreen: dict | None = None):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.m, self.k = int(n_live), int(n_delete)
        self.seed = int(seed)
        self.dlogz = float(dlogz)
        self.blocks = tuple(tuple(b) for b in blocks)
        self.like, self.prec = like, prec
        self.sweeps, self.w, self.max_out, self.max_shrink = sweeps, w, max_out, max_shrink
        self.async_sweep = bool(async_sweep)
        self.cache = bool(cache)
        self.marg = int(marg)
        if self.cache and (like != _lib.GW_FULL or not self.async_sweep):
            raise ValueError("the waveform cache needs like=GW_FULL and async_sweep=True")
        self.rng = np.random.default_rng(self.seed)
        self.dev = torch.device("cuda", ctx.device)
        x0 = self.rng.uniform(size=(self.m, N_DIM))
        self.x = torch.from_numpy(x0).to(self.dev)
        self.logl = torch.empty(self.m, dtype=torch.float64, device=self.dev)
        self._eval(self.x, self.logl)
        self.dead_logl: list[float] = []
        self.dead_logw: list[float] = []
        self.dead_x: list[np.ndarray] = []
        self._log_z_dead = -math.inf  # log-sum-exp of dead_logw, kept as points die
        self._host = None  # host copies (x, logL) of the live set, or None when stale
        self.log_x = 0.0
        self.iteration = 0
        self.counter = 0
        self.n_evals = self.m
        self.eval_kinds = np.zeros(3, np.int64)  # with the cache: full, cached waveform, cached sums
        self.wall = 0.0
        # learned prescreen: settings, network, counts and training time
        self.pre_cfg = None
        self.pre = None
        self.screen_stats = {"screened": 0, "audited": 0, "audited_inside": 0}
        self.pre_train_s = 0.0
        self.pre_trainings = 0
        self.moves = 0  # blocks that moved (accepted proposals)
        if prescreen is not None:
            from .prescreen import Prescreen
            cfg = dict(start=100, every=50, audit=0.01, steps=1500, retrain_steps=400, batch=1024, seed=7,
                       k_margin=3.0, fn_target=0.02, capacity=1 << 17)
            cfg.update(prescreen)
            self.pre_cfg = cfg
            self.pre = Prescreen(ctx, seed=int(cfg["seed"]))
            cap = int(cfg["capacity"])
            self.rec = (torch.empty((cap, N_DIM), dtype=torch.float64, device=self.dev),
                        torch.empty(cap, dtype=torch.float64, device=self.dev),
                        torch.zeros(1, dtype=torch.int64, device=self.dev))
            self._fn = [0, 0]  # audited, audited and inside since the margin last changed

    # -- likelihood of unit-cube points (initial live set) ------------------
    def _eval(self, x, out):
        torch = self.torch
        th = self._unit_to_theta(x)
        _lib.loglike_batch(self.ctx.handle, th, self.like, self.marg, self.prec, out=out)
        torch.cuda.synchronize()

    def _unit_to_theta(self, x):
        return _lib.gw_prior_transform(self.ctx.handle, x.contiguous(), marg=self.marg)

    # -- evidence ----------------------------------------------------------
    def log_z_dead(self):
        return self._log_z_dead

    def log_z_live(self, logl_host):
        return self.log_x + _logsumexp(logl_host) - math.log(self.m)

    def converged(self, logl_host) -> bool:
        zd = self.log_z_dead()
        if not np.isfinite(zd):
            return False
        return np.logaddexp(zd, self.log_z_live(logl_host)) - zd < self.dlogz

    # -- one iteration -----------------------------------------------------
    def step(self):
        torch = self.torch
        x_host, logl = self.live_host()
        order = np.argsort(logl, kind="stable")
        worst = order[: self.k]
        lstar = float(logl[worst[-1]])
        new_w = []
        for j, i in enumerate(worst):
            new_log_x = self.log_x - 1.0 / (self.m - j)
            self.dead_logl.append(float(logl[i]))
            new_w.append(float(logl[i]) + self.log_x + math.log1p(-math.exp(new_log_x - self.log_x)))
            self.dead_x.append(x_host[i].copy())
            self.log_x = new_log_x
        self.dead_logw.extend(new_w)
        self._log_z_dead = float(np.logaddexp(self._log_z_dead, _logsumexp(new_w)))
        survivors = order[self.k:]
        starts = self.rng.choice(survivors, size=self.k, replace=True)
        chols = []
        x_surv = x_host[survivors]
        for b in self.blocks:
            sub = x_surv[:, list(b)]
            cov = np.atleast_2d(np.cov(sub, rowvar=False)) + 1e-12 * np.eye(len(b))
            chols.append(np.linalg.cholesky(cov))
        idx = torch.from_numpy(starts).to(self.dev)
        xn = self.x.index_select(0, idx).contiguous()
        ln = self.logl.index_select(0, idx).contiguous()
        ne = torch.zeros(self.k, dtype=torch.int32, device=self.dev)
        caps = torch.zeros(self.k, dtype=torch.int32, device=self.dev)
        pre = self._prescreen(lstar)
        sums = []  # per call on the device: (likelihood calls, chains kept), read once per iteration
        moved = 0  # chain-blocks run by those calls
        if self.async_sweep:
            # the M sweeps' blocks in order, at most 16 per call: the same
            # moves as one call per sweep (block j of the sequence draws from
            # counter + j either way)
            seq = [bi for _ in range(self.sweeps) for bi in range(len(self.blocks))]
            for j0 in range(0, len(seq), 16):
                part = seq[j0:j0 + 16]
                st = {} if pre is not None else None
                kinds = _lib.slice_sweep(self.ctx.handle, xn, ln, lstar, [self.blocks[b] for b in part],
                                         [chols[b] for b in part], seed=self.seed, counter=self.counter, w=self.w,
                                         max_out=self.max_out, max_shrink=self.max_shrink, like=self.like,
                                         marg=self.marg, prec=self.prec, n_evals=ne, status=caps,
                                         use_cache=self.cache, prescreen=pre, screen_stats=st,
                                         record=self.rec if self.pre is not None else None)
                if kinds is not None:
                    self.eval_kinds += np.array(kinds, np.int64)
                if st:
                    self._count_screen(st)
                sums.append(torch.stack((ne.sum(), caps.sum())))
                moved += self.k * len(part)
                self.counter += len(part)
        for _ in range(0 if self.async_sweep else self.sweeps):
            for bi, b in enumerate(self.blocks):
                st = {} if pre is not None else None
                _lib.slice_step(self.ctx.handle, xn, ln, lstar, b, chols[bi], seed=self.seed, counter=self.counter,
                                w=self.w, max_out=self.max_out, max_shrink=self.max_shrink, like=self.like,
                                marg=self.marg, prec=self.prec, n_evals=ne, status=caps, prescreen=pre,
                                screen_stats=st, record=self.rec if self.pre is not None else None)
                if st:
                    self._count_screen(st)
                sums.append(torch.stack((ne.sum(), caps.sum())))
                moved += self.k
                self.counter += 1
        wi = torch.from_numpy(worst).to(self.dev)
        self.x.index_copy_(0, wi, xn)
        self.logl.index_copy_(0, wi, ln)
        # one copy back: the new points (to update the host copies) and the counts
        cnt = torch.cat(sums).reshape(-1, 2).sum(0).to(torch.float64) if sums else torch.zeros(2, dtype=torch.float64,
                                                                                                device=self.dev)
        pack = torch.cat((xn.reshape(-1), ln, cnt)).cpu().numpy()
        x_host[worst] = pack[: self.k * N_DIM].reshape(self.k, N_DIM)
        logl[worst] = pack[self.k * N_DIM: self.k * (N_DIM + 1)]
        self.n_evals += int(pack[-2])
        self.moves += moved - int(pack[-1])
        self.iteration += 1

    def live_host(self):
        """Host copies (x [m, 11], logL [m]) of the live set; the sampler keeps
        them current, so the caller must not change them."""
        if self._host is None:
            self._host = (self.x.cpu().numpy(), self.logl.cpu().numpy())
        return self._host

    def _count_screen(self, st):
        for key in self.screen_stats:
            self.screen_stats[key] += st[key]
        self._fn[0] += st["audited"]
        self._fn[1] += st["audited_inside"]
        # the audit estimates the share of screened-out candidates that were
        # inside; above the target the margin widens
        if self._fn[0] >= 50 and self._fn[1] > self.pre_cfg["fn_target"] * self._fn[0]:
            self.pre.margin *= 1.5
            self._fn = [0, 0]

    def _prescreen(self, lstar):
        """The (network, margin, audit fraction) for this iteration's sweeps,
        training it first when due, or None."""
        if self.pre is None or self.iteration < self.pre_cfg["start"]:
            return None
        cfg = self.pre_cfg
        if (self.iteration - cfg["start"]) % cfg["every"] == 0:
            t0 = time.perf_counter()
            cnt = int(self.rec[2].item())
            n_rec = min(cnt, self.rec[0].shape[0])
            x = np.concatenate([self.rec[0][:n_rec].cpu().numpy(), self.x.cpu().numpy()])
            y = np.concatenate([self.rec[1][:n_rec].cpu().numpy(), self.logl.cpu().numpy()])
            steps = cfg["steps"] if self.pre_trainings == 0 else cfg["retrain_steps"]
            n_train = int(0.9 * len(x))
            epochs = max(1, int(math.ceil(steps * cfg["batch"] / max(n_train, 1))))
            self.pre.train(x, y, self.x.cpu().numpy(), lstar, epochs=epochs, batch=cfg["batch"])
            self.pre.set_margin(lstar, k=cfg["k_margin"])
            self._fn = [0, 0]
            self.pre_train_s += time.perf_counter() - t0
            self.pre_trainings += 1
        return (self.pre.mlp, self.pre.margin, cfg["audit"])

    def run(self, max_iter: int = 100000, checkpoint: str | None = None, every: int = 50, verbose: bool = False):
        t0 = time.perf_counter()
        while self.iteration < max_iter:
            self.step()
            logl = self.live_host()[1]
            if verbose and self.iteration % 20 == 0:
                print(f"it {self.iteration} logL*={max(self.dead_logl[-self.k:]):.3f} "
                      f"logZ_dead={self.log_z_dead():.3f} evals={self.n_evals}", flush=True)
            if checkpoint and self.iteration % every == 0:
                self.save(checkpoint)
            if self.converged(logl):
                break
        self.torch.cuda.synchronize()
        self.wall += time.perf_counter() - t0
        return self.result()

    def result(self) -> dict:
        logl = self.logl.cpu().numpy()
        all_logw = np.concatenate([self.dead_logw, logl + self.log_x - math.log(self.m)])
        all_logl = np.concatenate([self.dead_logl, logl])
        log_z = _logsumexp(all_logw)
        p = np.exp(all_logw - log_z)
        h = float(np.sum(p * all_logl) - log_z)
        ess = float(1.0 / np.sum(p * p))
        out = dict(log_z=log_z, log_z_err=math.sqrt(max(h, 0.0) / self.m), h=h, iterations=self.iteration,
                   n_evals=self.n_evals, wall_s=self.wall, ess=ess)
        if self.cache:
            out["eval_kinds"] = [int(v) for v in self.eval_kinds]
        out["moves"] = self.moves
        if self.pre is not None:
            out["prescreen"] = dict(self.screen_stats, trainings=self.pre_trainings, train_s=self.pre_train_s,
                                    margin=self.pre.margin)
        return out

    def close(self):
        if self.pre is not None:
            self.pre.close()
            self.pre = None

    def samples(self):
        """(unit-cube points, normalised posterior weights) of dead + live points."""
        x = np.concatenate([np.array(self.dead_x).reshape(-1, N_DIM), self.x.cpu().numpy()])
        logl = self.logl.cpu().numpy()
        lw = np.concatenate([self.dead_logw, logl + self.log_x - math.log(self.m)])
        w = np.exp(lw - _logsumexp(lw))
        return x, w

    # -- checkpoint / resume -----------------------------------------------
    def save(self, path: str):
        if self.pre is not None:
            raise NotImplementedError("checkpoints of a prescreened run are not supported")
        np.savez(path, x=self.x.cpu().numpy(), logl=self.logl.cpu().numpy(),
                 dead_logl=np.array(self.dead_logl), dead_logw=np.array(self.dead_logw),
                 dead_x=np.array(self.dead_x).reshape(-1, N_DIM), log_x=self.log_x, iteration=self.iteration,
                 counter=self.counter, n_evals=self.n_evals, eval_kinds=self.eval_kinds,
                 rng=np.frombuffer(repr(self.rng.bit_generator.state).encode(), dtype=np.uint8))

    def load(self, path: str):
        import ast
        d = np.load(path, allow_pickle=False)
        self.x = self.torch.from_numpy(d["x"]).to(self.dev)
        self.logl = self.torch.from_numpy(d["logl"]).to(self.dev)
        self.dead_logl = list(d["dead_logl"])
        self.dead_logw = list(d["dead_logw"])
        self._log_z_dead = _logsumexp(self.dead_logw)
        self._host = None
        self.dead_x = list(d["dead_x"])
        self.log_x = float(d["log_x"])
        self.iteration = int(d["iteration"])
        self.counter = int(d["counter"])
        self.n_evals = int(d["n_evals"])
        self.eval_kinds = np.array(d["eval_kinds"], np.int64)
        self.rng.bit_generator.state = ast.literal_eval(bytes(d["rng"]).decode())

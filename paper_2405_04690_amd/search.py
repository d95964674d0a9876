"""Per-sub-band search for the loudest remaining source (appendix "Algorithm
for fitting proposal distributions"; the search RJ proposal of Sec. 4).

`Search` owns the device state of include/gbl.h's gbl_search_state and
forwards to the C ABI.  `run_search` follows the appendix's schedule:
iterate until every sub-band's best cold-chain likelihood has not improved
for n_stall iterations, relaunch from a ball around each best point and
converge again, keep the sub-bands whose best template passes the optimal
SNR limit, then run on and collect thinned cold-chain samples of every such
source (30 per walker after thinning by 25 in the paper).  Host work is
bookkeeping only (convergence flags, sample copies).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .gbl import Context, SearchConfig, SearchState

# restart-ball widths in sampling coordinates (log10 A, f0 [bins / T], fdot,
# phi0, cos iota, psi, lambda, sin beta)
BALL_SIGMA = (0.01, 0.05, 0.0, 0.05, 0.02, 0.05, 0.02, 0.02)


def make_config(n_bands, n_temps, n_walkers, N, width, k_band0, prior_lo, prior_hi, n_stall=500, stretch_a=2.0,
                seed=4242):
    c = SearchConfig()
    c.n_bands, c.n_temps, c.n_walkers, c.N, c.width, c.n_stall = n_bands, n_temps, n_walkers, N, width, n_stall
    c.k_band0, c.stretch_a, c.seed = int(k_band0), float(stretch_a), int(seed)
    for k in range(8):
        c.prior_lo[k], c.prior_hi[k] = float(prior_lo[k]), float(prior_hi[k])
    return c


class Search:
    def __init__(self, ctx: Context, cfg: SearchConfig, residual, psd):
        self.ctx, self.cfg = ctx, cfg
        dev = ctx.device
        nb, nt, nw = cfg.n_bands, cfg.n_temps, cfg.n_walkers
        f64 = dict(dtype=torch.float64, device=dev)
        self.residual = ctx._dev(residual, torch.complex128, "residual").reshape(2, ctx.n_bins)
        self.psd = ctx._dev(psd, torch.float64, "psd").reshape(2, ctx.n_bins)
        self.u = torch.zeros((nb, nt, nw, 8), **f64)
        self.logl = torch.zeros((nb, nt, nw), **f64)
        self.betas = torch.ones(nt, **f64)
        self.best_u = torch.zeros((nb, 8), **f64)
        self.best_logl = torch.full((nb,), float("-inf"), **f64)
        self.stall = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.stats = torch.zeros(4, dtype=torch.int64, device=dev)
        nbytes = ctypes.c_int64()
        ctx._check(ctx.lib.gb_search_workspace(ctypes.byref(cfg), ctypes.byref(nbytes)), "gb_search_workspace")
        self.workspace = torch.zeros(int(nbytes.value), dtype=torch.uint8, device=dev)
        self.iter = 0

    def _state(self):
        st = SearchState()
        for n in ("u", "logl", "betas", "best_u", "best_logl", "stall", "stats", "workspace"):
            setattr(st, n, getattr(self, n).data_ptr())
        return st

    def _call(self, name, *args):
        self.ctx._sync_stream()
        rc = getattr(self.ctx.lib, name)(self.ctx._h, ctypes.byref(self.cfg), ctypes.byref(self._state()), *args)
        self.ctx._check(rc, name)

    def box(self, b):
        """prior box of sub-band b in sampling coordinates"""
        c = self.cfg
        lo = np.array(list(c.prior_lo), float)
        hi = np.array(list(c.prior_hi), float)
        lo[1] = (c.k_band0 + b * c.width) / self.ctx.T
        hi[1] = (c.k_band0 + (b + 1) * c.width) / self.ctx.T
        for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
            lo[k], hi[k] = 0.0, P
        return lo, hi

    def start_uniform(self, seed: int):
        """every chain from a uniform draw in its band's box (input marshalling)"""
        rng = np.random.default_rng(seed)
        c = self.cfg
        u = np.empty((c.n_bands, c.n_temps, c.n_walkers, 8))
        for b in range(c.n_bands):
            lo, hi = self.box(b)
            u[b] = lo + (hi - lo) * rng.uniform(size=u[b].shape)
        self.u.copy_(torch.from_numpy(u))
        self.eval()

    def eval(self):
        self._call("gb_search_eval", self.residual.data_ptr(), self.psd.data_ptr())

    def step(self, it: int | None = None):
        it = self.iter if it is None else it
        self._call("gb_search_step", ctypes.c_int64(int(it)), self.residual.data_ptr(), self.psd.data_ptr())
        self.iter = it + 1

    def ball(self, sigma, it: int | None = None):
        it = self.iter if it is None else it
        sg = (ctypes.c_double * 8)(*[float(x) for x in sigma])
        self._call("gb_search_ball", ctypes.c_int64(int(it)), sg, self.residual.data_ptr(), self.psd.data_ptr())
        self.iter = it + 1

    def converged(self) -> bool:
        return bool((self.stall >= self.cfg.n_stall).all().item())


def converge(search: Search, max_iter: int, check_every: int = 25) -> int:
    """iterate until every band has converged (or max_iter); returns iterations run"""
    n = 0
    while n < max_iter:
        for _ in range(min(check_every, max_iter - n)):
            search.step()
            n += 1
        if search.converged():
            break
    return n


def run_search(search: Search, max_iter: int = 20000, snr_limit: float = 7.0, n_samples: int = 30, thin: int = 25):
    """the appendix's schedule; returns a dict with the best points, their
    optimal SNRs, the kept bands and, per kept band, cold-chain samples
    [n_samples * n_walkers][8] (sampling coordinates)"""
    ctx, c = search.ctx, search.cfg
    it1 = converge(search, max_iter)
    width_f = c.width / ctx.T
    sigma = list(BALL_SIGMA)
    sigma[1] = BALL_SIGMA[1] / ctx.T
    search.ball(sigma)
    it2 = converge(search, max_iter)
    best = search.best_u.clone()
    phys = best.clone()
    phys[:, 0] = torch.pow(10.0, best[:, 0])
    phys[:, 4] = torch.acos(best[:, 4])
    phys[:, 7] = torch.asin(best[:, 7])
    opt, _ = ctx.gb_snr(phys.contiguous(), c.N, search.psd.reshape(1, 2, ctx.n_bins).contiguous())
    keep = (opt > snr_limit).cpu().numpy()
    # sampling: the kept bands run on (no convergence freeze) and the cold rung
    # is copied every `thin` iterations
    saved_stall = search.stall.clone()
    search.stall.zero_()
    search.stall[torch.from_numpy(~keep).to(search.stall.device)] = c.n_stall   # the others stay frozen
    samples = []
    for _ in range(n_samples):
        for _ in range(thin):
            search.step()
            search.stall.masked_fill_(torch.from_numpy(keep).to(search.stall.device), 0)
        samples.append(search.u[:, 0].clone())
    search.stall.copy_(saved_stall)
    S = torch.stack(samples, dim=1)          # [n_b][n_samples][n_w][8]
    return {"iterations": [it1, it2], "best_u": best, "best_logl": search.best_logl.clone(), "snr": opt,
            "keep": keep, "samples": {int(b): S[b].reshape(-1, 8) for b in np.nonzero(keep)[0]},
            "band_width_hz": width_f}

"""Binding of the sampler sweep (Sec. 4; appendix algorithms gb1 and gb2).

`Sweep` owns the device tensors of the sampler state in the layouts of
include/gbl.h and forwards to the C ABI (argument marshalling only).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .gbl import (GBL_MOVE_INMODEL, GBL_MOVE_PT, GBL_MOVE_RJ, Context, PsdSweepConfig, PsdSweepState, SweepConfig,
                  SweepState, _ptr)

__all__ = ["Sweep", "PsdSweep", "make_config", "psd_config", "GBL_MOVE_INMODEL", "GBL_MOVE_RJ", "GBL_MOVE_PT"]

# default prior box of the sampling coordinates
# (log10 A, f0 [per band], fdot, phi0, cos iota, psi, lambda, sin beta)
DEFAULT_PRIOR_LO = (-23.0, 0.0, -1e-16, 0.0, -1.0, 0.0, 0.0, -1.0)
DEFAULT_PRIOR_HI = (-21.0, 0.0, 1e-15, 0.0, 1.0, 0.0, 0.0, 1.0)


def make_config(n_temps, n_walkers, n_bands, n_slots, N, k_band0, n_prop=10, n_friends=8, group_every=30,
                stretch_a=2.0, seed=1234, prior_lo=DEFAULT_PRIOR_LO, prior_hi=DEFAULT_PRIOR_HI, cls=SweepConfig,
                adapt_ladder=False, shift_ownership=False, adapt_lag=10000.0, adapt_time=100.0, band_width=0):
    """adapt_lag / adapt_time: t0 and nu of the ladder adaptation's step
    t0 / (nu (t + t0)) (defaults as commonly used with the Vousden scheme);
    band_width: sub-band width W in bins (even; 0: W = N)"""
    c = cls()
    c.n_temps, c.n_walkers, c.n_bands, c.n_slots = n_temps, n_walkers, n_bands, n_slots
    c.N, c.n_prop, c.n_friends, c.group_every = N, n_prop, n_friends, group_every
    c.k_band0, c.stretch_a, c.seed = k_band0, stretch_a, seed
    c.adapt_ladder, c.shift_ownership = int(bool(adapt_ladder)), int(bool(shift_ownership))
    c.adapt_lag, c.adapt_time = float(adapt_lag), float(adapt_time)
    c.band_width = int(band_width)
    for i in range(8):
        c.prior_lo[i] = prior_lo[i]
        c.prior_hi[i] = prior_hi[i]
    return c


def run_band_sets(sweeps, n_sweeps: int = 1):
    """Full sweeps of several band sets that cover adjacent frequency ranges
    with their own template and sub-band widths (the paper's widths by
    frequency) and share the walkers' cold-chain buffers: in every sweep each
    set runs one full sweep in turn, seeing the others' current cold-chain
    sources as subtracted.  For the odd/even scheme to continue across a
    boundary, every set but the last has an even number of sub-bands."""
    for sw in sweeps[:-1]:
        if sw.cfg.n_bands % 2:
            raise ValueError("every band set but the last needs an even number of sub-bands")
    for _ in range(n_sweeps):
        for sw in sweeps:
            sw.run(1)

class Sweep:
    """Device state of one set of sub-bands (gbl_sweep_state) and the calls on
    it.  resid / inv_psd: the walkers' cold-chain buffers and weights to share
    with other band sets (None: allocated here)."""

    def __init__(self, ctx: Context, cfg: SweepConfig, spectrum_pool: int = 1024, window_sums: bool = False,
                 resid=None, inv_psd=None):
        self.ctx, self.cfg = ctx, cfg
        dev = ctx.device
        nt, nw, nb, ns = cfg.n_temps, cfg.n_walkers, cfg.n_bands, cfg.n_slots
        f64 = dict(dtype=torch.float64, device=dev)
        self.u = torch.zeros((nt, nw, nb, ns, 8), **f64)
        self.exists = torch.zeros((nt, nw, nb, ns), dtype=torch.int32, device=dev)
        self.betas = torch.ones((nb, nt), **f64)
        if resid is None:
            resid = torch.zeros((2, nw, 2, ctx.n_bins), dtype=torch.complex128, device=dev)
        if inv_psd is None:
            inv_psd = torch.zeros((nw, 2, ctx.n_bins), **f64)
        if tuple(resid.shape) != (2, nw, 2, ctx.n_bins) or tuple(inv_psd.shape) != (nw, 2, ctx.n_bins):
            raise ValueError("shared buffers must have shapes [2, n_walkers, 2, n_bins] and [n_walkers, 2, n_bins]")
        self.resid, self.inv_psd = resid, inv_psd
        self.group = torch.zeros((nb, nw * ns, 8), **f64)
        self.group_count = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.stats = torch.zeros(10, dtype=torch.int64, device=dev)
        self.swap_acc = torch.zeros((nb, nt), dtype=torch.int32, device=dev)
        self.sweep_counter = torch.zeros(1, dtype=torch.int64, device=dev)
        # optional: RJ proposal arrays (flow proposals) and the cold-chain logL trace
        self.prop_u = None
        self.rj_logq = None
        self.cold_logl = None
        self.rj_mode = None
        # per-slot spectrum cache of the band loops (spectrum_pool entries)
        self.spec_pool = None
        self.pool_flags = None
        if spectrum_pool > 0:
            entry = max(ns * 2 * cfg.N, nt * 6 * cfg.N)
            self.spec_pool = torch.zeros((spectrum_pool, entry), dtype=torch.complex128, device=dev)
            self.pool_flags = torch.zeros(spectrum_pool, dtype=torch.int32, device=dev)
        # window sums of the source sets, written by the band passes for the
        # tempering pass (n_temps x n_walkers x n_bands x 2 (2W + N) complex
        # doubles); required for sub-bands wider than the template and for
        # N = 1024, whose windows live there during the band passes
        self.band_width = cfg.band_width if cfg.band_width > 0 else cfg.N
        self.window_sums = None
        if window_sums or self.band_width != cfg.N or cfg.N == 1024:
            L = 2 * self.band_width + cfg.N
            self.window_sums = torch.zeros((nt, nw, nb, 2 * L), dtype=torch.complex128, device=dev)
        self._graph = None

    def enable_proposals(self):
        """allocate prop_u / rj_logq (used by the flow RJ proposal, or filled by the caller)"""
        c = self.cfg
        dev = self.ctx.device
        self.prop_u = torch.zeros((c.n_temps, c.n_walkers, c.n_bands, c.n_slots, 8), dtype=torch.float64, device=dev)
        self.rj_logq = torch.zeros((c.n_temps, c.n_walkers, c.n_bands, c.n_slots), dtype=torch.float64, device=dev)
        self.rj_mode = torch.zeros((c.n_temps, c.n_walkers, c.n_bands, c.n_slots), dtype=torch.int32, device=dev)

    def disable_proposals(self):
        self.prop_u = None
        self.rj_logq = None
        self.rj_mode = None

    def enable_logl_trace(self):
        c = self.cfg
        self.cold_logl = torch.full((c.n_walkers, c.n_bands), float("nan"), dtype=torch.float64,
                                    device=self.ctx.device)

    def _state(self):
        st = SweepState()
        for n in ("u", "exists", "betas", "resid", "inv_psd", "group", "group_count", "stats", "sweep_counter",
                  "prop_u", "rj_logq", "cold_logl", "rj_mode", "spec_pool", "pool_flags", "swap_acc", "window_sums"):
            t = getattr(self, n)
            setattr(st, n, t.data_ptr() if t is not None else None)
        st.pool_size = self.spec_pool.shape[0] if self.spec_pool is not None else 0
        return st

    def _call(self, name, *args):
        self.ctx._sync_stream()
        rc = getattr(self.ctx.lib, name)(self.ctx._h, *args)
        self.ctx._check(rc, name)

    def step(self, move: int, parity: int):
        self._call("gb_sweep_step", ctypes.byref(self.cfg), ctypes.byref(self._state()), int(move), int(parity))

    def group_refresh(self):
        self._call("gb_sweep_group", ctypes.byref(self.cfg), ctypes.byref(self._state()))

    def advance(self):
        self._call("gb_sweep_advance", ctypes.byref(self._state()))

    def adapt_ladder(self):
        self._call("gb_sweep_adapt_ladder", ctypes.byref(self.cfg), ctypes.byref(self._state()))

    def shift_ownership(self):
        self._call("gb_sweep_shift_ownership", ctypes.byref(self.cfg), ctypes.byref(self._state()))

    def run(self, n_sweeps: int):
        self._call("gb_sweep_run", ctypes.byref(self.cfg), ctypes.byref(self._state()), int(n_sweeps))

    def rj_prepare(self, flow):
        """fill prop_u / rj_logq from the flow (births: flow samples; deaths: flow density)"""
        if self.prop_u is None:
            self.enable_proposals()
        self._call("gb_sweep_rj_prepare", ctypes.byref(self.cfg), ctypes.byref(self._state()),
                   ctypes.byref(flow.cfg), ctypes.byref(flow._state()))

    def run_flow(self, flow, n_sweeps: int):
        if self.prop_u is None:
            self.enable_proposals()
        self._call("gb_sweep_run_flow", ctypes.byref(self.cfg), ctypes.byref(self._state()), ctypes.byref(flow.cfg),
                   ctypes.byref(flow._state()), int(n_sweeps))

    def capture_flow(self, flow, n_sweeps: int):
        """capture n_sweeps sweeps with the flow RJ proposal into a HIP graph"""
        self.release_graph()
        if self.prop_u is None:
            self.enable_proposals()
        h = ctypes.c_void_p()
        self._call("gb_sweep_graph_create_flow", ctypes.byref(self.cfg), ctypes.byref(self._state()),
                   ctypes.byref(flow.cfg), ctypes.byref(flow._state()), int(n_sweeps), ctypes.byref(h))
        self._graph = h

    def capture(self, n_sweeps: int):
        """Capture n_sweeps full sweeps into a HIP graph (context stream must not be the default one)."""
        self.release_graph()
        h = ctypes.c_void_p()
        self._call("gb_sweep_graph_create", ctypes.byref(self.cfg), ctypes.byref(self._state()), int(n_sweeps),
                   ctypes.byref(h))
        self._graph = h

    def replay(self):
        rc = self.ctx.lib.gb_graph_launch(self._graph)
        self.ctx._check(rc, "gb_graph_launch")

    def release_graph(self):
        if self._graph is not None:
            self.ctx.lib.gb_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.release_graph()
        except Exception:
            pass

    @staticmethod
    def geometric_ladder(n_temps: int, ratio: float = 1.2, hottest_zero: bool = True):
        """Inverse temperatures 1, 1/r, 1/r^2, ... with an infinite-temperature top rung (Sec. 4)."""
        b = ratio ** -np.arange(n_temps, dtype=np.float64)
        if hottest_zero and n_temps > 1:
            b[-1] = 0.0
        return b


def psd_config(n_tn: int, n_walkers: int, prior_lo, prior_hi, stretch_a: float = 2.0, seed: int = 4321):
    """noise-step configuration; 4 prior bounds (instrument noise) or 9 (with the
    Galactic foreground (A_fg, alpha, f_k, s1, s2))"""
    n_par = len(prior_lo)
    if n_par not in (4, 9) or len(prior_hi) != n_par:
        raise ValueError("prior_lo/prior_hi must both have 4 or 9 entries")
    c = PsdSweepConfig()
    c.n_tn, c.n_walkers, c.n_par = int(n_tn), int(n_walkers), n_par
    c.stretch_a, c.seed = float(stretch_a), int(seed)
    for k in range(n_par):
        c.prior_lo[k], c.prior_hi[k] = float(prior_lo[k]), float(prior_hi[k])
    return c


class PsdSweep:
    """Noise-PSD step bound to a Sweep: its cold-chain buffers, 1/S and sweep
    counter; owns the PSD chains (theta, logl, betas) and the workspaces."""

    def __init__(self, sweep: Sweep, cfg: PsdSweepConfig, data):
        self.sweep, self.cfg = sweep, cfg
        ctx = sweep.ctx
        dev = ctx.device
        nt, nw = cfg.n_tn, cfg.n_walkers
        if nw != sweep.cfg.n_walkers:
            raise ValueError("the PSD step needs the sweep's walkers")
        self.data = ctx._dev(data, torch.complex128, "data")
        if self.data.shape != (2, ctx.n_bins):
            raise ValueError("data must have shape [2, n_bins]")
        f64 = dict(dtype=torch.float64, device=dev)
        self.theta = torch.zeros((nt, nw, cfg.n_par), **f64)
        self.logl = torch.zeros((nt, nw), **f64)
        self.betas = torch.ones(nt, **f64)
        self.full_resid = torch.zeros((nw, 2, ctx.n_bins), dtype=torch.complex128, device=dev)
        self.work = torch.zeros(7 * nt * nw, **f64)
        self.res_idx = torch.zeros(nt * nw, dtype=torch.int32, device=dev)
        self.stats = torch.zeros(4, dtype=torch.int64, device=dev)

    def _state(self):
        st = PsdSweepState()
        sw = self.sweep
        for n, t in (("theta", self.theta), ("logl", self.logl), ("betas", self.betas), ("data", self.data),
                     ("resid", sw.resid), ("full_resid", self.full_resid), ("inv_psd", sw.inv_psd),
                     ("work", self.work), ("res_idx", self.res_idx), ("stats", self.stats),
                     ("sweep_counter", sw.sweep_counter)):
            setattr(st, n, t.data_ptr())
        return st

    def step(self):
        ctx = self.sweep.ctx
        ctx._sync_stream()
        rc = ctx.lib.gb_psd_sweep_step(ctx._h, ctypes.byref(self.cfg), ctypes.byref(self._state()))
        ctx._check(rc, "gb_psd_sweep_step")

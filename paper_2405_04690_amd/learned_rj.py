"""Learned versus prior RJ proposal on one sampler problem: the comparison of
RJ acceptance and effective samples per second (Sec. 4 "Online updating of RJ
sampling distributions"; the flow replaces the paper's fitted mixtures).

Problem: sub-bands of W bins from bin k_band0 (templates of N bins; W = N, or
wider, e.g. 1e-4 Hz as in the learned-proposal configuration), each holding
one loud and one near-threshold injected source in stationary Gaussian noise;
every chain starts from the injections.  The sampler first runs with prior RJ draws and
collects cold-chain samples; the flow is trained on them with the library's
own training kernels.  Two measurements follow, each once with prior RJ
draws and once with the flow mixture (prior share 0.2) as the RJ proposal:
(1) stationary mixing: the state is first equilibrated with the flow mixture
(the better-mixing chain), then from that saved state the same number of
sweeps runs with each proposal, recording per sweep the cold chain's source
count and band log-likelihood per (walker, band) for their ESS per second;
both chains must then agree on the mean source count and mean cold
log-likelihood within their Monte Carlo errors (the check that the
comparison is stationary is reported next to the ratios; the error is the
larger of the autocorrelation-based one and the spread of the per-walker
means, the walkers being independent chains); (2) discovery: from every slot
empty, the fraction of (walker, injected source) pairs the cold chain has
recovered per sweep.  Everything runs through the C ABI; only the
bookkeeping (trace copies, ESS, recovery fractions) is host-side.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import ess as ess_mod
from . import inputs
from .flow import Flow, flow_config
from .gbl import Context
from .sampler import Sweep, make_config

# amplitude prior: log10 A from the amplitude of an SNR_MIN source at the
# injections' median sensitivity up to 2.5 decades above (sources too quiet to
# be resolved are outside the model, as with the paper's final SNR limit of 5
# in the search-to-PE schedule); fdot in a narrow symmetric range
SNR_MIN = 5.0
LOG10A_SPAN = 2.5
FDOT_MAX = 1e-17


@dataclass
class Problem:
    ctx: Context
    sweep: Sweep
    fcfg: object
    sources: np.ndarray
    snr: np.ndarray
    data: torch.Tensor


def _to_u(p):
    return np.stack([np.log10(p[:, 0]), p[:, 1], p[:, 2], p[:, 3], np.cos(p[:, 4]), p[:, 5], p[:, 6],
                     np.sin(p[:, 7])], axis=1)


def _physical(u):
    p = u.clone()
    p[:, 0] = torch.pow(10.0, u[:, 0])
    p[:, 4] = torch.acos(u[:, 4])
    p[:, 7] = torch.asin(u[:, 7])
    return p


def build(cfg=inputs.TINY, N=128, n_temps=4, n_walkers=32, n_bands=8, n_slots=6, snr=(20.0, 7.0), seed=60,
          f_start=3e-3, stream=None, snr_min: float = SNR_MIN, W: int | None = None) -> Problem:
    """W: sub-band width in bins (even; None: the template width N)"""
    dev = torch.device("cuda", torch.cuda.current_device())
    ctx = Context(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi, device=dev, stream=stream)
    T = cfg.T
    k_band0 = int(f_start * T)
    W = N if W is None else int(W)
    src = inputs.band_sources(seed, n_bands, len(snr), T, k_band0, W)
    noise = torch.tensor([[cfg.sqrt_oms, cfg.sqrt_acc, cfg.sqrt_oms, cfg.sqrt_acc]], dtype=torch.float64, device=dev)
    S = ctx.gb_psd_eval(noise)
    invS = ctx.gb_psd_eval(noise, inverse=True)
    # amplitude for the target SNR: a birth into noise-free data has dlnL = -SNR^2 / 2
    zero = torch.zeros((1, 2, ctx.n_bins), dtype=torch.complex128, device=dev)
    unit = torch.from_numpy(src).to(dev)
    none = unit.clone()
    none[:, 0] = 0.0
    dl = ctx.gb_delta_loglike(zero, invS, none, unit, N, psd_inverse=True)
    snr_unit = torch.sqrt(-2.0 * dl).cpu().numpy()
    target = np.tile(np.asarray(snr, dtype=np.float64), n_bands)
    src[:, 0] = target / snr_unit
    lo_a = float(np.log10(snr_min / np.median(snr_unit)))
    prior_lo = (lo_a, 0.0, -FDOT_MAX, 0.0, -1.0, 0.0, 0.0, -1.0)
    prior_hi = (lo_a + LOG10A_SPAN, 0.0, FDOT_MAX, 0.0, 1.0, 0.0, 0.0, 1.0)
    d = ctx.gb_make_noise(S, torch.from_numpy(inputs.complex_normals(seed + 1, (1, 2, ctx.n_bins))).to(dev))
    ctx.gb_scatter_add(torch.from_numpy(src).to(dev), N, 1.0, d)
    sc = make_config(n_temps, n_walkers, n_bands, n_slots, N, k_band0, n_prop=20, n_friends=8, group_every=10,
                     seed=seed + 2, prior_lo=prior_lo, prior_hi=prior_hi, band_width=0 if W == N else W)
    sw = Sweep(ctx, sc)
    u0 = np.zeros((n_bands, n_slots, 8))
    e0 = np.zeros((n_bands, n_slots), np.int32)
    us = _to_u(src)
    for b in range(n_bands):
        for j in range(len(snr)):
            u0[b, j] = us[b * len(snr) + j]
            e0[b, j] = 1
    sw.u.copy_(torch.from_numpy(u0).to(dev).expand(n_temps, n_walkers, -1, -1, -1))
    sw.exists.copy_(torch.from_numpy(e0).to(dev).expand(n_temps, n_walkers, -1, -1))
    sw.betas.copy_(torch.from_numpy(np.geomspace(1.0, 0.1, n_temps)).to(dev).expand(n_bands, -1))
    sw.inv_psd.copy_(invS.expand(n_walkers, -1, -1))
    band_par = (torch.arange(n_bands, device=dev) % 2).view(1, n_bands, 1).expand(n_walkers, -1, n_slots)
    walker = torch.arange(n_walkers, device=dev, dtype=torch.int32).view(n_walkers, 1, 1).expand(-1, n_bands, n_slots)
    for par in (0, 1):
        sw.resid[par].copy_(d.expand(n_walkers, -1, -1))
        sel = (sw.exists[0] != 0) & (band_par == par)
        ctx.gb_scatter_add(_physical(sw.u[0][sel].contiguous()), N, -1.0, sw.resid[par], walker[sel].contiguous())
    sw.enable_logl_trace()
    fcfg = flow_config(n_bands, W, k_band0, prior_lo, prior_hi)
    torch.cuda.synchronize()
    return Problem(ctx, sw, fcfg, src, target, d)


_STATE = ("u", "exists", "resid", "group", "group_count", "stats", "sweep_counter")


def save(sw: Sweep):
    return {k: getattr(sw, k).clone() for k in _STATE}


def restore(sw: Sweep, st):
    for k in _STATE:
        getattr(sw, k).copy_(st[k])


def collect(sw: Sweep, n_sweeps: int, every: int = 1):
    """run n_sweeps prior-RJ sweeps; return the cold chain's occupied (u, band) pairs"""
    c = sw.cfg
    band_of = torch.arange(c.n_bands, device=sw.u.device, dtype=torch.int32).view(1, c.n_bands, 1).expand(
        c.n_walkers, -1, c.n_slots)
    us, bs = [], []
    for i in range(n_sweeps):
        sw.run(1)
        if i % every == 0:
            m = sw.exists[0] != 0
            us.append(sw.u[0][m].clone())
            bs.append(band_of[m].clone())
    return torch.cat(us), torch.cat(bs).contiguous()


def source_weights(u, band, T: float, n_states: int, min_presence: float = 0.1, cell_bins: float = 4.0):
    """Per-sample training weights that give every recurring source the same
    total weight, the way the paper's refit proposal fits the sources that
    appear regularly and combines their mixtures with equal probability
    (Sec. 4, "refit RJ proposal"): samples are grouped into sources by
    sub-band and carrier-frequency cell (cell_bins frequency bins wide); a
    group present in at least min_presence of the n_states collected chain
    states shares weight 1, a rarer one gets none."""
    cell = torch.floor(u[:, 1].double() * T / cell_bins).to(torch.int64)
    key = band.to(torch.int64) * (1 << 40) + cell
    _, inv, counts = torch.unique(key, return_inverse=True, return_counts=True)
    c = counts[inv].double()
    return torch.where(c >= min_presence * n_states, 1.0 / c, torch.zeros_like(c))


def train(flow: Flow, u, band, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0, weights=None):
    """Adam steps on batches drawn from (u, band), uniformly or with the given
    per-sample weights"""
    gen = torch.Generator(device=u.device)
    gen.manual_seed(seed)
    losses = []
    for _ in range(steps):
        if weights is None:
            idx = torch.randint(0, u.shape[0], (batch,), generator=gen, device=u.device)
        else:
            idx = torch.multinomial(weights, batch, replacement=True, generator=gen)
        losses.append(flow.train_step(u[idx].contiguous(), band[idx].contiguous(), lr).clone())
    return torch.stack(losses).view(-1).cpu().numpy()


def measure(sw: Sweep, n_sweeps: int, flow: Flow | None = None):
    """n_sweeps sweeps (flow RJ proposal if given, else prior draws); traces and rates"""
    k_tr, l_tr = [], []
    st0 = sw.stats.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_sweeps):
        if flow is None:
            sw.disable_proposals()
            sw.run(1)
        else:
            sw.run_flow(flow, 1)
        k_tr.append(sw.exists[0].sum(dim=-1))
        l_tr.append(sw.cold_logl.clone())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = torch.stack(k_tr, dim=-1).double().cpu().numpy()   # [n_w][n_b][n_sweeps]
    lnl = torch.stack(l_tr, dim=-1).cpu().numpy()
    dst = (sw.stats - st0).cpu().numpy()
    ess_kb = [ess_mod.ess(k[:, b, :]) for b in range(k.shape[1])]
    ess_lb = [ess_mod.ess(lnl[:, b, :]) for b in range(lnl.shape[1])]
    ess_k = float(sum(ess_kb))
    ess_l = float(sum(ess_lb))
    # Monte Carlo error of the band-summed means: per band var / ESS, summed
    # over the (independent) bands, then divided by the band count squared;
    # and from the spread of the per-walker means (independent chains); the
    # larger of the two is reported
    nb, nw = k.shape[1], k.shape[0]
    se_k = float(np.sqrt(sum(k[:, b, :].var() / max(e, 1.0) for b, e in enumerate(ess_kb))) / nb)
    se_l = float(np.sqrt(sum(lnl[:, b, :].var() / max(e, 1.0) for b, e in enumerate(ess_lb))) / nb)
    se_k = max(se_k, float(k.mean(axis=(1, 2)).std(ddof=1) / np.sqrt(nw)))
    se_l = max(se_l, float(lnl.mean(axis=(1, 2)).std(ddof=1) / np.sqrt(nw)))
    return {"sweeps": n_sweeps, "wall_s": wall,
            "birth_acceptance": float(dst[3]) / max(1.0, float(dst[2])),
            "death_acceptance": float(dst[5]) / max(1.0, float(dst[4])),
            "rj_accepted_per_s": float(dst[3] + dst[5]) / wall,
            "ess_k": ess_k, "ess_logl": ess_l, "ess_k_per_s": ess_k / wall, "ess_logl_per_s": ess_l / wall,
            "mean_k": float(k.mean()), "se_mean_k": se_k,
            "mean_logl": float(lnl.mean()), "se_mean_logl": se_l}


def empty_state(problem: Problem):
    """every slot empty, both cold-chain buffers = the data"""
    sw = problem.sweep
    st = save(sw)
    st["exists"] = torch.zeros_like(sw.exists)
    st["resid"] = problem.data.expand(sw.resid.shape[1], -1, -1).unsqueeze(0).expand(2, -1, -1, -1).contiguous()
    st["stats"] = torch.zeros_like(sw.stats)
    return st


def recovered(problem: Problem, tol_bins: float = 1.0, tol_log10a: float = 0.3):
    """fraction of (walker, injected source) pairs whose source the cold chain holds:
    an occupied slot of its sub-band within tol_bins of its f0 and tol_log10a of its log10 A"""
    sw = problem.sweep
    c = sw.cfg
    per_band = len(problem.sources) // c.n_bands
    u = sw.u[0]                        # [n_w][n_b][n_slot][8]
    ex = sw.exists[0] != 0
    src = torch.from_numpy(problem.sources).to(u.device).view(c.n_bands, per_band, 8)
    f_inj = src[..., 1]
    a_inj = torch.log10(src[..., 0])
    df = (u[:, :, None, :, 1] - f_inj[None, :, :, None]).abs() * problem.ctx.T   # [w][b][j][s]
    da = (u[:, :, None, :, 0] - a_inj[None, :, :, None]).abs()
    hit = (df < tol_bins) & (da < tol_log10a) & ex[:, :, None, :]
    return hit.any(dim=-1).double().mean(dim=(0, 1)).cpu().numpy()   # per source rank j


def discover(problem: Problem, n_sweeps: int, flow: Flow | None, start):
    """from `start` (all slots empty), n_sweeps sweeps; recovered fractions per sweep"""
    sw = problem.sweep
    restore(sw, start)
    traj = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_sweeps):
        if flow is None:
            sw.disable_proposals()
            sw.run(1)
        else:
            sw.run_flow(flow, 1)
        traj.append(recovered(problem))
    wall = time.perf_counter() - t0
    traj = np.array(traj)              # [n_sweeps][per_band]
    return {"wall_s": wall, "final": traj[-1].tolist(), "mean": traj.mean(axis=0).tolist(),
            "sweeps_to_half": [int(np.argmax(traj[:, j] >= 0.5)) if np.any(traj[:, j] >= 0.5) else None
                               for j in range(traj.shape[1])]}


def stationarity(plain, learned):
    """z-scores of the differences of the two chains' mean source count and mean
    cold log-likelihood, in units of their combined Monte Carlo error"""
    zk = (plain["mean_k"] - learned["mean_k"]) / max(np.hypot(plain["se_mean_k"], learned["se_mean_k"]), 1e-300)
    zl = (plain["mean_logl"] - learned["mean_logl"]) / max(np.hypot(plain["se_mean_logl"],
                                                                    learned["se_mean_logl"]), 1e-300)
    return {"z_mean_k": float(zk), "z_mean_logl": float(zl), "stationary": bool(abs(zk) < 3 and abs(zl) < 3)}


def compare(problem: Problem, burn: int = 100, collect_sweeps: int = 200, train_steps: int = 300,
            measure_sweeps: int = 400, lr: float = 1e-3, seed: int = 0, balance: bool = False,
            equilibrate: int = 200):
    """burn-in and sample collection with prior RJ, flow training (samples
    weighted per source if balance), equilibration with the flow mixture, then
    the same number of sweeps from the same equilibrated state with each
    proposal"""
    from .flow import init_params
    sw = problem.sweep
    sw.run(burn)
    u, band = collect(sw, collect_sweeps)
    flow = Flow(problem.ctx, problem.fcfg, init_params(seed, problem.fcfg.n_emb))
    n_states = sw.cfg.n_walkers * collect_sweeps
    weights = source_weights(u, band, problem.ctx.cfg.T, n_states) if balance else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = train(flow, u, band, train_steps, lr=lr, seed=seed, weights=weights)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for _ in range(equilibrate):
        sw.run_flow(flow, 1)
    state = save(sw)
    plain = measure(sw, measure_sweeps, None)
    restore(sw, state)
    learned = measure(sw, measure_sweeps, flow)
    start = empty_state(problem)
    disc_plain = discover(problem, measure_sweeps, None, start)
    disc_learned = discover(problem, measure_sweeps, flow, start)
    restore(sw, state)
    return {"training_samples": int(u.shape[0]), "train_steps": train_steps,
            "train_ms_per_step": 1e3 * t_train / max(1, train_steps),
            "loss_first": float(np.mean(losses[:10])), "loss_last": float(np.mean(losses[-10:])),
            "equilibration_sweeps": equilibrate, "plain": plain, "learned": learned,
            "stationarity": stationarity(plain, learned),
            "discovery": {"plain": disc_plain, "learned": disc_learned},
            "gain_ess_k_per_s": learned["ess_k_per_s"] / max(plain["ess_k_per_s"], 1e-300),
            "gain_ess_logl_per_s": learned["ess_logl_per_s"] / max(plain["ess_logl_per_s"], 1e-300),
            "gain_birth_acceptance": learned["birth_acceptance"] / max(plain["birth_acceptance"], 1e-300)}, flow

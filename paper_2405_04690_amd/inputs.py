"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no waveform, response, PSD or likelihood).  The source
populations follow the shapes of the paper's LDC2A ("Sangria") workload, which
is not available here: 1 yr of data at 5 s cadence, A/E channels, ~1e4
resolvable binaries, stationary noise.  No dataset item is reproduced.

Parameter vectors are in physical units, in the order
(A, f0 [Hz], fdot [Hz/s], phi0, iota, psi, lambda, beta).
Recipes (each array drawn in the listed order from numpy's PCG64 seeded
generator):
  log10 A ~ U(-23, -21); f0 = 10**U(log10 f_lo, log10 f_hi);
  fdot = 0 or 10**U(-19, -15); lambda ~ U(0, 2 pi); sin beta ~ U(-1, 1);
  psi ~ U(0, pi); cos iota ~ U(-1, 1); phi0 ~ U(0, 2 pi).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

YEAR = 31557600.0  # Julian year [s]


@dataclass(frozen=True)
class RunConfig:
    name: str
    T: float
    dt: float
    N: int
    L: float = 2.5e9
    f_lo: float = 1e-4
    f_hi: float = 3e-2
    sqrt_oms: float = 15e-12  # m / sqrt(Hz)
    sqrt_acc: float = 3e-15   # m s^-2 / sqrt(Hz)


# 256 sources, 0.25 yr at 15 s, N = 128: the small case the oracle finishes in seconds.
TINY = RunConfig("tiny-0.25yr-dt15-N128", T=0.25 * YEAR, dt=15.0, N=128)
# Paper scale: 1 yr at 5 s, N = 256 (the paper's most common template width).
PAPER = RunConfig("paper-1yr-dt5-N256", T=YEAR, dt=5.0, N=256)


def draw_sources(seed: int, n: int, f_range=(1e-4, 1e-2), log10_fdot_range=None) -> np.ndarray:
    """Draw n source parameter vectors [n, 8] following the recipe above."""
    rng = np.random.default_rng(seed)
    log10A = rng.uniform(-23.0, -21.0, n)
    f0 = 10.0 ** rng.uniform(np.log10(f_range[0]), np.log10(f_range[1]), n)
    if log10_fdot_range is None:
        fdot = np.zeros(n)
    else:
        fdot = 10.0 ** rng.uniform(log10_fdot_range[0], log10_fdot_range[1], n)
    lam = rng.uniform(0.0, 2 * np.pi, n)
    sinb = rng.uniform(-1.0, 1.0, n)
    psi = rng.uniform(0.0, np.pi, n)
    cosi = rng.uniform(-1.0, 1.0, n)
    phi0 = rng.uniform(0.0, 2 * np.pi, n)
    return np.stack([10.0 ** log10A, f0, fdot, phi0, np.arccos(cosi), psi, lam, np.arcsin(sinb)], axis=1)


def complex_normals(seed: int, shape) -> np.ndarray:
    """g1 + i g2 with g1, g2 ~ N(0, 1) independent (complex128)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def _wrap(x, period):
    return np.mod(x, period)


def perturb(seed: int, params: np.ndarray, T: float, kind: str = "inmodel") -> np.ndarray:
    """Proposal-like perturbation of parameter vectors.

    inmodel: df0 ~ N(0, (0.3/T)^2), dlog10 A ~ N(0, 0.02^2),
             dlog10 fdot ~ N(0, 0.05^2) (fdot > 0 only), angles ~ N(0, 0.03^2)
             (phi0, psi, lambda wrapped; cos iota and sin beta clipped to [-1, 1]).
    jitter:  df0 ~ N(0, (0.1/T)^2) only.
    """
    rng = np.random.default_rng(seed)
    p = np.array(params, dtype=np.float64, copy=True)
    n = p.shape[0]
    if kind == "jitter":
        p[:, 1] += rng.normal(0.0, 0.1 / T, n)
        return p
    if kind != "inmodel":
        raise ValueError(kind)
    p[:, 1] += rng.normal(0.0, 0.3 / T, n)
    p[:, 0] *= 10.0 ** rng.normal(0.0, 0.02, n)
    dfd = rng.normal(0.0, 0.05, n)
    p[:, 2] = np.where(p[:, 2] > 0, p[:, 2] * 10.0 ** dfd, p[:, 2])
    p[:, 3] = _wrap(p[:, 3] + rng.normal(0.0, 0.03, n), 2 * np.pi)
    ci = np.clip(np.cos(p[:, 4]) + rng.normal(0.0, 0.03, n), -1.0, 1.0)
    p[:, 4] = np.arccos(ci)
    p[:, 5] = _wrap(p[:, 5] + rng.normal(0.0, 0.03, n), np.pi)
    p[:, 6] = _wrap(p[:, 6] + rng.normal(0.0, 0.03, n), 2 * np.pi)
    sb = np.clip(np.sin(p[:, 7]) + rng.normal(0.0, 0.03, n), -1.0, 1.0)
    p[:, 7] = np.arcsin(sb)
    return p


@dataclass
class SwapBatch:
    """A batch of (old, new) template pairs against per-walker residuals."""
    sources: np.ndarray     # [n_src, 8] injected sources
    params_old: np.ndarray  # [B, 8]
    params_new: np.ndarray  # [B, 8]
    res_idx: np.ndarray     # [B] int32 walker index
    n_walkers: int
    n_temps: int


def paper_swap_batch(n_walkers: int = 32, n_temps: int = 24, n_src: int = 130, seed_src: int = 2,
                     seed_prop: int = 1000, T: float = YEAR, mix: str = "inmodel") -> SwapBatch:
    """Batch of 32 walkers x 24 temperatures x 130 sources = 99,840 pairs.

    Templates are ordered b = (t * n_walkers + w) * n_src + i.  params_old is
    the source plus a small f0 jitter; params_new an in-model perturbation of
    it.  mix == "full": 10% births (old amplitude 0) and 10% deaths (new
    amplitude 0) mixed into the in-model moves.
    """
    src = draw_sources(seed_src, n_src, (1e-4, 1e-2), (-19.0, -15.0))
    B = n_walkers * n_temps * n_src
    base = np.tile(src, (n_walkers * n_temps, 1))
    old = perturb(seed_prop, base, T, "jitter")
    new = perturb(seed_prop + 1, old, T, "inmodel")
    if mix == "full":
        u = np.random.default_rng(seed_prop + 2).uniform(size=B)
        birth = u < 0.1
        death = (u >= 0.1) & (u < 0.2)
        old[birth, 0] = 0.0
        new[death, 0] = 0.0
    elif mix != "inmodel":
        raise ValueError(mix)
    walker = (np.arange(B) // n_src) % n_walkers
    return SwapBatch(src, old, new, walker.astype(np.int32), n_walkers, n_temps)


def band_slots(sources: np.ndarray, T: float, k_band0: int, width: int, n_bands: int, max_slots: int):
    """Assign sources to sub-bands of `width` bins starting at bin k_band0 by
    their carrier bin floor(f0 T), and lay them out as per-band slot lists in
    sampling coordinates (log10 A, f0, fdot, phi0, cos iota, psi, lambda,
    sin beta).

    Returns (u [n_bands, n_slot, 8], exists [n_bands, n_slot] int32, dropped)
    with n_slot = min(max_slots, largest band count + 8); sources beyond a
    band's capacity or outside the band range are dropped (count returned).
    """
    q = np.floor(sources[:, 1] * T).astype(np.int64)
    b = (q - k_band0) // width
    keep = (b >= 0) & (b < n_bands)
    counts = np.bincount(b[keep], minlength=n_bands)
    n_slot = int(min(max_slots, counts.max() + 8))
    u = np.zeros((n_bands, n_slot, 8))
    ex = np.zeros((n_bands, n_slot), np.int32)
    fill = np.zeros(n_bands, np.int64)
    dropped = int((~keep).sum())
    for i in np.nonzero(keep)[0]:
        bb = b[i]
        if fill[bb] >= n_slot:
            dropped += 1
            continue
        p = sources[i]
        u[bb, fill[bb]] = [np.log10(p[0]), p[1], p[2], p[3], np.cos(p[4]), p[5], p[6], np.sin(p[7])]
        ex[bb, fill[bb]] = 1
        fill[bb] += 1
    return u, ex, dropped


def band_sources(seed: int, n_bands: int, per_band: int, T: float, k_band0: int, width: int) -> np.ndarray:
    """per_band sources in each sub-band b (carrier bin inside [k_band0 + (b + 0.2) W,
    k_band0 + (b + 0.8) W)), unit amplitude, other parameters as in draw_sources
    (fdot = 0); rows ordered band-major."""
    rng = np.random.default_rng(seed)
    n = n_bands * per_band
    b = np.repeat(np.arange(n_bands), per_band)
    f0 = (k_band0 + (b + rng.uniform(0.2, 0.8, n)) * width) / T
    lam = rng.uniform(0.0, 2 * np.pi, n)
    sinb = rng.uniform(-1.0, 1.0, n)
    psi = rng.uniform(0.0, np.pi, n)
    cosi = rng.uniform(-1.0, 1.0, n)
    phi0 = rng.uniform(0.0, 2 * np.pi, n)
    return np.stack([np.ones(n), f0, np.zeros(n), phi0, np.arccos(cosi), psi, lam, np.arcsin(sinb)], axis=1)

"""Effective sample size of the sampler's ensemble traces (source-count and
log-likelihood traces of the cold chain), for the RJ acceptance and
effective-samples-per-second accounting.

tau_int: walker-averaged normalised autocorrelation (computed by zero-padded
FFT), Sokal's automatic window (smallest M with M >= c tau(M), c = 5),
capped to [1, n]; walkers with a constant trace are left out of the average
and a trace constant in every walker counts as one sample per walker.
ESS = n_walkers * n_sweeps / tau_int.
"""
from __future__ import annotations

import numpy as np

__all__ = ["autocorr", "tau_int", "ess"]


def autocorr(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    d = x - x.mean(axis=1, keepdims=True)
    v = np.sum(d * d, axis=1)
    keep = v > 0
    if not np.any(keep):
        return np.full(n, np.nan)
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(d[keep], m, axis=1)
    ac = np.fft.irfft(f * np.conj(f), m, axis=1)[:, :n]
    return np.mean(ac / v[keep, None], axis=0)


def tau_int(x, c: float = 5.0) -> float:
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    rho = autocorr(x)
    if np.isnan(rho[0]):
        return float(n)
    taus = 2.0 * np.cumsum(rho) - 1.0   # tau(M) = 1 + 2 sum_{k=1..M} rho(k)
    M = np.arange(n)
    ok = (M >= c * taus) & (M >= 1)
    tau = taus[np.argmax(ok)] if np.any(ok) else taus[-1]
    return float(min(max(tau, 1.0), n))


def ess(x, c: float = 5.0) -> float:
    x = np.asarray(x)
    return x.shape[0] * x.shape[1] / tau_int(x, c)

"""Plain O(n^2) integrated autocorrelation time and effective sample size of
ensemble traces.  TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU
leg); shares no code with the package.

Reading (the paper reports none): for traces X[w, n] of n_w walkers over n
sweeps, each walker's normalised autocorrelation
  rho_w(k) = sum_{i < n-k} (x_i - m_w)(x_{i+k} - m_w) / sum_i (x_i - m_w)^2
is averaged over the walkers with non-zero variance; tau(M) = 1 + 2 sum_{k=1..M}
rho(k); Sokal's automatic window takes the smallest M with M >= c tau(M)
(c = 5) and tau_int = tau(M), capped to [1, n] (a frozen trace counts as one
sample per walker); ESS = n_w n / tau_int.
"""
import numpy as np


def autocorr(x: np.ndarray) -> np.ndarray:
    """walker-averaged normalised autocorrelation rho(k), k = 0..n-1 (NaN if every walker is constant)"""
    x = np.asarray(x, dtype=np.float64)
    nw, n = x.shape
    acc = np.zeros(n)
    used = 0
    for w in range(nw):
        d = x[w] - x[w].mean()
        v = float(np.dot(d, d))
        if v == 0.0:
            continue
        for k in range(n):
            acc[k] += float(np.dot(d[: n - k], d[k:])) / v
        used += 1
    return acc / used if used else np.full(n, np.nan)


def tau_int(x: np.ndarray, c: float = 5.0) -> float:
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    rho = autocorr(x)
    if np.isnan(rho[0]):
        return float(n)
    tau = 1.0
    for M in range(1, n):
        tau += 2.0 * rho[M]
        if M >= c * tau:
            break
    return float(min(max(tau, 1.0), n))


def ess(x: np.ndarray, c: float = 5.0) -> float:
    x = np.asarray(x)
    return x.shape[0] * x.shape[1] / tau_int(x, c)

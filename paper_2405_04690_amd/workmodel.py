"""Algorithmic work per likelihood evaluation, for roofline reporting.

Bytes: what one fused swap evaluation must move from HBM: both parameter
vectors (2 x 64 B), the residual (16 B) and inverse-PSD (8 B) values of
channels A and E over the union U of the two template windows, and the 8-byte
result.  The templates themselves never leave the chip.

FP64 flops (an FMA counts 2): counted by hand from the formulation the
kernel evaluates, per template of width N (the per-template decode, done once
per source, is left out):
  slow part, per midpoint sample; every projection on the orbit is an affine
  function of (cos a, sin a, cos 2a, sin 2a) with per-source coefficients
    receiver terms, 3 craft: k.x/c 8, phase 5, f_r 2               -> 15 each
      phase factor: octant reduction in cycles + degree-15/16 Taylor  40 each
      (templates whose link phases stay below 0.25, about f0 < 4.7 mHz:
      40 for craft 0, and for craft 1, 2 the offset from craft 0 through
      the short link series and one complex product: 32 each)
    arm terms: k.n 8, q.n 8, p.n 4 for two arms, the third by closure 3,
      G 10 for each of the three arms                               -> 73
    links, 6: amplitude/phase 5, sinc & cos Taylor 45 (short series 23),
      envelope products 16                                   -> 66 (44) each
    TDI pieces and A/E combinations                                 -> 28
    common phase terms                                              -> 9
  FFT: 5 N log2 N per series (the standard radix-2 count), 4 series
  per bin: delay factor 6, 1 - D^2 1, per channel 23 (x2)          -> 53
inner products: 20 flops per union bin.
"""
from __future__ import annotations

import math

import numpy as np

PARAM_BYTES = 64
BIN_BYTES = 2 * (16 + 8)  # A and E: complex128 residual + float64 inverse PSD


C_LIGHT = 299792458.0


def flops_per_sample(small_u: bool = False) -> int:
    receivers = 3 * 15 + (40 + 2 * 32 if small_u else 3 * 40)
    return 9 + receivers + 73 + 6 * (44 if small_u else 66) + 28


def flops_per_template(N: int, n_series: int = 4, small_u: bool = False) -> int:
    return N * flops_per_sample(small_u) + n_series * 5 * N * int(math.log2(N)) + N * 53


AU = 1.495978707e11


def small_link_phase(params: np.ndarray, T: float, L: float = 2.5e9) -> np.ndarray:
    """templates whose link phases and receiver phase offsets stay below 0.25
    (the kernel's rule)"""
    Lc = L / C_LIGHT
    fd = np.abs(params[:, 2])
    f_max = np.abs(params[:, 1]) + fd * (T + 1100.0)
    return 2 * math.pi * Lc * (f_max + fd * (AU / C_LIGHT + 2 * Lc)) <= 0.25


def union_bins(params_old: np.ndarray, params_new: np.ndarray, T: float, N: int) -> np.ndarray:
    """Union size U of the two windows per pair (a zero-amplitude side has none)."""
    ko = np.floor(params_old[:, 1] * T)
    kn = np.floor(params_new[:, 1] * T)
    d = np.minimum(np.abs(kn - ko), N)
    u = N + d
    only_one = (params_old[:, 0] == 0) | (params_new[:, 0] == 0)
    both_zero = (params_old[:, 0] == 0) & (params_new[:, 0] == 0)
    u = np.where(only_one, N, u)
    return np.where(both_zero, 0, u).astype(np.int64)


def launch_work(params_old: np.ndarray, params_new: np.ndarray, T: float, N: int):
    """(algorithmic bytes, algorithmic FP64 flops) of one batched launch."""
    U = union_bins(params_old, params_new, T, N)
    B = params_old.shape[0]
    bytes_ = int(B * (2 * PARAM_BYTES + 8) + BIN_BYTES * U.sum())
    flops = 20 * int(U.sum())
    for p in (params_old, params_new):
        live = p[:, 0] != 0
        small = small_link_phase(p, T) & live
        flops += int(small.sum()) * flops_per_template(N, small_u=True)
        flops += int((live & ~small).sum()) * flops_per_template(N)
    return bytes_, flops

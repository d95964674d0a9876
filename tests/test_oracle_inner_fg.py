"""Pins of the oracle's stored-slice inner products, SNRs (Sec. 2 eq. inner
and the SNR definitions after eq. like) and of the Galactic-foreground PSD
term (Sec. 3, "Galactic foreground noise parameterization") against closed
forms, limits, invariants and matched-filter statistics."""
import numpy as np
import pytest

import oracle
from paper_2405_04690_amd import inputs

CFG = inputs.TINY
FG_EXAMPLE = np.array([3.3e-44, 1.2, 2.8e-3, 1763.3, 1686.3])  # the paper's example foreground


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)


def _noise4():
    return np.array([CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc])


def _sources(n, seed, f_lo=5e-4, f_hi=2e-2):
    """n sources spread in f0 so that their N = 128 windows never overlap"""
    rng = np.random.default_rng(seed)
    f0 = np.linspace(f_lo, f_hi, n) + rng.uniform(0, 1, n) / CFG.T
    return np.stack([10 ** rng.uniform(-22.5, -21.5, n), f0, np.zeros(n), rng.uniform(0, 2 * np.pi, n),
                     np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, np.pi, n), rng.uniform(0, 2 * np.pi, n),
                     np.arcsin(rng.uniform(-1, 1, n))], axis=1)


# --------------------------------------------------------------------------
# Galactic foreground
# --------------------------------------------------------------------------
def test_zero_foreground_amplitude_gives_the_instrument_psd(orc):
    th = np.concatenate([_noise4(), FG_EXAMPLE])
    th[4] = 0.0
    assert np.array_equal(orc.psd_eval_n(th, 9), orc.psd_eval(_noise4()))


def test_foreground_low_frequency_power_law(orc):
    """s1 = s2 = 0: S_fg = 3 A x^2 sin^2 x f^(-7/3) -> slope 4 - 7/3 = 5/3 in
    log-log as x -> 0 (pins the -7/3 and the x^2 sin^2 x factor)"""
    fg = np.array([1e-44, 1.2, 2.8e-3, 0.0, 0.0])
    f1, f2 = 1e-6, 2e-6
    s1, s2 = orc.foreground_value(f1, fg), orc.foreground_value(f2, fg)
    assert abs(np.log(s2 / s1) / np.log(2.0) - 5.0 / 3.0) < 1e-7  # sin x = x (1 - x^2/6): 4e-9
    x = 2 * np.pi * f1 * CFG.L / oracle.C_LIGHT
    assert abs(s1 / (3 * fg[0] * x ** 4 * f1 ** (-7 / 3)) - 1) < 1e-8


def test_foreground_knee_and_exponential_cut(orc):
    """tanh step: twice the knee value well below f_k, zero well above (the
    sign of the tanh argument); exp(-s1 f^alpha) recovers alpha"""
    fg = np.array([1e-44, 1.2, 2.8e-3, 0.0, 1e6])
    g = lambda f, p: orc.foreground_value(f, p) / orc.foreground_value(f, np.r_[p[0], p[1], p[2], 0.0, 0.0])
    assert abs(g(2.8e-3, fg) - 1.0) < 1e-12           # tanh(0) = 0 at the knee
    assert abs(g(2.7e-3, fg) - 2.0) < 1e-12           # below the knee the foreground is on
    assert g(2.9e-3, fg) < 1e-12                      # above it, off
    fg2 = np.array([1e-44, 1.2, 2.8e-3, 1763.3, 0.0])
    r = [-np.log(g(f, fg2)) for f in (1e-3, 4e-3)]    # = s1 f^alpha
    assert abs(np.log(r[1] / r[0]) / np.log(4.0) - 1.2) < 1e-9
    assert abs(r[0] / (1763.3 * 1e-3 ** 1.2) - 1) < 1e-9


def test_paper_example_foreground_shape(orc):
    """the paper's example point: the confusion noise exceeds the instrument
    noise around 1 mHz and has vanished (relative 1e-10) by 10 mHz"""
    th = np.concatenate([_noise4(), FG_EXAMPLE])
    S9 = orc.psd_eval_n(th, 9)[0]
    S4 = orc.psd_eval(_noise4())[0]
    f = (orc.k_min + np.arange(orc.n_bins)) / CFG.T
    i1, i10 = np.searchsorted(f, 1e-3), np.searchsorted(f, 1e-2)
    assert S9[0, i1] > 2 * S4[0, i1]
    assert abs(S9[0, i10] / S4[0, i10] - 1) < 1e-10
    # shared by A and E: their difference is the instrument difference
    th2 = th.copy()
    th2[2] *= 1.3
    S9b = orc.psd_eval_n(th2, 9)[0]
    S4b = orc.psd_eval(th2[:4])[0]
    assert np.allclose(S9b[1] - S9b[0], S4b[1] - S4b[0], rtol=1e-12, atol=1e-12 * S9b.max())


def test_foreground_likelihood_is_stationary_at_the_truth(orc):
    """noise drawn at S = S_n + S_fg(theta0): the PSD log-likelihood's
    derivative in the foreground amplitude at the truth is a zero-mean score
    with variance sum (S_fg/S)^2 (Fisher); 5 sigma.  At twice the amplitude it
    is strongly negative."""
    th = np.concatenate([_noise4(), FG_EXAMPLE])
    S = orc.psd_eval_n(th, 9)
    R = np.sqrt(S[0] / (4 * orc.df)) * inputs.complex_normals(91, (2, orc.n_bins))
    def lnl(scale):
        t = th.copy()
        t[4] *= scale
        return orc.psd_loglike_n(R[None], t, 9, np.zeros(1, np.int32))[0]
    eps = 1e-4
    d = (lnl(1 + eps) - lnl(1 - eps)) / (2 * eps)
    Sfg = S[0] - orc.psd_eval(_noise4())[0]
    sigma = np.sqrt(np.sum((Sfg / S[0]) ** 2))
    assert abs(d) < 5 * sigma, (d, sigma)
    d2 = (lnl(2 + eps) - lnl(2 - eps)) / (2 * eps)
    assert d2 < -10 * sigma


# --------------------------------------------------------------------------
# Stored-slice inner products and SNRs
# --------------------------------------------------------------------------
def test_inner_noise_free_and_scaling(orc):
    src = _sources(20, 1)
    A, E, _, sb = orc.waveform(src, 128, with_T=False)
    S = orc.psd_eval(_noise4())
    data = np.zeros((1, 2, orc.n_bins), complex)
    orc.scatter_add(src, 128, 1.0, data)
    out = orc.inner(A, E, sb, data, S)
    assert np.allclose(out[:, 1], out[:, 0], rtol=1e-13, atol=0)     # R = h: <R|h> = <h|h>
    # eq. addsource with R = h: dlnL = <h|h> - 1/2 <h|h>
    zero = src.copy()
    zero[:, 0] = 0.0
    dl = orc.delta_loglike(data, S, zero, src, 128)
    assert np.allclose(dl, 0.5 * out[:, 0], rtol=1e-12, atol=0)
    out2 = orc.inner(2 * A, 2 * E, sb, data, S)
    assert np.array_equal(out2[:, 0], 4 * out[:, 0]) and np.array_equal(out2[:, 1], 2 * out[:, 1])
    outi = orc.inner(A, E, sb, data, 1.0 / S, psd_is_inverse=True)
    assert np.allclose(outi, out, rtol=1e-14, atol=0)


def test_inner_matched_filter_statistics(orc):
    """<n|h> over 400 disjoint windows of one noise realisation at PSD S:
    independent N(0, <h|h>) draws (normalisation of eq. inner with the noise
    convention E[<n|n>] = 2 per bin and channel)"""
    src = _sources(400, 2, 2e-4, 2.9e-2)
    A, E, _, sb = orc.waveform(src, 128, with_T=False)
    S = orc.psd_eval(_noise4())
    n = np.sqrt(S[0] / (4 * orc.df)) * inputs.complex_normals(3, (2, orc.n_bins))
    out = orc.inner(A, E, sb, n[None], S)
    z = out[:, 1] / np.sqrt(out[:, 0])
    assert abs(z.mean()) < 5 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))


def test_inner_clips_to_the_band(orc):
    """P11: a slice straddling k_min counts only its in-band bins"""
    rng = np.random.default_rng(4)
    N = 128
    A = rng.normal(size=(1, N)) + 1j * rng.normal(size=(1, N))
    E = rng.normal(size=(1, N)) + 1j * rng.normal(size=(1, N))
    sb = np.array([orc.k_min - 40])
    S = orc.psd_eval(_noise4())
    R = rng.normal(size=(1, 2, orc.n_bins)) + 1j * rng.normal(size=(1, 2, orc.n_bins))
    out = orc.inner(A, E, sb, R, S)
    A2, E2 = A.copy(), E.copy()
    A2[:, :40] = 0
    E2[:, :40] = 0
    out2 = orc.inner(A2, E2, sb, R, S)
    assert np.array_equal(out, out2)
    hh = 4 * orc.df * (np.sum(np.abs(A[0, 40:]) ** 2 / S[0, 0, :N - 40]) + np.sum(np.abs(E[0, 40:]) ** 2 / S[0, 1, :N - 40]))
    assert abs(out[0, 0] / hh - 1) < 1e-13


def test_snr_definitions(orc):
    """optimal SNR^2 = <h|h>; noise-free data: observed = optimal; data =
    signal + noise: observed - optimal ~ N(0, 1); zero amplitude: 0 and NaN"""
    src = _sources(300, 5, 2e-4, 2.9e-2)
    S = orc.psd_eval(_noise4())
    A, E, _, sb = orc.waveform(src, 128, with_T=False)
    hh = orc.inner(A, E, sb, np.zeros((1, 2, orc.n_bins), complex), S)[:, 0]
    data = np.zeros((1, 2, orc.n_bins), complex)
    orc.scatter_add(src, 128, 1.0, data)
    opt, obs = orc.snr(src, 128, S, data=data)
    assert np.allclose(opt ** 2, hh, rtol=1e-13, atol=0)
    assert np.allclose(obs, opt, rtol=1e-12, atol=0)
    noisy = data + np.sqrt(S[0] / (4 * orc.df)) * inputs.complex_normals(6, (2, orc.n_bins))
    opt2, obs2 = orc.snr(src, 128, S, data=noisy)
    assert np.array_equal(opt2, opt)
    z = obs2 - opt2
    assert abs(z.mean()) < 5 / np.sqrt(len(z)) and abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))
    zero = src[:2].copy()
    zero[:, 0] = 0.0
    o, b = orc.snr(zero, 128, S, data=data)
    assert np.all(o == 0) and np.all(np.isnan(b))
    o3, b3 = orc.snr(src[:3], 128, S)
    assert b3 is None and np.array_equal(o3, opt[:3])

"""Oracle noise-PSD step: at zero inverse temperature the stretch moves keep
the uniform prior box (eq. stretch's z^(d-1) factor), equal inverse
temperatures always swap, the cold chain's 1/S is eq. psd at its parameters,
and the stored log-likelihoods are eq. like at the final parameters."""
import numpy as np
import pytest
from scipy import stats as sps

import oracle
from paper_2405_04690_amd import inputs

CFG = inputs.TINY
LO = (10e-12, 2e-15, 10e-12, 2e-15)
HI = (20e-12, 4e-15, 20e-12, 4e-15)


def _setup(nt, nw, seed, f_lo=CFG.f_lo, f_hi=CFG.f_hi):
    orc = oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=f_lo, f_hi=f_hi)
    pc = oracle.PsdSweepConfig()
    pc.n_tn, pc.n_walkers, pc.n_par, pc.stretch_a, pc.seed = nt, nw, 4, 2.0, seed
    for k in range(4):
        pc.prior_lo[k], pc.prior_hi[k] = LO[k], HI[k]
    S = orc.psd_eval(np.array([CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc]))[0]
    data = np.sqrt(S / (4 * orc.df)) * inputs.complex_normals(seed, (2, orc.n_bins))
    resid = np.zeros((2, nw, 2, orc.n_bins), np.complex128)
    resid[0] = data          # buffer 0 = data, buffer 1 = data: full residual = data
    resid[1] = data
    rng = np.random.default_rng(seed + 1)
    theta = np.array(LO) + (np.array(HI) - np.array(LO)) * rng.uniform(size=(nt, nw, 4))
    return orc, pc, data, resid, theta


def test_zero_temperature_keeps_the_prior_box():
    """final states of 20 independent ensembles (32 walkers, 80 steps, a narrow
    band so the likelihood is cheap; it does not enter at beta = 0) are
    uniform in the box; dropping the z^(d-1) factor fails this at p ~ 1e-6"""
    finals = []
    acc = []
    for rep in range(20):
        orc, pc, data, resid, theta = _setup(1, 32, 100 + rep, f_lo=1e-3, f_hi=1.1e-3)
        logl = np.zeros((1, 32))
        inv = np.zeros((32, 2, orc.n_bins))
        st = np.zeros(4, np.int64)
        for s in range(80):
            oracle.psd_sweep_step(orc, pc, s, theta, logl, np.zeros(1), data, resid, inv, st)
        finals.append(theta[0].copy())
        acc.append(st[1] / st[0])
    x = np.concatenate(finals)
    assert np.mean(acc) > 0.3
    for k in range(4):
        u = (x[:, k] - LO[k]) / (HI[k] - LO[k])
        assert sps.kstest(u, "uniform").pvalue > 1e-4, k


def test_swaps_equal_betas_and_cold_psd():
    orc, pc, data, resid, theta = _setup(3, 4, 5)
    logl = np.zeros((3, 4))
    inv = np.zeros((4, 2, orc.n_bins))
    st = np.zeros(4, np.int64)
    oracle.psd_sweep_step(orc, pc, 0, theta, logl, np.ones(3), data, resid, inv, st)
    assert st[2] == 2 * 4 and st[3] == st[2]     # equal inverse temperatures: every swap accepted
    S = orc.psd_eval(theta[0])
    assert np.allclose(inv, 1.0 / S, rtol=1e-15, atol=0)
    full = resid[0] + resid[1] - data
    ref = orc.psd_loglike(np.broadcast_to(full, (4, 2, orc.n_bins)).copy(), theta.reshape(-1, 4),
                          np.tile(np.arange(4, dtype=np.int32), 3))
    assert np.allclose(logl.ravel(), ref, rtol=1e-14, atol=0)


FG_LO = (1e-44, 0.8, 1.5e-3, 500.0, 500.0)
FG_HI = (1e-43, 1.6, 4.0e-3, 3000.0, 3000.0)


def test_zero_temperature_keeps_the_prior_box_with_the_foreground():
    """nine parameters (instrument + Galactic foreground, Sec. 3): the z^(d-1)
    factor with d = 9 keeps the uniform box at beta = 0 on every coordinate"""
    lo9 = np.array(LO + FG_LO)
    hi9 = np.array(HI + FG_HI)
    finals, acc = [], []
    for rep in range(12):
        orc, pc, data, resid, _ = _setup(1, 32, 200 + rep, f_lo=1e-3, f_hi=1.1e-3)
        pc.n_par = 9
        for k in range(9):
            pc.prior_lo[k], pc.prior_hi[k] = lo9[k], hi9[k]
        rng = np.random.default_rng(300 + rep)
        theta = lo9 + (hi9 - lo9) * rng.uniform(size=(1, 32, 9))
        logl = np.zeros((1, 32))
        inv = np.zeros((32, 2, orc.n_bins))
        st = np.zeros(4, np.int64)
        for s in range(80):
            oracle.psd_sweep_step(orc, pc, s, theta, logl, np.zeros(1), data, resid, inv, st)
        finals.append(theta[0].copy())
        acc.append(st[1] / st[0])
    x = np.concatenate(finals)
    assert np.mean(acc) > 0.15
    for k in range(9):
        u = (x[:, k] - lo9[k]) / (hi9[k] - lo9[k])
        assert sps.kstest(u, "uniform").pvalue > 1e-4, k
    # the cold chain's 1/S includes the foreground of its parameters
    S = orc.psd_eval_n(theta[0, :2], 9)
    assert np.allclose(inv[:2], 1.0 / S, rtol=1e-15, atol=0)

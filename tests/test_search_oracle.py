"""Pins of the oracle's per-sub-band source search (appendix "Algorithm for
fitting proposal distributions"): at zero inverse temperature the stretch
chains keep the band-confined prior box; the target never exceeds its closed-
form maximum 1/2 <d|d> and the search reaches it for an injected source in
noise-free data; equal temperatures always swap; converged bands freeze; the
restart ball stays in the box."""
import numpy as np
import pytest
from scipy import stats as sps

import oracle
from paper_2405_04690_amd import inputs

CFG = inputs.TINY
N = 128
W = 128
LO = (-23.0, 0.0, -1e-17, 0.0, -1.0, 0.0, 0.0, -1.0)
HI = (-20.5, 0.0, 1e-17, 0.0, 1.0, 0.0, 0.0, 1.0)


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)


@pytest.fixture(scope="module")
def psd(orc):
    return orc.psd_eval(np.array([CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc]))[0]


def _config(nb, nt, nw, seed, k_band0, n_stall=10 ** 9):
    sc = oracle.SearchConfig()
    sc.n_bands, sc.n_temps, sc.n_walkers, sc.N, sc.width, sc.n_stall = nb, nt, nw, N, W, n_stall
    sc.k_band0, sc.stretch_a, sc.seed = k_band0, 2.0, seed
    for k in range(8):
        sc.prior_lo[k], sc.prior_hi[k] = LO[k], HI[k]
    return sc


def _box(sc, b):
    lo, hi = np.array(LO, float), np.array(HI, float)
    lo[1] = (sc.k_band0 + b * W) / CFG.T
    hi[1] = (sc.k_band0 + (b + 1) * W) / CFG.T
    for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
        lo[k], hi[k] = 0.0, P
    return lo, hi


def _start(sc, st, rng):
    for b in range(sc.n_bands):
        lo, hi = _box(sc, b)
        st.u[b] = lo + (hi - lo) * rng.uniform(size=st.u[b].shape)


def test_zero_temperature_keeps_the_band_box(orc, psd):
    """beta = 0: every coordinate of the final states is uniform in the band's
    box (f0 confined to the band, angles on their circles)"""
    k0 = int(4e-3 * CFG.T)
    R = np.sqrt(psd / (4 * orc.df)) * inputs.complex_normals(11, (2, orc.n_bins))
    finals = []
    acc = []
    for rep in range(10):
        sc = _config(2, 1, 32, 100 + rep, k0)
        st = oracle.SearchState(sc)
        st.betas[:] = 0.0
        _start(sc, st, np.random.default_rng(200 + rep))
        oracle.search_eval(orc, sc, st, R, psd)
        for it in range(60):
            oracle.search_step(orc, sc, st, it, R, psd)
        acc.append(st.stats[1] / st.stats[0])
        for b in range(2):
            lo, hi = _box(sc, b)
            finals.append((st.u[b, 0] - lo) / (hi - lo))
    x = np.concatenate(finals)
    assert np.mean(acc) > 0.1
    for k in range(8):
        assert sps.kstest(x[:, k], "uniform").pvalue > 1e-4, k


def test_search_finds_an_injected_source(orc, psd):
    """noise-free data holding one source per band: the target is bounded by
    1/2 <d|d> (equality at h = d) and the search gets within a few units of
    it, at the source's frequency and amplitude"""
    k0 = int(3e-3 * CFG.T)
    sc = _config(2, 6, 32, 7, k0, n_stall=100)
    rng = np.random.default_rng(8)
    src = inputs.draw_sources(9, 2, (3e-3, 3e-3), (-19.0, -18.0))
    src[:, 2] = 0.0
    src[:, 1] = (k0 + np.array([0.55, 1.45]) * W + 0.3) / CFG.T
    opt, _ = orc.snr(src, N, psd[None])
    src[:, 0] *= 25.0 / opt
    d = np.zeros((1, 2, orc.n_bins), np.complex128)
    orc.scatter_add(src, N, 1.0, d)
    st = oracle.SearchState(sc)
    st.betas[:] = np.geomspace(1.0, 0.003, 6)
    _start(sc, st, rng)
    oracle.search_eval(orc, sc, st, d, psd)
    half_dd = 0.5 * 25.0 ** 2
    for it in range(3000):
        oracle.search_step(orc, sc, st, it, d, psd)
        assert np.all(st.logl <= half_dd * (1 + 1e-9))
        if np.all(st.stall >= sc.n_stall):
            break
    assert np.all(st.stall >= sc.n_stall)
    # a restart ball around the best points, then converge again
    sigma = np.array([0.01, 0.05 / CFG.T, 0.0, 0.05, 0.02, 0.05, 0.02, 0.02])
    oracle.search_ball(orc, sc, st, 10 ** 6, sigma, d, psd)
    assert np.all(st.stall == 0)
    for it in range(3000):
        oracle.search_step(orc, sc, st, 10 ** 6 + 1 + it, d, psd)
        if np.all(st.stall >= sc.n_stall):
            break
    # the parameters are partly degenerate (amplitude with inclination, f0
    # with sky position at 0.25 yr): the found template is compared with the
    # injected one by their overlap
    bu = st.best_u
    best = np.stack([10 ** bu[:, 0], bu[:, 1], bu[:, 2], bu[:, 3], np.arccos(bu[:, 4]), bu[:, 5], bu[:, 6],
                     np.arcsin(bu[:, 7])], axis=1)
    ov = orc.overlap(best, src, N, psd[None])[:, 3]
    for b in range(2):
        assert st.best_logl[b] > half_dd - 4.0, (b, st.best_logl[b], half_dd)
        assert ov[b] > 0.99, ov


def test_swaps_converged_bands_and_the_ball(orc, psd):
    k0 = int(5e-3 * CFG.T)
    R = np.sqrt(psd / (4 * orc.df)) * inputs.complex_normals(13, (2, orc.n_bins))
    sc = _config(3, 3, 8, 21, k0, n_stall=5)
    st = oracle.SearchState(sc)
    _start(sc, st, np.random.default_rng(22))
    oracle.search_eval(orc, sc, st, R, psd)
    ref = st.logl.copy()
    oracle.search_eval(orc, sc, st, R, psd)
    assert np.array_equal(ref, st.logl)
    st.betas[:] = 1.0
    st.stall[1] = sc.n_stall             # band 1 has converged: it must not move
    frozen = st.u[1].copy()
    oracle.search_step(orc, sc, st, 0, R, psd)
    assert np.array_equal(st.u[1], frozen)
    assert st.stats[2] == 2 * 8 * 2 and st.stats[3] == st.stats[2]   # equal betas: every swap accepted
    # the ball: inside the box, logl re-evaluated, stall cleared
    st.best_u[:] = st.u[:, 0, 0]
    sigma = np.array([0.5, 1e3 / CFG.T, 0.0, 4.0, 0.8, 4.0, 4.0, 0.8])   # wide: exercises clamping and wrapping
    oracle.search_ball(orc, sc, st, 5, sigma, R, psd)
    assert np.all(st.stall == 0)
    for b in range(3):
        lo, hi = _box(sc, b)
        x = st.u[b].reshape(-1, 8)
        assert np.all(x >= lo) and np.all(x[:, [0, 2, 4, 7]] <= hi[[0, 2, 4, 7]]) and np.all(x[:, 1] < hi[1])
        assert np.all(x[:, [3, 5, 6]] < hi[[3, 5, 6]])
    chk = st.logl.copy()
    oracle.search_eval(orc, sc, st, R, psd)
    assert np.array_equal(chk, st.logl)

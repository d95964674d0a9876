"""Pins of the oracle's sampler arithmetic (CPU)."""
import numpy as np
import pytest

import oracle
import sampler_setup


def test_philox_matches_numpy_bit_generator():
    """Philox4x64-10 equals numpy's Philox (which pre-increments its counter)."""
    for key in ([0, 0], [123, 456], [2**63 + 5, 17]):
        g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.zeros(4, dtype=np.uint64))
        raw = g.random_raw(4 * 5)
        for blk in range(5):
            got = oracle.philox([blk + 1, 0, 0, 0], key)
            assert got == [int(x) for x in raw[4 * blk:4 * blk + 4]]


def test_rng_uniform_range_and_moments():
    u = np.array([oracle.rng_uniform(9, 3, 1, 77, i) for i in range(20000)])
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))
    hist = np.histogram(u, bins=20, range=(0, 1))[0]
    chi2 = np.sum((hist - len(u) / 20) ** 2 / (len(u) / 20))
    assert chi2 < 19 + 5 * np.sqrt(2 * 19)


def test_residual_aware_swap_reduces_to_standard_swap():
    """eq. temp-final equals eq. temp-orig when both walkers see one likelihood."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        bI, bII = rng.uniform(0, 1, 2)
        Ln, Lm = rng.normal(0, 100, 2)
        la = oracle.pt_log_alpha(bI, bII, Lm, Ln, Ln, Lm)
        # (L_n / L_m)^(beta_j - beta_i) with walker i at beta_I holding n
        assert abs(la - (bII - bI) * (Ln - Lm)) <= 1e-12 * (1 + abs(Ln) + abs(Lm))


def test_rj_pass_keeps_the_prior_at_zero_inverse_temperature():
    """At beta = 0 every flip is accepted: occupied slots are emptied and empty
    slots receive prior draws, so slot occupancy stays Bernoulli(1/2) and the
    parameters of occupied slots are prior draws."""
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=6, n_b=4, n_slots=6, beta_top=1.0)
    rng = np.random.default_rng(1)
    st.exists[:] = (rng.uniform(size=st.exists.shape) < 0.5).astype(np.int32)
    st.betas[:] = 0.0
    before = st.exists.copy()
    oracle.sweep_step(orc, sc, st, oracle.MOVE_RJ, 1, sweep=5)
    oracle.sweep_step(orc, sc, st, oracle.MOVE_RJ, 0, sweep=5)
    assert np.array_equal(st.exists, 1 - before)
    born = (before == 0)
    uu = st.u[born]
    assert st.stats[3] == born.sum() and st.stats[5] == before.sum()
    # log10 A uniform on the prior box; cos iota and sin beta uniform on [-1, 1]
    for k, (lo, hi) in ((0, (sc.prior_lo[0], sc.prior_hi[0])), (4, (-1, 1)), (7, (-1, 1))):
        x = (uu[:, k] - lo) / (hi - lo)
        assert x.min() >= 0 and x.max() <= 1
        assert abs(x.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(x))


# --------------------------------------------------------------------------
# Group stretch (eq. stretch with the stationary group, appendix on in-model
# GB proposals): at beta = 0 the target is the uniform prior box, so a chain
# built from the oracle's proposal and the z^(d-1) factor must leave every
# coordinate uniform, the periodic angles included.
# --------------------------------------------------------------------------
def _band_box(sc, T, b):
    W = sc.band_width or sc.N
    lo = np.array(list(sc.prior_lo))
    hi = np.array(list(sc.prior_hi))
    lo[1] = (sc.k_band0 + (b - 0.5) * W) / T
    hi[1] = (sc.k_band0 + (b + 1.5) * W) / T
    for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
        lo[k], hi[k] = 0.0, P
    return lo, hi


def test_stretch_proposal_keeps_the_uniform_box_invariant():
    """6000 independent chains started uniform, 25 steps each with a fixed group
    of 10 friends: the marginals stay uniform (KS) on all eight coordinates.
    The wrapped stretch without its reversibility check fails this test on the
    non-periodic coordinates (p ~ 1e-9): a move that cannot be undone
    mis-weights z."""
    from scipy import stats as sps
    cfg, orc, sc, st = sampler_setup.problem(n_t=1, n_w=4, n_b=2, n_slots=3, n_friends=64)
    b = 1
    lo, hi = _band_box(sc, cfg.T, b)
    rng = np.random.default_rng(0)
    group = lo + (hi - lo) * rng.uniform(size=(10, 8))
    group = group[np.argsort(group[:, 1], kind="stable")]
    x = lo + (hi - lo) * rng.uniform(size=(6000, 8))
    acc = 0
    for _ in range(25):
        for c in range(len(x)):
            ok, un, lr = oracle.stretch_propose(sc, x[c], group, rng.uniform(), rng.uniform())
            if ok and oracle.in_prior(orc, sc, b, un) and np.log(rng.uniform()) < lr:
                x[c] = un
                acc += 1
    assert acc > 0.1 * 25 * len(x)
    for k in range(8):
        p = sps.kstest((x[:, k] - lo[k]) / (hi[k] - lo[k]), "uniform").pvalue
        assert p > 1e-4, (k, p)


def test_stretch_proposal_is_an_involution():
    """the move from u' with the same friend and 1/z returns to u (mod the
    periods); a rejected proposal is one whose reverse would not return"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=1, n_w=4, n_b=2, n_slots=3, n_friends=64)
    lo, hi = _band_box(sc, cfg.T, 1)
    rng = np.random.default_rng(1)
    X = lo + (hi - lo) * rng.uniform(size=(1, 8))
    a = sc.stretch_a
    n_rej = 0
    for _ in range(2000):
        u = lo + (hi - lo) * rng.uniform(size=8)
        uz = rng.uniform()
        ok, un, lr = oracle.stretch_propose(sc, u, X, 0.5, uz)
        z = ((a - 1) * uz + 1) ** 2 / a
        assert abs(lr - 7 * np.log(z)) < 1e-14
        # the uniform giving 1/z: ((a-1) v + 1)^2 / a = 1/z
        v = (np.sqrt(a / z) - 1) / (a - 1)
        ok2, back, _ = oracle.stretch_propose(sc, un, X, 0.5, v)
        d = np.abs(back - u)
        for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
            d[k] = min(d[k], P - d[k])
        if ok:
            assert ok2 and np.max(d / (hi - lo)) < 1e-12
        else:
            n_rej += 1
    assert 0 < n_rej < 2000


@pytest.mark.parametrize("W", [None, 200])
def test_inmodel_band_loop_keeps_the_prior_at_zero_inverse_temperature(W):
    """the band loop's wiring of the move (slot pick, friend window, prior box,
    acceptance) at beta = 0 with a fixed group no larger than n_friends: all
    eight coordinates of 768 independent slot chains stay uniform (one final
    snapshot: successive snapshots of one chain are correlated, which KS does
    not allow for; the exactness itself is pinned with more power by the
    stand-alone chain test above)"""
    from scipy import stats as sps
    cfg, orc, sc, st = sampler_setup.problem(n_t=16, n_w=4, n_b=4, n_slots=3, n_prop=6, n_friends=16, seed=9, W=W)
    rng = np.random.default_rng(2)
    for b in range(sc.n_bands):
        lo, hi = _band_box(sc, cfg.T, b)
        st.u[:, :, b] = lo + (hi - lo) * rng.uniform(size=st.u[:, :, b].shape)
    st.exists[:] = 1
    st.betas[:] = 0.0
    oracle.sweep_group(sc, st)
    assert st.group_count.max() <= sc.n_friends
    for it in range(12):
        oracle.sweep_step(orc, sc, st, oracle.MOVE_INMODEL, 1, it)
        oracle.sweep_step(orc, sc, st, oracle.MOVE_INMODEL, 0, it)
    assert st.stats[1] > 0.1 * st.stats[0]
    x = []
    for b in range(sc.n_bands):
        lo, hi = _band_box(sc, cfg.T, b)
        x.append((st.u[:, :, b].reshape(-1, 8) - lo) / (hi - lo))
    x = np.concatenate(x)
    for k in range(8):
        p = sps.kstest(x[:, k], "uniform").pvalue
        assert p > 1e-3, (k, p)


# --------------------------------------------------------------------------
# Alg. gb2 pieces: the window likelihood, the pairing, the write-back
# --------------------------------------------------------------------------
def _full_lnl(orc, sc, R, inv_psd, U, ex):
    """-1/2 <R - H|R - H> over the whole analysis band, H = the sources U[ex]
    (eq. like without the PSD term, which cancels in differences)"""
    x = R.copy()
    for u in U[ex.astype(bool)]:
        orc.scatter_add(sampler_setup._phys(u)[None], sc.N, -1.0, x)
    return -0.5 * 4 * orc.df * np.sum((x.real ** 2 + x.imag ** 2) * inv_psd)


@pytest.mark.parametrize("W", [None, 384, 200])
def test_band_loglike_differences_equal_full_band_likelihood_differences(W):
    """band_loglike over the band's window (2W + N bins) differs between two
    source sets by exactly what the full-band eq. like does (every template
    of band b lies inside the window, also at the ends of the f0 range); it
    reads walker w_res's opposite-parity buffer"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=3, n_b=4, n_slots=4, seed=13, W=W)
    rng = np.random.default_rng(14)
    for b in (1, 2):
        par = b & 1
        for k, ((t1, w1), (t2, w2), wr) in enumerate((((0, 0), (1, 2), 1), ((1, 1), (0, 2), 0))):
            st.exists[t1, w1, b, 2] = 1  # a third source in one set
            lo, hi = _band_box(sc, cfg.T, b)
            st.u[t1, w1, b, 2] = lo + (hi - lo) * rng.uniform(size=8)
            st.u[t1, w1, b, 2, 0] = -21.5
            # at the lowest f0 of the band's range, or just below its top
            st.u[t1, w1, b, 2, 1] = lo[1] if k == 0 else hi[1] - 0.01 / cfg.T
            l1 = oracle.band_loglike(orc, sc, st, t1, w1, b, wr)
            l2 = oracle.band_loglike(orc, sc, st, t2, w2, b, wr)
            R = st.resid[1 - par, wr]
            f1 = _full_lnl(orc, sc, R, st.inv_psd[wr], st.u[t1, w1, b], st.exists[t1, w1, b])
            f2 = _full_lnl(orc, sc, R, st.inv_psd[wr], st.u[t2, w2, b], st.exists[t2, w2, b])
            assert abs((l1 - l2) - (f1 - f2)) <= 1e-9 * max(1.0, abs(f1), abs(f2)), (b, l1 - l2, f1 - f2)
            assert abs(l1 - l2) > 1.0  # the sets differ measurably


@pytest.mark.parametrize("W", [None, 384])
def test_cold_chain_buffers_stay_consistent_through_every_move(W):
    """after in-model, RJ and tempering steps each parity buffer equals the data
    minus the current cold-chain sources of its bands (rebuilt from scratch)"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=3, n_w=3, n_b=4, n_slots=4, n_prop=6, seed=17, beta_top=0.5, W=W)
    oracle.sweep_group(sc, st)
    for move in (oracle.MOVE_INMODEL, oracle.MOVE_RJ, oracle.MOVE_PT):
        for parity in (1, 0):
            oracle.sweep_step(orc, sc, st, move, parity, 3)
        for par in (0, 1):
            for w in range(sc.n_walkers):
                ref = sampler_setup.rebuild_buffer(orc, sc, st, par, w)
                assert np.max(np.abs(st.resid[par, w] - ref)) <= 1e-9 * np.abs(ref).max(), (move, par, w)
    assert st.stats[1] > 0 and st.stats[3] + st.stats[5] > 0 and st.stats[7] > 0


def _pt_perm(sc, sweep, b, t):
    perm = list(range(sc.n_walkers))
    for j in range(sc.n_walkers - 1, 0, -1):
        r = int(np.floor(oracle.rng_uniform(sc.seed, sweep, 3, b * sc.n_temps + t, j) * (j + 1)))
        perm[j], perm[r] = perm[r], perm[j]
    return perm


def test_equal_temperatures_with_shared_residuals_always_swap():
    """one band (so every walker sees the same residual) and equal inverse
    temperatures: eq. temp-final gives ln alpha = 0 exactly, so every swap is
    accepted; each set then moves down one rung along the walkers that the
    Fisher-Yates pairing names, the hottest set ends in the cold chain, and the
    cold chain's buffer follows it"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=4, n_w=5, n_b=1, n_slots=3, seed=19)
    for w in range(sc.n_walkers):
        st.resid[1, w] = st.data
    st.betas[:] = 1.0
    before_u, before_ex = st.u.copy(), st.exists.copy()
    sweep = 6
    oracle.sweep_step(orc, sc, st, oracle.MOVE_PT, 0, sweep)
    assert st.stats[6] == sc.n_walkers * (sc.n_temps - 1) and st.stats[7] == st.stats[6]
    perms = [_pt_perm(sc, sweep, 0, t) for t in range(sc.n_temps)]
    for i in range(sc.n_walkers):
        wt = [perms[t][i] for t in range(sc.n_temps)]
        # swaps from the hottest pair down: set of (t - 1) <- old set of t for t = n_t - 1 ... 1 in turn,
        # so (0, w_0) ends with the hottest set and (t, w_t) with the old set of (t - 1)
        assert np.array_equal(st.u[0, wt[0], 0], before_u[sc.n_temps - 1, wt[-1], 0])
        assert np.array_equal(st.exists[0, wt[0], 0], before_ex[sc.n_temps - 1, wt[-1], 0])
        for t in range(1, sc.n_temps):
            assert np.array_equal(st.u[t, wt[t], 0], before_u[t - 1, wt[t - 1], 0])
    for w in range(sc.n_walkers):
        ref = sampler_setup.rebuild_buffer(orc, sc, st, 0, w)
        assert np.max(np.abs(st.resid[0, w] - ref)) <= 1e-9 * np.abs(ref).max()


# --------------------------------------------------------------------------
# Reversible jump with a given proposal density (eq. rj-acceptance): at
# beta = 0 the chain must keep the prior (occupancy 1/2, uniform parameters)
# whatever q is, provided ln q is the density the candidates are drawn from
# --------------------------------------------------------------------------
def test_rj_with_a_given_proposal_keeps_the_prior_at_zero_inverse_temperature():
    from scipy import stats as sps
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=6, n_b=4, n_slots=8, seed=23)
    rng = np.random.default_rng(24)
    for b in range(sc.n_bands):
        lo, hi = _band_box(sc, cfg.T, b)
        st.u[:, :, b] = lo + (hi - lo) * rng.uniform(size=st.u[:, :, b].shape)
    st.exists[:] = (rng.uniform(size=st.exists.shape) < 0.5).astype(np.int32)
    st.betas[:] = 0.0
    boxes = [_band_box(sc, cfg.T, b) for b in range(sc.n_bands)]

    def lnq(u, b):
        # q: f0 ~ Beta(3, 3) over the band's range, the rest uniform over the box
        lo, hi = boxes[b]
        x = (u[1] - lo[1]) / (hi[1] - lo[1])
        return sps.beta.logpdf(x, 3, 3) - np.log(hi[1] - lo[1]) - np.sum(np.log(np.delete(hi - lo, 1)))

    f0s = []
    for it in range(30):
        prop = np.zeros_like(st.u)
        logq = np.zeros(st.exists.shape)
        for (t, w, b, s) in np.ndindex(*st.exists.shape):
            lo, hi = boxes[b]
            if st.exists[t, w, b, s]:
                logq[t, w, b, s] = lnq(st.u[t, w, b, s], b)
            else:
                cand = lo + (hi - lo) * rng.uniform(size=8)
                cand[1] = lo[1] + (hi[1] - lo[1]) * rng.beta(3, 3)
                prop[t, w, b, s] = cand
                logq[t, w, b, s] = lnq(cand, b)
        for parity in (1, 0):
            oracle.sweep_step(orc, sc, st, oracle.MOVE_RJ, parity, it, prop_u=prop, rj_logq=logq)
        if it >= 10 and it % 4 == 0:
            for b in range(sc.n_bands):
                lo, hi = boxes[b]
                ex = st.exists[:, :, b].astype(bool)
                f0s.append((st.u[:, :, b][ex][:, 1] - lo[1]) / (hi[1] - lo[1]))
    assert st.stats[3] > 0.1 * st.stats[2] and st.stats[5] > 0.1 * st.stats[4]
    assert abs(st.exists.mean() - 0.5) < 0.08
    x = np.concatenate(f0s)
    assert sps.kstest(x, "uniform").pvalue > 1e-4
    # under q the centre fifth would hold 35% of the sources; under the prior 20%
    assert abs(np.mean(np.abs(x - 0.5) < 0.1) - 0.2) < 0.05


# --------------------------------------------------------------------------
# P16: textbook high-SNR limit.  For an isolated source at SNR 100 in
# noise-free data and a flat prior, the posterior is Gaussian around the
# truth with covariance F^-1, F_ij = <d_i h|d_j h> (Fisher matrix from
# central differences of the waveform in the sampling coordinates).  The
# oracle's in-model band loop (group stretch, beta = 1) must sample it.
# --------------------------------------------------------------------------
def test_posterior_of_an_isolated_loud_source_matches_the_inverse_fisher_matrix():
    from paper_2405_04690_amd import inputs
    cfg = inputs.TINY
    orc = oracle.Oracle(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi)
    N, n_w = 128, 32
    phys = sampler_setup._phys
    f0 = 12e-3 + 0.37 / cfg.T
    u0 = np.array([-22.0, f0, 3e-16, 1.1, 0.45, 0.7, 2.3, 0.3])
    S = orc.psd_eval(np.array([cfg.sqrt_oms, cfg.sqrt_acc, cfg.sqrt_oms, cfg.sqrt_acc]))[0]

    def window(u, k_lo):
        A, E, _, sb = orc.waveform(phys(u)[None], N, with_T=False)
        out = np.zeros((2, 3 * N), complex)
        out[:, sb[0] - k_lo:sb[0] - k_lo + N] = np.stack([A[0], E[0]])
        return out

    k_lo = int(np.floor(f0 * cfg.T)) - N // 2 - N
    wgt = 1.0 / S[:, k_lo - orc.k_min:k_lo - orc.k_min + 3 * N]
    inner = lambda a, b: 4 * orc.df * np.sum((np.conj(a) * b).real * wgt)
    h = window(u0, k_lo)
    u0[0] += np.log10(100.0 / np.sqrt(inner(h, h)))  # SNR 100
    steps = np.array([1e-4, 1e-4 / cfg.T, 1e-4 / cfg.T ** 2, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4])
    D = []
    for i in range(8):
        e = np.zeros(8)
        e[i] = steps[i]
        D.append((window(u0 + e, k_lo) - window(u0 - e, k_lo)) / (2 * steps[i]))
    F = np.array([[inner(D[i], D[j]) for j in range(8)] for i in range(8)])
    C = np.linalg.inv(F)
    sig = np.sqrt(np.diag(C))
    # one band centred on the source, one slot per walker, a prior box far wider than the posterior
    sc = oracle.SweepConfig()
    sc.n_temps, sc.n_walkers, sc.n_bands, sc.n_slots = 1, n_w, 1, 1
    sc.N, sc.n_prop, sc.n_friends, sc.group_every = N, 10, n_w, 1
    sc.k_band0, sc.stretch_a, sc.seed = k_lo + N, 2.0, 5
    lo = (-24.0, 0.0, -1e-13, 0.0, -1.0, 0.0, 0.0, -1.0)
    hi = (-19.0, 0.0, 1e-13, 0.0, 1.0, 0.0, 0.0, 1.0)
    for i in range(8):
        sc.prior_lo[i], sc.prior_hi[i] = lo[i], hi[i]
    st = oracle.SweepState(sc, orc.n_bins)
    data = np.zeros((2, orc.n_bins), complex)
    orc.scatter_add(phys(u0)[None], N, 1.0, data)
    rng = np.random.default_rng(6)
    chol = np.linalg.cholesky(C / np.outer(sig, sig))
    st.u[0, :, 0, 0] = u0 + sig * (rng.standard_normal((n_w, 8)) @ chol.T)  # start in the Gaussian
    st.exists[:] = 1
    for w in range(n_w):
        st.inv_psd[w] = 1.0 / S
        st.resid[1, w] = data
        st.resid[0, w] = data
        orc.scatter_add(phys(st.u[0, w, 0, 0])[None], N, -1.0, st.resid[0, w])
    samples = []
    for it in range(100):
        oracle.sweep_group(sc, st)
        oracle.sweep_step(orc, sc, st, oracle.MOVE_INMODEL, 0, it)
        if it >= 20:
            samples.append(st.u[0, :, 0, 0].copy())
    assert 0.2 < st.stats[1] / st.stats[0] < 0.8
    d = np.array(samples).reshape(-1, 8) - u0
    ratio = (d ** 2).mean(axis=0) / np.diag(C)
    assert np.all((ratio > 0.8) & (ratio < 1.25)), ratio
    # E[(u - u0)^T F (u - u0)] = 8 for the Gaussian limit
    m = np.einsum("ni,ij,nj->n", d, F, d).mean()
    assert abs(m - 8.0) < 1.0, m


def test_parallel_sweep_schedule_is_bitwise_the_sequential_one():
    """The oracle runs the units of a step (band loops, tempering chains) on
    several threads and adds their cold-chain changes in the sequential
    order: one thread and eight give bitwise identical states."""
    lib = oracle._load()
    before = lib.gblo_set_threads(0)
    runs = []
    try:
        for n in (1, 8):
            cfg, orc, sc, st = sampler_setup.problem(n_t=4, n_w=6, n_b=5, n_slots=8, n_prop=5, seed=123)
            lib.gblo_set_threads(n)
            oracle.sweep_group(sc, st)
            cl = np.zeros((sc.n_walkers, sc.n_bands))
            for mv in (0, 1, 2):
                for par in (1, 0):
                    oracle.sweep_step(orc, sc, st, mv, par, 3, cold_logl=cl if mv == 2 else None)
            runs.append((st.u.copy(), st.exists.copy(), st.resid.copy(), st.stats.copy(), cl))
    finally:
        lib.gblo_set_threads(before)
    for a, b in zip(*runs):
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
    assert runs[0][3][1] > 0 and runs[0][3][3] + runs[0][3][5] > 0 and runs[0][3][7] > 0


# --------------------------------------------------------------------------
# temperature-ladder adaptation and sub-band ownership
# --------------------------------------------------------------------------
def _ladder_config(nt, nw, nb, lag=1e9, time_scale=2.0):
    sc = oracle.SweepConfig()
    sc.n_temps, sc.n_walkers, sc.n_bands, sc.n_slots = nt, nw, nb, 1
    sc.adapt_ladder, sc.adapt_lag, sc.adapt_time = 1, lag, time_scale
    return sc


def test_ladder_adaptation_converges_to_the_equal_acceptance_ladder():
    """Swap acceptance that depends only on the ratio of neighbouring
    temperatures, A = (T_j / T_(j+1))^c: equal acceptance on every pair
    (the adaptation's fixed point) is the geometric ladder between the fixed
    end rungs, T_j = T_max^(j / (n_t - 1)).  Starting from a badly spaced
    ladder, the adapted ladder reaches it; the end rungs never move and the
    ladder stays ordered."""
    nt, nw, nb = 8, 1 << 20, 3
    sc = _ladder_config(nt, nw, nb)
    st = oracle.SweepState(sc, 1)
    T_max = 50.0
    start = [np.r_[1.0, np.linspace(1.01, 1.3, nt - 2), T_max],           # crowded at the bottom
             np.r_[1.0, np.linspace(20.0, 45.0, nt - 2), T_max],          # crowded at the top
             np.r_[1.0, np.geomspace(1.5, 40.0, nt - 2), T_max]]
    st.betas[:] = 1.0 / np.array(start)
    c = 1.5
    for sweep in range(4000):
        T = 1.0 / st.betas
        A = (T[:, :-1] / T[:, 1:]) ** c                    # pair (t-1, t) at entry t
        st.swap_acc[:, 1:] = np.rint(A * nw).astype(np.int32)
        st.swap_acc[:, 0] = 0
        oracle.adapt_ladder(sc, st, sweep)
        assert np.all(st.swap_acc == 0)
        assert np.all(st.betas[:, 0] == 1.0) and np.all(st.betas[:, -1] == 1.0 / T_max)
        assert np.all(np.diff(st.betas, axis=1) < 0)
    target = T_max ** (np.arange(nt) / (nt - 1))
    assert np.max(np.abs(1.0 / st.betas / target - 1)) < 1e-3


def test_ladder_adaptation_leaves_an_equal_acceptance_ladder_and_decays():
    """equal acceptance on every pair: nothing moves; the step size decays as
    t0 / (t + t0): after a sweep index far beyond t0 an unequal acceptance
    barely moves the ladder, while at t = 0 it moves it visibly"""
    nt, nw = 6, 100
    sc = _ladder_config(nt, nw, 1, lag=10.0, time_scale=1.0)
    st = oracle.SweepState(sc, 1)
    ladder = np.r_[1.0 / np.geomspace(1.0, 30.0, nt - 1), 0.0]   # hottest rung at beta = 0
    st.betas[0] = ladder
    st.swap_acc[0, 1:] = 37
    oracle.adapt_ladder(sc, st, 0)
    assert np.allclose(st.betas[0], ladder, rtol=1e-14, atol=0)
    moved = []
    for sweep in (0, 10 ** 9):
        st.betas[0] = ladder
        st.swap_acc[0, 1:] = [90, 10, 10, 10, 10]
        oracle.adapt_ladder(sc, st, sweep)
        moved.append(np.max(np.abs(st.betas[0, :-1] / ladder[:-1] - 1)))
        assert st.betas[0, -1] == 0.0
    assert moved[0] > 0.3 and moved[1] < 1e-7


@pytest.mark.parametrize("W", [None, 200])
def test_ownership_shift_moves_cold_sources_and_keeps_the_buffers(W):
    """cold-chain sources pushed past their band edge move to the
    neighbouring band's lowest free slot; the multiset of cold sources is
    unchanged, hot chains are untouched, moved sources sit in their new
    band's nominal range, and both parity buffers equal a rebuild from the
    data minus every cold source of that parity"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=3, n_b=5, n_slots=4, seed=131, W=W)
    T, kb = cfg.T, sc.k_band0
    N = sc.band_width or sc.N   # the sub-band width
    rng = np.random.default_rng(132)
    # move some cold sources across an edge: up to 0.45 band into the neighbour
    pushed = []
    for w in range(sc.n_walkers):
        for b in range(sc.n_bands):
            for s in range(2):
                if rng.uniform() < 0.5:
                    side = rng.choice([-1, 1])
                    f = (kb + (b + (1.0 + rng.uniform(0.02, 0.45) if side > 0 else -rng.uniform(0.02, 0.45))) * N) / T
                    st.u[0, w, b, s, 1] = f
                    pushed.append((w, b, s, side))
    # fill the top band's slots of walker 0 so that a push into it finds no room
    st.exists[0, 0, 4, :] = 1
    st.u[0, 0, 4, 2:] = st.u[0, 0, 4, 0]
    st.u[0, 0, 4, 2:, 1] = (kb + 4.5 * N) / T
    for par in (0, 1):
        for w in range(sc.n_walkers):
            st.resid[par, w] = sampler_setup.rebuild_buffer(orc, sc, st, par, w)
    before = {w: sorted(map(tuple, st.u[0, w][st.exists[0, w].astype(bool)])) for w in range(sc.n_walkers)}
    hot_u, hot_e = st.u[1].copy(), st.exists[1].copy()
    stats = np.zeros(2, np.int64)
    oracle.shift_ownership(orc, sc, st, stats)
    assert stats[0] > 0
    for w in range(sc.n_walkers):
        after = sorted(map(tuple, st.u[0, w][st.exists[0, w].astype(bool)]))
        assert after == before[w]
        for b in range(sc.n_bands):
            for s in range(sc.n_slots):
                if not st.exists[0, w, b, s]:
                    continue
                kk = st.u[0, w, b, s, 1] * T - kb
                inside = b * N <= kk < (b + 1) * N
                edge = (kk < 0 and b == 0) or (kk >= sc.n_bands * N and b == sc.n_bands - 1)
                full = not np.any(st.exists[0, w, b + (1 if kk >= (b + 1) * N else -1)] == 0) if not (inside or edge) else False
                assert inside or edge or full, (w, b, s, kk / N)
    assert np.array_equal(st.u[1], hot_u) and np.array_equal(st.exists[1], hot_e)
    for par in (0, 1):
        for w in range(sc.n_walkers):
            ref = sampler_setup.rebuild_buffer(orc, sc, st, par, w)
            assert np.max(np.abs(st.resid[par, w] - ref)) <= 1e-12 * np.abs(ref).max()
    assert stats[1] >= 1   # the push into walker 0's full top band stayed

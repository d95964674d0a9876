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

"""ESS accounting: the oracle's plain autocorrelation against the AR(1)
closed form tau = (1 + rho) / (1 - rho) and iid samples (tau = 1); the
package's FFT estimator equal to the oracle's on the same traces."""
import numpy as np
import pytest

from oracle import ess as oess
from paper_2405_04690_amd import ess


def _ar1(seed, rho, nw, n):
    rng = np.random.default_rng(seed)
    x = np.zeros((nw, n))
    x[:, 0] = rng.standard_normal(nw) / np.sqrt(1 - rho * rho)
    e = rng.standard_normal((nw, n))
    for i in range(1, n):
        x[:, i] = rho * x[:, i - 1] + e[:, i]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_oracle_tau_matches_ar1_closed_form(rho):
    x = _ar1(1, rho, 16, 3000)
    tau = oess.tau_int(x)
    ref = (1 + rho) / (1 - rho)
    assert abs(tau - ref) <= 0.12 * ref, (tau, ref)


def test_fft_estimator_equals_the_plain_one():
    for seed, rho in ((2, 0.7), (3, 0.95)):
        x = _ar1(seed, rho, 8, 700)
        assert np.allclose(ess.autocorr(x), oess.autocorr(x), rtol=0, atol=1e-12)
        assert abs(ess.tau_int(x) - oess.tau_int(x)) <= 1e-9 * oess.tau_int(x)
        assert abs(ess.ess(x) - oess.ess(x)) <= 1e-9 * oess.ess(x)


def test_frozen_and_partly_frozen_traces():
    x = np.ones((4, 100))
    assert oess.tau_int(x) == 100 and ess.tau_int(x) == 100 and ess.ess(x) == 4
    y = _ar1(4, 0.5, 4, 400)
    y[0] = 3.0
    assert abs(ess.tau_int(y) - oess.tau_int(y)) <= 1e-9 * oess.tau_int(y)

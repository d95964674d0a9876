"""Pins of the oracle's correlated-channel noise matrix and matrix-weighted
likelihoods (Sec. 2: with unequal noise the A and E channels correlate and the
likelihood needs the noise matrix across channels): the equal-noise limit is
eq. psd with no cross term; relabelling the spacecraft rotates (A, E) as the
TDI algebra says; the likelihood is invariant under unitary channel mixing;
matched-noise statistics; the diagonal case and full-band differences agree
with the existing likelihood paths."""
import numpy as np
import pytest

import oracle
from paper_2405_04690_amd import inputs

CFG = inputs.TINY


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)


def _levels(rng, spread=0.3):
    so = CFG.sqrt_oms * (1 + spread * rng.uniform(-1, 1, 6))
    sa = CFG.sqrt_acc * (1 + spread * rng.uniform(-1, 1, 6))
    return np.concatenate([so, sa])


def _C(v):
    K = np.array([[v[0], v[2] + 1j * v[3]], [v[2] - 1j * v[3], v[1]]])
    return np.linalg.inv(K), K


LINKS = [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]


def test_equal_noise_is_eq_psd_without_cross_term(orc):
    lv = np.concatenate([np.full(6, CFG.sqrt_oms), np.full(6, CFG.sqrt_acc)])
    for f in np.geomspace(1.1e-4, 2.9e-2, 23):
        v = orc.noise_matrix_value(f, lv)
        S = orc.psd_value(f, CFG.sqrt_oms, CFG.sqrt_acc)
        assert abs(v[0] * S - 1) < 1e-12 and abs(v[1] * S - 1) < 1e-12
        assert abs(v[2]) * S < 1e-12 and abs(v[3]) * S < 1e-12
        assert abs(v[4] - 2 * np.log(S)) < 1e-10


def test_relabelling_the_spacecraft_rotates_a_and_e(orc):
    """craft i -> i+1 (mod 3) maps (X, Y, Z) -> (Z, X, Y); with the A, E rows M
    of the TDI transform, C' = U C U^T with U = M P M^T (a rotation, as the
    T direction is invariant)"""
    rng = np.random.default_rng(3)
    M = np.array([[-1, 0, 1] / np.sqrt(2), [1, -2, 1] / np.sqrt(6)])
    P = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]])       # new (X, Y, Z) = old (Z, X, Y)
    U = M @ P @ M.T
    assert np.allclose(U @ U.T, np.eye(2), atol=1e-15)
    sig = [1, 2, 0]
    for _ in range(4):
        lv = _levels(rng)
        lp = np.empty(12)
        for j, (s, r) in enumerate(LINKS):
            jn = LINKS.index((sig[s], sig[r]))
            lp[jn] = lv[j]
            lp[6 + jn] = lv[6 + j]
        for f in (3e-4, 2.2e-3, 9e-3, 2.4e-2):
            C, _ = _C(orc.noise_matrix_value(f, lv))
            Cp, _ = _C(orc.noise_matrix_value(f, lp))
            assert np.allclose(Cp, U @ C @ U.T, rtol=1e-10, atol=1e-10 * np.abs(C).max())


def test_matrix_is_hermitian_positive_and_scales(orc):
    rng = np.random.default_rng(4)
    lv = _levels(rng, 0.6)
    for f in np.geomspace(2e-4, 2.5e-2, 9):
        v = orc.noise_matrix_value(f, lv)
        C, K = _C(v)
        ev = np.linalg.eigvalsh(C)
        assert np.all(ev > 0)
        assert abs(np.log(np.linalg.det(C).real) - v[4]) < 1e-10
        assert abs(v[2]) + abs(v[3]) > 1e-6 * max(v[0], v[1])        # unequal noise: channels correlate
        v2 = orc.noise_matrix_value(f, 3.0 * lv)
        assert np.allclose(v2[:4], v[:4] / 9.0, rtol=1e-12) and abs(v2[4] - v[4] - 2 * np.log(9.0)) < 1e-10


def _cov(K):
    """C = K^-1 per bin, as (c11, c22, c12) arrays"""
    kae = K[2] + 1j * K[3]
    det = K[0] * K[1] - np.abs(kae) ** 2
    return K[1] / det, K[0] / det, -kae / det


def _noise_draw(orc, K, seed):
    """n with covariance 2 C / (4 df) per bin (complex normals with unit real
    and imaginary variances through the Cholesky factor of C / (4 df))"""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((2, orc.n_bins)) + 1j * rng.standard_normal((2, orc.n_bins))
    c11, c22, c12 = (x / (4 * orc.df) for x in _cov(K))
    l11 = np.sqrt(c11)
    l21 = np.conj(c12) / l11
    l22 = np.sqrt(c22 - np.abs(l21) ** 2)
    return np.stack([l11 * z[0], l21 * z[0] + l22 * z[1]])


def test_unitary_invariance_and_matched_noise_statistics(orc):
    rng = np.random.default_rng(5)
    K = orc.noise_matrix(_levels(rng, 0.5))[0]
    n = _noise_draw(orc, K, 6)
    ll = orc.loglike_matrix(n, K)
    # <n|n>_K = -2 (ll + sum ln det): the whitened draw has 4 unit real
    # normals per bin, so it is chi^2 with 4 n_bins degrees of freedom
    q = -2 * (ll + K[4].sum())
    dof = 4 * orc.n_bins
    assert abs(q - dof) < 5 * np.sqrt(2 * dof)
    # a unitary mixing of the channels with K -> U K U^H leaves the likelihood unchanged
    th, ph = 0.7, 1.3
    U = np.array([[np.cos(th), -np.exp(1j * ph) * np.sin(th)], [np.exp(-1j * ph) * np.sin(th), np.cos(th)]])
    n2 = U @ n
    Km = np.array([[K[0], K[2] + 1j * K[3]], [K[2] - 1j * K[3], K[1]]])      # [2][2][nb]
    Km2 = np.einsum("ij,jkn,lk->iln", U, Km, U.conj())
    Kp = np.stack([Km2[0, 0].real, Km2[1, 1].real, Km2[0, 1].real, Km2[0, 1].imag, K[4]])
    assert abs(orc.loglike_matrix(n2, Kp) / ll - 1) < 1e-12


def test_matrix_delta_loglike_reduces_and_equals_full_differences(orc):
    rng = np.random.default_rng(7)
    S = orc.psd_eval(np.array([CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc]))
    src = inputs.draw_sources(8, 12, (5e-4, 1e-2), (-19.0, -16.0))
    src[:, 0] *= 30
    R = np.sqrt(S[0] / (4 * orc.df)) * inputs.complex_normals(9, (2, orc.n_bins))
    orc.scatter_add(src, 128, 1.0, R)
    old = inputs.perturb(10, src, CFG.T, "jitter")
    new = inputs.perturb(11, old, CFG.T, "inmodel")
    # diagonal K: the existing path
    Kd = np.zeros((5, orc.n_bins))
    Kd[0], Kd[1] = 1 / S[0, 0], 1 / S[0, 1]
    Kd[4] = np.log(S[0, 0] * S[0, 1])
    got = orc.delta_loglike_matrix(R[None], Kd, old, new, 128)
    ref, terms = orc.delta_loglike(R[None], S, old, new, 128, return_terms=True)
    scale = np.maximum(1.0, np.abs(terms[:, :5]).max(axis=1))
    assert np.max(np.abs(got - ref) / scale) <= 1e-10
    # correlated K: equals the difference of two full-band likelihoods
    K = orc.noise_matrix(_levels(rng, 0.5))[0]
    got = orc.delta_loglike_matrix(R[None], K, old[:4], new[:4], 128)
    for i in range(4):
        R2 = R.copy()
        orc.scatter_add(old[i:i + 1], 128, 1.0, R2)     # swap: R' = R + r - a
        orc.scatter_add(new[i:i + 1], 128, -1.0, R2)
        full = orc.loglike_matrix(R2, K) - orc.loglike_matrix(R, K)
        assert abs(got[i] - full) <= 1e-8 * abs(full) + 1e-6   # the full-band sums cancel to ~1e-7

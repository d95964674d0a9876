"""Pins of the FP64 flow oracle (CPU): exact inverse, log-determinant against
a finite-difference Jacobian, a closed form (constant conditioner = Gaussian
with affine maps, checked with scipy), normalisation of q_u over the prior
box by Monte Carlo, the hand-written gradient against central differences,
Adam's first step, and bfloat16 rounding against torch."""
import numpy as np
import pytest
import torch
from scipy import stats

from oracle import flow

N_EMB = 5
T = 7889400.0
K0, W = 23668, 128
LO = (-23.0, 0.0, -1e-16, 0.0, -1.0, 0.0, 0.0, -1.0)
HI = (-21.0, 0.0, 1e-15, 0.0, 1.0, 0.0, 0.0, 1.0)


def _theta(seed=1, out_scale=1.0):
    th = flow.init_params(seed, N_EMB, out_scale=out_scale)
    rng = np.random.default_rng(seed + 100)
    layers, _ = flow.unpack(th, N_EMB)
    for L in layers:
        L["b1"][:] = rng.normal(0, 0.1, L["b1"].shape)
        L["b3"][:] = rng.normal(0, 0.1, L["b3"].shape)
    return th


def test_inverse_is_exact():
    th = _theta()
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1.5, (200, 8))
    band = rng.integers(0, N_EMB, 200)
    z, ld = flow.forward(th, N_EMB, x, band)
    x2, ld2 = flow.inverse(th, N_EMB, z, band)
    assert np.max(np.abs(x2 - x)) <= 1e-12 * max(1.0, np.abs(x).max())
    assert np.max(np.abs(ld - ld2)) <= 1e-12
    lo, hi = flow.box(band, T, K0, W, LO, HI)
    u, lj = flow.from_real(x, lo, hi)
    x3, lj3 = flow.to_real(u, lo, hi)
    assert np.max(np.abs(x3 - x)) <= 1e-9 and np.max(np.abs(lj - lj3)) <= 1e-9


def test_logdet_matches_finite_difference_jacobian():
    th = _theta(seed=2)
    rng = np.random.default_rng(4)
    for trial in range(5):
        x = rng.normal(0, 1, (1, 8))
        band = np.array([trial % N_EMB])
        _, ld = flow.forward(th, N_EMB, x, band)
        h = 1e-5
        J = np.zeros((8, 8))
        for j in range(8):
            xp, xm = x.copy(), x.copy()
            xp[0, j] += h
            xm[0, j] -= h
            J[:, j] = (flow.forward(th, N_EMB, xp, band)[0][0] - flow.forward(th, N_EMB, xm, band)[0][0]) / (2 * h)
        sign, logdet = np.linalg.slogdet(J)
        assert sign > 0
        assert abs(logdet - ld[0]) <= 1e-7 * max(1.0, abs(ld[0]))


def test_constant_conditioner_is_a_gaussian():
    """W3 = 0: every layer applies the same affine map y = x e^{s} + t with
    s = 2 tanh(c_s), so each coordinate (moved in 3 of 6 layers) follows a
    Gaussian whose density scipy gives directly."""
    th = _theta(seed=5)
    layers, _ = flow.unpack(th, N_EMB)
    cs = np.array([0.3, -0.2, 0.1, 0.05])
    ct = np.array([0.5, -1.0, 0.25, 2.0])
    for L in layers:
        L["W3"][:] = 0.0
        L["b3"][:4] = cs
        L["b3"][4:] = ct
    s = 2 * np.tanh(cs)
    a = np.ones(8)
    b = np.zeros(8)
    for l in range(flow.N_LAYERS):
        _, moved = flow.masks(l)
        for j, d in enumerate(moved):
            a[d], b[d] = a[d] * np.exp(s[j]), b[d] * np.exp(s[j]) + ct[j]
    rng = np.random.default_rng(6)
    x = rng.normal(0, 2, (50, 8))
    band = rng.integers(0, N_EMB, 50)
    ref = stats.norm.logpdf(x, loc=-b / a, scale=1.0 / a).sum(axis=1)
    got = flow.log_prob_x(th, N_EMB, x, band)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(ref).max()


def test_density_on_the_prior_box_is_normalised():
    """E_{u ~ uniform box}[q_u(u) V] = 1 (Monte Carlo, 5 sigma)"""
    th = _theta(seed=7, out_scale=0.5)
    rng = np.random.default_rng(8)
    n = 400_000
    band = rng.integers(0, N_EMB, n)
    lo, hi = flow.box(band, T, K0, W, LO, HI)
    u = lo + (hi - lo) * rng.uniform(size=(n, 8))
    lq = flow.log_prob_u(th, N_EMB, u, band, lo, hi)
    w = np.exp(lq + np.sum(np.log(hi - lo), axis=1))
    mean, se = w.mean(), w.std() / np.sqrt(n)
    assert abs(mean - 1.0) < 5 * se + 1e-3, (mean, se)


def test_samples_follow_the_density():
    """sample_u returns ln q_u consistent with log_prob_u at the samples"""
    th = _theta(seed=9)
    rng = np.random.default_rng(10)
    z = rng.standard_normal((300, 8))
    band = rng.integers(0, N_EMB, 300)
    lo, hi = flow.box(band, T, K0, W, LO, HI)
    u, lq = flow.sample_u(th, N_EMB, z, band, lo, hi)
    assert np.all((u > lo) & (u < hi))
    lq2 = flow.log_prob_u(th, N_EMB, u, band, lo, hi)
    ok = np.all((lo < u) & (u < hi), axis=1)
    assert np.max(np.abs(lq[ok] - lq2[ok])) <= 1e-8 * np.abs(lq).max()


def test_gradient_matches_central_differences():
    th = _theta(seed=11)
    rng = np.random.default_rng(12)
    x = rng.normal(0, 1, (16, 8))
    band = rng.integers(0, N_EMB, 16)
    loss, g = flow.nll_grad(th, N_EMB, x, band)
    assert np.isclose(loss, -np.mean(flow.log_prob_x(th, N_EMB, x, band)), rtol=1e-13)
    layers_off = flow.LAYER_SIZE
    # a sample of indices from every block: each layer's W1, b1, W2, b2, W3, b3, and the embedding
    idx = []
    for l in range(flow.N_LAYERS):
        base = l * layers_off
        sizes = [128 * 20, 128, 128 * 128, 128, 8 * 128, 8]
        o = base
        for n in sizes:
            idx += list(o + rng.integers(0, n, 3))
            o += n
    idx += list(flow.N_LAYERS * layers_off + rng.integers(0, N_EMB * flow.EMB, 10))
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (flow.nll_grad(tp, N_EMB, x, band)[0] - flow.nll_grad(tm, N_EMB, x, band)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_adam_first_step_moves_by_lr_against_the_gradient_sign():
    rng = np.random.default_rng(13)
    th = rng.normal(size=1000)
    g = rng.normal(size=1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    th1, m1, v1 = flow.adam(th, g, m, v, 1, lr=1e-3)
    assert np.all(np.abs((th - th1) - 1e-3 * np.sign(g)) <= 1e-3 * 1e-8 / np.abs(g) + 1e-15)


def test_training_reduces_the_loss_towards_the_entropy():
    """fit a correlated Gaussian in x: the loss falls from the identity-flow
    value towards the target's entropy"""
    th = flow.init_params(14, 1, out_scale=0.0)
    rng = np.random.default_rng(15)
    A = np.eye(8) + 0.4 * rng.normal(size=(8, 8)) / np.sqrt(8)
    mu = rng.normal(0, 0.5, 8)
    cov = A @ A.T
    entropy = 0.5 * np.linalg.slogdet(2 * np.pi * np.e * cov)[1]
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    losses = []
    for step in range(1, 151):
        x = mu + rng.standard_normal((512, 8)) @ A.T
        loss, g = flow.nll_grad(th, 1, x, np.zeros(512, int))
        th, m, v = flow.adam(th, g, m, v, step, lr=3e-3)
        losses.append(loss)
    start = np.mean(losses[:5])
    end = np.mean(losses[-10:])
    assert end < start - 0.5 * (start - entropy), (start, end, entropy)
    assert end > entropy - 0.2


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(16)
    a = np.concatenate([rng.normal(0, 1, 10000) * 10.0 ** rng.uniform(-5, 5, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.0 - 2 ** -7]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(flow.bf16_round(a), ref)

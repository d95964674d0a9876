"""GPU flow (BF16 MFMA) against the FP64 flow oracle.

Tolerances: densities within twice the first-order BF16 error bound of
tests/flow_bounds.py (computed per sample from the oracle's activations and
adjoints); the density a sample is returned with equals the
GPU density at that sample to FP64 rounding (what exact Metropolis-Hastings
needs); gradients within 3% norm-wise per parameter block (each weight
gradient sums products of two BF16-rounded factors whose upstream chain
passes through at most three more BF16 roundings: 5 u ~ 2%, plus FP32);
Adam to FP32 rounding."""
import numpy as np
import pytest
import torch

import flow_bounds
from oracle import flow as oflow
from paper_2405_04690_amd import inputs
from paper_2405_04690_amd.flow import Flow, flow_config
from paper_2405_04690_amd.gbl import Context

pytestmark = pytest.mark.gpu

CFG = inputs.TINY
N_EMB, WIDTH, K0 = 7, 128, 23668
LO = (-23.0, 0.0, -1e-16, 0.0, -1.0, 0.0, 0.0, -1.0)
HI = (-21.0, 0.0, 1e-15, 0.0, 1.0, 0.0, 0.0, 1.0)


def _master(seed=1, out_scale=1.0):
    th = oflow.init_params(seed, N_EMB, out_scale=out_scale)
    rng = np.random.default_rng(seed + 50)
    layers, _ = oflow.unpack(th, N_EMB)
    for L in layers:
        L["b1"][:] = rng.normal(0, 0.1, L["b1"].shape)
        L["b2"][:] = rng.normal(0, 0.1, L["b2"].shape)
        L["b3"][:] = rng.normal(0, 0.1, L["b3"].shape)
    return th.astype(np.float32)


def _setup(seed=1, out_scale=1.0):
    ctx = Context(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)
    fc = flow_config(N_EMB, WIDTH, K0, LO, HI)
    m = _master(seed, out_scale)
    fl = Flow(ctx, fc, m)
    return ctx, fl, m, flow_bounds.oracle_theta(m, N_EMB)


def _points(seed, B):
    rng = np.random.default_rng(seed)
    band = rng.integers(0, N_EMB, B).astype(np.int32)
    lo, hi = oflow.box(band, CFG.T, K0, WIDTH, LO, HI)
    u = lo + (hi - lo) * rng.uniform(0.002, 0.998, (B, 8))
    return u, band, lo, hi


def _dev(a, dt=None):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda() if dt is None else torch.from_numpy(
        np.ascontiguousarray(a)).to(dt).cuda()


@pytest.mark.parametrize("B", [1, 15, 16, 1000, 4133])
def test_log_prob_matches_oracle_within_bf16_bound(B):
    ctx, fl, m, th = _setup()
    u, band, lo, hi = _points(B, B)
    got = fl.log_prob(_dev(u), _dev(band)).cpu().numpy()
    x, lj = oflow.to_real(u, lo, hi)
    _, lnq, e = flow_bounds.forward_bound(th, N_EMB, x, band)
    ref = lnq + lj
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= 2 * e + 1e-9), np.max(np.abs(got - ref) / (2 * e + 1e-9))
    ctx.close()


def test_sample_density_is_exact_and_matches_oracle():
    ctx, fl, m, th = _setup(seed=3)
    B = 3000
    rng = np.random.default_rng(4)
    z = rng.standard_normal((B, 8))
    band = rng.integers(0, N_EMB, B).astype(np.int32)
    ug, lq = fl.sample(_dev(z), _dev(band))
    lq2 = fl.log_prob(ug, _dev(band)).cpu().numpy()
    ug = ug.cpu().numpy()
    lq = lq.cpu().numpy()
    lo, hi = oflow.box(band, CFG.T, K0, WIDTH, LO, HI)
    inside = np.all((ug > lo) & (ug < hi), axis=1)
    assert inside.mean() > 0.99
    # the density returned with a sample = the density evaluated at it (FP64 rounding)
    assert np.max(np.abs(lq[inside] - lq2[inside]) / np.maximum(1.0, np.abs(lq[inside]))) <= 1e-9
    # oracle at the GPU's samples: latent point and density within the bound
    x, lj = oflow.to_real(ug[inside], lo[inside], hi[inside])
    _, lnq, e = flow_bounds.forward_bound(th, N_EMB, x, band[inside])
    assert np.all(np.abs(lnq + lj - lq[inside]) <= 2 * e + 1e-9)
    ctx.close()


def test_out_of_box_points_and_bad_bands_give_nan():
    ctx, fl, m, th = _setup()
    u, band, lo, hi = _points(5, 4)
    u[0, 1] = hi[0, 1]          # on the upper f0 edge: outside the open box
    u[1, 4] = -1.0              # on the cos iota edge
    band[2] = N_EMB             # no such band
    got = fl.log_prob(_dev(u), _dev(band)).cpu().numpy()
    assert np.isnan(got[:3]).all() and np.isfinite(got[3])
    ctx.close()


def test_gradient_matches_oracle():
    ctx, fl, m, th = _setup(seed=6, out_scale=0.5)
    B = 4096 + 77
    u, band, lo, hi = _points(7, B)
    loss = fl.compute_grad(_dev(u), _dev(band)).item()
    g = fl.grad.cpu().numpy().astype(np.float64)
    x, _ = oflow.to_real(u, lo, hi)
    lo_, go = oflow.nll_grad(th, N_EMB, x, band)
    _, _, e = flow_bounds.forward_bound(th, N_EMB, x, band)
    assert abs(loss - lo_) <= 2 * e.mean() + 1e-9
    gl, ge = oflow.unpack(g, N_EMB)
    ol, oe = oflow.unpack(go, N_EMB)
    for l in range(oflow.N_LAYERS):
        for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
            a, b = gl[l][k], ol[l][k]
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert rel <= 0.03, (l, k, rel)
    assert np.linalg.norm(ge - oe) / np.linalg.norm(oe) <= 0.03
    ctx.close()


def test_adam_matches_oracle():
    ctx, fl, m, th = _setup(seed=8)
    u, band, lo, hi = _points(9, 512)
    fl.compute_grad(_dev(u), _dev(band))
    g = fl.grad.cpu().numpy().astype(np.float64)
    p0 = fl.params.cpu().numpy().astype(np.float64)
    mom = np.zeros_like(p0)
    vel = np.zeros_like(p0)
    p_ref = p0
    for step in (1, 2, 3):
        fl.adam(lr=1e-3)
        p_ref, mom, vel = oflow.adam(p_ref, g, mom, vel, step, lr=1e-3)
    got = fl.params.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - p_ref)) <= 1e-6 * max(1.0, np.abs(p0).max())
    ctx.close()


def test_training_follows_the_oracle():
    """150 Adam steps on samples of a band-dependent correlated Gaussian (in
    the flow's real coordinates): the GPU loss falls like the oracle's."""
    ctx = Context(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)
    fc = flow_config(N_EMB, WIDTH, K0, LO, HI)
    m = oflow.init_params(10, N_EMB, out_scale=0.0).astype(np.float32)
    fl = Flow(ctx, fc, m)
    th = m.astype(np.float64)
    mo, vo = np.zeros_like(th), np.zeros_like(th)
    rng = np.random.default_rng(11)
    A = np.eye(8) + 0.4 * rng.normal(size=(8, 8)) / np.sqrt(8)
    gpu_l, orc_l = [], []
    for step in range(1, 151):
        band = rng.integers(0, N_EMB, 1024).astype(np.int32)
        x = 0.3 * band[:, None] + rng.standard_normal((1024, 8)) @ A.T
        lo, hi = oflow.box(band, CFG.T, K0, WIDTH, LO, HI)
        u, _ = oflow.from_real(x, lo, hi)
        gpu_l.append(fl.train_step(_dev(u), _dev(band), lr=3e-3).item())
        lo_, g = oflow.nll_grad(flow_bounds.oracle_theta(th.astype(np.float32), N_EMB), N_EMB, x, band)
        th, mo, vo = oflow.adam(th, g, mo, vo, step, lr=3e-3)
        th = th.astype(np.float32).astype(np.float64)
        orc_l.append(lo_)
    g0, g1 = np.mean(gpu_l[:5]), np.mean(gpu_l[-10:])
    o0, o1 = np.mean(orc_l[:5]), np.mean(orc_l[-10:])
    assert g1 < g0 - 0.5 * (o0 - o1)
    assert abs(g1 - o1) <= 0.1 * (o0 - o1)
    ctx.close()


def test_large_batch_sampled_against_oracle():
    ctx, fl, m, th = _setup(seed=12)
    B = 300_000
    u, band, lo, hi = _points(13, B)
    got = fl.log_prob(_dev(u), _dev(band)).cpu().numpy()
    idx = np.random.default_rng(14).choice(B, 2000, replace=False)
    idx = np.concatenate([idx, [0, B - 1]])
    x, lj = oflow.to_real(u[idx], lo[idx], hi[idx])
    _, lnq, e = flow_bounds.forward_bound(th, N_EMB, x, band[idx])
    assert np.all(np.abs(got[idx] - (lnq + lj)) <= 2 * e + 1e-9)
    assert np.all(np.isfinite(got))
    ctx.close()

"""GPU parity of the template overlaps (gb_overlap) and of the cataloging
operation (Sec. 4) against the oracle: overlaps to 1e-9 of the terms' scale,
the catalog's groups and confidences exactly."""
import numpy as np
import pytest
import torch

import oracle
from oracle.catalog import catalog as oracle_catalog
from paper_2405_04690_amd import inputs
from paper_2405_04690_amd.catalog import catalog
from paper_2405_04690_amd.gbl import Context

pytestmark = pytest.mark.gpu

CFG = inputs.TINY


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda", 0))


@pytest.fixture(scope="module")
def tiny():
    ctx = Context(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)
    orc = oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)
    S = orc.psd_eval(np.array([[CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc],
                               [1.3 * CFG.sqrt_oms, 0.8 * CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc]]))
    yield ctx, orc, S
    ctx.close()


@pytest.mark.parametrize("N", [128, 256, 1024])
def test_overlap_matches_oracle(tiny, N):
    ctx, orc, S = tiny
    a = inputs.draw_sources(700 + N, 40, (2e-4, 2e-2), (-19.0, -15.0))
    b = inputs.perturb(701, a, CFG.T, "inmodel")
    b[::3, 1] += 17.0 / CFG.T                  # partial window overlap
    b[1::7, 1] += 3.0 * N / CFG.T              # disjoint windows
    edge = a[:4].copy()
    edge[0, 1] = (orc.k_min + 3.5) / CFG.T     # straddling the band edge
    edge[1, 0] = 0.0                           # zero amplitude: NaN overlap
    edge[2, 3] = np.nan                        # undefined
    edge[3, 1] = (orc.k_min + orc.n_bins + 20.5) / CFG.T
    A = np.vstack([a, edge])
    Bp = np.vstack([b, a[:4]])
    pi = (np.arange(len(A)) % 2).astype(np.int32)
    print(f"gb_overlap N={N} B={len(A)}", flush=True)
    got = ctx.gb_overlap(_t(A), _t(Bp), N, _t(S), _t(pi)).cpu().numpy()
    ref = orc.overlap(A, Bp, N, S, pi)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    rows = fin[:, 0] & fin[:, 1]
    scale = np.maximum(np.abs(ref[rows, :2]).max(axis=1, keepdims=True), 1e-300)
    assert np.max(np.abs(got[rows, :3] - ref[rows, :3]) / scale) <= 1e-9
    ok = fin[:, 3]
    assert np.max(np.abs(got[ok, 3] - ref[ok, 3])) <= 1e-9
    assert np.all(got[1:len(a):7, 2] == 0.0)                        # disjoint windows: exactly 0
    assert np.isnan(got[len(a) + 1, 3]) and np.all(np.isnan(got[len(a) + 2]))
    inv = ctx.gb_overlap(_t(A), _t(Bp), N, _t(1.0 / S), _t(pi), psd_inverse=True).cpu().numpy()
    assert np.max(np.abs(inv[ok, 3] - ref[ok, 3])) <= 1e-9


def _samples(orc, S, seed, n_src=12, M=8):
    """M chain samples of a small catalog: loud sources present in every
    sample, others in some; jittered per sample"""
    rng = np.random.default_rng(seed)
    base = inputs.draw_sources(seed, n_src, (1e-3, 1.2e-2), (-19.0, -16.0))
    base[:, 1] = (np.sort(rng.choice(np.arange(30, 2500), n_src, replace=False)) * 80 + 0.4) / CFG.T
    opt, _ = orc.snr(base, 128, S[:1])
    snr = rng.choice([5.0, 9.0, 15.0, 40.0], n_src)
    base[:, 0] *= snr / opt
    presence = rng.uniform(0.3, 1.0, n_src)
    presence[::3] = 1.0
    samples = []
    for m in range(M):
        rows = []
        for k in range(n_src):
            if rng.uniform() < presence[k]:
                p = base[k].copy()
                p[1] += rng.normal(0, 0.02) / CFG.T
                p[0] *= 1 + rng.normal(0, 0.02)
                p[3] += rng.normal(0, 0.02)
                rows.append(p)
        samples.append(np.array(rows)[rng.permutation(len(rows))])
    return samples


def test_catalog_matches_oracle(tiny):
    ctx, orc, S = tiny
    samples = _samples(orc, S, 710)
    print(f"catalog: {sum(len(s) for s in samples)} templates in {len(samples)} samples", flush=True)
    st = {}
    g_gpu, c_gpu = catalog(ctx, samples, 128, _t(S[:1]), stats=st)
    g_ref, c_ref = oracle_catalog(orc, samples, 128, S[:1])
    assert g_gpu == g_ref
    assert c_gpu == c_ref
    assert len(g_ref) >= 5 and st["overlaps"] > 0
    assert any(c < 1.0 for c in c_ref) and any(c == 1.0 for c in c_ref)

"""Pins of the oracle's template overlap and of the cataloging operation
(Sec. 4 "Cataloging Operation") against closed forms, invariants, an
independent inner-product path, and constructed samples with known groups."""
import numpy as np
import pytest

import oracle
from oracle.catalog import catalog
from paper_2405_04690_amd import inputs

CFG = inputs.TINY
N = 128


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)


@pytest.fixture(scope="module")
def psd(orc):
    return orc.psd_eval(np.array([CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc]))


def _src(seed, n, f=(2e-3, 8e-3)):
    return inputs.draw_sources(seed, n, f, (-18.0, -16.0))


def test_overlap_closed_forms(orc, psd):
    """self-overlap 1; phi0 + pi (the waveform's sign flip) gives -1; the
    amplitude drops out; symmetric; Cauchy-Schwarz; disjoint windows give 0"""
    a = _src(1, 12)
    out = orc.overlap(a, a, N, psd)
    assert np.allclose(out[:, 3], 1.0, rtol=0, atol=1e-13)
    assert np.allclose(out[:, 0], out[:, 1], rtol=1e-15)
    flip = a.copy()
    flip[:, 3] += np.pi
    assert np.allclose(orc.overlap(a, flip, N, psd)[:, 3], -1.0, rtol=0, atol=1e-12)
    louder = a.copy()
    louder[:, 0] *= 7.5
    o2 = orc.overlap(a, louder, N, psd)
    assert np.allclose(o2[:, 3], 1.0, rtol=0, atol=1e-13)
    assert np.allclose(o2[:, 1], 7.5 ** 2 * out[:, 0], rtol=1e-13)
    b = inputs.perturb(2, a, CFG.T, "inmodel")
    ab, ba = orc.overlap(a, b, N, psd), orc.overlap(b, a, N, psd)
    assert np.allclose(ab[:, 2], ba[:, 2], rtol=1e-12) and np.allclose(ab[:, 3], ba[:, 3], rtol=1e-12)
    assert np.all(np.abs(ab[:, 3]) <= 1.0 + 1e-12) and np.all(ab[:, 3] < 1.0)
    far = a.copy()
    far[:, 1] += 3 * N / CFG.T
    assert np.all(orc.overlap(a, far, N, psd)[:, 2] == 0.0)


def test_overlap_equals_the_stored_slice_inner_product(orc, psd):
    """<a|b> from the overlap equals <R|a> of the stored-slice inner product
    with R = b scattered into an empty residual (a separate code path:
    waveform slices, scatter, inner product over slices)"""
    a = _src(3, 10)
    b = inputs.perturb(4, a, CFG.T, "inmodel")
    b[:, 1] += 3.0 / CFG.T          # shift the windows against each other by 3 bins
    out = orc.overlap(a, b, N, psd)
    A, E, _, sb = orc.waveform(a, N, with_T=False)
    for i in range(len(a)):
        R = np.zeros((1, 2, orc.n_bins), np.complex128)
        orc.scatter_add(b[i:i + 1], N, 1.0, R)
        got = orc.inner(A[i:i + 1], E[i:i + 1], sb[i:i + 1], R, psd[:1])
        assert abs(got[0, 1] - out[i, 2]) <= 1e-12 * out[i, 0]
        assert abs(got[0, 0] - out[i, 0]) <= 1e-12 * out[i, 0]


def _loud(p, orc, psd, snr):
    """rescale amplitudes to the given optimal SNRs"""
    p = p.copy()
    opt, _ = orc.snr(p, N, psd)
    p[:, 0] *= snr / opt
    return p


def test_catalog_recovers_constructed_groups(orc, psd):
    """six samples: three loud sources in every sample (jittered per sample),
    one loud source in four of them, one below the SNR cut everywhere, one
    spurious source in a single sample, and in sample 0 a near-duplicate of a
    loud source (two templates fitting one source: merged by the final step)"""
    rng = np.random.default_rng(5)
    base = _src(6, 6, (2e-3, 6e-3))
    base[:, 1] = (np.array([20000, 26000, 33000, 41000, 47000, 54000]) + 0.3) / CFG.T
    base = _loud(base, orc, psd, np.array([40.0, 30.0, 25.0, 20.0, 4.0, 15.0]))
    M = 6
    samples = []
    for m in range(M):
        s = []
        for k in range(5):
            if k == 3 and m in (1, 4):
                continue                                   # source 3: absent from two samples
            p = base[k].copy()
            p[1] += rng.normal(0, 0.01) / CFG.T
            p[0] *= 1 + rng.normal(0, 0.01)
            s.append(p)
        if m == 2:
            s.append(base[5])                              # spurious, one sample
        if m == 0:
            d = base[0].copy()
            d[1] += 0.02 / CFG.T
            s.append(d)                                    # duplicate of source 0
        samples.append(np.array(s)[rng.permutation(len(s))])
    groups, conf = catalog(orc, samples, N, psd)
    # identify groups by their mean carrier frequency
    f = [np.mean([samples[m][i][1] for m, i in g]) * CFG.T for g in groups]
    order = np.argsort(f)
    got = [(round(f[j]), len(groups[j]), conf[j]) for j in order]
    exp = [(20000, 7, 1.0), (26000, 6, 1.0), (33000, 6, 1.0), (41000, 4, 4 / 6), (54000, 1, 1 / 6)]
    assert [(a, b) for a, b, _ in got] == [(a, b) for a, b, _ in exp]
    assert np.allclose([c for _, _, c in got], [c for _, _, c in exp])
    # every group holds templates of one carrier cell only
    for g in groups:
        q = {int(samples[m][i][1] * CFG.T) for m, i in g}
        assert max(q) - min(q) <= 1


def test_catalog_threshold_is_strict(orc, psd):
    """two samples whose single templates overlap just below / above the
    threshold end in two groups / one group"""
    p = _loud(_src(8, 1, (3e-3, 3e-3)), orc, psd, np.array([30.0]))
    q = p.copy()
    # find a phase offset giving an overlap of about 0.9
    dphi = np.arccos(0.9)
    for delta, n_groups in ((dphi + 0.02, 2), (dphi - 0.02, 1)):
        q2 = q.copy()
        q2[0, 3] += delta
        ov = orc.overlap(p, q2, N, psd)[0, 3]
        assert (ov > 0.9) == (n_groups == 1)
        groups, conf = catalog(orc, [p, q2], N, psd)
        assert len(groups) == n_groups
        assert sum(len(g) for g in groups) == 2

"""GPU noise-PSD step against the oracle's, on the same Philox streams: accept
decisions and counters exact, parameters and log-likelihoods to rounding."""
import numpy as np
import pytest
import torch

import oracle
from paper_2405_04690_amd import inputs
from paper_2405_04690_amd.gbl import Context
from paper_2405_04690_amd.sampler import PsdSweep, Sweep, make_config, psd_config

pytestmark = pytest.mark.gpu

CFG = inputs.TINY
LO = (10e-12, 2e-15, 10e-12, 2e-15)
HI = (20e-12, 4e-15, 20e-12, 4e-15)


# (3, 6): sets in launch order; (8, 6) and the benchmark's 36 x 32: the
# temperature count is a multiple of four, so the likelihood launches hand
# each block four temperatures of one walker (sets taken walker-major)
@pytest.mark.parametrize("nt,nw", [(3, 6), (8, 6), (36, 32)])
def test_psd_step_matches_oracle(nt, nw):
    print(f"psd step parity nt={nt} nw={nw}", flush=True)
    orc = oracle.Oracle(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)
    S = orc.psd_eval(np.array([CFG.sqrt_oms, CFG.sqrt_acc, CFG.sqrt_oms, CFG.sqrt_acc]))[0]
    amp = np.sqrt(S / (4 * orc.df))
    data = amp * inputs.complex_normals(801, (2, orc.n_bins))
    x = amp * inputs.complex_normals(802, (nw, 2, orc.n_bins))
    y = 0.3 * amp * inputs.complex_normals(803, (nw, 2, orc.n_bins))
    resid = np.stack([data[None] + x, data[None] - x + y])       # full residual = data + y
    rng = np.random.default_rng(804)
    theta = np.array(LO) + (np.array(HI) - np.array(LO)) * rng.uniform(size=(nt, nw, 4))
    betas = np.array([1.0, 0.5, 0.2]) if nt == 3 else np.geomspace(1.0, 0.05, nt)
    pco = oracle.PsdSweepConfig()
    pco.n_tn, pco.n_walkers, pco.n_par, pco.stretch_a, pco.seed = nt, nw, 4, 2.0, 805
    for k in range(4):
        pco.prior_lo[k], pco.prior_hi[k] = LO[k], HI[k]

    ctx = Context(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi)
    sc = make_config(1, nw, 2, 1, 128, int(3e-3 * CFG.T))
    sw = Sweep(ctx, sc)
    sw.resid.copy_(torch.from_numpy(resid))
    ps = PsdSweep(sw, psd_config(nt, nw, LO, HI, seed=805), torch.from_numpy(data).cuda())
    ps.theta.copy_(torch.from_numpy(theta))
    ps.betas.copy_(torch.from_numpy(betas))
    logl = np.zeros((nt, nw))
    inv = np.zeros((nw, 2, orc.n_bins))
    st = np.zeros(4, np.int64)
    th = theta.copy()
    for s in range(4):
        sw.sweep_counter.fill_(s)
        ps.step()
        oracle.psd_sweep_step(orc, pco, s, th, logl, betas, data, resid, inv, st)
        torch.cuda.synchronize()
        assert np.array_equal(ps.stats.cpu().numpy(), st), s
        assert np.allclose(ps.theta.cpu().numpy(), th, rtol=1e-12, atol=0), s
        assert np.allclose(ps.logl.cpu().numpy(), logl, rtol=1e-12, atol=0), s
        assert np.allclose(sw.inv_psd.cpu().numpy(), inv, rtol=1e-13, atol=0), s
    assert st[1] > 0 and st[1] < st[0] and st[3] > 0
    ctx.close()

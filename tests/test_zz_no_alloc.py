"""The allocation-free PSD likelihood (gb_psd_loglike_noalloc) through the C
ABI against gb_psd_loglike_n: two calls in a row on one device, the second
with fewer parameter sets, for 4 and 9 noise parameters; over-large batches
rejected."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2405_04690_amd import inputs
from paper_2405_04690_amd.gbl import GBL_EINVAL, Context

pytestmark = pytest.mark.gpu

CFG = inputs.TINY


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_psd_loglike_matches_the_workspace_path():
    dev = torch.device("cuda", 0)
    ctx = Context(T=CFG.T, dt=CFG.dt, L=CFG.L, f_lo=CFG.f_lo, f_hi=CFG.f_hi, device=dev)
    rng = np.random.default_rng(990)
    n_res = 3
    R = torch.from_numpy(inputs.complex_normals(991, (n_res, 2, ctx.n_bins)) * 1e-20).to(dev)
    fg = np.array([3.3e-44, 1.2, 2.8e-3, 1763.3, 1686.3])
    for n_par in (4, 9):
        for P in (1500, 37):   # two calls in a row, the second smaller
            lv = np.column_stack([CFG.sqrt_oms * rng.uniform(0.5, 2, P), CFG.sqrt_acc * rng.uniform(0.5, 2, P),
                                  CFG.sqrt_oms * rng.uniform(0.5, 2, P), CFG.sqrt_acc * rng.uniform(0.5, 2, P)])
            if n_par == 9:
                lv = np.hstack([lv, fg * rng.uniform(0.8, 1.2, (P, 5))])
            noise = torch.from_numpy(np.ascontiguousarray(lv)).to(dev)
            ri = torch.from_numpy(rng.integers(0, n_res, P).astype(np.int32)).to(dev)
            print(f"noalloc psd loglike n_par={n_par} P={P}", flush=True)
            got = torch.full((P,), float("nan"), dtype=torch.float64, device=dev)
            ctx._sync_stream()
            rc = ctx.lib.gb_psd_loglike_noalloc(ctx._h, _p(R), n_res, _p(noise), n_par, _p(ri), P, _p(got))
            assert rc == 0
            ref = ctx.gb_psd_loglike(R, noise, ri)
            torch.cuda.synchronize()
            assert torch.equal(got, ref)          # same kernels and summation order: bitwise
            assert torch.isfinite(got).all()
    big = torch.zeros((2049, 4), dtype=torch.float64, device=dev)
    ri = torch.zeros(2049, dtype=torch.int32, device=dev)
    out = torch.zeros(2049, dtype=torch.float64, device=dev)
    assert ctx.lib.gb_psd_loglike_noalloc(ctx._h, _p(R), n_res, _p(big), 4, _p(ri), 2049, _p(out)) == GBL_EINVAL
    ctx.close()

"""Launch-shape knobs and the autotuner: results do not depend on the knobs
(bitwise), out-of-range knobs are rejected, and the autotuner returns one of
its candidates."""
import numpy as np
import pytest
import torch

from paper_2405_04690_amd import autotune, inputs
from paper_2405_04690_amd.gbl import GBL_MIXED, Context, GblError

pytestmark = pytest.mark.gpu


def _problem(ctx, seed=700, B=3000):
    dev = ctx.device
    cfg = inputs.TINY
    noise = torch.tensor([[cfg.sqrt_oms, cfg.sqrt_acc, cfg.sqrt_oms, cfg.sqrt_acc]], dtype=torch.float64, device=dev)
    S = ctx.gb_psd_eval(noise)
    R = ctx.gb_make_noise(S, torch.from_numpy(inputs.complex_normals(seed, (1, 2, ctx.n_bins))).to(dev))
    src = inputs.draw_sources(seed + 1, B, log10_fdot_range=(-19, -15))
    old = inputs.perturb(seed + 2, src, cfg.T, "jitter")
    new = inputs.perturb(seed + 3, old, cfg.T, "inmodel")
    f0 = old[:, 1]
    w = np.where(f0 < 1e-3, 128, np.where(f0 < 3e-3, 256, np.where(f0 < 6e-3, 512, 1024))).astype(np.int32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return R, S, t(old), t(new), t(w)


@pytest.mark.parametrize("precision", [0, GBL_MIXED])
def test_results_do_not_depend_on_the_knobs(precision):
    cfg = inputs.TINY
    ctx = Context(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi, precision=precision)
    R, S, old, new, w = _problem(ctx)
    ref = ctx.gb_delta_loglike_var(R, S, old, new, w).cpu().numpy()
    for knobs in ({"bucket_chunk": 4096, "widest_first": 0}, {"bucket_chunk": 1 << 16, "widest_first": 1},
                  {"exact_grids": 0}, {"exact_grids": 1, "bucket_chunk": 1 << 20}):
        ctx.set_tuning(**knobs)
        got = ctx.gb_delta_loglike_var(R, S, old, new, w).cpu().numpy()
        assert np.array_equal(got, ref, equal_nan=True)
    best, table = autotune.tune_delta_var(ctx, (R, S, old, new, w), reps=2)
    assert best["bucket_chunk"] in autotune.CHUNKS and len(table) >= 16
    got = ctx.gb_delta_loglike_var(R, S, old, new, w).cpu().numpy()
    assert np.array_equal(got, ref, equal_nan=True)
    ctx.close()


def test_out_of_range_knobs_are_rejected():
    cfg = inputs.TINY
    ctx = Context(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi)
    for bad in ({"bucket_chunk": 5000}, {"bucket_chunk": 1 << 21}, {"flow_grid": 1}, {"flow_grid": 10 ** 6},
                {"widest_first": 2}, {"exact_grids": 2}):
        with pytest.raises(GblError):
            ctx.set_tuning(**bad)
    ctx.close()


@pytest.mark.parametrize("precision", [0, GBL_MIXED])
def test_uneven_widths_under_capture_match_eager(precision):
    """With exact grids requested, the eager call reads its bucket sizes back;
    captured, it cannot and runs upper-bound grids.  Three replays (with eager
    work in between) give the eager result bit for bit."""
    cfg = inputs.TINY
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = Context(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi, precision=precision,
                      stream=stream)
        R, S, old, new, w = _problem(ctx, seed=710)
        ctx.set_tuning(exact_grids=1)
        ref = ctx.gb_delta_loglike_var(R, S, old, new, w).clone()
        out = torch.full_like(ref, 7.0)
        ctx.graph_begin()
        ctx.gb_delta_loglike_var(R, S, old, new, w, out=out)
        g = ctx.graph_end()
        for _ in range(3):
            out.fill_(7.0)
            g.launch()
            stream.synchronize()
            assert torch.equal(torch.nan_to_num(out, nan=-1.0), torch.nan_to_num(ref, nan=-1.0))
        g.destroy()
        ctx.close()

"""GPU sampler sweep against the oracle sweep on identical random streams.

The accept/reject decisions are integers decided in FP64 on both sides, so
slot occupancy and the proposal/acceptance counters must agree exactly;
sampling coordinates and the cold-chain residual buffers agree to rounding
(1e-10 of their scale).
"""
import numpy as np
import pytest
import torch

import oracle
import sampler_setup
from paper_2405_04690_amd.gbl import Context, SweepConfig
from paper_2405_04690_amd.sampler import Sweep

pytestmark = pytest.mark.gpu


def _gpu_sweep(cfg, sc, st, stream=None, pool=1024, window_sums=False, precision=None):
    kw = {} if precision is None else {"precision": precision}
    ctx = Context(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi, stream=stream, **kw)
    gc = SweepConfig()
    for name, _ in oracle.SweepConfig._fields_:
        v = getattr(sc, name)
        if name in ("prior_lo", "prior_hi"):
            for i in range(8):
                getattr(gc, name)[i] = v[i]
        else:
            setattr(gc, name, v)
    sw = Sweep(ctx, gc, spectrum_pool=pool, window_sums=window_sums)
    for name in ("u", "exists", "betas", "resid", "inv_psd", "group", "group_count", "stats", "swap_acc"):
        getattr(sw, name).copy_(torch.from_numpy(np.ascontiguousarray(getattr(st, name))))
    return ctx, sw


def _compare(sw, st, what, T=None):
    torch.cuda.synchronize()
    ex = sw.exists.cpu().numpy()
    assert np.array_equal(ex, st.exists), f"{what}: occupancy differs"
    assert np.array_equal(sw.stats.cpu().numpy(), st.stats), f"{what}: counters differ"
    u = sw.u.cpu().numpy()
    occ = st.exists.astype(bool)
    # per-coordinate scale: log10 A, f0 (one band), fdot, phi0, cos iota, psi, lambda, sin beta
    T = sampler_setup.inputs.TINY.T if T is None else T
    width = np.array([2.5, 512 / T, 1e-15, 2 * np.pi, 2.0, np.pi, 2 * np.pi, 2.0])
    scale = np.maximum(np.abs(st.u[occ]), width)
    assert np.max(np.abs(u[occ] - st.u[occ]) / scale) <= 1e-10, f"{what}: coordinates differ"
    r = sw.resid.cpu().numpy()
    assert np.max(np.abs(r - st.resid)) <= 1e-10 * np.abs(st.resid).max(), f"{what}: residual buffers differ"


@pytest.mark.parametrize("N,pool,ws", [(128, 1024, False), (256, 1024, False), (512, 1024, False), (128, 0, False),
                                       (256, 2, False), (256, 1024, True), (128, 0, True), (512, 1024, True),
                                       (512, 0, True)])
def test_sweep_parity_each_move(N, pool, ws):
    """pool: the per-slot spectrum cache (0: recomputed spectra; 2: most band
    loops find no free entry and recompute, the others use the cache); ws:
    the tempering pass takes the window sums the band passes leave"""
    cfg, orc, sc, st = sampler_setup.problem(N=N, n_b=6 if N == 128 else 4)
    ctx, sw = _gpu_sweep(cfg, sc, st, pool=pool, window_sums=ws)
    s0 = 11
    sw.sweep_counter.fill_(s0)
    oracle.sweep_group(sc, st)
    sw.group_refresh()
    torch.cuda.synchronize()
    assert np.array_equal(sw.group_count.cpu().numpy(), st.group_count)
    assert np.array_equal(sw.group.cpu().numpy(), st.group)
    for move, name in ((0, "in-model"), (1, "rj"), (2, "tempering")):
        for parity in (1, 0):
            print(f"sweep parity: {name} parity {parity}", flush=True)
            oracle.sweep_step(orc, sc, st, move, parity, s0)
            sw.step(move, parity)
            _compare(sw, st, f"{name}/{parity}")
    assert st.stats[1] > 0 and st.stats[0] > st.stats[1]  # some in-model moves accepted, some not
    assert st.stats[3] + st.stats[5] > 0                   # some births or deaths accepted
    ctx.close()


@pytest.mark.parametrize("N,W,pool", [(128, 384, 1024), (256, 200, 0), (256, 1000, 1024), (512, 640, 0),
                                     (1024, 1024, 1024), (1024, 1024, 0)])
def test_sweep_parity_wide_subbands(N, W, pool):
    """sub-bands of W bins with templates of N bins (the band loops keep their
    2W + N-bin windows in global memory, in the window-sum entries), and N =
    1024 sub-bands (512 threads per band loop): every move against the
    oracle, decisions and counters exact"""
    cfg, orc, sc, st = sampler_setup.problem(N=N, n_b=4, W=W)
    ctx, sw = _gpu_sweep(cfg, sc, st, pool=pool)
    assert sw.window_sums is not None and sw.window_sums.shape[-1] == 2 * (2 * W + N)
    s0 = 12
    sw.sweep_counter.fill_(s0)
    oracle.sweep_group(sc, st)
    sw.group_refresh()
    for move, name in ((0, "in-model"), (1, "rj"), (2, "tempering")):
        for parity in (1, 0):
            print(f"wide sub-bands N={N} W={W}: {name} parity {parity}", flush=True)
            oracle.sweep_step(orc, sc, st, move, parity, s0)
            sw.step(move, parity)
            _compare(sw, st, f"W={W} {name}/{parity}")
    assert st.stats[1] > 0 and st.stats[3] + st.stats[5] > 0 and st.stats[7] > 0
    ctx.close()


def test_sweep_run_and_graph_replay():
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=3, n_b=4, n_slots=3, n_prop=4, group_every=2, seed=5)
    st_ref = oracle.SweepState(sc, orc.n_bins)
    for name in ("u", "exists", "betas", "resid", "inv_psd", "group", "group_count", "stats"):
        setattr(st_ref, name, getattr(st, name).copy())
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx, sw = _gpu_sweep(cfg, sc, st, stream=stream)
        ctx2, sw2 = _gpu_sweep(cfg, sc, st, stream=stream)
        sw.sweep_counter.fill_(4)
        sw2.sweep_counter.fill_(4)
        sw.run(4)
        sw2.capture(2)
        sw2.replay()
        sw2.replay()
        stream.synchronize()
    for s in range(4, 8):
        oracle.sweep_full(orc, sc, st_ref, s)
    _compare(sw, st_ref, "gb_sweep_run")
    _compare(sw2, st_ref, "graph replay")
    assert int(sw2.sweep_counter.item()) == 8
    sw2.release_graph()
    ctx.close()
    ctx2.close()


def test_inmodel_moves_keep_the_prior_at_zero_inverse_temperature():
    """beta = 0: the group-stretch chain must leave the uniform prior of the
    occupied slots invariant on all eight coordinates, the periodic angles
    included.  3072 independent slot chains, a fixed group no larger than
    n_friends (so that the friend window does not depend on the current f0),
    one final snapshot after 40 sweeps."""
    from scipy import stats as sps
    cfg, orc, sc, st = sampler_setup.problem(n_t=64, n_w=4, n_b=4, n_slots=3, n_prop=6, n_friends=16, seed=9)
    rng = np.random.default_rng(2)
    lo = np.array(list(sc.prior_lo))
    hi = np.array(list(sc.prior_hi))
    boxes = []
    for b in range(sc.n_bands):
        box_lo, box_hi = lo.copy(), hi.copy()
        box_lo[1] = (sc.k_band0 + (b - 0.5) * sc.N) / cfg.T
        box_hi[1] = (sc.k_band0 + (b + 1.5) * sc.N) / cfg.T
        for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
            box_lo[k], box_hi[k] = 0.0, P
        boxes.append((box_lo, box_hi))
        st.u[:, :, b] = box_lo + (box_hi - box_lo) * rng.uniform(size=st.u[:, :, b].shape)
    st.exists[:] = 1
    st.betas[:] = 0.0
    ctx, sw = _gpu_sweep(cfg, sc, st)
    sw.group_refresh()
    for it in range(40):
        sw.step(0, 1)
        sw.step(0, 0)
        sw.advance()
    torch.cuda.synchronize()
    assert int(sw.group_count.max().item()) <= sc.n_friends
    u = sw.u.cpu().numpy()
    stats = sw.stats.cpu().numpy()
    assert stats[1] > 0.1 * stats[0]
    x = np.concatenate([(u[:, :, b].reshape(-1, 8) - boxes[b][0]) / (boxes[b][1] - boxes[b][0])
                        for b in range(sc.n_bands)])
    for k in range(8):
        p = sps.kstest(x[:, k], "uniform").pvalue
        assert p > 1e-3, (k, p)
    ctx.close()


def _given_proposals(sc, T, seed):
    """seeded RJ proposal arrays (not from any flow): candidates inside the
    band's prior box (a tenth with f0 outside it) and arbitrary ln q values"""
    rng = np.random.default_rng(seed)
    nt, nw, nb, ns = sc.n_temps, sc.n_walkers, sc.n_bands, sc.n_slots
    lo = np.array(list(sc.prior_lo))
    hi = np.array(list(sc.prior_hi))
    prop = np.zeros((nt, nw, nb, ns, 8))
    for b in range(nb):
        blo, bhi = lo.copy(), hi.copy()
        blo[1] = (sc.k_band0 + (b - 0.5) * sc.N) / T
        bhi[1] = (sc.k_band0 + (b + 1.5) * sc.N) / T
        for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
            blo[k], bhi[k] = 0.0, P
        prop[:, :, b] = blo + (bhi - blo) * rng.uniform(size=(nt, nw, ns, 8))
    out = rng.uniform(size=(nt, nw, nb, ns)) < 0.1
    prop[..., 1] = np.where(out, prop[..., 1] + 2.5 * sc.N / T, prop[..., 1])
    logq = rng.normal(-5.0, 3.0, (nt, nw, nb, ns))
    return prop, logq


def test_rj_with_given_proposal_densities_and_cold_logl_trace():
    cfg, orc, sc, st = sampler_setup.problem(seed=21)
    ctx, sw = _gpu_sweep(cfg, sc, st)
    prop, logq = _given_proposals(sc, cfg.T, 22)
    sw.enable_proposals()
    sw.prop_u.copy_(torch.from_numpy(prop))
    sw.rj_logq.copy_(torch.from_numpy(logq))
    sw.enable_logl_trace()
    s0 = 3
    sw.sweep_counter.fill_(s0)
    for parity in (1, 0):
        oracle.sweep_step(orc, sc, st, 1, parity, s0, prop_u=prop, rj_logq=logq)
        sw.step(1, parity)
        _compare(sw, st, f"rj given proposals/{parity}")
    assert st.stats[3] > 0 and st.stats[5] > 0
    cl = np.full((sc.n_walkers, sc.n_bands), np.nan)
    for parity in (1, 0):
        oracle.sweep_step(orc, sc, st, 2, parity, s0, cold_logl=cl)
        sw.step(2, parity)
        _compare(sw, st, f"tempering/{parity}")
    got = sw.cold_logl.cpu().numpy()
    assert np.all(np.isfinite(cl))
    assert np.max(np.abs(got - cl)) <= 1e-10 * np.abs(cl).max()
    ctx.close()


def _flow_for(sc, cfg, s_bias=0.0, seed=31, identity=False, prior_weight=0.2):
    from oracle import flow as oflow
    from paper_2405_04690_amd.flow import flow_config
    fc = flow_config(sc.n_bands, sc.N, sc.k_band0, list(sc.prior_lo), list(sc.prior_hi), prior_weight)
    th = oflow.init_params(seed, sc.n_bands, out_scale=0.0 if identity else 0.3)
    layers, _ = oflow.unpack(th, sc.n_bands)
    for l, L in enumerate(layers):
        if l % 2 == 0:
            L["b3"][0] = s_bias   # contracts coordinate 1 (f0) in the even layers
    return fc, th


def test_rj_prepare_mixture_with_identity_flow():
    """identity flow (W3 = b3 = 0) in a 3:1 flow/prior mixture: each empty
    slot's candidate is either the box image of the stream's Box-Muller
    normals or a prior draw from the same uniforms (choice by the stream), and
    ln q = ln(3/4 q_flow + 1/4 p) at candidates and current sources alike"""
    from oracle import flow as oflow
    from paper_2405_04690_amd.flow import Flow
    cfg, orc, sc, st = sampler_setup.problem(seed=41)
    ctx, sw = _gpu_sweep(cfg, sc, st)
    w = 0.25
    fc, th = _flow_for(sc, cfg, identity=True, prior_weight=w)
    fl = Flow(ctx, fc, th.astype(np.float32))
    s0 = 9
    sw.sweep_counter.fill_(s0)
    sw.rj_prepare(fl)
    torch.cuda.synchronize()
    pu = sw.prop_u.cpu().numpy()
    lq = sw.rj_logq.cpu().numpy()
    mode = sw.rj_mode.cpu().numpy()
    ex = st.exists.astype(bool)
    nt, nw, nb, ns = ex.shape
    lo8 = np.array(list(sc.prior_lo))
    hi8 = np.array(list(sc.prior_hi))

    def lnq_mix(u, b):
        lo, hi = oflow.box(np.array([b]), cfg.T, sc.k_band0, sc.N, lo8, hi8)
        lnV = np.sum(np.log(hi - lo))
        if np.all((u > lo) & (u < hi)):
            x, lj = oflow.to_real(u[None], lo, hi)
            lf = oflow.log_normal(x)[0] + lj[0]
            return np.logaddexp(np.log1p(-w) + lf, np.log(w) - lnV)
        return np.log(w) - lnV

    n_prior = 0
    for (t, wk, b, s) in np.argwhere(~ex)[:300]:
        unit = (t * nw + wk) * nb + b
        d0 = 2048 + 16 * s
        uu = np.array([oracle.rng_uniform(sc.seed, s0, 1, unit, d0 + k) for k in range(8)])
        c = oracle.rng_uniform(sc.seed, s0, 1, unit, d0 + 8)
        lo, hi = oflow.box(np.array([b]), cfg.T, sc.k_band0, sc.N, lo8, hi8)
        if c < w:
            n_prior += 1
            assert mode[t, wk, b, s] == 2
            u_ref = lo[0] + (hi[0] - lo[0]) * uu
        else:
            assert mode[t, wk, b, s] == 1
            z = np.zeros(8)
            for p in range(4):
                r = np.sqrt(-2 * np.log(uu[2 * p]))
                z[2 * p], z[2 * p + 1] = r * np.cos(2 * np.pi * uu[2 * p + 1]), r * np.sin(2 * np.pi * uu[2 * p + 1])
            u_ref = oflow.from_real(z[None], lo, hi)[0][0]
        assert np.allclose(pu[t, wk, b, s], u_ref, rtol=1e-12, atol=1e-12 * np.abs(hi - lo).max())
        ref = lnq_mix(pu[t, wk, b, s], b)
        assert abs(lq[t, wk, b, s] - ref) <= 1e-9 * max(1.0, abs(ref))
    assert 0 < n_prior < 300
    for (t, wk, b, s) in np.argwhere(ex)[:100]:
        assert mode[t, wk, b, s] == 0
        ref = lnq_mix(st.u[t, wk, b, s], b)
        assert abs(lq[t, wk, b, s] - ref) <= 1e-9 * max(1.0, abs(ref))
    ctx.close()


def test_flow_rj_keeps_the_prior_at_zero_inverse_temperature():
    """beta = 0 with a flow proposal concentrated in f0: the exact MH ratio
    keeps each slot occupied with probability 1/2 and the occupied f0
    uniform over the band's range (without the ln q terms they would follow q)"""
    from paper_2405_04690_amd.flow import Flow
    from scipy import stats as sps
    cfg, orc, sc, st = sampler_setup.problem(n_t=1, n_w=16, n_b=4, n_slots=16, seed=51)
    rng = np.random.default_rng(52)
    lo = np.array(list(sc.prior_lo))
    hi = np.array(list(sc.prior_hi))
    for b in range(sc.n_bands):
        blo, bhi = lo.copy(), hi.copy()
        blo[1] = (sc.k_band0 + (b - 0.5) * sc.N) / cfg.T
        bhi[1] = (sc.k_band0 + (b + 1.5) * sc.N) / cfg.T
        for k, P in ((3, 2 * np.pi), (5, np.pi), (6, 2 * np.pi)):
            blo[k], bhi[k] = 0.0, P
        st.u[:, :, b] = blo + (bhi - blo) * rng.uniform(size=st.u[:, :, b].shape)
    st.exists[:] = (rng.uniform(size=st.exists.shape) < 0.5).astype(np.int32)
    st.betas[:] = 0.0
    ctx, sw = _gpu_sweep(cfg, sc, st)
    fc, th = _flow_for(sc, cfg, s_bias=-0.5)
    fl = Flow(ctx, fc, th.astype(np.float32))
    f0s, occ = [], []
    for it in range(400):
        sw.rj_prepare(fl)
        sw.step(1, 1)
        sw.step(1, 0)
        sw.advance()
        if it >= 100 and it % 25 == 0:
            ex = sw.exists.cpu().numpy().astype(bool)
            u = sw.u.cpu().numpy()
            occ.append(ex.mean())
            for b in range(sc.n_bands):
                flo = (sc.k_band0 + (b - 0.5) * sc.N) / cfg.T
                fhi = (sc.k_band0 + (b + 1.5) * sc.N) / cfg.T
                f0s.append((u[:, :, b][ex[:, :, b]][:, 1] - flo) / (fhi - flo))
    stats = sw.stats.cpu().numpy()
    assert stats[3] > 0.02 * stats[2] and stats[5] > 0.02 * stats[4]
    assert abs(np.mean(occ) - 0.5) < 0.05, np.mean(occ)
    x = np.concatenate(f0s)
    # the flow's f0 density peaks at the band centre; the occupied f0 must not
    # (snapshots 25 sweeps apart are correlated: a loose KS threshold)
    assert sps.kstest(x, "uniform").pvalue > 1e-6
    assert abs(np.mean(np.abs(x - 0.5) < 0.1) - 0.2) < 0.05
    ctx.close()


def test_general_capture_of_flow_sweep_and_psd_step():
    """one graph holding a sweep with the flow RJ proposal and the noise-PSD
    step: two replays give what two direct calls give"""
    from paper_2405_04690_amd.flow import Flow
    from paper_2405_04690_amd.sampler import PsdSweep, psd_config
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=4, n_b=4, n_slots=4, seed=61)
    lo, hi = (10e-12, 2e-15, 10e-12, 2e-15), (20e-12, 4e-15, 20e-12, 4e-15)
    rng = np.random.default_rng(62)
    theta = np.array(lo) + (np.array(hi) - np.array(lo)) * rng.uniform(size=(2, sc.n_walkers, 4))
    stream = torch.cuda.Stream()
    runs = []
    with torch.cuda.stream(stream):
        for captured in (False, True):
            ctx, sw = _gpu_sweep(cfg, sc, st, stream=stream)
            fc, th = _flow_for(sc, cfg, s_bias=-0.3)
            fl = Flow(ctx, fc, th.astype(np.float32))
            data = sw.resid[0][0].clone()
            ps = PsdSweep(sw, psd_config(2, sc.n_walkers, lo, hi, seed=63), data)
            ps.theta.copy_(torch.from_numpy(theta))
            ps.betas.copy_(torch.tensor([1.0, 0.5], dtype=torch.float64))
            sw.enable_proposals()
            sw.sweep_counter.fill_(7)
            if captured:
                ctx.graph_begin()
                sw.run_flow(fl, 1)
                ps.step()
                g = ctx.graph_end()
                g.launch()
                g.launch()
            else:
                for _ in range(2):
                    sw.run_flow(fl, 1)
                    ps.step()
            stream.synchronize()
            runs.append({k: getattr(sw, k).cpu().numpy().copy() for k in ("u", "exists", "resid", "stats",
                                                                          "sweep_counter", "inv_psd")} |
                        {k: getattr(ps, k).cpu().numpy().copy() for k in ("theta", "logl")} |
                        {"psd_stats": ps.stats.cpu().numpy().copy()})
            if captured:
                g.destroy()
            ctx.close()
    a, b = runs
    assert int(a["sweep_counter"][0]) == 9 and int(b["sweep_counter"][0]) == 9
    for k in ("exists", "stats", "psd_stats"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("u", "theta", "logl", "inv_psd"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=0), k
    assert np.max(np.abs(a["resid"] - b["resid"])) <= 1e-10 * np.abs(a["resid"]).max()


def test_sweep_parity_at_the_slot_limit():
    """64 slots per band (the kernel's limit), every slot occupied at the start"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=2, n_b=3, n_slots=64, n_prop=8, seed=71)
    rng = np.random.default_rng(72)
    for b in range(sc.n_bands):
        flo = (sc.k_band0 + (b + 0.05) * sc.N) / cfg.T
        fhi = (sc.k_band0 + (b + 0.95) * sc.N) / cfg.T
        occ = ~st.exists.astype(bool)[:, :, b]
        n = int(occ.sum())
        st.u[:, :, b][occ] = np.stack([rng.uniform(-23, -22, n), rng.uniform(flo, fhi, n), np.zeros(n),
                                       rng.uniform(0, 6.28, n), rng.uniform(-1, 1, n), rng.uniform(0, 3.14, n),
                                       rng.uniform(0, 6.28, n), rng.uniform(-1, 1, n)], axis=1)
    st.exists[:] = 1
    # rebuild the cold-chain buffers for the new slot contents
    data = st.resid[0, 0].copy()   # buffer 0 = data minus the even bands' original sources: any fixed data will do
    for par in (0, 1):
        for w in range(sc.n_walkers):
            st.resid[par, w] = data
            for b in range(par, sc.n_bands, 2):
                phys = np.array([sampler_setup._phys(st.u[0, w, b, s]) for s in range(sc.n_slots)])
                orc.scatter_add(phys, sc.N, -1.0, st.resid[par, w])
    ctx, sw = _gpu_sweep(cfg, sc, st)
    sw.sweep_counter.fill_(2)
    oracle.sweep_group(sc, st)
    sw.group_refresh()
    for move in (0, 1, 2):
        for parity in (1, 0):
            oracle.sweep_step(orc, sc, st, move, parity, 2)
            sw.step(move, parity)
            _compare(sw, st, f"slot limit {move}/{parity}")
    ctx.close()


@pytest.mark.timeout(900)
def test_sweep_parity_at_the_bench_shape():
    """The benchmark's chain shape: 36 temperatures x 32 walkers x 60 slots,
    1 yr at 5 s, N = 256, four sub-bands with every slot occupied, so each
    stationary group holds 1,920 cold-chain sources (the 64-way friend search
    over them) and tempering runs 36 rungs; one group refresh and one full
    sweep (in-model, RJ, tempering; odd then even) against the oracle"""
    from paper_2405_04690_amd import inputs
    print("bench shape: building the problem on the host", flush=True)
    cfg, orc, sc, st = sampler_setup.problem(n_t=36, n_w=32, n_b=4, n_slots=60, n_prop=4, n_friends=40,
                                             group_every=1, seed=91, beta_top=0.02, N=256, cfg=inputs.PAPER,
                                             per_band=60)
    ctx, sw = _gpu_sweep(cfg, sc, st, window_sums=True)   # the benchmark's configuration
    s0 = 5
    sw.sweep_counter.fill_(s0)
    oracle.sweep_group(sc, st)
    sw.group_refresh()
    torch.cuda.synchronize()
    assert np.array_equal(sw.group_count.cpu().numpy(), st.group_count)
    assert st.group_count.min() == 32 * 60
    assert np.array_equal(sw.group.cpu().numpy(), st.group)
    for move, name in ((0, "in-model"), (1, "rj"), (2, "tempering")):
        for parity in (1, 0):
            print(f"bench shape: {name} parity {parity}", flush=True)
            sw.step(move, parity)
            oracle.sweep_step(orc, sc, st, move, parity, s0)
            _compare(sw, st, f"bench shape {name}/{parity}", T=cfg.T)
    assert st.stats[1] > 0 and st.stats[5] > 0 and st.stats[7] > 0
    ctx.close()


def test_inmodel_draws_refill_past_64_proposals():
    """n_prop = 70: the in-model loop's counter-based draws are computed 64
    proposals at a time, so the second run (6 proposals) is a partial one"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=2, n_w=3, n_b=4, n_slots=4, n_prop=70, seed=93)
    ctx, sw = _gpu_sweep(cfg, sc, st)
    s0 = 6
    sw.sweep_counter.fill_(s0)
    oracle.sweep_group(sc, st)
    sw.group_refresh()
    for parity in (1, 0):
        print(f"n_prop=70 in-model parity {parity}", flush=True)
        oracle.sweep_step(orc, sc, st, 0, parity, s0)
        sw.step(0, parity)
        _compare(sw, st, f"n_prop=70/{parity}")
    assert st.stats[0] == 70 * 2 * 3 * 4
    ctx.close()


def _push_over_edges(cfg, orc, sc, st, seed):
    """move some cold-chain sources up to 0.45 band past an edge of their band
    (inside the prior box) and rebuild the buffers"""
    rng = np.random.default_rng(seed)
    T, N, kb = cfg.T, sc.N, sc.k_band0
    for w in range(sc.n_walkers):
        for b in range(sc.n_bands):
            for s in range(sc.n_slots):
                if st.exists[0, w, b, s] and rng.uniform() < 0.4:
                    d = rng.uniform(0.02, 0.45)
                    st.u[0, w, b, s, 1] = (kb + (b + 1.0 + d if rng.uniform() < 0.5 else b - d) * N) / T
    for par in (0, 1):
        for w in range(sc.n_walkers):
            st.resid[par, w] = sampler_setup.rebuild_buffer(orc, sc, st, par, w)


def test_ladder_adaptation_and_ownership_shift_match_the_oracle():
    """the two per-sweep steps on their own (given swap counts; strayed
    sources), then three full sweeps with both switched on"""
    cfg, orc, sc, st = sampler_setup.problem(n_t=5, n_w=4, n_b=5, n_slots=4, n_prop=6, seed=141)
    sc.adapt_ladder, sc.shift_ownership, sc.adapt_lag, sc.adapt_time = 1, 1, 10.0, 2.0
    _push_over_edges(cfg, orc, sc, st, 142)
    st.swap_acc[:] = np.random.default_rng(143).integers(0, sc.n_walkers + 1, st.swap_acc.shape).astype(np.int32)
    ctx, sw = _gpu_sweep(cfg, sc, st)
    s0 = 4
    sw.sweep_counter.fill_(s0)
    print("ladder adaptation step", flush=True)
    sw.adapt_ladder()
    oracle.adapt_ladder(sc, st, s0)
    torch.cuda.synchronize()
    assert np.array_equal(sw.swap_acc.cpu().numpy(), st.swap_acc)
    assert np.allclose(sw.betas.cpu().numpy(), st.betas, rtol=1e-14, atol=0)
    sw.betas.copy_(torch.from_numpy(st.betas))          # both sides continue from the oracle's ladder
    print("ownership shift step", flush=True)
    sw.shift_ownership()
    oracle.shift_ownership(orc, sc, st, st.stats[8:])
    _compare(sw, st, "ownership shift")
    assert st.stats[8] > 0
    print("three full sweeps with adaptation and shifts", flush=True)
    _push_over_edges(cfg, orc, sc, st, 144)
    ctx.close()
    ctx, sw = _gpu_sweep(cfg, sc, st)
    sw.sweep_counter.fill_(s0)
    sw.run(3)
    for s in range(s0, s0 + 3):
        oracle.sweep_full(orc, sc, st, s)
    _compare(sw, st, "full sweeps with adaptation and shifts")
    assert np.allclose(sw.betas.cpu().numpy(), st.betas, rtol=1e-13, atol=0)
    assert np.array_equal(sw.swap_acc.cpu().numpy(), st.swap_acc)
    assert st.stats[8] > 0 and st.stats[7] > 0
    ctx.close()


def test_band_sets_share_the_cold_chain_buffers():
    """two band sets over adjacent ranges -- four N = 128 sub-bands, then two
    of N = 256 from where the first set ends -- sharing the walkers'
    cold-chain buffers: full sweeps of one set after the other against the
    oracle doing the same on one shared buffer array"""
    from paper_2405_04690_amd.sampler import run_band_sets
    cfg, orc, scA, stA = sampler_setup.problem(N=128, n_b=4, n_t=2, n_w=3, n_slots=3, seed=71)
    kB = scA.k_band0 + 4 * 128
    _, _, scB, stB = sampler_setup.problem(N=256, n_b=2, n_t=2, n_w=3, n_slots=3, seed=72, f_band0=(kB + 0.5) / cfg.T)
    assert scB.k_band0 == kB
    # one data set holding both sets' injections; the shared buffers: the
    # data minus the cold-chain sources of every band of that parity
    data = stA.data.copy()
    orc.scatter_add(stB.src, 256, 1.0, data)
    for par in (0, 1):
        for w in range(scA.n_walkers):
            buf = data.copy()
            for st, sc in ((stA, scA), (stB, scB)):
                for b in range(par, sc.n_bands, 2):
                    occ = [sampler_setup._phys(st.u[0, w, b, s]) for s in range(sc.n_slots) if st.exists[0, w, b, s]]
                    if occ:
                        orc.scatter_add(np.array(occ), sc.N, -1.0, buf)
            stA.resid[par, w] = buf
    stB.resid = stA.resid                     # one array for both oracle states
    stB.inv_psd = stA.inv_psd
    ctx, swA = _gpu_sweep(cfg, scA, stA)
    gcB = SweepConfig()
    for name, _ in oracle.SweepConfig._fields_:
        v = getattr(scB, name)
        if name in ("prior_lo", "prior_hi"):
            for i in range(8):
                getattr(gcB, name)[i] = v[i]
        else:
            setattr(gcB, name, v)
    swB = Sweep(ctx, gcB, resid=swA.resid, inv_psd=swA.inv_psd)
    for name in ("u", "exists", "betas", "group", "group_count", "stats", "swap_acc"):
        getattr(swB, name).copy_(torch.from_numpy(np.ascontiguousarray(getattr(stB, name))))
    for sw in (swA, swB):
        sw.sweep_counter.fill_(4)
    for s in range(4, 7):
        print(f"band sets: sweep {s}", flush=True)
        oracle.sweep_full(orc, scA, stA, s)
        oracle.sweep_full(orc, scB, stB, s)
        run_band_sets([swA, swB], 1)
        _compare(swA, stA, f"set A, sweep {s}")
        _compare(swB, stB, f"set B, sweep {s}")
    assert stA.stats[1] > 0 and stB.stats[1] > 0 and stA.stats[7] > 0
    ctx.close()


def test_mixed_precision_sweep_takes_the_fp64_decisions_but_near_the_threshold():
    """Mixed-precision band loops (FP32 response and FFT; decode, phases,
    spectra at the bins, windows and every sum in FP64) at the bench shape
    (36 temperatures x 32 walkers x 60 slots, 1 yr): one full sweep from the
    same state as the FP64 sweep.  A decision can differ only where the FP32
    template error moves the log acceptance ratio across the draw, so almost
    every (temperature, walker, sub-band) unit ends in the same state, the
    acceptance counts agree closely, and a walker whose cold-chain units all
    agree holds the same cold-chain buffers up to the FP32 template error."""
    from paper_2405_04690_amd import inputs
    from paper_2405_04690_amd.gbl import GBL_MIXED
    print("mixed sweep: building the problem on the host", flush=True)
    cfg, orc, sc, st = sampler_setup.problem(n_t=36, n_w=32, n_b=4, n_slots=60, n_prop=8, n_friends=40,
                                             group_every=1, seed=92, beta_top=0.02, N=256, cfg=inputs.PAPER,
                                             per_band=60)
    ctx_bad, sw_bad = _gpu_sweep(cfg, sc, st, precision=GBL_MIXED)   # no window sums: refused
    with pytest.raises(RuntimeError, match="window_sums"):
        sw_bad.step(0, 1)
    ctx_bad.close()
    runs = {}
    for name, prec in (("fp64", None), ("mixed", GBL_MIXED)):
        print(f"mixed sweep: {name} sweep", flush=True)
        ctx, sw = _gpu_sweep(cfg, sc, st, window_sums=True, precision=prec)
        sw.sweep_counter.fill_(7)
        sw.group_refresh()
        for move in (0, 1, 2):
            for parity in (1, 0):
                sw.step(move, parity)
        torch.cuda.synchronize()
        runs[name] = {k: getattr(sw, k).cpu().numpy() for k in ("u", "exists", "resid", "stats")}
        ctx.close()
    a, b = runs["fp64"], runs["mixed"]
    same = np.all(a["exists"] == b["exists"], axis=-1) & np.all(a["u"] == b["u"], axis=(-1, -2))  # [t][w][b]
    frac = float(same.mean())
    print(f"mixed sweep: identical units {frac:.4f}, stats fp64 {a['stats'][:8]} mixed {b['stats'][:8]}", flush=True)
    assert frac >= 0.95
    sa, sb = a["stats"].astype(np.float64), b["stats"].astype(np.float64)
    # proposal counts follow the occupancy the RJ pass starts from, which the
    # in-model pass does not change: equal; acceptance counts close
    assert np.array_equal(sa[[0, 2, 4, 6]], sb[[0, 2, 4, 6]])
    for acc in (1, 3, 5, 7):
        assert abs(sa[acc] - sb[acc]) <= max(3.0, 0.02 * sa[acc]), acc
    cold_same = np.all(same[0], axis=-1)  # walkers whose cold-chain units all agree
    assert cold_same.sum() >= 0.75 * cold_same.size
    for w in np.nonzero(cold_same)[0]:
        ra, rb = a["resid"][:, w], b["resid"][:, w]
        assert np.max(np.abs(ra - rb)) <= 1e-3 * np.max(np.abs(ra)), w


@pytest.mark.parametrize("shape", [(3, 4, 6, 4), (16, 32, 16, 40), (32, 32, 16, 40), (36, 32, 16, 60)])
def test_rj_prepare_densities_equal_the_flow_density_call(shape):
    """The RJ preparation's masked flow passes (current sources; prior
    candidates) gather their slots into tiles by ballot before the flow runs
    when there are at least 2^18 slots; each slot must still get the flow
    density that the plain density call gives at its point (a non-identity
    flow, mixed with the prior as in the sweep).  Shapes: 288 slots (no
    gathering), 327,680 / 655,360 / 1,105,920 slots (gathering windows of 64,
    128 and 256 slots)."""
    from oracle import flow as oflow
    from paper_2405_04690_amd.flow import Flow
    n_t, n_w, n_b, n_s = shape
    print(f"rj_prepare densities: shape {shape}", flush=True)
    cfg, orc, sc, st = sampler_setup.problem(n_t=n_t, n_w=n_w, n_b=n_b, n_slots=n_s, seed=43)
    ctx, sw = _gpu_sweep(cfg, sc, st)
    w = 0.2
    fc, th = _flow_for(sc, cfg, prior_weight=w)
    fl = Flow(ctx, fc, th.astype(np.float32))
    sw.sweep_counter.fill_(5)
    sw.rj_prepare(fl)
    torch.cuda.synchronize()
    lo8, hi8 = np.array(list(sc.prior_lo)), np.array(list(sc.prior_hi))
    lnV = np.array([np.sum(np.log(np.subtract(*oflow.box(np.array([b]), cfg.T, sc.k_band0, sc.N, lo8, hi8)[::-1])))
                    for b in range(n_b)])
    dev = sw.u.device
    band = torch.arange(n_b, device=dev, dtype=torch.int32).view(1, 1, n_b, 1).expand(n_t, n_w, n_b, n_s)
    mode, lq = sw.rj_mode, sw.rj_logq
    for m, pts in ((0, sw.u), (2, sw.prop_u)):
        sel = mode == m
        assert int(sel.sum()) > 0
        bb = band[sel].contiguous()
        lf = fl.log_prob(pts[sel].contiguous(), bb).cpu().numpy()
        lv = lnV[bb.cpu().numpy()]
        ref = np.where(np.isnan(lf), np.log(w) - lv, np.logaddexp(np.log1p(-w) + lf, np.log(w) - lv))
        got = lq[sel].cpu().numpy()
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-10), m
    ctx.close()


def test_sweep_parity_with_sources_on_the_prior_edges():
    """every injected source and every slot holding it sits on the edges of
    the angle ranges (cos iota = +-1, sin beta = +-1, phi0 = psi = lambda =
    0): the band loops decode such coordinates directly (cos beta = 0 at sin
    beta = +-1), and the stretch moves from them leave the box or wrap; one
    full sweep against the oracle, decisions exact"""
    cfg, orc, sc, st = sampler_setup.problem(seed=95, edge=True)
    u = st.u[st.exists.astype(bool)]
    assert np.all(np.abs(u[:, 4]) == 1.0) and np.all(np.abs(u[:, 7]) == 1.0) and np.all(u[:, [3, 5, 6]] == 0.0)
    ctx, sw = _gpu_sweep(cfg, sc, st)
    s0 = 13
    sw.sweep_counter.fill_(s0)
    oracle.sweep_group(sc, st)
    sw.group_refresh()
    for move, name in ((0, "in-model"), (1, "rj"), (2, "tempering")):
        for parity in (1, 0):
            print(f"prior edges: {name} parity {parity}", flush=True)
            oracle.sweep_step(orc, sc, st, move, parity, s0)
            sw.step(move, parity)
            _compare(sw, st, f"edges {name}/{parity}")
    assert st.stats[0] > 0 and st.stats[2] + st.stats[4] > 0
    ctx.close()


@pytest.mark.parametrize("N", [128, 512, 1024])
def test_mixed_precision_band_loops_at_every_template_width(N):
    """the FP32-response band loops at the other template widths (N = 512 and
    1024 keep their windows in global memory), one full sweep against the
    FP64 one from the same state: the same proposal counts, acceptance counts
    within two, and at most one (temperature, walker, sub-band) unit in ten
    ending elsewhere"""
    from paper_2405_04690_amd.gbl import GBL_MIXED
    cfg, orc, sc, st = sampler_setup.problem(N=N, n_b=4, n_t=3, n_w=8, n_slots=4, seed=97)
    runs = {}
    for name, prec in (("fp64", None), ("mixed", GBL_MIXED)):
        print(f"mixed band loops N={N}: {name}", flush=True)
        ctx, sw = _gpu_sweep(cfg, sc, st, window_sums=True, precision=prec)
        sw.sweep_counter.fill_(3)
        sw.group_refresh()
        for move in (0, 1, 2):
            for parity in (1, 0):
                sw.step(move, parity)
        torch.cuda.synchronize()
        runs[name] = {k: getattr(sw, k).cpu().numpy() for k in ("u", "exists", "stats")}
        ctx.close()
    a, b = runs["fp64"], runs["mixed"]
    same = np.all(a["exists"] == b["exists"], axis=-1) & np.all(a["u"] == b["u"], axis=(-1, -2))
    assert same.mean() >= 0.9
    sa, sb = a["stats"].astype(np.int64), b["stats"].astype(np.int64)
    assert np.array_equal(sa[[0, 2, 4, 6]], sb[[0, 2, 4, 6]])
    assert np.all(np.abs(sa[[1, 3, 5, 7]] - sb[[1, 3, 5, 7]]) <= 2)
    assert sa[1] > 0 and sa[3] + sa[5] > 0

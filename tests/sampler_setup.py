"""Shared construction of a small sampler problem (tests only).

Data = noise + injected sources around 3 mHz on the 0.25 yr configuration;
the initial state puts jittered copies of the injections into the slots of
every (temperature, walker, band), and builds the odd/even cold-chain buffers
(data minus the cold-chain sources of the bands of that parity) with the
oracle.
"""
import numpy as np

import oracle
from paper_2405_04690_amd import inputs

N = 128


def problem(n_t=3, n_w=4, n_b=6, n_slots=4, n_prop=6, n_friends=4, group_every=1, seed=77, beta_top=0.3, N=N,
            cfg=None, per_band=2, f_band0=3e-3, W=None, edge=False):
    """per_band injections per sub-band, each held by one slot of every chain
    (jittered); cfg defaults to the 0.25 yr configuration; W: sub-band width
    in bins (None: the template width N); edge: the injections' angles on the
    edges of their ranges (cos iota = +-1, sin beta = +-1, phi0 = psi =
    lambda = 0), which the chains' slots then hold exactly"""
    cfg = inputs.TINY if cfg is None else cfg
    orc = oracle.Oracle(T=cfg.T, dt=cfg.dt, L=cfg.L, f_lo=cfg.f_lo, f_hi=cfg.f_hi)
    k_band0 = int(f_band0 * cfg.T)
    sc = oracle.SweepConfig()
    sc.n_temps, sc.n_walkers, sc.n_bands, sc.n_slots = n_t, n_w, n_b, n_slots
    sc.N, sc.n_prop, sc.n_friends, sc.group_every = N, n_prop, n_friends, group_every
    sc.k_band0, sc.stretch_a, sc.seed = k_band0, 2.0, seed
    sc.band_width = 0 if W is None else W
    Wb = N if W is None else W
    lo = (-23.0, 0.0, -1e-16, 0.0, -1.0, 0.0, 0.0, -1.0)
    hi = (-20.5, 0.0, 1e-15, 0.0, 1.0, 0.0, 0.0, 1.0)
    for i in range(8):
        sc.prior_lo[i], sc.prior_hi[i] = lo[i], hi[i]
    st = oracle.SweepState(sc, orc.n_bins)
    rng = np.random.default_rng(seed)
    # injections: per_band per band, loud enough to matter
    src = []
    for b in range(n_b):
        for _ in range(per_band):
            f0 = (k_band0 + (b + rng.uniform(0.1, 0.9)) * Wb) / cfg.T
            src.append([10 ** rng.uniform(-22.0, -21.3), f0, 0.0, rng.uniform(0, 2 * np.pi),
                        np.arccos(rng.uniform(-1, 1)), rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi),
                        np.arcsin(rng.uniform(-1, 1))])
    src = np.array(src)
    if edge:
        for i in range(len(src)):
            src[i, 3] = src[i, 5] = src[i, 6] = 0.0
            src[i, 4] = 0.0 if i % 2 == 0 else np.pi             # cos iota = +1, -1
            src[i, 7] = np.pi / 2 if (i // 2) % 2 == 0 else -np.pi / 2  # sin beta = +1, -1
    S = orc.psd_eval(np.array([cfg.sqrt_oms, cfg.sqrt_acc, cfg.sqrt_oms, cfg.sqrt_acc]))[0]
    data = np.sqrt(S / (4 * orc.df)) * inputs.complex_normals(seed + 1, (2, orc.n_bins))
    orc.scatter_add(src, N, 1.0, data)
    # slots: jittered injections (first per_band slots of each band), the rest empty
    for t in range(n_t):
        for w in range(n_w):
            for b in range(n_b):
                for s in range(per_band):
                    p = src[per_band * b + s]
                    st.u[t, w, b, s] = [np.log10(p[0]) + rng.normal(0, 0.02), p[1] + rng.normal(0, 0.2) / cfg.T,
                                        p[2], p[3], np.cos(p[4]), p[5], p[6], np.sin(p[7])]
                    st.exists[t, w, b, s] = 1
    for w in range(n_w):
        st.inv_psd[w] = 1.0 / S
        for par in (0, 1):
            st.resid[par, w] = data
            occ = [_phys(st.u[0, w, b, s]) for b in range(par, n_b, 2) for s in range(n_slots) if st.exists[0, w, b, s]]
            if occ:
                orc.scatter_add(np.array(occ), N, -1.0, st.resid[par, w])
    ladder = np.geomspace(1.0, beta_top, n_t) if n_t > 1 else np.ones(1)
    st.betas[:] = ladder[None, :]
    st.data = data
    st.src = src
    return cfg, orc, sc, st


def rebuild_buffer(orc, sc, st, par, w):
    """parity-par cold-chain buffer of walker w from scratch: the data minus
    every cold-chain (t = 0) source of the bands with b % 2 == par"""
    buf = st.data.copy()
    for b in range(par, sc.n_bands, 2):
        for s in range(sc.n_slots):
            if st.exists[0, w, b, s]:
                orc.scatter_add(_phys(st.u[0, w, b, s])[None], sc.N, -1.0, buf)
    return buf


def _phys(u):
    return np.array([10 ** u[0], u[1], u[2], u[3], np.arccos(u[4]), u[5], u[6], np.arcsin(u[7])])

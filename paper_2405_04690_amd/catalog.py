"""Cataloging operation (Sec. 4 "Cataloging Operation") on the GPU library.

Every SNR and overlap is computed by the library (`gb_snr`, `gb_overlap`);
this module only builds the candidate pairs and does the group bookkeeping
(integer work) on the host:
  1. keep the templates of every sample whose optimal SNR exceeds snr_min;
  2. for each sample c in turn, its still-ungrouped templates found one group
     each (the control set), and every ungrouped template of the other samples
     joins the control template it overlaps most, when that overlap exceeds
     `threshold`; the overlaps of one round are one batched `gb_overlap` call;
  3. groups whose founders overlap by more than `threshold` are merged;
  4. confidence = number of samples with a member / number of samples.
Two templates of width N can only overlap when their carrier bins differ by
less than N, so only those pairs are evaluated (the others have overlap 0,
below any positive threshold).  Ties in the largest overlap go to the lowest
control index.
"""
from __future__ import annotations

import numpy as np
import torch

from .gbl import Context


def _candidate_pairs(q_test, q_ctrl, N):
    """all (test, control) index pairs with |q_test - q_ctrl| < N"""
    order = np.argsort(q_ctrl, kind="stable")
    qs = q_ctrl[order]
    lo = np.searchsorted(qs, q_test - N + 1, side="left")
    hi = np.searchsorted(qs, q_test + N - 1, side="right")
    counts = hi - lo
    ti = np.repeat(np.arange(len(q_test)), counts)
    starts = np.repeat(lo, counts)
    within = np.arange(counts.sum()) - np.repeat(np.cumsum(counts) - counts, counts)
    ci = order[starts + within]
    return ti, ci


def catalog(ctx: Context, samples, N: int, psd, snr_min: float = 7.0, threshold: float = 0.9, stats=None):
    """samples: list of [n_m][8] parameter arrays; psd: [1, 2, n_bins] S_n on the
    device.  Returns (groups, confidence) as the oracle's catalog: groups are
    lists of (sample, index) pairs ordered by founder, confidence per group.
    stats (dict, optional) receives the number of overlaps evaluated."""
    dev = ctx.device
    M = len(samples)
    arrs = [np.asarray(p, np.float64).reshape(-1, 8) for p in samples]
    sample_of = np.concatenate([np.full(len(a), m, np.int64) for m, a in enumerate(arrs)]) if M else np.zeros(0, int)
    index_in = np.concatenate([np.arange(len(a)) for a in arrs]) if M else np.zeros(0, int)
    allp = np.concatenate(arrs) if M else np.zeros((0, 8))
    n_all = len(allp)
    P = torch.from_numpy(np.ascontiguousarray(allp)).to(dev)
    opt, _ = ctx.gb_snr(P, N, psd)
    keep = (opt.cpu().numpy() > snr_min)
    q = np.floor(allp[:, 1] * ctx.T).astype(np.int64)
    group = np.full(n_all, -1, np.int64)
    founders = []
    n_overlaps = 0
    for c in range(M):
        ctrl = np.nonzero(keep & (sample_of == c) & (group < 0))[0]
        for i in ctrl:
            group[i] = len(founders)
            founders.append(i)
        if len(ctrl) == 0:
            continue
        test = np.nonzero(keep & (sample_of != c) & (group < 0))[0]
        if len(test) == 0:
            continue
        ti, ci = _candidate_pairs(q[test], q[ctrl], N)
        if len(ti) == 0:
            continue
        a = P[torch.from_numpy(test[ti]).to(dev)].contiguous()
        b = P[torch.from_numpy(ctrl[ci]).to(dev)].contiguous()
        ov = ctx.gb_overlap(a, b, N, psd)[:, 3].cpu().numpy()
        n_overlaps += len(ti)
        # per test template: the largest overlap, lowest control index on ties
        srt = np.lexsort((ci, -ov, ti))
        first = np.ones(len(srt), bool)
        first[1:] = ti[srt][1:] != ti[srt][:-1]
        best = srt[first]
        ok = ov[best] > threshold
        group[test[ti[best[ok]]]] = group[ctrl[ci[best[ok]]]]
    # merge groups whose founders overlap above the threshold
    G = len(founders)
    parent = np.arange(G)
    if G > 1:
        fidx = np.array(founders)
        ti, ci = _candidate_pairs(q[fidx], q[fidx], N)
        sel = ti < ci
        ti, ci = ti[sel], ci[sel]
        if len(ti):
            ov = ctx.gb_overlap(P[torch.from_numpy(fidx[ti]).to(dev)].contiguous(),
                                P[torch.from_numpy(fidx[ci]).to(dev)].contiguous(), N, psd)[:, 3].cpu().numpy()
            n_overlaps += len(ti)

            def find(x):
                while parent[x] != x:
                    parent[x] = parent[parent[x]]
                    x = parent[x]
                return x

            for g, h in zip(ti[ov > threshold], ci[ov > threshold]):
                rg, rh = find(g), find(h)
                if rg != rh:
                    parent[max(rg, rh)] = min(rg, rh)
            for g in range(G):
                parent[g] = find(g)
    out = {}
    for i in np.nonzero(group >= 0)[0]:
        out.setdefault(int(parent[group[i]]), []).append((int(sample_of[i]), int(index_in[i])))
    groups = [sorted(out[r]) for r in sorted(out)]
    confidence = [len({m for m, _ in g}) / M for g in groups]
    if stats is not None:
        stats["overlaps"] = n_overlaps
        stats["templates"] = int(n_all)
        stats["kept"] = int(keep.sum())
    return groups, confidence

"""Test infrastructure (the oracle): a plain implementation of the cataloging
operation of Sec. 4 ("Cataloging Operation") for small inputs, on the C
oracle's SNRs and overlaps.  Only tests/, the smoke entry point and the
benchmark's CPU leg may use it.

Steps, in the paper's order:
  1. keep the templates of every sample whose optimal SNR exceeds snr_min (7);
  2. for each sample c in turn: its still-ungrouped templates are the control
     set and found one group each; every ungrouped template of the other
     samples (the test set) joins the group of the control template it has
     the largest overlap with, when that overlap exceeds `threshold` (0.9);
  3. groups whose founding templates overlap by more than `threshold` are
     merged (transitively);
  4. a group's confidence is the number of samples with a member in it
     divided by the number of samples.
Readings where the paper is silent: the overlap is the normalised inner
product of eq. inner over A and E without maximising over phase or time; a
tie in the largest overlap goes to the lowest control index; merging compares
founders.
"""
from __future__ import annotations

import numpy as np


def catalog(orc, samples, N: int, psd, snr_min: float = 7.0, threshold: float = 0.9):
    """samples: list of [n_m][8] parameter arrays (one per MCMC sample).
    Returns (groups, confidence): groups is a list of lists of (sample,
    index) pairs (index into that sample's array), confidence a list of
    floats, both ordered by group founder (sample, index)."""
    M = len(samples)
    psd = np.asarray(psd, np.float64).reshape(-1, 2, orc.n_bins)
    keep = []
    for m, p in enumerate(samples):
        p = np.asarray(p, np.float64).reshape(-1, 8)
        opt, _ = orc.snr(p, N, psd) if len(p) else (np.zeros(0), None)
        keep.append([i for i in range(len(p)) if opt[i] > snr_min])
    grouped = {}             # (m, i) -> group id
    founders = []            # group id -> (m, i)
    members = []             # group id -> list of (m, i)
    for c in range(M):
        control = [(c, i) for i in keep[c] if (c, i) not in grouped]
        for key in control:
            grouped[key] = len(founders)
            founders.append(key)
            members.append([key])
        if not control:
            continue
        ctrl_p = np.array([samples[c][i] for _, i in control], np.float64)
        for m in range(M):
            if m == c:
                continue
            for i in keep[m]:
                if (m, i) in grouped:
                    continue
                test_p = np.repeat(np.asarray(samples[m][i], np.float64)[None], len(control), axis=0)
                ov = orc.overlap(test_p, ctrl_p, N, psd)[:, 3]
                best = -np.inf
                arg = -1
                for j in range(len(control)):   # first maximum wins ties
                    if ov[j] > best:
                        best, arg = ov[j], j
                if best > threshold:
                    g = grouped[control[arg]]
                    grouped[(m, i)] = g
                    members[g].append((m, i))
    # merge groups whose founders overlap above the threshold (union-find)
    G = len(founders)
    parent = list(range(G))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for g in range(G):
        for h in range(g + 1, G):
            pa = np.asarray(samples[founders[g][0]][founders[g][1]], np.float64)[None]
            pb = np.asarray(samples[founders[h][0]][founders[h][1]], np.float64)[None]
            if orc.overlap(pa, pb, N, psd)[0, 3] > threshold:
                rg, rh = find(g), find(h)
                if rg != rh:
                    parent[max(rg, rh)] = min(rg, rh)
    out = {}
    for g in range(G):
        out.setdefault(find(g), []).extend(members[g])
    groups = [sorted(out[r]) for r in sorted(out)]
    confidence = [len({m for m, _ in grp}) / M for grp in groups]
    return groups, confidence

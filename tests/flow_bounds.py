"""Error bound of the BF16-MFMA flow against the FP64 oracle (tests only).

The GPU evaluates the same network as the oracle (same BF16 weights and
embeddings, FP32 biases) but rounds the conditioner inputs x_C and both hidden
activations h1, h2 to bfloat16 (relative error at most u = 2^-8) before each
MFMA, accumulates in FP32 and evaluates SiLU / tanh in FP32.  To first order
the change of ln q is the sum over these rounding points of (d ln q / d h) *
delta h, so

  |ln q_gpu - ln q| <= u * sum_p |g_p| |h_p|  +  g * sum_p |g_p| |h_p|_acc

with g_p the adjoint of ln q at rounding point p (computed here by a
backward pass through the oracle's FP64 activations) and g = 2^-19 covering
FP32 accumulation over at most 128 terms and the FP32 elementwise functions
(|h|_acc = |W| |h_in| + |b| for pre-activations).  The tests allow twice
this first-order bound.
"""
import numpy as np

from oracle import flow

U_BF16 = 2.0 ** -8
G32 = 2.0 ** -19


def oracle_theta(master32: np.ndarray, n_emb: int) -> np.ndarray:
    """the network the GPU evaluates: BF16 weights and embeddings, FP32 biases"""
    th = np.asarray(master32, dtype=np.float32).astype(np.float64)
    layers, E = flow.unpack(th, n_emb)
    for L in layers:
        for k in ("W1", "W2", "W3"):
            L[k][:] = flow.bf16_round(L[k])
    E[:] = flow.bf16_round(E)
    return th


def forward_bound(theta, n_emb, x, band):
    """z, ln q_x (oracle) and the first-order bound on |ln q_gpu - ln q_x| per sample"""
    layers, E = flow.unpack(theta, n_emb)
    e = E[np.asarray(band)]
    y = np.array(x, dtype=np.float64, copy=True)
    ys, caches = [], []
    logdet = np.zeros(y.shape[0])
    for l, L in enumerate(layers):
        kept, moved = flow.masks(l)
        ys.append(y.copy())
        s, t, cache = flow.conditioner(L, y[:, kept], e)
        caches.append((s, t, cache))
        y[:, moved] = y[:, moved] * np.exp(s) + t
        logdet += s.sum(axis=1)
    z = y
    lnq = flow.log_normal(z) + logdet
    bound = np.zeros(z.shape[0])
    gy = -z  # d lnq / d z
    for l in reversed(range(flow.N_LAYERS)):
        L = layers[l]
        kept, moved = flow.masks(l)
        s, t, (h0, a1, h1, a2, h2, o) = caches[l]
        xin = ys[l]
        es = np.exp(s)
        gym = gy[:, moved]
        gs = gym * xin[:, moved] * es + 1.0
        go = np.concatenate([gs * 2.0 * (1.0 - np.tanh(o[:, :4]) ** 2), gym], axis=1)
        acc3 = np.abs(h2) @ np.abs(L["W3"]).T + np.abs(L["b3"])
        bound += G32 * np.sum(np.abs(go) * acc3, axis=1) + G32 * np.sum(np.abs(gs * s), axis=1)
        gh2 = go @ L["W3"]
        bound += (U_BF16 + G32) * np.sum(np.abs(gh2 * h2), axis=1)
        ga2 = gh2 * flow.silu_grad(a2)
        acc2 = np.abs(h1) @ np.abs(L["W2"]).T + np.abs(L["b2"])
        bound += G32 * np.sum(np.abs(ga2) * acc2, axis=1)
        gh1 = ga2 @ L["W2"]
        bound += (U_BF16 + G32) * np.sum(np.abs(gh1 * h1), axis=1)
        ga1 = gh1 * flow.silu_grad(a1)
        acc1 = np.abs(h0) @ np.abs(L["W1"]).T + np.abs(L["b1"])
        bound += G32 * np.sum(np.abs(ga1) * acc1, axis=1)
        gh0 = ga1 @ L["W1"]
        bound += (U_BF16 + G32) * np.sum(np.abs(gh0[:, :4] * h0[:, :4]), axis=1)
        gx = gy.copy()
        gx[:, moved] = gym * es
        gx[:, kept] += gh0[:, :4]
        gy = gx
    return z, lnq, bound

"""FP64 CPU oracle of the learned reversible-jump proposal (a conditional
affine-coupling flow).  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
and the benchmark's CPU-baseline leg may use it; the product path never does.
It shares no code with the HIP library.

The paper fits its RJ proposal distributions (Sec. "Online updating of RJ
sampling distributions"; appendix "Algorithm for fitting proposal
distributions") with Gaussian mixtures and names normalizing flows as the
planned replacement (Discussion, "Single source search-to-parameter
estimation information transfer").  The flow built here is that replacement.
Its form is a reading (the paper gives none):

* coordinates: the sampler's coordinates u = (log10 A, f0, fdot, phi0,
  cos iota, psi, lambda, sin beta) inside the prior box of sub-band b are
  mapped to the real line by x_i = logit((u_i - lo_i) / (hi_i - lo_i));
* six affine coupling layers; layer l keeps the dimensions C_l =
  (0, 2, 4, 6) (l even) or (1, 3, 5, 7) (l odd) and moves the other four:
  y_T = x_T * exp(s) + t, with (s_hat, t) = MLP([x_C, E[b]]), s = 2 tanh(s_hat);
* MLP: 20 -> 128 -> 128 -> 8 with SiLU, E = learned 16-wide embedding of the
  sub-band index b;
* density: ln q_x(x) = sum_i ln N(z_i; 0, 1) + sum over layers of sum(s),
  z = the output of the last layer; ln q_u(u) = ln q_x(x) + sum_i ln|dx_i/du_i|;
* training: the mean of -ln q_x over a batch (the u -> x term does not depend
  on the weights), Adam with bias correction.

Parameter vector layout (float64 here, FP32 master copy on the GPU): for each
layer l = 0..5: W1 [128][20], b1 [128], W2 [128][128], b2 [128], W3 [8][128],
b3 [8] (row-major, output-major); then the embedding E [n_emb][16].
"""
from __future__ import annotations

import numpy as np

D = 8
N_LAYERS = 6
HIDDEN = 128
EMB = 16
COND_IN = 4 + EMB
OUT = 8
LAYER_SIZE = HIDDEN * COND_IN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + OUT * HIDDEN + OUT
LN_2PI = np.log(2.0 * np.pi)


def n_params(n_emb: int) -> int:
    return N_LAYERS * LAYER_SIZE + EMB * n_emb


def masks(l: int):
    """(kept, moved) dimension lists of coupling layer l"""
    even = [0, 2, 4, 6]
    odd = [1, 3, 5, 7]
    return (even, odd) if l % 2 == 0 else (odd, even)


def unpack(theta: np.ndarray, n_emb: int):
    """views of the parameter vector: list of per-layer dicts and E"""
    layers = []
    o = 0

    def take(shape):
        nonlocal o
        n = int(np.prod(shape))
        v = theta[o:o + n].reshape(shape)
        o += n
        return v

    for _ in range(N_LAYERS):
        layers.append({"W1": take((HIDDEN, COND_IN)), "b1": take((HIDDEN,)),
                       "W2": take((HIDDEN, HIDDEN)), "b2": take((HIDDEN,)),
                       "W3": take((OUT, HIDDEN)), "b3": take((OUT,))})
    E = take((n_emb, EMB))
    assert o == theta.size
    return layers, E


def init_params(seed: int, n_emb: int, out_scale: float = 0.0) -> np.ndarray:
    """Seeded initial weights: W1, W2 ~ U(+-1/sqrt(fan_in)), biases 0,
    W3 ~ U(+-out_scale/sqrt(128)) (0: the flow starts as the identity map),
    E ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(n_params(n_emb))
    layers, E = unpack(theta, n_emb)
    for L in layers:
        L["W1"][:] = rng.uniform(-1, 1, L["W1"].shape) / np.sqrt(COND_IN)
        L["W2"][:] = rng.uniform(-1, 1, L["W2"].shape) / np.sqrt(HIDDEN)
        L["W3"][:] = rng.uniform(-1, 1, L["W3"].shape) * out_scale / np.sqrt(HIDDEN)
    E[:] = rng.standard_normal(E.shape)
    return theta


# --------------------------------------------------------------------------
# prior box and the map to the real line
# --------------------------------------------------------------------------
PERIODS = {3: 2 * np.pi, 5: np.pi, 6: 2 * np.pi}


def box(band: np.ndarray, T: float, k_band0: int, width: int, prior_lo, prior_hi):
    """per-sample box [B, 8] (lo, hi): f0 over [k_band0 + (b - 1/2) W,
    k_band0 + (b + 3/2) W) / T, angles over their periods, the rest from the
    prior bounds"""
    band = np.asarray(band)
    lo = np.tile(np.asarray(prior_lo, float), (band.size, 1))
    hi = np.tile(np.asarray(prior_hi, float), (band.size, 1))
    lo[:, 1] = (k_band0 + (band - 0.5) * width) / T
    hi[:, 1] = (k_band0 + (band + 1.5) * width) / T
    for i, P in PERIODS.items():
        lo[:, i] = 0.0
        hi[:, i] = P
    return lo, hi


def to_real(u, lo, hi):
    """x = logit(p), p = (u - lo)/(hi - lo); returns x and sum_i ln|dx_i/du_i|"""
    w = hi - lo
    p = (u - lo) / w
    x = np.log(p) - np.log1p(-p)
    logjac = np.sum(-np.log(w) - np.log(p) - np.log1p(-p), axis=1)
    return x, logjac


def from_real(x, lo, hi):
    p = 1.0 / (1.0 + np.exp(-x))
    u = lo + (hi - lo) * p
    logjac = np.sum(-np.log(hi - lo) - np.log(p) - np.log1p(-p), axis=1)
    return u, logjac


# --------------------------------------------------------------------------
# conditioner and coupling layers
# --------------------------------------------------------------------------
def silu(a):
    return a / (1.0 + np.exp(-a))


def silu_grad(a):
    sg = 1.0 / (1.0 + np.exp(-a))
    return sg * (1.0 + a * (1.0 - sg))


def conditioner(L, xc, e):
    """(s, t, cache) for kept coordinates xc [B, 4] and embeddings e [B, 16]"""
    h0 = np.concatenate([xc, e], axis=1)
    a1 = h0 @ L["W1"].T + L["b1"]
    h1 = silu(a1)
    a2 = h1 @ L["W2"].T + L["b2"]
    h2 = silu(a2)
    o = h2 @ L["W3"].T + L["b3"]
    s = 2.0 * np.tanh(o[:, :4])
    t = o[:, 4:]
    return s, t, (h0, a1, h1, a2, h2, o)


def forward(theta, n_emb, x, band):
    """x [B, 8] -> z [B, 8] and sum of s over the layers [B]"""
    layers, E = unpack(theta, n_emb)
    e = E[np.asarray(band)]
    y = np.array(x, dtype=np.float64, copy=True)
    logdet = np.zeros(y.shape[0])
    for l, L in enumerate(layers):
        kept, moved = masks(l)
        s, t, _ = conditioner(L, y[:, kept], e)
        y[:, moved] = y[:, moved] * np.exp(s) + t
        logdet += s.sum(axis=1)
    return y, logdet


def inverse(theta, n_emb, z, band):
    """z [B, 8] -> x [B, 8] and the sum of s over the layers [B]"""
    layers, E = unpack(theta, n_emb)
    e = E[np.asarray(band)]
    x = np.array(z, dtype=np.float64, copy=True)
    logdet = np.zeros(x.shape[0])
    for l in reversed(range(N_LAYERS)):
        kept, moved = masks(l)
        s, t, _ = conditioner(layers[l], x[:, kept], e)
        x[:, moved] = (x[:, moved] - t) * np.exp(-s)
        logdet += s.sum(axis=1)
    return x, logdet


def log_normal(z):
    return np.sum(-0.5 * z * z - 0.5 * LN_2PI, axis=1)


def log_prob_x(theta, n_emb, x, band):
    z, ld = forward(theta, n_emb, x, band)
    return log_normal(z) + ld


def log_prob_u(theta, n_emb, u, band, lo, hi):
    """ln q_u(u) for sampler coordinates inside the box"""
    x, lj = to_real(u, lo, hi)
    return log_prob_x(theta, n_emb, x, band) + lj


def sample_u(theta, n_emb, z, band, lo, hi):
    """push standard normals z through the inverse flow: u and ln q_u(u)"""
    x, ld = inverse(theta, n_emb, z, band)
    u, lj = from_real(x, lo, hi)
    return u, log_normal(z) + ld + lj


# --------------------------------------------------------------------------
# training: mean negative log-density and its gradient (hand-written backward)
# --------------------------------------------------------------------------
def nll_grad(theta, n_emb, x, band):
    """loss = -mean ln q_x(x) and d loss / d theta"""
    layers, E = unpack(theta, n_emb)
    band = np.asarray(band)
    B = x.shape[0]
    e = E[band]
    grad = np.zeros_like(theta)
    glayers, gE = unpack(grad, n_emb)
    # forward, keeping every layer's input and conditioner cache
    ys = [np.array(x, dtype=np.float64, copy=True)]
    caches = []
    logdet = np.zeros(B)
    for l, L in enumerate(layers):
        kept, moved = masks(l)
        y = ys[-1].copy()
        s, t, cache = conditioner(L, y[:, kept], e)
        y[:, moved] = y[:, moved] * np.exp(s) + t
        logdet += s.sum(axis=1)
        ys.append(y)
        caches.append((s, t, cache))
    z = ys[-1]
    loss = -np.mean(log_normal(z) + logdet)
    # backward
    gy = z / B  # d loss / d z
    for l in reversed(range(N_LAYERS)):
        L, G = layers[l], glayers[l]
        kept, moved = masks(l)
        s, t, (h0, a1, h1, a2, h2, o) = caches[l]
        xin = ys[l]
        es = np.exp(s)
        g_moved = gy[:, moved]
        gx = gy.copy()
        gx[:, moved] = g_moved * es                    # through y_T = x_T e^s + t
        gs = g_moved * xin[:, moved] * es - 1.0 / B    # incl. the log-det term
        gt = g_moved
        go = np.concatenate([gs * 2.0 * (1.0 - np.tanh(o[:, :4]) ** 2), gt], axis=1)
        G["W3"] += go.T @ h2
        G["b3"] += go.sum(axis=0)
        ga2 = (go @ L["W3"]) * silu_grad(a2)
        G["W2"] += ga2.T @ h1
        G["b2"] += ga2.sum(axis=0)
        ga1 = (ga2 @ L["W2"]) * silu_grad(a1)
        G["W1"] += ga1.T @ h0
        G["b1"] += ga1.sum(axis=0)
        gh0 = ga1 @ L["W1"]
        gx[:, kept] += gh0[:, :4]
        np.add.at(gE, band, gh0[:, 4:])
        gy = gx
    return loss, grad


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """one Adam update (step counts from 1); returns new (theta, m, v)"""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """round float64 values to the nearest bfloat16 (ties to even), via float32"""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)

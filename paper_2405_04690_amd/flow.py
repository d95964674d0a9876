"""Binding of the learned RJ proposal (the conditional affine-coupling flow of
include/gbl.h): device buffers and argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .gbl import Context, FlowConfig, FlowState, load_library

__all__ = ["Flow", "FlowConfig", "flow_config", "init_params", "LAYER_PARAMS"]

LAYER_PARAMS = 20232
N_LAYERS, HIDDEN, EMB, COND_IN, OUT = 6, 128, 16, 20, 8


def init_params(seed: int, n_emb: int) -> np.ndarray:
    """Seeded starting weights in the layout of include/gbl.h: W1, W2 uniform in
    +-1/sqrt(fan_in), W3 and all biases zero (the flow starts as the identity
    map, i.e. as a logit-normal proposal), embedding N(0, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(N_LAYERS):
        out.append(rng.uniform(-1, 1, HIDDEN * COND_IN) / np.sqrt(COND_IN))
        out.append(np.zeros(HIDDEN))
        out.append(rng.uniform(-1, 1, HIDDEN * HIDDEN) / np.sqrt(HIDDEN))
        out.append(np.zeros(HIDDEN))
        out.append(np.zeros(OUT * HIDDEN))
        out.append(np.zeros(OUT))
    out.append(rng.standard_normal(EMB * n_emb))
    return np.concatenate(out).astype(np.float32)


def flow_config(n_emb: int, width: int, k_band0: int, prior_lo, prior_hi, prior_weight: float = 0.2) -> FlowConfig:
    """prior_weight: share of prior draws in the sampler's RJ proposal mixture"""
    c = FlowConfig()
    c.n_emb, c.width, c.k_band0 = int(n_emb), int(width), int(k_band0)
    c.prior_weight = float(prior_weight)
    for i in range(8):
        c.prior_lo[i] = float(prior_lo[i])
        c.prior_hi[i] = float(prior_hi[i])
    return c


class Flow:
    """Flow weights (FP32 master, Adam moments, gradient), BF16 fragments and
    the gradient workspace on the context's device."""

    def __init__(self, ctx: Context, cfg: FlowConfig, params=None):
        self.ctx, self.cfg = ctx, cfg
        lib = load_library()
        n, pb, wb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        rc = lib.gb_flow_sizes(ctypes.byref(cfg), ctypes.byref(n), ctypes.byref(pb), ctypes.byref(wb))
        if rc != 0:
            raise ValueError("invalid flow configuration")
        dev = ctx.device
        self.n_params = n.value
        f32 = dict(dtype=torch.float32, device=dev)
        self.params = torch.zeros(self.n_params, **f32)
        self.adam_m = torch.zeros(self.n_params, **f32)
        self.adam_v = torch.zeros(self.n_params, **f32)
        self.grad = torch.zeros(self.n_params, **f32)
        self.packed = torch.zeros(pb.value, dtype=torch.uint8, device=dev)
        self.workspace = torch.zeros(wb.value, dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.step = 0
        if params is not None:
            self.set_params(params)

    def _state(self):
        st = FlowState()
        for k in ("params", "adam_m", "adam_v", "grad", "packed", "workspace", "loss"):
            setattr(st, k, getattr(self, k).data_ptr())
        return st

    def _call(self, name, *args):
        self.ctx._sync_stream()
        rc = getattr(self.ctx.lib, name)(self.ctx._h, ctypes.byref(self.cfg), ctypes.byref(self._state()), *args)
        self.ctx._check(rc, name)

    def set_params(self, params):
        p = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(self.ctx.device)
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self.params.copy_(p)
        self.pack()

    def pack(self):
        self._call("gb_flow_pack")

    def _uband(self, u, band, name):
        u = self.ctx._dev(u, torch.float64, name)
        band = self.ctx._dev(band, torch.int32, "band")
        if u.dim() != 2 or u.shape[1] != 8 or band.shape != (u.shape[0],):
            raise ValueError(f"{name} must be [B, 8] with band [B]")
        return u, band

    def log_prob(self, u, band):
        u, band = self._uband(u, band, "u")
        out = torch.empty(u.shape[0], dtype=torch.float64, device=self.ctx.device)
        self._call("gb_flow_log_prob", ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(band.data_ptr()),
                   u.shape[0], ctypes.c_void_p(out.data_ptr()))
        return out

    def sample(self, z, band):
        z, band = self._uband(z, band, "z")
        u = torch.empty_like(z)
        lq = torch.empty(z.shape[0], dtype=torch.float64, device=self.ctx.device)
        self._call("gb_flow_sample", ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(band.data_ptr()), z.shape[0],
                   ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(lq.data_ptr()))
        return u, lq

    def compute_grad(self, u, band):
        u, band = self._uband(u, band, "u")
        self._call("gb_flow_grad", ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(band.data_ptr()), u.shape[0])
        return self.loss

    def adam(self, lr: float = 1e-3):
        self.step += 1
        self._call("gb_flow_adam", self.step, ctypes.c_float(lr))

    def train_step(self, u, band, lr: float = 1e-3):
        u, band = self._uband(u, band, "u")
        self.step += 1
        self._call("gb_flow_train_step", ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(band.data_ptr()),
                   u.shape[0], self.step, ctypes.c_float(lr))
        return self.loss

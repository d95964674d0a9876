"""Thin Python binding of libgbl.so (the C ABI in include/gbl.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors must be CUDA (HIP) tensors on the context's device; outputs
are allocated here and filled by the library on the current torch stream.
There is no CPU fallback: if libgbl.so is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

from .build import LIB_PATH

GBL_OK = 0
GBL_EINVAL = -1
GBL_EUNSUPPORTED = -2
GBL_EHIP = -3
GBL_FP64 = 0
GBL_MIXED = 1
GBL_PSD_INVERSE = 1
GBL_MIXED_UNROUTED = 1  # config flags
GBL_DETERMINISTIC = 2

SUPPORTED_N = (128, 256, 512, 1024)

EXPORTED = ("gbl_create", "gbl_destroy", "gbl_set_stream", "gbl_last_error", "gbl_band", "gb_waveform",
            "gb_waveform_var", "gb_delta_loglike", "gb_delta_loglike_var", "gb_psd_eval", "gb_psd_loglike",
            "gb_scatter_add", "gb_make_noise", "gb_sweep_step", "gb_sweep_group", "gb_sweep_advance",
            "gb_sweep_run", "gb_sweep_graph_create", "gb_graph_launch", "gb_graph_destroy", "gb_flow_sizes",
            "gb_flow_pack", "gb_flow_log_prob", "gb_flow_sample", "gb_flow_grad", "gb_flow_adam",
            "gb_flow_train_step", "gb_sweep_rj_prepare", "gb_sweep_run_flow", "gb_sweep_graph_create_flow",
            "gbl_get_tuning", "gbl_set_tuning", "gb_psd_sweep_step", "gb_graph_begin", "gb_graph_end",
            "gb_psd_eval_n", "gb_psd_loglike_n", "gb_inner", "gb_snr", "gb_sweep_adapt_ladder",
            "gb_sweep_shift_ownership", "gb_overlap", "gb_search_workspace", "gb_search_eval",
            "gb_search_step", "gb_search_ball", "gb_psd_loglike_noalloc", "gb_noise_matrix",
            "gb_delta_loglike_matrix", "gb_loglike_matrix")

GBL_MOVE_INMODEL, GBL_MOVE_RJ, GBL_MOVE_PT = 0, 1, 2


class GblError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gbl status {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("dt", ctypes.c_double), ("L", ctypes.c_double),
                ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class SweepConfig(ctypes.Structure):
    """gbl_sweep_config"""
    _fields_ = [("n_temps", ctypes.c_int32), ("n_walkers", ctypes.c_int32), ("n_bands", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("N", ctypes.c_int32), ("n_prop", ctypes.c_int32),
                ("n_friends", ctypes.c_int32), ("group_every", ctypes.c_int32), ("k_band0", ctypes.c_int64),
                ("stretch_a", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("prior_lo", ctypes.c_double * 8), ("prior_hi", ctypes.c_double * 8),
                ("adapt_ladder", ctypes.c_int32), ("shift_ownership", ctypes.c_int32),
                ("adapt_lag", ctypes.c_double), ("adapt_time", ctypes.c_double), ("band_width", ctypes.c_int32)]


class SweepState(ctypes.Structure):
    """gbl_sweep_state (device pointers)"""
    _fields_ = [(n, ctypes.c_void_p) for n in ("u", "exists", "betas", "resid", "inv_psd", "group", "group_count",
                                              "stats", "sweep_counter", "prop_u", "rj_logq", "cold_logl",
                                              "rj_mode", "spec_pool", "pool_flags")] + [("pool_size", ctypes.c_int32),
                                                                                        ("swap_acc", ctypes.c_void_p),
                                                                                        ("window_sums", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """gbl_tuning: launch-shape knobs of a context"""
    _fields_ = [("flow_grid", ctypes.c_int32), ("bucket_chunk", ctypes.c_int32), ("widest_first", ctypes.c_int32),
                ("exact_grids", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PsdSweepConfig(ctypes.Structure):
    """gbl_psd_sweep_config"""
    _fields_ = [("n_tn", ctypes.c_int32), ("n_walkers", ctypes.c_int32), ("n_par", ctypes.c_int32),
                ("stretch_a", ctypes.c_double), ("seed", ctypes.c_uint64), ("prior_lo", ctypes.c_double * 9),
                ("prior_hi", ctypes.c_double * 9)]


class PsdSweepState(ctypes.Structure):
    """gbl_psd_sweep_state (device pointers)"""
    _fields_ = [(n, ctypes.c_void_p) for n in ("theta", "logl", "betas", "data", "resid", "full_resid", "inv_psd",
                                              "work", "res_idx", "stats", "sweep_counter")]


class SearchConfig(ctypes.Structure):
    """gbl_search_config"""
    _fields_ = [("n_bands", ctypes.c_int32), ("n_temps", ctypes.c_int32), ("n_walkers", ctypes.c_int32),
                ("N", ctypes.c_int32), ("width", ctypes.c_int32), ("n_stall", ctypes.c_int32),
                ("k_band0", ctypes.c_int64), ("stretch_a", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("prior_lo", ctypes.c_double * 8), ("prior_hi", ctypes.c_double * 8)]


class SearchState(ctypes.Structure):
    """gbl_search_state (device pointers)"""
    _fields_ = [(n, ctypes.c_void_p) for n in ("u", "logl", "betas", "best_u", "best_logl", "stall", "stats",
                                              "workspace")]


class FlowConfig(ctypes.Structure):
    """gbl_flow_config"""
    _fields_ = [("n_emb", ctypes.c_int32), ("width", ctypes.c_int32), ("k_band0", ctypes.c_int64),
                ("prior_lo", ctypes.c_double * 8), ("prior_hi", ctypes.c_double * 8), ("prior_weight", ctypes.c_double)]


class FlowState(ctypes.Structure):
    """gbl_flow (device pointers)"""
    _fields_ = [(n, ctypes.c_void_p) for n in ("params", "adam_m", "adam_v", "grad", "packed", "workspace", "loss")]


_lib = None


def load_library(path: str = LIB_PATH):
    """dlopen libgbl.so and declare the C signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build the HIP library first (python -m paper_2405_04690_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sigs = {
        "gbl_create": [ctypes.POINTER(vp), ctypes.POINTER(Config), vp],
        "gbl_destroy": [vp],
        "gbl_set_stream": [vp, vp],
        "gbl_band": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "gb_waveform": [vp, vp, i64, i32, dbl, dbl, vp, vp, vp, vp],
        "gb_waveform_var": [vp, vp, vp, vp, i64, vp, vp, vp, vp],
        "gb_delta_loglike": [vp, vp, i32, vp, i32, i32, vp, vp, i32, vp, vp, i64, vp],
        "gb_delta_loglike_var": [vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, i64, vp],
        "gb_psd_eval": [vp, vp, i64, i32, vp],
        "gb_psd_loglike": [vp, vp, i32, vp, vp, i64, vp],
        "gb_psd_eval_n": [vp, vp, i32, i64, i32, vp],
        "gb_psd_loglike_n": [vp, vp, i32, vp, i32, vp, i64, vp],
        "gb_psd_loglike_noalloc": [vp, vp, i32, vp, i32, vp, i64, vp],
        "gb_noise_matrix": [vp, vp, i64, vp],
        "gb_delta_loglike_matrix": [vp, vp, i32, vp, i32, vp, vp, i32, vp, vp, i64, vp],
        "gb_loglike_matrix": [vp, vp, i32, vp, i32, vp, vp, i64, vp],
        "gb_inner": [vp, vp, vp, vp, i32, vp, i32, vp, i32, i32, vp, vp, i64, vp],
        "gb_snr": [vp, vp, i64, i32, vp, i32, i32, vp, vp, i32, vp, vp, vp],
        "gb_overlap": [vp, vp, vp, i32, vp, i32, i32, vp, i64, vp],
        "gb_search_workspace": [ctypes.POINTER(SearchConfig), ctypes.POINTER(i64)],
        "gb_search_eval": [vp, ctypes.POINTER(SearchConfig), ctypes.POINTER(SearchState), vp, vp],
        "gb_search_step": [vp, ctypes.POINTER(SearchConfig), ctypes.POINTER(SearchState), i64, vp, vp],
        "gb_search_ball": [vp, ctypes.POINTER(SearchConfig), ctypes.POINTER(SearchState), i64,
                           ctypes.POINTER(dbl), vp, vp],
        "gb_scatter_add": [vp, vp, i64, i32, dbl, vp, i32, vp],
        "gb_make_noise": [vp, vp, vp, i64, vp],
        "gb_sweep_step": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState), i32, i32],
        "gb_sweep_group": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState)],
        "gb_sweep_advance": [vp, ctypes.POINTER(SweepState)],
        "gb_sweep_adapt_ladder": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState)],
        "gb_sweep_shift_ownership": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState)],
        "gb_sweep_run": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState), i32],
        "gb_sweep_graph_create": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState), i32,
                                  ctypes.POINTER(vp)],
        "gb_graph_launch": [vp],
        "gbl_get_tuning": [vp, ctypes.POINTER(Tuning)],
        "gb_graph_begin": [vp],
        "gb_graph_end": [vp, ctypes.POINTER(vp)],
        "gb_psd_sweep_step": [vp, ctypes.POINTER(PsdSweepConfig), ctypes.POINTER(PsdSweepState)],
        "gbl_set_tuning": [vp, ctypes.POINTER(Tuning)],
        "gb_flow_sizes": [ctypes.POINTER(FlowConfig), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "gb_flow_pack": [vp, ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState)],
        "gb_flow_log_prob": [vp, ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), vp, vp, i64, vp],
        "gb_flow_sample": [vp, ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), vp, vp, i64, vp, vp],
        "gb_flow_grad": [vp, ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), vp, vp, i64],
        "gb_flow_adam": [vp, ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), i64, ctypes.c_float],
        "gb_flow_train_step": [vp, ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), vp, vp, i64, i64,
                               ctypes.c_float],
        "gb_sweep_rj_prepare": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState),
                                ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState)],
        "gb_sweep_run_flow": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState),
                              ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), i32],
        "gb_sweep_graph_create_flow": [vp, ctypes.POINTER(SweepConfig), ctypes.POINTER(SweepState),
                                       ctypes.POINTER(FlowConfig), ctypes.POINTER(FlowState), i32,
                                       ctypes.POINTER(vp)],
        "gb_graph_destroy": [vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.gbl_last_error.argtypes = [vp]
    lib.gbl_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """One library context: a run configuration bound to a device and stream."""

    def __init__(self, T: float, dt: float, L: float = 2.5e9, f_lo: float = 1e-4, f_hi: float = 3e-2,
                 precision: int = GBL_FP64, device=None, stream=None, flags: int = 0):
        self.lib = load_library()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.cfg = Config(T, dt, L, f_lo, f_hi, precision, flags)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            rc = self.lib.gbl_create(ctypes.byref(self._h), ctypes.byref(self.cfg), ctypes.c_void_p(s.cuda_stream))
        if rc != GBL_OK:
            raise GblError(rc, "gbl_create failed")
        kmin, nb = ctypes.c_int64(), ctypes.c_int64()
        self.lib.gbl_band(self._h, ctypes.byref(kmin), ctypes.byref(nb))
        self.k_min, self.n_bins = kmin.value, nb.value
        self.T, self.dt, self.L = T, dt, L
        self.df = 1.0 / T

    def close(self):
        if self._h:
            self.lib.gbl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.lib.gbl_get_tuning(self._h, ctypes.byref(t)), "gbl_get_tuning")
        return t

    def set_tuning(self, **knobs) -> Tuning:
        t = self.get_tuning()
        for k, v in knobs.items():
            if k not in dict(Tuning._fields_):
                raise KeyError(k)
            setattr(t, k, int(v))
        self._check(self.lib.gbl_set_tuning(self._h, ctypes.byref(t)), "gbl_set_tuning")
        return t

    def graph_begin(self):
        """start recording every library call on this context's stream (non-default stream)"""
        self._sync_stream()
        self._check(self.lib.gb_graph_begin(self._h), "gb_graph_begin")

    def graph_end(self) -> "Graph":
        h = ctypes.c_void_p()
        self._check(self.lib.gb_graph_end(self._h, ctypes.byref(h)), "gb_graph_end")
        return Graph(self.lib, h)

    # -- helpers ---------------------------------------------------------
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device)
        self.lib.gbl_set_stream(self._h, ctypes.c_void_p(s.cuda_stream))

    def _check(self, rc: int, what: str):
        if rc != GBL_OK:
            msg = self.lib.gbl_last_error(self._h)
            raise GblError(rc, f"{what}: {msg.decode() if msg else ''}")

    def _dev(self, t, dtype, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _params(self, p, name="params"):
        p = self._dev(p, torch.float64, name)
        if p.dim() != 2 or p.shape[1] != 8:
            raise ValueError(f"{name} must have shape [B, 8]")
        return p

    def _residual(self, r):
        r = self._dev(r, torch.complex128, "residual")
        if r.dim() != 3 or r.shape[1] != 2 or r.shape[2] != self.n_bins:
            raise ValueError(f"residual must have shape [n_res, 2, {self.n_bins}]")
        return r

    # -- C ABI calls -----------------------------------------------------
    def gb_waveform(self, params, N: int, with_T: bool = True):
        params = self._params(params)
        B = params.shape[0]
        kw = dict(device=self.device)
        A = torch.empty((B, N), dtype=torch.complex128, **kw)
        E = torch.empty((B, N), dtype=torch.complex128, **kw)
        Tc = torch.empty((B, N), dtype=torch.complex128, **kw) if with_T else None
        sb = torch.empty(B, dtype=torch.int64, **kw)
        self._sync_stream()
        rc = self.lib.gb_waveform(self._h, _ptr(params), B, int(N), self.T, self.dt, _ptr(A), _ptr(E), _ptr(Tc),
                                  _ptr(sb))
        self._check(rc, "gb_waveform")
        return A, E, Tc, sb

    def gb_waveform_var(self, params, N, with_T: bool = True):
        """Templates of per-template width N[b]; slices packed back to back.

        Returns (A, E, T, start_bin, offsets) with A/E/T flat complex arrays of
        length sum(N) and offsets[b] the first element of template b."""
        params = self._params(params)
        N = self._dev(N, torch.int32, "N")
        B = params.shape[0]
        if N.numel() != B:
            raise ValueError("N must have B entries")
        Nl = N.to(torch.int64)
        # widths outside the supported set occupy no output space
        ok = (Nl == 128) | (Nl == 256) | (Nl == 512) | (Nl == 1024)
        sizes = torch.where(ok, Nl, torch.zeros_like(Nl))
        offsets = torch.cumsum(sizes, 0) - sizes
        total = int(sizes.sum().item()) if B else 0
        kw = dict(device=self.device, dtype=torch.complex128)
        A = torch.empty(max(total, 1), **kw)
        E = torch.empty(max(total, 1), **kw)
        Tc = torch.empty(max(total, 1), **kw) if with_T else None
        sb = torch.empty(B, dtype=torch.int64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_waveform_var(self._h, _ptr(params), _ptr(N), _ptr(offsets), B, _ptr(A), _ptr(E), _ptr(Tc),
                                      _ptr(sb))
        self._check(rc, "gb_waveform_var")
        return A[:total], E[:total], (Tc[:total] if with_T else None), sb, offsets

    def gb_delta_loglike(self, residual, psd, params_old, params_new, N: int, res_idx=None, psd_idx=None,
                         psd_inverse: bool = False, out=None):
        residual = self._residual(residual)
        psd = self._dev(psd, torch.float64, "psd")
        if psd.dim() != 3 or psd.shape[1] != 2 or psd.shape[2] != self.n_bins:
            raise ValueError("psd must have shape [n_psd, 2, n_bins]")
        po = self._params(params_old, "params_old")
        pn = self._params(params_new, "params_new")
        B = po.shape[0]
        if pn.shape[0] != B:
            raise ValueError("params_old and params_new differ in length")
        if res_idx is None:
            res_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        if psd_idx is None:
            psd_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        psd_idx = self._dev(psd_idx, torch.int32, "psd_idx")
        if res_idx.numel() != B or psd_idx.numel() != B:
            raise ValueError("res_idx/psd_idx must have B entries")
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_delta_loglike(self._h, _ptr(residual), residual.shape[0], _ptr(psd), psd.shape[0],
                                       GBL_PSD_INVERSE if psd_inverse else 0, _ptr(po), _ptr(pn), int(N),
                                       _ptr(res_idx), _ptr(psd_idx), B, _ptr(out))
        self._check(rc, "gb_delta_loglike")
        return out

    def gb_delta_loglike_var(self, residual, psd, params_old, params_new, N, res_idx=None, psd_idx=None,
                             psd_inverse: bool = False, out=None):
        """As gb_delta_loglike with a per-pair template width N[b] (int32 tensor)."""
        residual = self._residual(residual)
        psd = self._dev(psd, torch.float64, "psd")
        if psd.dim() != 3 or psd.shape[1] != 2 or psd.shape[2] != self.n_bins:
            raise ValueError("psd must have shape [n_psd, 2, n_bins]")
        po = self._params(params_old, "params_old")
        pn = self._params(params_new, "params_new")
        B = po.shape[0]
        N = self._dev(N, torch.int32, "N")
        if pn.shape[0] != B or N.numel() != B:
            raise ValueError("params_old, params_new and N differ in length")
        if res_idx is None:
            res_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        if psd_idx is None:
            psd_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        psd_idx = self._dev(psd_idx, torch.int32, "psd_idx")
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_delta_loglike_var(self._h, _ptr(residual), residual.shape[0], _ptr(psd), psd.shape[0],
                                           GBL_PSD_INVERSE if psd_inverse else 0, _ptr(po), _ptr(pn), _ptr(N),
                                           _ptr(res_idx), _ptr(psd_idx), B, _ptr(out))
        self._check(rc, "gb_delta_loglike_var")
        return out

    def _noise(self, noise):
        noise = self._dev(noise, torch.float64, "noise")
        if noise.dim() != 2 or noise.shape[1] not in (4, 9):
            raise ValueError("noise must have shape [P, 4] or [P, 9] (with the Galactic foreground)")
        return noise

    def gb_psd_eval(self, noise, inverse: bool = False):
        """S (or 1/S) [P, 2, n_bins] for noise sets [P, 4] or [P, 9]"""
        noise = self._noise(noise)
        P = noise.shape[0]
        S = torch.empty((P, 2, self.n_bins), dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_psd_eval_n(self._h, _ptr(noise), noise.shape[1], P, GBL_PSD_INVERSE if inverse else 0,
                                    _ptr(S))
        self._check(rc, "gb_psd_eval")
        return S

    def gb_psd_loglike(self, residual, noise, res_idx=None):
        residual = self._residual(residual)
        noise = self._noise(noise)
        P = noise.shape[0]
        if res_idx is None:
            res_idx = torch.zeros(P, dtype=torch.int32, device=self.device)
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        out = torch.empty(P, dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_psd_loglike_n(self._h, _ptr(residual), residual.shape[0], _ptr(noise), noise.shape[1],
                                       _ptr(res_idx), P, _ptr(out))
        self._check(rc, "gb_psd_loglike")
        return out

    def gb_inner(self, A, E, start_bin, residual, psd, res_idx=None, psd_idx=None, psd_inverse: bool = False,
                 out=None):
        """[B, 2] = (<h|h>, <R|h>) of stored slices A, E [B, N] starting at start_bin [B]"""
        A = self._dev(A, torch.complex128, "A")
        E = self._dev(E, torch.complex128, "E")
        if A.dim() != 2 or A.shape != E.shape:
            raise ValueError("A and E must have the same shape [B, N]")
        B, N = A.shape
        start_bin = self._dev(start_bin, torch.int64, "start_bin")
        residual = self._residual(residual)
        psd = self._dev(psd, torch.float64, "psd")
        if psd.dim() != 3 or psd.shape[1] != 2 or psd.shape[2] != self.n_bins:
            raise ValueError("psd must have shape [n_psd, 2, n_bins]")
        if res_idx is None:
            res_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        if psd_idx is None:
            psd_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        psd_idx = self._dev(psd_idx, torch.int32, "psd_idx")
        if start_bin.numel() != B or res_idx.numel() != B or psd_idx.numel() != B:
            raise ValueError("start_bin/res_idx/psd_idx must have B entries")
        if out is None:
            out = torch.empty((B, 2), dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_inner(self._h, _ptr(A), _ptr(E), _ptr(start_bin), int(N), _ptr(residual),
                               residual.shape[0], _ptr(psd), psd.shape[0], GBL_PSD_INVERSE if psd_inverse else 0,
                               _ptr(res_idx), _ptr(psd_idx), B, _ptr(out))
        self._check(rc, "gb_inner")
        return out

    def gb_overlap(self, params_a, params_b, N: int, psd, psd_idx=None, psd_inverse: bool = False, out=None):
        """[B, 4] = (<a|a>, <b|b>, <a|b>, normalised overlap) of template pairs"""
        params_a = self._params(params_a, "params_a")
        params_b = self._params(params_b, "params_b")
        if params_a.shape != params_b.shape:
            raise ValueError("params_a and params_b must have the same shape")
        B = params_a.shape[0]
        psd = self._dev(psd, torch.float64, "psd")
        if psd.dim() != 3 or psd.shape[1] != 2 or psd.shape[2] != self.n_bins:
            raise ValueError("psd must have shape [n_psd, 2, n_bins]")
        if psd_idx is None:
            psd_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        psd_idx = self._dev(psd_idx, torch.int32, "psd_idx")
        if out is None:
            out = torch.empty((B, 4), dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_overlap(self._h, _ptr(params_a), _ptr(params_b), int(N), _ptr(psd), psd.shape[0],
                                 GBL_PSD_INVERSE if psd_inverse else 0, _ptr(psd_idx), B, _ptr(out))
        self._check(rc, "gb_overlap")
        return out

    def gb_noise_matrix(self, levels):
        """[P, 5, n_bins]: K_AA, K_EE, Re K_AE, Im K_AE, ln det C for link noise levels [P, 12]"""
        levels = self._dev(levels, torch.float64, "levels")
        if levels.dim() != 2 or levels.shape[1] != 12:
            raise ValueError("levels must have shape [P, 12]")
        P = levels.shape[0]
        out = torch.empty((P, 5, self.n_bins), dtype=torch.float64, device=self.device)
        self._sync_stream()
        self._check(self.lib.gb_noise_matrix(self._h, _ptr(levels), P, _ptr(out)), "gb_noise_matrix")
        return out

    def _kmat(self, K):
        K = self._dev(K, torch.float64, "K")
        if K.dim() != 3 or K.shape[1] != 5 or K.shape[2] != self.n_bins:
            raise ValueError("K must have shape [n_K, 5, n_bins]")
        return K

    def gb_delta_loglike_matrix(self, residual, K, params_old, params_new, N: int, res_idx=None, k_idx=None):
        residual = self._residual(residual)
        K = self._kmat(K)
        po = self._params(params_old, "params_old")
        pn = self._params(params_new, "params_new")
        B = po.shape[0]
        if pn.shape[0] != B:
            raise ValueError("params_old and params_new must have the same length")
        res_idx = torch.zeros(B, dtype=torch.int32, device=self.device) if res_idx is None else res_idx
        k_idx = torch.zeros(B, dtype=torch.int32, device=self.device) if k_idx is None else k_idx
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        k_idx = self._dev(k_idx, torch.int32, "k_idx")
        out = torch.empty(B, dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_delta_loglike_matrix(self._h, _ptr(residual), residual.shape[0], _ptr(K), K.shape[0],
                                              _ptr(po), _ptr(pn), int(N), _ptr(res_idx), _ptr(k_idx), B, _ptr(out))
        self._check(rc, "gb_delta_loglike_matrix")
        return out

    def gb_loglike_matrix(self, residual, K, res_idx=None, k_idx=None, P=None):
        residual = self._residual(residual)
        K = self._kmat(K)
        if P is None:
            P = res_idx.numel() if res_idx is not None else K.shape[0]
        res_idx = torch.zeros(P, dtype=torch.int32, device=self.device) if res_idx is None else res_idx
        k_idx = torch.arange(P, dtype=torch.int32, device=self.device) if k_idx is None else k_idx
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        k_idx = self._dev(k_idx, torch.int32, "k_idx")
        out = torch.empty(P, dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_loglike_matrix(self._h, _ptr(residual), residual.shape[0], _ptr(K), K.shape[0],
                                        _ptr(res_idx), _ptr(k_idx), P, _ptr(out))
        self._check(rc, "gb_loglike_matrix")
        return out

    def gb_snr(self, params, N: int, psd, psd_idx=None, data=None, data_idx=None, psd_inverse: bool = False):
        """(optimal SNR [B], observed SNR [B] or None)"""
        params = self._params(params)
        B = params.shape[0]
        psd = self._dev(psd, torch.float64, "psd")
        if psd.dim() != 3 or psd.shape[1] != 2 or psd.shape[2] != self.n_bins:
            raise ValueError("psd must have shape [n_psd, 2, n_bins]")
        if psd_idx is None:
            psd_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        psd_idx = self._dev(psd_idx, torch.int32, "psd_idx")
        opt = torch.empty(B, dtype=torch.float64, device=self.device)
        obs = None
        if data is not None:
            data = self._residual(data)
            if data_idx is None:
                data_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
            data_idx = self._dev(data_idx, torch.int32, "data_idx")
            obs = torch.empty(B, dtype=torch.float64, device=self.device)
        self._sync_stream()
        rc = self.lib.gb_snr(self._h, _ptr(params), B, int(N), _ptr(psd), psd.shape[0],
                             GBL_PSD_INVERSE if psd_inverse else 0, _ptr(psd_idx), _ptr(data),
                             data.shape[0] if data is not None else 0, _ptr(data_idx) if data is not None else None,
                             _ptr(opt), _ptr(obs))
        self._check(rc, "gb_snr")
        return opt, obs

    def gb_scatter_add(self, params, N: int, sign: float, residual, res_idx=None):
        params = self._params(params)
        residual = self._residual(residual)
        B = params.shape[0]
        if res_idx is None:
            res_idx = torch.zeros(B, dtype=torch.int32, device=self.device)
        res_idx = self._dev(res_idx, torch.int32, "res_idx")
        self._sync_stream()
        rc = self.lib.gb_scatter_add(self._h, _ptr(params), B, int(N), float(sign), _ptr(residual),
                                     residual.shape[0], _ptr(res_idx))
        self._check(rc, "gb_scatter_add")
        return residual

    def gb_make_noise(self, S, normals):
        S = self._dev(S, torch.float64, "S")
        normals = self._dev(normals, torch.complex128, "normals")
        if S.shape != normals.shape or S.dim() != 3 or S.shape[1] != 2 or S.shape[2] != self.n_bins:
            raise ValueError("S and normals must both have shape [n, 2, n_bins]")
        out = torch.empty_like(normals)
        self._sync_stream()
        rc = self.lib.gb_make_noise(self._h, _ptr(S), _ptr(normals), S.shape[0], _ptr(out))
        self._check(rc, "gb_make_noise")
        return out


class Graph:
    """an instantiated HIP graph of library calls (gb_graph_end)"""

    def __init__(self, lib, handle):
        self.lib, self.h = lib, handle

    def launch(self):
        rc = self.lib.gb_graph_launch(self.h)
        if rc != GBL_OK:
            raise GblError(rc, "gb_graph_launch")

    def destroy(self):
        if self.h:
            self.lib.gb_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

"""FP64 CPU oracle for the GB template + likelihood hot path (arXiv:2405.04690).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP library.  The C source is ``gbl_oracle.c``; this
module compiles it with gcc and exposes numpy-level wrappers.

Every function follows the paper's statement of the problem (Sec. 2,
eqs. like/inner/addsource/swapsource; Sec. 3, eq. psd) plus the waveform
reading documented in ``gbl_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gbl_oracle.c")
_LIB = os.path.join(_HERE, "libgbl_oracle.so")

C_LIGHT = 299792458.0
AU = 1.495978707e11
YEAR = 31557600.0


def build() -> str:
    """Compile the oracle with gcc (plain -O2; OpenMP over independent templates,
    parameter sets and sampler units, never inside one sum)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Config(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("dt", ctypes.c_double), ("L", ctypes.c_double),
                ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double)]


class SweepConfig(ctypes.Structure):
    """Sampler configuration (field order of gblo_sweep_config)."""
    _fields_ = [("n_temps", ctypes.c_int32), ("n_walkers", ctypes.c_int32), ("n_bands", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("N", ctypes.c_int32), ("n_prop", ctypes.c_int32),
                ("n_friends", ctypes.c_int32), ("group_every", ctypes.c_int32), ("k_band0", ctypes.c_int64),
                ("stretch_a", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("prior_lo", ctypes.c_double * 8), ("prior_hi", ctypes.c_double * 8),
                ("adapt_ladder", ctypes.c_int32), ("shift_ownership", ctypes.c_int32),
                ("adapt_lag", ctypes.c_double), ("adapt_time", ctypes.c_double), ("band_width", ctypes.c_int32)]


class SearchConfig(ctypes.Structure):
    """Per-sub-band search configuration (field order of gblo_search_config)."""
    _fields_ = [("n_bands", ctypes.c_int32), ("n_temps", ctypes.c_int32), ("n_walkers", ctypes.c_int32),
                ("N", ctypes.c_int32), ("width", ctypes.c_int32), ("n_stall", ctypes.c_int32),
                ("k_band0", ctypes.c_int64), ("stretch_a", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("prior_lo", ctypes.c_double * 8), ("prior_hi", ctypes.c_double * 8)]


MOVE_INMODEL, MOVE_RJ, MOVE_PT = 0, 1, 2
MOVE_PSD, MOVE_PSDPT = 4, 5


class PsdSweepConfig(ctypes.Structure):
    """Noise-PSD step configuration (field order of gblo_psd_sweep_config);
    n_par = 4 (instrument noise) or 9 (with the Galactic foreground)."""
    _fields_ = [("n_tn", ctypes.c_int32), ("n_walkers", ctypes.c_int32), ("n_par", ctypes.c_int32),
                ("stretch_a", ctypes.c_double), ("seed", ctypes.c_uint64), ("prior_lo", ctypes.c_double * 9),
                ("prior_hi", ctypes.c_double * 9)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I32 = ctypes.POINTER(ctypes.c_int32)
        I64 = ctypes.POINTER(ctypes.c_int64)
        C = ctypes.POINTER(Config)
        sig = {
            "gblo_set_threads": (ctypes.c_int, [ctypes.c_int]),
            "gblo_band": (ctypes.c_int, [C, I64, I64]),
            "gblo_orbit_position": (None, [C, ctypes.c_int, ctypes.c_double, D]),
            "gblo_source_frame": (None, [D, D, D]),
            "gblo_link_response": (ctypes.c_double, [C, D, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
            "gblo_link_envelope": (None, [C, D, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double, D]),
            "gblo_fft": (ctypes.c_int, [ctypes.c_int, D]),
            "gblo_waveform": (ctypes.c_int, [C, D, ctypes.c_int64, ctypes.c_int, D, D, D, I64]),
            "gblo_psd_value": (ctypes.c_double, [C, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "gblo_psd_eval": (ctypes.c_int, [C, D, ctypes.c_int64, D]),
            "gblo_psd_eval_n": (ctypes.c_int, [C, D, ctypes.c_int32, ctypes.c_int64, D]),
            "gblo_foreground_value": (ctypes.c_double, [C, ctypes.c_double, D]),
            "gblo_psd_loglike_n": (ctypes.c_int, [C, D, ctypes.c_int32, D, ctypes.c_int32, I32, ctypes.c_int64, D]),
            "gblo_inner": (ctypes.c_int, [C, D, D, I64, ctypes.c_int32, D, ctypes.c_int32, D, ctypes.c_int32,
                                          ctypes.c_int32, I32, I32, ctypes.c_int64, D]),
            "gblo_snr": (ctypes.c_int, [C, D, ctypes.c_int64, ctypes.c_int32, D, ctypes.c_int32, ctypes.c_int32, I32,
                                        D, ctypes.c_int32, I32, D, D]),
            "gblo_overlap": (ctypes.c_int, [C, D, D, ctypes.c_int64, ctypes.c_int32, D, ctypes.c_int32,
                                            ctypes.c_int32, I32, D]),
            "gblo_loglike": (ctypes.c_double, [C, D, D]),
            "gblo_noise_matrix_value": (None, [C, ctypes.c_double, D, D]),
            "gblo_noise_matrix": (ctypes.c_int, [C, D, ctypes.c_int64, D]),
            "gblo_loglike_matrix": (ctypes.c_double, [C, D, D]),
            "gblo_delta_loglike_matrix": (ctypes.c_int, [C, D, ctypes.c_int32, D, ctypes.c_int32, D, D,
                                                         ctypes.c_int32, I32, I32, ctypes.c_int64, D]),
            "gblo_psd_loglike": (ctypes.c_int, [C, D, ctypes.c_int32, D, I32, ctypes.c_int64, D]),
            "gblo_delta_loglike": (ctypes.c_int, [C, D, ctypes.c_int32, D, ctypes.c_int32, ctypes.c_int32, D, D,
                                                  ctypes.c_int32, I32, I32, ctypes.c_int64, D, D]),
            "gblo_scatter_add": (ctypes.c_int, [C, D, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, D,
                                                ctypes.c_int32, I32]),
            "gblo_philox": (None, [ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]),
            "gblo_rng_uniform": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                                   ctypes.c_uint64]),
            "gblo_pt_log_alpha": (ctypes.c_double, [ctypes.c_double] * 6),
            "gblo_sweep_step": (ctypes.c_int, [C, ctypes.POINTER(SweepConfig), ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int64, D, I32, D, D, D, D, I32, I64, D, D, D, I32]),
            "gblo_sweep_adapt_ladder": (ctypes.c_int, [ctypes.POINTER(SweepConfig), ctypes.c_int64, D, I32]),
            "gblo_sweep_shift_ownership": (ctypes.c_int, [C, ctypes.POINTER(SweepConfig), D, I32, D, I64]),
            "gblo_sweep_group": (ctypes.c_int, [ctypes.POINTER(SweepConfig), D, I32, D, I32]),
            "gblo_search_eval": (ctypes.c_int, [C, ctypes.POINTER(SearchConfig), D, D, D, D]),
            "gblo_search_step": (ctypes.c_int, [C, ctypes.POINTER(SearchConfig), ctypes.c_int64, D, D, D, D, D,
                                                D, D, I32, I64]),
            "gblo_search_ball": (ctypes.c_int, [C, ctypes.POINTER(SearchConfig), ctypes.c_int64, D, D, D, D, D,
                                                D, I32]),
            "gblo_stretch_propose": (ctypes.c_int, [ctypes.POINTER(SweepConfig), D, D, ctypes.c_int, ctypes.c_double,
                                                    ctypes.c_double, D, D]),
            "gblo_in_prior": (ctypes.c_int, [C, ctypes.POINTER(SweepConfig), ctypes.c_int, D]),
            "gblo_band_loglike": (ctypes.c_double, [C, ctypes.POINTER(SweepConfig), ctypes.c_int, ctypes.c_int,
                                                    ctypes.c_int, ctypes.c_int, D, I32, D, D]),
            "gblo_psd_sweep_step": (ctypes.c_int, [C, ctypes.POINTER(PsdSweepConfig), ctypes.c_int64, D, D, D, D, D,
                                                   D, I64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


class Oracle:
    """Oracle bound to one run configuration (T, dt, L, band)."""

    def __init__(self, T: float, dt: float, L: float = 2.5e9, f_lo: float = 1e-4, f_hi: float = 3e-2):
        self.lib = _load()
        self.cfg = Config(T, dt, L, f_lo, f_hi)
        kmin = np.zeros(1, np.int64)
        nb = np.zeros(1, np.int64)
        self.lib.gblo_band(ctypes.byref(self.cfg), _i64(kmin), _i64(nb))
        self.k_min = int(kmin[0])
        self.n_bins = int(nb[0])
        self.T, self.dt, self.L = T, dt, L
        self.df = 1.0 / T

    # threads used by the batched calls (OpenMP over templates)
    def set_threads(self, n: int) -> int:
        return int(self.lib.gblo_set_threads(int(n)))

    def orbit_position(self, i: int, t: float) -> np.ndarray:
        x = np.zeros(3)
        self.lib.gblo_orbit_position(ctypes.byref(self.cfg), int(i), float(t), _d(x))
        return x

    def source_frame(self, p):
        p = _f64(p)
        k = np.zeros(3)
        H = np.zeros((3, 3, 2))
        self.lib.gblo_source_frame(_d(p), _d(k), _d(H))
        return k, H[..., 0] + 1j * H[..., 1]

    def link_response(self, p, s: int, r: int, t: float) -> float:
        p = _f64(p)
        return float(self.lib.gblo_link_response(ctypes.byref(self.cfg), _d(p), s, r, float(t)))

    def link_envelope(self, p, q: int, s: int, r: int, t: float) -> complex:
        p = _f64(p)
        out = np.zeros(2)
        self.lib.gblo_link_envelope(ctypes.byref(self.cfg), _d(p), int(q), s, r, float(t), _d(out))
        return complex(out[0], out[1])

    def fft(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.complex128).copy()
        v = x.view(np.float64)
        _check(self.lib.gblo_fft(len(x), _d(v)), "fft")
        return x

    def waveform(self, params, N: int, with_T: bool = True):
        params = _f64(params).reshape(-1, 8)
        B = params.shape[0]
        A = np.zeros((B, N), np.complex128)
        E = np.zeros((B, N), np.complex128)
        Tc = np.zeros((B, N), np.complex128) if with_T else None
        sb = np.zeros(B, np.int64)
        rc = self.lib.gblo_waveform(ctypes.byref(self.cfg), _d(params), B, int(N), _d(A.view(np.float64)),
                                    _d(E.view(np.float64)),
                                    _d(Tc.view(np.float64)) if with_T else None, _i64(sb))
        _check(rc, "waveform")
        return A, E, Tc, sb

    def psd_value(self, f: float, sqrt_oms: float, sqrt_acc: float) -> float:
        return float(self.lib.gblo_psd_value(ctypes.byref(self.cfg), float(f), float(sqrt_oms), float(sqrt_acc)))

    def psd_eval(self, noise) -> np.ndarray:
        noise = _f64(noise).reshape(-1, 4)
        P = noise.shape[0]
        S = np.zeros((P, 2, self.n_bins))
        _check(self.lib.gblo_psd_eval(ctypes.byref(self.cfg), _d(noise), P, _d(S)), "psd_eval")
        return S

    def foreground_value(self, f: float, fg) -> float:
        fg = _f64(fg)
        return float(self.lib.gblo_foreground_value(ctypes.byref(self.cfg), float(f), _d(fg)))

    def psd_eval_n(self, noise, n_par: int) -> np.ndarray:
        """S [P][2][n_bins] for noise sets of 4 or 9 (with the foreground) parameters"""
        noise = _f64(noise).reshape(-1, n_par)
        P = noise.shape[0]
        S = np.zeros((P, 2, self.n_bins))
        _check(self.lib.gblo_psd_eval_n(ctypes.byref(self.cfg), _d(noise), int(n_par), P, _d(S)), "psd_eval_n")
        return S

    def psd_loglike_n(self, residual, noise, n_par: int, res_idx) -> np.ndarray:
        residual = np.ascontiguousarray(residual, dtype=np.complex128).reshape(-1, 2, self.n_bins)
        noise = _f64(noise).reshape(-1, n_par)
        res_idx = np.ascontiguousarray(res_idx, dtype=np.int32)
        out = np.zeros(noise.shape[0])
        rc = self.lib.gblo_psd_loglike_n(ctypes.byref(self.cfg), _d(residual.view(np.float64)), residual.shape[0],
                                         _d(noise), int(n_par), _i32(res_idx), noise.shape[0], _d(out))
        _check(rc, "psd_loglike_n")
        return out

    def inner(self, A, E, start_bin, residual, psd, res_idx=None, psd_idx=None, psd_is_inverse=False):
        """[B][2] = (<h|h>, <R|h>) of stored slices A, E [B][N] starting at start_bin [B]"""
        A = np.ascontiguousarray(A, np.complex128)
        E = np.ascontiguousarray(E, np.complex128)
        B, N = A.shape
        sb = np.ascontiguousarray(start_bin, np.int64)
        residual = np.ascontiguousarray(residual, dtype=np.complex128).reshape(-1, 2, self.n_bins)
        psd = _f64(psd).reshape(-1, 2, self.n_bins)
        res_idx = np.zeros(B, np.int32) if res_idx is None else np.ascontiguousarray(res_idx, np.int32)
        psd_idx = np.zeros(B, np.int32) if psd_idx is None else np.ascontiguousarray(psd_idx, np.int32)
        out = np.zeros((B, 2))
        rc = self.lib.gblo_inner(ctypes.byref(self.cfg), _d(A.view(np.float64)), _d(E.view(np.float64)), _i64(sb),
                                 int(N), _d(residual.view(np.float64)), residual.shape[0], _d(psd), psd.shape[0],
                                 int(bool(psd_is_inverse)), _i32(res_idx), _i32(psd_idx), B, _d(out))
        _check(rc, "inner")
        return out

    def snr(self, params, N: int, psd, psd_idx=None, data=None, data_idx=None, psd_is_inverse=False):
        """(optimal SNR [B], observed SNR [B] or None)"""
        params = _f64(params).reshape(-1, 8)
        B = params.shape[0]
        psd = _f64(psd).reshape(-1, 2, self.n_bins)
        psd_idx = np.zeros(B, np.int32) if psd_idx is None else np.ascontiguousarray(psd_idx, np.int32)
        opt = np.zeros(B)
        obs = np.zeros(B) if data is not None else None
        if data is not None:
            data = np.ascontiguousarray(data, dtype=np.complex128).reshape(-1, 2, self.n_bins)
            data_idx = np.zeros(B, np.int32) if data_idx is None else np.ascontiguousarray(data_idx, np.int32)
        rc = self.lib.gblo_snr(ctypes.byref(self.cfg), _d(params), B, int(N), _d(psd), psd.shape[0],
                               int(bool(psd_is_inverse)), _i32(psd_idx),
                               _d(data.view(np.float64)) if data is not None else None,
                               data.shape[0] if data is not None else 0,
                               _i32(data_idx) if data is not None else None, _d(opt),
                               _d(obs) if obs is not None else None)
        _check(rc, "snr")
        return opt, obs

    def overlap(self, params_a, params_b, N: int, psd, psd_idx=None, psd_is_inverse=False):
        """[B][4] = (<a|a>, <b|b>, <a|b>, normalised overlap) of template pairs"""
        pa = _f64(params_a).reshape(-1, 8)
        pb = _f64(params_b).reshape(-1, 8)
        assert pa.shape == pb.shape
        B = pa.shape[0]
        psd = _f64(psd).reshape(-1, 2, self.n_bins)
        psd_idx = np.zeros(B, np.int32) if psd_idx is None else np.ascontiguousarray(psd_idx, np.int32)
        out = np.zeros((B, 4))
        rc = self.lib.gblo_overlap(ctypes.byref(self.cfg), _d(pa), _d(pb), B, int(N), _d(psd), psd.shape[0],
                                   int(bool(psd_is_inverse)), _i32(psd_idx), _d(out))
        _check(rc, "overlap")
        return out

    def noise_matrix_value(self, f: float, levels) -> np.ndarray:
        """(K_AA, K_EE, Re K_AE, Im K_AE, ln det C) at frequency f for 12 link noise levels"""
        levels = _f64(levels)
        out = np.zeros(5)
        self.lib.gblo_noise_matrix_value(ctypes.byref(self.cfg), float(f), _d(levels), _d(out))
        return out

    def noise_matrix(self, levels) -> np.ndarray:
        """[P][5][n_bins] inverse channel covariance and ln det for level sets [P][12]"""
        levels = _f64(levels).reshape(-1, 12)
        out = np.zeros((levels.shape[0], 5, self.n_bins))
        _check(self.lib.gblo_noise_matrix(ctypes.byref(self.cfg), _d(levels), levels.shape[0], _d(out)),
               "noise_matrix")
        return out

    def loglike_matrix(self, R, K) -> float:
        R = np.ascontiguousarray(R, dtype=np.complex128).reshape(2, self.n_bins)
        K = _f64(K).reshape(5, self.n_bins)
        return float(self.lib.gblo_loglike_matrix(ctypes.byref(self.cfg), _d(R.view(np.float64)), _d(K)))

    def delta_loglike_matrix(self, residual, K, params_old, params_new, N: int, res_idx=None, k_idx=None):
        residual = np.ascontiguousarray(residual, dtype=np.complex128).reshape(-1, 2, self.n_bins)
        K = _f64(K).reshape(-1, 5, self.n_bins)
        po = _f64(params_old).reshape(-1, 8)
        pn = _f64(params_new).reshape(-1, 8)
        B = po.shape[0]
        res_idx = np.zeros(B, np.int32) if res_idx is None else np.ascontiguousarray(res_idx, np.int32)
        k_idx = np.zeros(B, np.int32) if k_idx is None else np.ascontiguousarray(k_idx, np.int32)
        out = np.zeros(B)
        rc = self.lib.gblo_delta_loglike_matrix(ctypes.byref(self.cfg), _d(residual.view(np.float64)),
                                                residual.shape[0], _d(K), K.shape[0], _d(po), _d(pn), int(N),
                                                _i32(res_idx), _i32(k_idx), B, _d(out))
        _check(rc, "delta_loglike_matrix")
        return out

    def loglike(self, R, S) -> float:
        R = np.ascontiguousarray(R, dtype=np.complex128).reshape(2, self.n_bins)
        S = _f64(S).reshape(2, self.n_bins)
        return float(self.lib.gblo_loglike(ctypes.byref(self.cfg), _d(R.view(np.float64)), _d(S)))

    def psd_loglike(self, residual, noise, res_idx) -> np.ndarray:
        residual = np.ascontiguousarray(residual, dtype=np.complex128).reshape(-1, 2, self.n_bins)
        noise = _f64(noise).reshape(-1, 4)
        res_idx = np.ascontiguousarray(res_idx, dtype=np.int32)
        P = noise.shape[0]
        out = np.zeros(P)
        rc = self.lib.gblo_psd_loglike(ctypes.byref(self.cfg), _d(residual.view(np.float64)), residual.shape[0],
                                       _d(noise), _i32(res_idx), P, _d(out))
        _check(rc, "psd_loglike")
        return out

    def delta_loglike(self, residual, psd, params_old, params_new, N: int, res_idx=None, psd_idx=None,
                      psd_is_inverse: bool = False, return_terms: bool = False):
        residual = np.ascontiguousarray(residual, dtype=np.complex128).reshape(-1, 2, self.n_bins)
        psd = _f64(psd).reshape(-1, 2, self.n_bins)
        po = _f64(params_old).reshape(-1, 8)
        pn = _f64(params_new).reshape(-1, 8)
        B = po.shape[0]
        if res_idx is None:
            res_idx = np.zeros(B, np.int32)
        if psd_idx is None:
            psd_idx = np.zeros(B, np.int32)
        res_idx = np.ascontiguousarray(res_idx, dtype=np.int32)
        psd_idx = np.ascontiguousarray(psd_idx, dtype=np.int32)
        out = np.zeros(B)
        terms = np.zeros((B, 6))
        rc = self.lib.gblo_delta_loglike(ctypes.byref(self.cfg), _d(residual.view(np.float64)), residual.shape[0],
                                         _d(psd), psd.shape[0], int(bool(psd_is_inverse)), _d(po), _d(pn), int(N),
                                         _i32(res_idx), _i32(psd_idx), B, _d(out), _d(terms))
        _check(rc, "delta_loglike")
        return (out, terms) if return_terms else out

    def scatter_add(self, params, N: int, sign: float, residual, res_idx=None):
        """In place: residual[res_idx[b]] += sign * template b (A, E)."""
        params = _f64(params).reshape(-1, 8)
        B = params.shape[0]
        assert residual.dtype == np.complex128 and residual.flags.c_contiguous
        res3 = residual.reshape(-1, 2, self.n_bins)
        if res_idx is None:
            res_idx = np.zeros(B, np.int32)
        res_idx = np.ascontiguousarray(res_idx, dtype=np.int32)
        rc = self.lib.gblo_scatter_add(ctypes.byref(self.cfg), _d(params), B, int(N), float(sign),
                                       _d(res3.view(np.float64)), res3.shape[0], _i32(res_idx))
        _check(rc, "scatter_add")
        return residual


def philox(ctr, key):
    """Philox4x64-10 block for a 4-word counter and 2-word key."""
    lib = _load()
    c = (ctypes.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib.gblo_philox(c, k, o)
    return [int(x) for x in o]


def rng_uniform(seed, sweep, move, unit, idx):
    return float(_load().gblo_rng_uniform(int(seed), int(sweep), int(move), int(unit), int(idx)))


def pt_log_alpha(bI, bII, lnL_im, lnL_in, lnL_jn, lnL_jm):
    return float(_load().gblo_pt_log_alpha(bI, bII, lnL_im, lnL_in, lnL_jn, lnL_jm))


class SweepState:
    """Host arrays of the sampler state (layouts as documented in gbl_oracle.c)."""

    def __init__(self, sc: SweepConfig, n_bins: int):
        nt, nw, nb, ns = sc.n_temps, sc.n_walkers, sc.n_bands, sc.n_slots
        self.u = np.zeros((nt, nw, nb, ns, 8))
        self.exists = np.zeros((nt, nw, nb, ns), np.int32)
        self.betas = np.ones((nb, nt))
        self.resid = np.zeros((2, nw, 2, n_bins), np.complex128)
        self.inv_psd = np.zeros((nw, 2, n_bins))
        self.group = np.zeros((nb, nw * ns, 8))
        self.group_count = np.zeros(nb, np.int32)
        self.stats = np.zeros(10, np.int64)              # [8], [9]: ownership shifts (moved, no free slot)
        self.swap_acc = np.zeros((nb, nt), np.int32)   # accepted swaps of rungs (t-1, t) since the last adaptation


def sweep_step(orc: "Oracle", sc: SweepConfig, st: SweepState, move: int, parity: int, sweep: int,
               prop_u=None, rj_logq=None, cold_logl=None):
    """One move over the bands of one parity.  prop_u [n_t][n_w][n_b][n_slot][8]
    and rj_logq [n_t][n_w][n_b][n_slot] give an RJ proposal (None: the prior);
    cold_logl [n_w][n_b] receives the cold chain's band logL after tempering;
    tempering also counts its accepted swaps per band and rung in st.swap_acc."""
    pu_a = np.ascontiguousarray(prop_u, np.float64) if prop_u is not None else None
    lq_a = np.ascontiguousarray(rj_logq, np.float64) if rj_logq is not None else None
    pu = _d(pu_a) if pu_a is not None else None
    lq = _d(lq_a) if lq_a is not None else None
    if cold_logl is not None:
        assert cold_logl.dtype == np.float64 and cold_logl.flags.c_contiguous
    rc = orc.lib.gblo_sweep_step(ctypes.byref(orc.cfg), ctypes.byref(sc), int(move), int(parity), int(sweep),
                                 _d(st.u), _i32(st.exists), _d(st.betas), _d(st.resid.view(np.float64)),
                                 _d(st.inv_psd), _d(st.group), _i32(st.group_count), _i64(st.stats), pu, lq,
                                 _d(cold_logl) if cold_logl is not None else None, _i32(st.swap_acc))
    _check(rc, "sweep_step")


def adapt_ladder(sc: SweepConfig, st: SweepState, sweep: int):
    """each band's ladder from the swap acceptance counted since the last call
    (Vousden-Farr-Mandel gap dynamics); clears st.swap_acc"""
    rc = _load().gblo_sweep_adapt_ladder(ctypes.byref(sc), int(sweep), _d(st.betas), _i32(st.swap_acc))
    _check(rc, "sweep_adapt_ladder")


def shift_ownership(orc: "Oracle", sc: SweepConfig, st: SweepState, stats=None):
    """cold-chain sources whose f0 left their band move to the neighbouring band
    (lowest free slot), buffers updated; stats [2]: moved, no free slot"""
    if stats is not None:
        assert stats.dtype == np.int64 and stats.flags.c_contiguous
    rc = orc.lib.gblo_sweep_shift_ownership(ctypes.byref(orc.cfg), ctypes.byref(sc), _d(st.u), _i32(st.exists),
                                            _d(st.resid.view(np.float64)),
                                            _i64(stats) if stats is not None else None)
    _check(rc, "sweep_shift_ownership")


def sweep_group(sc: SweepConfig, st: SweepState):
    rc = _load().gblo_sweep_group(ctypes.byref(sc), _d(st.u), _i32(st.exists), _d(st.group), _i32(st.group_count))
    _check(rc, "sweep_group")


def stretch_propose(sc: SweepConfig, u, group, uf: float, uz: float):
    """Group-stretch proposal from u with friend uniform uf and stretch uniform uz
    against the sorted group [G][8]: (ok, u_new, ln proposal factor)."""
    u = _f64(u)
    group = _f64(group).reshape(-1, 8)
    un = np.zeros(8)
    lr = np.zeros(1)
    ok = _load().gblo_stretch_propose(ctypes.byref(sc), _d(u), _d(group), group.shape[0], float(uf), float(uz),
                                      _d(un), _d(lr))
    return bool(ok), un, float(lr[0])


def in_prior(orc: "Oracle", sc: SweepConfig, b: int, u) -> bool:
    u = _f64(u)
    return bool(orc.lib.gblo_in_prior(ctypes.byref(orc.cfg), ctypes.byref(sc), int(b), _d(u)))


def band_loglike(orc: "Oracle", sc: SweepConfig, st: SweepState, t: int, w_src: int, b: int, w_res: int) -> float:
    """-1/2 <r'|r'> over the window of band b: r' = walker w_res's opposite-parity
    cold-chain buffer minus the sources of (t, w_src, b) (Alg. gb2)."""
    return float(orc.lib.gblo_band_loglike(ctypes.byref(orc.cfg), ctypes.byref(sc), int(t), int(w_src), int(b),
                                           int(w_res), _d(st.u), _i32(st.exists), _d(st.resid.view(np.float64)),
                                           _d(st.inv_psd)))


def sweep_full(orc: "Oracle", sc: SweepConfig, st: SweepState, sweep: int):
    """One full sweep in the library's order: group refresh (when due),
    in-model (odd, even), RJ (odd, even), tempering (odd, even), then the
    ladder adaptation and the ownership shift when the configuration asks."""
    if sc.group_every > 0 and sweep % sc.group_every == 0:
        sweep_group(sc, st)
    for move in (MOVE_INMODEL, MOVE_RJ, MOVE_PT):
        for parity in (1, 0):
            sweep_step(orc, sc, st, move, parity, sweep)
    if sc.adapt_ladder:
        adapt_ladder(sc, st, sweep)
    if sc.shift_ownership:
        shift_ownership(orc, sc, st, st.stats[8:])


def psd_sweep_step(orc: "Oracle", pc: PsdSweepConfig, sweep: int, theta, logl, betas, data, resid, inv_psd, stats):
    """Noise-PSD step (stretch moves with vertical tempering) on host arrays, in place:
    theta [n_tn][n_w][n_par], logl [n_tn][n_w], betas [n_tn], data [2][n_bins] complex,
    resid [2][n_w][2][n_bins] complex (the sweep's cold-chain buffers), inv_psd [n_w][2][n_bins],
    stats [4]."""
    data = np.ascontiguousarray(data, np.complex128)
    resid = np.ascontiguousarray(resid, np.complex128)
    betas = np.ascontiguousarray(betas, np.float64)
    for a, dt in ((theta, np.float64), (logl, np.float64), (inv_psd, np.float64), (stats, np.int64)):
        assert a.dtype == dt and a.flags.c_contiguous
    rc = orc.lib.gblo_psd_sweep_step(ctypes.byref(orc.cfg), ctypes.byref(pc), int(sweep), _d(theta), _d(logl),
                                     _d(betas), _d(data.view(np.float64)), _d(resid.view(np.float64)), _d(inv_psd),
                                     _i64(stats))
    _check(rc, "psd_sweep_step")


class SearchState:
    """Host arrays of the per-sub-band search (layouts of gblo_search_step)."""

    def __init__(self, sc: SearchConfig):
        nb, nt, nw = sc.n_bands, sc.n_temps, sc.n_walkers
        self.u = np.zeros((nb, nt, nw, 8))
        self.logl = np.zeros((nb, nt, nw))
        self.betas = np.ones(nt)
        self.best_u = np.zeros((nb, 8))
        self.best_logl = np.full(nb, -np.inf)
        self.stall = np.zeros(nb, np.int32)
        self.stats = np.zeros(4, np.int64)


def search_eval(orc: "Oracle", sc: SearchConfig, st: SearchState, residual, psd):
    """logl of every chain at its current point (residual [2][n_bins], psd [2][n_bins] = S_n)"""
    residual = np.ascontiguousarray(residual, np.complex128).reshape(2, orc.n_bins)
    psd = _f64(psd).reshape(2, orc.n_bins)
    _check(orc.lib.gblo_search_eval(ctypes.byref(orc.cfg), ctypes.byref(sc), _d(residual.view(np.float64)), _d(psd),
                                    _d(st.u), _d(st.logl)), "search_eval")


def search_step(orc: "Oracle", sc: SearchConfig, st: SearchState, it: int, residual, psd):
    residual = np.ascontiguousarray(residual, np.complex128).reshape(2, orc.n_bins)
    psd = _f64(psd).reshape(2, orc.n_bins)
    rc = orc.lib.gblo_search_step(ctypes.byref(orc.cfg), ctypes.byref(sc), int(it), _d(residual.view(np.float64)),
                                  _d(psd), _d(st.u), _d(st.logl), _d(st.betas), _d(st.best_u), _d(st.best_logl),
                                  _i32(st.stall), _i64(st.stats))
    _check(rc, "search_step")


def search_ball(orc: "Oracle", sc: SearchConfig, st: SearchState, it: int, sigma, residual, psd):
    residual = np.ascontiguousarray(residual, np.complex128).reshape(2, orc.n_bins)
    psd = _f64(psd).reshape(2, orc.n_bins)
    sigma = _f64(sigma)
    rc = orc.lib.gblo_search_ball(ctypes.byref(orc.cfg), ctypes.byref(sc), int(it), _d(sigma),
                                  _d(residual.view(np.float64)), _d(psd), _d(st.u), _d(st.logl), _d(st.best_u),
                                  _i32(st.stall))
    _check(rc, "search_ball")

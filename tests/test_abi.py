"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/gbl.h, and rejects a null context on
the host before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2405_04690_amd import build, gbl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(build.LIB_PATH):
        build.build()
    return gbl.load_library()


def _declared():
    txt = open(os.path.join(ROOT, "include", "gbl.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(gbl?_\w+)\s*\(", txt, re.M)))


def test_header_declares_expected_calls():
    names = _declared()
    assert names == sorted(gbl.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_null_context_rejected_on_host(lib):
    null = None
    assert lib.gbl_set_stream(null, null) == gbl.GBL_EINVAL
    assert lib.gbl_band(null, None, None) == gbl.GBL_EINVAL
    assert lib.gb_waveform(null, null, 1, 256, 1.0, 1.0, null, null, null, null) == gbl.GBL_EINVAL
    assert lib.gb_delta_loglike(null, null, 1, null, 1, 0, null, null, 256, null, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_delta_loglike_var(null, null, 1, null, 1, 0, null, null, null, null, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_waveform_var(null, null, null, null, 1, null, null, null, null) == gbl.GBL_EINVAL
    assert lib.gb_psd_eval(null, null, 1, 0, null) == gbl.GBL_EINVAL
    assert lib.gb_psd_loglike(null, null, 1, null, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_scatter_add(null, null, 1, 256, 1.0, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_make_noise(null, null, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_psd_eval_n(null, null, 9, 1, 0, null) == gbl.GBL_EINVAL
    assert lib.gb_psd_loglike_n(null, null, 1, null, 9, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_inner(null, null, null, null, 256, null, 1, null, 1, 0, null, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_snr(null, null, 1, 256, null, 1, 0, null, null, 0, null, null, null) == gbl.GBL_EINVAL
    assert lib.gbl_destroy(null) == gbl.GBL_OK
    assert lib.gbl_last_error(null) == b"null context"


def test_create_rejects_bad_config_on_host(lib):
    h = ctypes.c_void_p()
    bad = [
        gbl.Config(0.0, 5.0, 2.5e9, 1e-4, 3e-2, 0, 0),      # T <= 0
        gbl.Config(1e7, 5.0, 2.5e9, 3e-2, 1e-4, 0, 0),      # f_hi < f_lo
        gbl.Config(1e7, 50.0, 2.5e9, 1e-4, 3e-2, 0, 0),     # f_hi above Nyquist
        gbl.Config(1e7, 5.0, 2.5e9, 1e-4, 3e-2, 0, 7),      # unknown flags
    ]
    for cfg in bad:
        assert lib.gbl_create(ctypes.byref(h), ctypes.byref(cfg), None) == gbl.GBL_EINVAL
        assert not h.value
    cfg = gbl.Config(1e7, 5.0, 2.5e9, 1e-4, 3e-2, 99, 0)    # unknown precision
    assert lib.gbl_create(ctypes.byref(h), ctypes.byref(cfg), None) == gbl.GBL_EUNSUPPORTED
    assert lib.gbl_create(None, ctypes.byref(cfg), None) == gbl.GBL_EINVAL


def test_null_context_rejected_by_sampler_flow_and_tuning_calls(lib):
    null = None
    assert lib.gbl_get_tuning(null, null) == gbl.GBL_EINVAL
    assert lib.gbl_set_tuning(null, null) == gbl.GBL_EINVAL
    assert lib.gb_sweep_step(null, null, null, 0, 0) == gbl.GBL_EINVAL
    assert lib.gb_sweep_rj_prepare(null, null, null, null, null) == gbl.GBL_EINVAL
    assert lib.gb_sweep_run_flow(null, null, null, null, null, 1) == gbl.GBL_EINVAL
    assert lib.gb_flow_pack(null, null, null) == gbl.GBL_EINVAL
    assert lib.gb_flow_log_prob(null, null, null, null, null, 1, null) == gbl.GBL_EINVAL
    assert lib.gb_flow_train_step(null, null, null, null, null, 1, 1, 1e-3) == gbl.GBL_EINVAL
    cfg = gbl.FlowConfig()
    assert lib.gb_flow_sizes(ctypes.byref(cfg), None, None, None) == gbl.GBL_EINVAL   # n_emb = 0
    cfg.n_emb = 3
    n, pb, wb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert lib.gb_flow_sizes(ctypes.byref(cfg), ctypes.byref(n), ctypes.byref(pb), ctypes.byref(wb)) == gbl.GBL_OK
    assert n.value == 6 * 20232 + 16 * 3 and pb.value == 6 * 92 * 64 * 16

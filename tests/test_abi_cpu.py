"""The C-ABI library loads, exports every symbol include/rtcal.h declares,
and rejects bad arguments on the host with the documented status codes (no
kernel is launched, so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtcal.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(rtc_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (binds the HIP runtime first)
    from paper_2311_18558_amd import lib as rl
    return rl


def test_library_exports_every_declared_symbol(lib):
    so = lib.load()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(so, n), n
    assert set(names) == set(lib.exported_names())


def test_abi_version(lib):
    m = re.search(r"#define RTC_ABI_VERSION (\d+)", open(HEADER).read())
    assert lib.load().rtc_abi_version() == int(m.group(1))


def _radio(lib, n_sc=256, n_elem=4):
    return lib.make_radio(3.5e9, 50e6 / n_sc, n_sc, n_elem)


def test_null_arguments(lib):
    so = lib.load()
    st = so.rtc_cfr(None, None, None, None, None, None, None)
    assert st == -1
    assert b"radio is NULL" in so.rtc_last_error()
    r = _radio(lib)
    st = so.rtc_cfr(ctypes.byref(r), None, None, None, None, None, None)
    assert st == -1 and b"paths is NULL" in so.rtc_last_error()


def test_bad_shapes_and_ranges(lib):
    so = lib.load()
    r = _radio(lib)
    p = lib.Paths()
    p.n_links, p.n_paths, p.max_depth = 1, 1, 9
    st = so.rtc_cfr(ctypes.byref(r), ctypes.byref(p), None, None, None, None, None)
    assert st == -3 and b"max_depth" in so.rtc_last_error()
    bad = lib.make_radio(3.5e9, 1e5, 0, 1)
    st = so.rtc_cfr(ctypes.byref(bad), ctypes.byref(p), None, None, None, None, None)
    assert st == -2 and b"n_sc" in so.rtc_last_error()


def test_loss_needs_power_of_two_and_workspace(lib):
    so = lib.load()
    r = lib.make_radio(3.5e9, 1e5, 200, 1)
    loss = ctypes.c_void_p(16)
    st = so.rtc_cfr_loss(ctypes.byref(r), 4, ctypes.c_void_p(16), ctypes.c_void_p(32), None,
                         None, 1.0, 1.0, loss, None, None, 0, None)
    assert st == -6 and b"power of two" in so.rtc_last_error()
    r = _radio(lib)
    st = so.rtc_cfr_loss(ctypes.byref(r), 4, ctypes.c_void_p(16), ctypes.c_void_p(32), None,
                         None, 1.0, 1.0, loss, None, ctypes.c_void_p(64), 8, None)
    assert st == -4 and b"workspace" in so.rtc_last_error()


def test_noalloc_loss_rejects_batches_beyond_its_scratch(lib):
    """The allocation-free loss checks its size limit on the host (before
    any device work) and says which entry point takes larger batches."""
    so = lib.load()
    max_rows = so.rtc_cfr_loss_noalloc_max_rows()
    assert max_rows == 1 << 19
    r = _radio(lib, n_sc=1024, n_elem=32)
    loss = ctypes.c_void_p(16)
    n_links = max_rows // 32 + 1
    st = so.rtc_cfr_loss_noalloc(ctypes.byref(r), n_links, ctypes.c_void_p(16),
                                 ctypes.c_void_p(32), None, None, 1.0, 1.0, loss, None, None)
    assert st == -3
    msg = so.rtc_last_error()
    assert b"exceed" in msg and b"rtc_cfr_loss" in msg
    r = lib.make_radio(3.5e9, 1e5, 200, 1)
    st = so.rtc_cfr_loss_noalloc(ctypes.byref(r), 4, ctypes.c_void_p(16), ctypes.c_void_p(32),
                                 None, None, 1.0, 1.0, loss, None, None)
    assert st == -6 and b"power of two" in so.rtc_last_error()


def test_materials_mode_checks(lib):
    so = lib.load()
    r = _radio(lib)
    p = lib.Paths()
    p.n_links, p.n_paths, p.max_depth = 1, 1, 0
    p.link_off = p.tx_pos = p.rx_pos = p.depth = p.tau = 16
    m = lib.Materials()
    m.n_mat = 1
    st = so.rtc_trace_fields(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m), None, None, None)
    assert st == -1 and b"exactly one" in so.rtc_last_error()
    m.raw = 16
    m.n_mat = 5000
    st = so.rtc_trace_fields(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m), None, None, None)
    assert st == -3 and b"n_mat" in so.rtc_last_error()


def test_adam_argument_checks(lib):
    so = lib.load()
    st = so.rtc_adam_step(None, None, None, None, 10, 0, 0.01, 0.9, 0.999, 1e-8, None)
    assert st == -1 and b"step" in so.rtc_last_error()
    st = so.rtc_adam_step(None, None, None, None, 10, 1, 0.01, 1.0, 0.999, 1e-8, None)
    assert st == -1 and b"betas" in so.rtc_last_error()
    assert so.rtc_adam_step(None, None, None, None, 0, 1, 0.01, 0.9, 0.999, 1e-8, None) == 0


def test_workspace_sizes(lib):
    r = lib.make_radio(3.5e9, 48828.125, 1024, 32)
    n_loss = lib.workspace_size(lib.RTC_OP_CFR_LOSS, r, 512, 100000)
    assert n_loss >= 512 * 32 * 4 * 8
    n_adj = lib.workspace_size(lib.RTC_OP_CFR_ADJOINT, r, 512, 100000)
    assert n_adj >= 512 * 32 * 16
    assert lib.workspace_size(lib.RTC_OP_TRACE_FIELDS_ADJOINT, r, 512, 100000, 10) > 0
    assert lib.workspace_size(99, r, 1, 1) == 0


def test_paper_loss_argument_checks(lib):
    so = lib.load()
    r = lib.make_radio(3.5e9, 1e5, 200, 1)
    st = so.rtc_cir_stats(ctypes.byref(r), 4, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert st == -6 and b"power of two" in so.rtc_last_error()
    r = _radio(lib)
    st = so.rtc_cir_stats(ctypes.byref(r), 0, ctypes.c_void_p(16), ctypes.c_void_p(32), None)
    assert st == -2 and b"n_links" in so.rtc_last_error()
    st = so.rtc_cir_stats(ctypes.byref(r), 4, None, ctypes.c_void_p(32), None)
    assert st == -1
    p = ctypes.c_void_p(16)
    st = so.rtc_paper_loss(ctypes.byref(r), 4, p, p, p, 1, 1.5, 1.0, 1.0, p, None, None, p,
                           1 << 20, None)
    assert st == -1 and b"delta" in so.rtc_last_error()
    st = so.rtc_paper_loss(ctypes.byref(r), 4, p, p, p, 1, 0.9, 1.0, 1.0, p, None, None, p, 8,
                           None)
    assert st == -4 and b"workspace" in so.rtc_last_error()
    st = so.rtc_paper_loss(ctypes.byref(r), 4, p, None, p, 0, 0.9, 1.0, 1.0, p, None, None, p,
                           1 << 20, None)
    assert st == -1 and b"tgt_stats" in so.rtc_last_error()
    st = so.rtc_eval_ale_rae(3, 0, p, p, None, p, None)
    assert st == -2
    st = so.rtc_eval_ale_rae(3, 2, p, None, None, p, None)
    assert st == -1
    n = lib.workspace_size(lib.RTC_OP_PAPER_LOSS, r, 512, 0)
    assert n >= 512 * 4 * 2 * 8


def test_pattern_argument_checks(lib):
    so = lib.load()
    r = _radio(lib)
    p = lib.Paths()
    p.n_links, p.n_paths, p.max_depth = 1, 1, 0
    p.link_off = p.tx_pos = p.rx_pos = p.depth = p.tau = 16
    m = lib.Materials()
    m.n_mat, m.raw = 2, 16
    pat = lib.Patterns()
    pat.n_vmf = 9
    st = so.rtc_trace_fields_pat(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m),
                                 ctypes.byref(pat), None, None, None)
    assert st == -3 and b"n_vmf" in so.rtc_last_error()
    pat.n_vmf = 2
    st = so.rtc_trace_fields_pat(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m),
                                 ctypes.byref(pat), None, None, None)
    assert st == -1 and b"tx_raw" in so.rtc_last_error()
    pat.n_vmf = 0
    q = ctypes.c_void_p(16)
    # a Tx gradient without a Tx gain
    st = so.rtc_trace_fields_adjoint_pat(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m),
                                         ctypes.byref(pat), q, q, None, q, None, q, 1 << 20, None)
    assert st == -1 and b"dLd_tx" in so.rtc_last_error()
    # pattern gradients without mat_raw, then with per-interaction materials
    st = so.rtc_trace_fields_adjoint_pat(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m),
                                         ctypes.byref(pat), q, q, None, None, q, q, 1 << 20, None)
    assert st == -1 and b"mat_raw" in so.rtc_last_error()
    pat.mat_raw = 16
    mi = lib.Materials()
    mi.n_mat, mi.per_inter = 1, 16
    st = so.rtc_trace_fields_adjoint_pat(ctypes.byref(r), ctypes.byref(p), ctypes.byref(mi),
                                         ctypes.byref(pat), q, None, q, None, q, q, 1 << 20, None)
    assert st == -6 and b"per-id" in so.rtc_last_error()
    # workspace too small for the pattern gradients
    st = so.rtc_trace_fields_adjoint_pat(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m),
                                         ctypes.byref(pat), q, q, None, None, q, q, 8, None)
    assert st == -4 and b"workspace" in so.rtc_last_error()
    n0 = lib.workspace_size(lib.RTC_OP_TRACE_FIELDS_ADJOINT, r, 4, 1000, 3)
    n1 = lib.workspace_size(lib.RTC_OP_TRACE_FIELDS_ADJOINT_PAT, r, 4, 1000, 3)
    assert n1 > n0 > 0


def test_embed_argument_checks(lib):
    so = lib.load()
    q = ctypes.c_void_p(16)
    st = so.rtc_embed_readout(0, 30, q, q, q, None, None)
    assert st == -3 and b"n_mat" in so.rtc_last_error()
    st = so.rtc_embed_readout(3, 1025, q, q, q, None, None)
    assert st == -3 and b"L must" in so.rtc_last_error()
    st = so.rtc_embed_readout(3, 30, None, q, q, None, None)
    assert st == -1
    st = so.rtc_embed_readout(3, 30, q, q, None, None, None)
    assert st == -1 and b"raw" in so.rtc_last_error()
    st = so.rtc_embed_readout_backward(3, 30, q, q, None, None, q, q, None)
    assert st == -1 and b"dLd_raw" in so.rtc_last_error()


def test_compact_rows_argument_check(lib):
    so = lib.load()
    r = _radio(lib)
    p = lib.Paths()
    p.n_links, p.n_paths, p.max_depth = 1, 4, 2
    p.link_off = p.tx_pos = p.rx_pos = p.depth = p.tau = 16
    p.px = p.py = p.pz = p.nx = p.ny = p.nz = p.mat = 16
    m = lib.Materials()
    m.n_mat, m.per_inter, m.inter_idx, m.n_inter = 1, 16, 16, 9
    st = so.rtc_trace_fields(ctypes.byref(r), ctypes.byref(p), ctypes.byref(m), None, None, None)
    assert st == -2 and b"n_inter" in so.rtc_last_error()


def test_validate_argument_checks(lib):
    so = lib.load()
    p = lib.Paths()
    p.n_links, p.n_paths, p.max_depth = 1, 1, 1
    p.link_off = p.tx_pos = p.rx_pos = p.depth = p.tau = 16
    p.px = p.py = p.pz = p.nx = p.ny = p.nz = p.mat = 16
    q = ctypes.c_void_p(16)
    st = so.rtc_validate_paths(ctypes.byref(p), 3, None, q, 1 << 20, None)
    assert st == -1 and b"counts" in so.rtc_last_error()
    st = so.rtc_validate_paths(ctypes.byref(p), 3, q, q, 8, None)
    assert st == -4 and b"workspace" in so.rtc_last_error()
    assert lib.workspace_size(lib.RTC_OP_VALIDATE_PATHS, None, 0, 0, 0) > 0


def test_delay_domain_target_argument_checks(lib):
    """rtc_cfr_target_cir and rtc_cfr_loss_adjoint_cir reject missing or
    aliased targets, non-power-of-two grids, unsupported shapes and short
    workspaces on the host."""
    so = lib.load()
    r = _radio(lib)
    vp = ctypes.c_void_p
    st = so.rtc_cfr_target_cir(ctypes.byref(r), 4, vp(16), vp(32), None, vp(64), 1 << 20, None)
    assert st == -1 and b"X_tgt" in so.rtc_last_error()
    st = so.rtc_cfr_target_cir(ctypes.byref(r), 4, vp(16), vp(32), vp(16), vp(64), 1 << 20, None)
    assert st == -1 and b"alias" in so.rtc_last_error()
    odd = lib.make_radio(3.5e9, 1e5, 200, 4)
    st = so.rtc_cfr_target_cir(ctypes.byref(odd), 4, vp(16), vp(32), vp(48), vp(64), 1 << 20,
                               None)
    assert st == -6 and b"power of two" in so.rtc_last_error()
    st = so.rtc_cfr_target_cir(ctypes.byref(r), 4, vp(16), vp(32), vp(48), vp(64), 8, None)
    assert st == -4 and b"workspace" in so.rtc_last_error()
    # the fused pass with delay-domain targets
    off = (ctypes.c_int64 * 2)(0, 0)
    p = lib.Paths()
    p.n_links, p.n_paths, p.max_depth = 1, 0, 0
    p.link_off = ctypes.cast(off, ctypes.c_void_p)
    st = so.rtc_cfr_loss_adjoint_cir(ctypes.byref(r), ctypes.byref(p), None, None, vp(16), None,
                                     vp(32), 1.0, 1.0, vp(48), None, None, vp(64), 1 << 20, None)
    assert st == -1 and b"X_tgt" in so.rtc_last_error()
    st = so.rtc_cfr_loss_adjoint_cir(ctypes.byref(r), ctypes.byref(p), None, None, vp(16), vp(24),
                                     None, 1.0, 1.0, vp(48), None, None, vp(64), 1 << 20, None)
    assert st == -1 and b"tgt_stats" in so.rtc_last_error()
    big = lib.make_radio(3.5e9, 1e5, 2048, 4)
    st = so.rtc_cfr_loss_adjoint_cir(ctypes.byref(big), ctypes.byref(p), None, None, vp(16),
                                     vp(24), vp(32), 1.0, 1.0, vp(48), None, None, vp(64),
                                     1 << 20, None)
    assert st == -6 and b"rtc_cfr_loss_adjoint_cir" in so.rtc_last_error()
    st = so.rtc_cfr_loss_adjoint_cir(ctypes.byref(r), ctypes.byref(p), None, None, vp(16), vp(24),
                                     vp(32), 1.0, 1.0, vp(48), None, None, vp(64), 8, None)
    assert st == -4 and b"workspace" in so.rtc_last_error()


def test_loss_with_delay_domain_targets_argument_checks(lib):
    """rtc_cfr_loss_cir needs X_tgt, the statistics when it forms dL/dH, a
    power-of-two grid and its workspace, all checked on the host."""
    so = lib.load()
    r = _radio(lib)
    vp = ctypes.c_void_p
    st = so.rtc_cfr_loss_cir(ctypes.byref(r), 4, vp(16), None, vp(32), 1.0, 1.0, vp(48), None,
                             vp(64), 1 << 20, None)
    assert st == -1 and b"X_tgt" in so.rtc_last_error()
    st = so.rtc_cfr_loss_cir(ctypes.byref(r), 4, vp(16), vp(24), None, 1.0, 1.0, vp(48), vp(16),
                             vp(64), 1 << 20, None)
    assert st == -1 and b"tgt_stats" in so.rtc_last_error()
    st = so.rtc_cfr_loss_cir(ctypes.byref(r), 4, vp(16), vp(24), vp(32), 1.0, 1.0, vp(48), vp(24),
                             vp(64), 1 << 20, None)
    assert st == -1 and b"alias" in so.rtc_last_error()
    odd = lib.make_radio(3.5e9, 1e5, 200, 4)
    st = so.rtc_cfr_loss_cir(ctypes.byref(odd), 4, vp(16), vp(24), vp(32), 1.0, 1.0, vp(48),
                             None, vp(64), 1 << 20, None)
    assert st == -6 and b"power of two" in so.rtc_last_error()
    st = so.rtc_cfr_loss_cir(ctypes.byref(r), 4, vp(16), vp(24), vp(32), 1.0, 1.0, vp(48), None,
                             vp(64), 8, None)
    assert st == -4 and b"workspace" in so.rtc_last_error()

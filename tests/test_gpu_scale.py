"""Parity at the full scale workload (16,384 links x 32 elements x 1,024
subcarriers, 3.05 M paths up to fifth order) in the launch configuration the
bench times: every kernel runs over the whole batch and sampled links are
checked one by one against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import channel as och
from oracle.trace import trace_fields_per_id as o_trace_id

pytestmark = pytest.mark.gpu

f64 = torch.float64
c128 = torch.complex128


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scale(gpu_lib):
    from paper_2311_18558_amd import lib
    from synth import workloads
    w = workloads.scale()
    say(f"scale workload: {w.store.n_links} links, {w.store.n_paths} paths")
    rng = np.random.default_rng(2024)
    links = np.sort(rng.choice(w.store.n_links, 12, replace=False))
    return lib, w, links


def _sel(st, links):
    return np.concatenate([np.arange(st.link_off[l], st.link_off[l + 1]) for l in links])


def test_scale_trace_and_cfr_sampled_links(scale):
    rl, w, links = scale
    st, radio = w.store, w.radio
    L, M, N, P = st.n_links, radio.n_elem, radio.n_sc, st.n_paths
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    raw = torch.tensor(w.raw, device="cuda")
    a = torch.empty(P, dtype=torch.complex64, device="cuda")
    psi = torch.empty(P, dtype=torch.float32, device="cuda")
    g = torch.tensor(w.g, device="cuda")
    say("trace_fields + cfr over the whole batch")
    rl.trace_fields(rc, dp, rl.materials_per_id(raw), a, psi)
    H = torch.empty((L, M, N), dtype=torch.complex64, device="cuda")
    rl.cfr(rc, dp, a, psi, g, H)
    torch.cuda.synchronize()
    sel = _sel(st, links)
    a_ref, psi_ref = o_trace_id(st, torch.tensor(w.raw, dtype=f64), radio.fc, sel=sel,
                                ula_axis=radio.ula_axis)
    a_got = a[torch.tensor(sel, device="cuda")].cpu().to(c128)
    off = np.concatenate([[0], np.cumsum(np.diff(st.link_off)[links])])
    worst = 0.0
    for k in range(len(links)):
        lo, hi = off[k], off[k + 1]
        worst = max(worst, (torch.linalg.norm(a_got[lo:hi] - a_ref[lo:hi]) /
                            torch.linalg.norm(a_ref[lo:hi])).item())
    say(f"sampled links: path coefficients max per-link error {worst:.2e}")
    assert worst <= 1e-5
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    H_ref = och.cfr(off, st.tau[sel], a_ref, psi_ref, torch.tensor(w.g, dtype=c128), f)
    H_got = H[torch.tensor(links, device="cuda")].cpu().to(c128)
    err = (torch.linalg.norm((H_got - H_ref).reshape(len(links), -1), dim=1) /
           torch.linalg.norm(H_ref.reshape(len(links), -1), dim=1)).max().item()
    say(f"sampled links: CFR max per-link error {err:.2e}")
    assert err <= 1e-5


def test_scale_cfr_adjoint_sampled_links(scale):
    """dL/dH is random on the sampled links and zero elsewhere; every wave of
    the full launch still runs and the dL/dg reduction spans all of them."""
    rl, w, links = scale
    st, radio = w.store, w.radio
    L, M, N, P = st.n_links, radio.n_elem, radio.n_sc, st.n_paths
    rng = np.random.default_rng(7)
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    a = torch.empty(P, dtype=torch.complex64, device="cuda")
    psi = torch.empty(P, dtype=torch.float32, device="cuda")
    rl.trace_fields(rc, dp, rl.materials_per_id(torch.tensor(w.raw, device="cuda")), a, psi)
    dH_s = (rng.normal(size=(len(links), M, N)) + 1j * rng.normal(size=(len(links), M, N))
            ).astype(np.complex64)
    dH = torch.zeros((L, M, N), dtype=torch.complex64, device="cuda")
    dH[torch.tensor(links, device="cuda")] = torch.tensor(dH_s, device="cuda")
    ws = rl.workspace(rl.RTC_OP_CFR_ADJOINT, rc, L, P)
    dLda = torch.empty(P, dtype=torch.complex64, device="cuda")
    dLdg = torch.empty(M, dtype=torch.complex64, device="cuda")
    say("cfr_adjoint over the whole batch")
    rl.cfr_adjoint(rc, dp, a, psi, torch.tensor(w.g, device="cuda"), dH, dLda, dLdg, ws)
    torch.cuda.synchronize()
    sel = _sel(st, links)
    a64 = a[torch.tensor(sel, device="cuda")].cpu().to(c128).requires_grad_(True)
    g64 = torch.tensor(w.g, dtype=c128, requires_grad=True)
    p64 = psi[torch.tensor(sel, device="cuda")].cpu().double()
    off = np.concatenate([[0], np.cumsum(np.diff(st.link_off)[links])])
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    H = och.cfr(off, st.tau[sel], a64, p64, g64, f)
    da_ref, dg_ref = torch.autograd.grad(H, (a64, g64), grad_outputs=torch.tensor(dH_s).to(c128))
    da = dLda[torch.tensor(sel, device="cuda")].cpu().to(c128)
    worst = 0.0
    for k in range(len(links)):
        lo, hi = off[k], off[k + 1]
        worst = max(worst, (torch.linalg.norm(da[lo:hi] - da_ref[lo:hi]) /
                            torch.linalg.norm(da_ref[lo:hi])).item())
    eg = (torch.linalg.norm(dLdg.cpu().to(c128) - dg_ref) / torch.linalg.norm(dg_ref)).item()
    say(f"sampled links: dL/da max per-link error {worst:.2e}, dL/dg error {eg:.2e}")
    assert worst <= 1e-5 and eg <= 1e-5
    # links without a gradient get exactly zero
    other = np.setdiff1d(np.arange(P), sel)[:100000]
    assert torch.count_nonzero(dLda[torch.tensor(other, device="cuda")]).item() == 0


def test_scale_loss_at_truth_is_zero(scale):
    rl, w, links = scale
    st, radio = w.store, w.radio
    L, M, N, P = st.n_links, radio.n_elem, radio.n_sc, st.n_paths
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    a = torch.empty(P, dtype=torch.complex64, device="cuda")
    psi = torch.empty(P, dtype=torch.float32, device="cuda")
    rl.trace_fields(rc, dp, rl.materials_per_id(torch.tensor(w.raw, device="cuda")), a, psi)
    H = torch.empty((L, M, N), dtype=torch.complex64, device="cuda")
    rl.cfr(rc, dp, a, psi, torch.tensor(w.g, device="cuda"), H)
    ws = rl.workspace(rl.RTC_OP_CFR_LOSS, rc, L, 0)
    stats = torch.empty(2, dtype=torch.float64, device="cuda")
    p_tgt = torch.empty((L, M, N), dtype=torch.float32, device="cuda")
    say("target statistics and loss at the truth over the whole batch")
    rl.cfr_target_stats(rc, L, H, stats, ws, p_tgt=p_tgt)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    dLdH = torch.full_like(H, float("nan"))
    rl.cfr_loss(rc, L, H, H, stats, 1.0, 1.0, loss, dLdH, ws, p_tgt=p_tgt)
    torch.cuda.synchronize()
    # coherent term exactly zero; the PDP term up to rounding of the two
    # kernels' transforms of the same rows
    assert loss[1].item() == 0.0
    assert loss[0].item() <= 1e-10, loss.tolist()
    assert torch.isfinite(dLdH).all()
    # the energy normaliser against a plain FP64 sum of the same tensor (the
    # kernel forms per-lane partials of 16 values in FP32, then FP64)
    zc = (H.abs().double() ** 2).sum().item()
    assert abs(stats[0].item() - zc) <= 1e-6 * zc
    # sampled rows of the target PDP against the oracle's
    rows = H[torch.tensor(links, device="cuda")].cpu().to(c128)
    p_ref = och.pdp(rows)
    p_got = p_tgt[torch.tensor(links, device="cuda")].cpu().double()
    assert (torch.linalg.norm(p_got - p_ref) / torch.linalg.norm(p_ref)).item() <= 1e-5

"""The torch.autograd layer (paper_2311_18558_amd.ops) end to end: a loss
built from the library's Functions, loss.backward(), and the gradients that
reach the leaves compared with the oracle's FP64 autograd gradient.

  per-id:  raw --TraceFields--> a --CFR(g)--> H --CFRLoss--> L
  neural:  params --MaterialMLP--> rows --TraceFieldsPerInteraction--> a
           --CFR(g)--> H --CFRLoss--> L
"""
import sys

import numpy as np
import pytest
import torch

from oracle import channel as och
from oracle import mlp as omlp
from oracle.trace import trace_fields as o_trace
from oracle.trace import trace_fields_per_id
from synth.params import Radio, mlp_init
from tests.helpers import multi_material_box

pytestmark = pytest.mark.gpu
f64 = torch.float64
c128 = torch.complex128
GAINS = np.array([1.0, 0.9 + 0.1j, 1.1 - 0.2j, 0.8j], np.complex64)


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


def _rel(a, b):
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def _setup(seed=8):
    st, raw = multi_material_box(seed=seed, n_rx=12, n_mat=3, max_depth=3)
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=256, n_elem=4)
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    return st, raw, radio, f


@pytest.mark.parametrize("upstream", [1.0, 2.5])
def test_per_id_chain_backward(rl, upstream):
    from paper_2311_18558_amd import ops
    st, raw, radio, f = _setup()
    # target at shifted materials and gains
    raw_t = raw.copy()
    raw_t[:, 0] += np.array([0.3, -0.2, 0.1])
    raw_t[:, 1] += 0.4
    g_t = GAINS * np.exp(1j * 0.2)
    a_t, p_t = trace_fields_per_id(st, torch.tensor(raw_t, dtype=f64), radio.fc)
    Ht = och.cfr(st.link_off, st.tau, a_t, p_t, torch.tensor(g_t, dtype=c128), f)
    # oracle gradient at (raw, GAINS)
    rr = torch.tensor(raw, dtype=f64, requires_grad=True)
    gg = torch.tensor(GAINS, dtype=c128, requires_grad=True)
    a, psi = trace_fields_per_id(st, rr, radio.fc)
    tot_ref, coh_ref, pdp_ref = och.cfr_loss(och.cfr(st.link_off, st.tau, a, psi, gg, f), Ht)
    d_raw_ref, d_g_ref = torch.autograd.grad(upstream * tot_ref, (rr, gg))

    say(f"autograd per-id chain, upstream {upstream}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    raw_d = torch.tensor(raw, device="cuda", requires_grad=True)
    g_d = torch.tensor(GAINS, device="cuda", requires_grad=True)
    a_d, psi_d = ops.TraceFields.apply(raw_d, dp, rc)
    H = ops.CFR.apply(a_d, psi_d, g_d, dp, rc)
    total, terms = ops.CFRLoss.apply(H, Ht.to(torch.complex64).cuda(), rc)
    assert total.requires_grad and not terms.requires_grad
    (upstream * total).backward()
    torch.cuda.synchronize()
    assert abs(total.item() - tot_ref.item()) <= 1e-4 * tot_ref.item()
    assert abs(terms[1].item() - coh_ref.item()) <= 1e-4 * coh_ref.item()
    assert abs(terms[2].item() - pdp_ref.item()) <= 1e-4 * pdp_ref.item()
    e_raw = _rel(raw_d.grad.cpu().double(), d_raw_ref)
    e_g = _rel(g_d.grad.cpu().to(c128), d_g_ref)
    print(f"per-id chain: loss {total.item():.6e} vs {tot_ref.item():.6e}, "
          f"materials {e_raw:.2e}, gains {e_g:.2e}")
    assert e_raw <= 1e-3 and e_g <= 1e-3, (e_raw, e_g)


def test_neural_chain_backward(rl):
    from paper_2311_18558_amd import ops
    st, _, radio, f = _setup(seed=9)
    rng = np.random.default_rng(4)
    params = mlp_init(rng, out_bias=(1.5, -2.5, -1.0))
    box_lo, box_hi = np.zeros(3), np.array([10.0, 8.0, 3.0])
    c = 0.5 * (box_lo + box_hi)
    inv = np.float32(1.0 / np.max(box_hi - box_lo))
    D, P = st.max_depth, st.n_paths
    pts = st.pts.T.astype(np.float64)
    gt = torch.tensor(GAINS, dtype=c128)
    params_gt = mlp_init(np.random.default_rng(98), out_bias=(2.0, -2.0, -1.5))
    (e_t, s_t, S_t), _ = omlp.forward(torch.tensor(params_gt, dtype=f64), torch.tensor(pts), c,
                                      inv, "bf16")
    a_t, p_t = o_trace(st, e_t.reshape(D, P), s_t.reshape(D, P), S_t.reshape(D, P), radio.fc)
    Ht = och.cfr(st.link_off, st.tau, a_t, p_t, gt, f)
    # oracle: BF16-emulating MLP (the kernels' rounding points), FP64 after it
    p64 = torch.tensor(params, dtype=f64)
    (e, s, S), inter = omlp.forward(p64, torch.tensor(pts), c, inv, "bf16")
    ee, ss, SS = (x.detach().clone().requires_grad_(True) for x in (e, s, S))
    gg = gt.clone().requires_grad_(True)
    a, psi = o_trace(st, ee.reshape(D, P), ss.reshape(D, P), SS.reshape(D, P), radio.fc)
    tot_ref, _, _ = och.cfr_loss(och.cfr(st.link_off, st.tau, a, psi, gg, f), Ht)
    de, ds, dS, d_g_ref = torch.autograd.grad(tot_ref, (ee, ss, SS, gg))
    d_prm_ref = omlp.backward(p64, inter, de, ds, dS, mode="bf16")
    d_rows_ref = torch.stack([de, ds, dS])

    say("autograd neural chain")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    prm = torch.tensor(params, device="cuda", requires_grad=True)
    g_d = torch.tensor(GAINS, device="cuda", requires_grad=True)
    pts_d = torch.tensor(st.pts, device="cuda")
    rows = ops.MaterialMLP.apply(prm, pts_d, box_lo, box_hi)
    rows.retain_grad()
    a_d, psi_d = ops.TraceFieldsPerInteraction.apply(rows, dp, rc)
    H = ops.CFR.apply(a_d, psi_d, g_d, dp, rc)
    total, _ = ops.CFRLoss.apply(H, Ht.to(torch.complex64).cuda(), rc)
    total.backward()
    torch.cuda.synchronize()
    assert abs(total.item() - tot_ref.item()) <= 1e-3 * tot_ref.item()
    e_rows = _rel(rows.grad.cpu().double(), d_rows_ref)
    e_prm = _rel(prm.grad.cpu().double(), d_prm_ref)
    e_g = _rel(g_d.grad.cpu().to(c128), d_g_ref)
    print(f"neural chain: loss {total.item():.6e} vs {tot_ref.item():.6e}, per-interaction "
          f"{e_rows:.2e}, MLP {e_prm:.2e}, gains {e_g:.2e}")
    assert e_rows <= 1e-3 and e_prm <= 1e-3 and e_g <= 1e-3, (e_rows, e_prm, e_g)


def test_loss_without_grad_request(rl):
    """A loss on a tensor that does not require a gradient computes no
    dL/dH and returns a detached total."""
    from paper_2311_18558_amd import ops
    st, raw, radio, f = _setup()
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    raw_d = torch.tensor(raw, device="cuda")
    g_d = torch.tensor(GAINS, device="cuda")
    with torch.no_grad():
        a_d, psi_d = ops.TraceFields.apply(raw_d, dp, rc)
        H = ops.CFR.apply(a_d, psi_d, g_d, dp, rc)
    total, terms = ops.CFRLoss.apply(H, H.clone(), rc)
    torch.cuda.synchronize()
    assert not total.requires_grad
    assert total.item() == 0.0 and terms[0].item() == 0.0

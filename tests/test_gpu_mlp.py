"""GPU parity of the neural-material kernels (BF16 MFMA, FP32 accumulate)
against the oracle's BF16-emulation mode (same rounding points), and the
full neural-material chain against the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import channel as och
from oracle import mlp as omlp
from oracle.trace import trace_fields as o_trace
from synth.params import mlp_init
from tests.helpers import multi_material_box

pytestmark = pytest.mark.gpu
f64 = torch.float64
c128 = torch.complex128


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


AABB = (np.array([0.0, 0.0, 0.0]), np.array([60.0, 40.0, 3.0]))


def _rel(a, b):
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


@pytest.mark.parametrize("n_points,seed", [(1000, 0), (37, 1), (65536 + 13, 2)])
def test_mlp_forward_backward_parity(rl, n_points, seed):
    rng = np.random.default_rng(seed)
    params = mlp_init(rng, out_bias=(1.5, -2.5, -1.0))
    pts = rng.uniform(AABB[0], AABB[1], (n_points, 3)).astype(np.float32)
    dout = rng.normal(size=(3, n_points)).astype(np.float32)
    say(f"mlp forward/backward n={n_points}")
    prm_d = torch.tensor(params, device="cuda")
    net = rl.make_mlp(prm_d, *AABB)
    P = torch.tensor(pts.T.copy(), device="cuda")
    out = torch.full((3, n_points), float("nan"), device="cuda")
    saved = rl.mlp_saved(n_points)
    ws = rl.mlp_workspace(n_points)
    rl.mlp_forward(net, n_points, P[0], P[1], P[2], out, saved, ws)
    dprm = torch.full((rl.mlp_n_params(),), float("nan"), device="cuda")
    rl.mlp_backward(net, n_points, torch.tensor(dout, device="cuda"), saved, dprm, ws)
    torch.cuda.synchronize()
    c = 0.5 * (AABB[0] + AABB[1])
    inv = 1.0 / np.max(AABB[1] - AABB[0])
    p64 = torch.tensor(params, dtype=f64)
    (e, s, S), inter = omlp.forward(p64, torch.tensor(pts, dtype=f64), c, np.float32(inv), "bf16")
    (e64, s64, S64), _ = omlp.forward(p64, torch.tensor(pts, dtype=f64), c, inv, "fp64")
    got = out.cpu().double()
    for i, (ref, ref64) in enumerate(((e, e64), (s, s64), (S, S64))):
        err = _rel(got[i], ref)
        print(f"output {i}: rel err vs BF16-emulating oracle {err:.2e}, "
              f"BF16 cost vs FP64 {_rel(ref, ref64):.2e}")
        assert err <= 1e-3, (i, err)
    g_ref = omlp.backward(p64, inter, *(torch.tensor(d, dtype=f64) for d in dout), mode="bf16")
    g = dprm.cpu().double()
    assert torch.isfinite(g).all()
    off = 0
    for li, (o, i) in enumerate(omlp.SHAPES):
        for name, n in (("W", o * i), ("b", o)):
            err = _rel(g[off:off + n], g_ref[off:off + n])
            print(f"layer {li} {name}: rel err {err:.2e}")
            assert err <= 1e-3, (li, name, err)
            off += n


def test_neural_material_chain(rl):
    """points -> MLP -> per-interaction materials -> trace_fields -> cfr ->
    loss -> adjoints -> MLP backward, against the oracle (BF16-emulating
    MLP, FP64 everything else)."""
    st, _ = multi_material_box(seed=8, n_rx=12, n_mat=3, max_depth=3)
    from synth.params import Radio
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=256, n_elem=4)
    rng = np.random.default_rng(3)
    g = np.array([1.0, 0.9 + 0.1j, 1.1 - 0.2j, 0.8j], np.complex64)
    params = mlp_init(rng, out_bias=(1.5, -2.5, -1.0))
    box_lo, box_hi = np.zeros(3), np.array([10.0, 8.0, 3.0])
    c = 0.5 * (box_lo + box_hi)
    inv = np.float32(1.0 / np.max(box_hi - box_lo))
    D, P, L = st.max_depth, st.n_paths, st.n_links
    pts = st.pts.T.astype(np.float64)  # [D*P, 3]
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    gt = torch.tensor(g, dtype=c128)
    # target: ground-truth materials from a second parameter vector
    params_gt = mlp_init(np.random.default_rng(99), out_bias=(2.0, -2.0, -1.5))
    (e_t, s_t, S_t), _ = omlp.forward(torch.tensor(params_gt, dtype=f64), torch.tensor(pts), c, inv, "bf16")
    a_t, p_t = o_trace(st, e_t.reshape(D, P), s_t.reshape(D, P), S_t.reshape(D, P), radio.fc)
    Ht = och.cfr(st.link_off, st.tau, a_t, p_t, gt, f)
    # oracle gradient at params
    p64 = torch.tensor(params, dtype=f64)
    (e, s, S), inter = omlp.forward(p64, torch.tensor(pts), c, inv, "bf16")
    ee, ss, SS = (x.detach().clone().requires_grad_(True) for x in (e, s, S))
    a, psi = o_trace(st, ee.reshape(D, P), ss.reshape(D, P), SS.reshape(D, P), radio.fc)
    H = och.cfr(st.link_off, st.tau, a, psi, gt, f)
    tot, _, _ = och.cfr_loss(H, Ht)
    de, ds, dS = torch.autograd.grad(tot, (ee, ss, SS))
    g_ref = omlp.backward(p64, inter, de, ds, dS, mode="bf16")
    say("neural-material chain")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    prm_d = torch.tensor(params, device="cuda")
    net = rl.make_mlp(prm_d, box_lo, box_hi)
    Q = D * P
    Pd = torch.tensor(st.pts, device="cuda")
    per = torch.empty((3, Q), device="cuda")
    saved = rl.mlp_saved(Q)
    ws = rl.mlp_workspace(Q)
    rl.mlp_forward(net, Q, Pd[0], Pd[1], Pd[2], per, saved, ws)
    mats = rl.materials_per_interaction(per)
    a_d = torch.empty(P, dtype=torch.complex64, device="cuda")
    psi_d = torch.empty(P, dtype=torch.float32, device="cuda")
    rl.trace_fields(rc, dp, mats, a_d, psi_d)
    Hd = torch.empty((L, radio.n_elem, radio.n_sc), dtype=torch.complex64, device="cuda")
    g_d = torch.tensor(g, device="cuda")
    rl.cfr(rc, dp, a_d, psi_d, g_d, Hd)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    rl.cfr_loss(rc, L, Hd, Ht.to(torch.complex64).cuda(), None, 1.0, 1.0, loss, Hd,
                rl.workspace(rl.RTC_OP_CFR_LOSS, rc, L, P))
    dLda = torch.empty(P, dtype=torch.complex64, device="cuda")
    dLdg = torch.empty(radio.n_elem, dtype=torch.complex64, device="cuda")
    rl.cfr_adjoint(rc, dp, a_d, psi_d, g_d, Hd, dLda, dLdg,
                   rl.workspace(rl.RTC_OP_CFR_ADJOINT, rc, L, P))
    dint = torch.empty((3, Q), device="cuda")
    rl.trace_fields_adjoint(rc, dp, mats, dLda, None, dint, None)
    dprm = torch.empty(rl.mlp_n_params(), device="cuda")
    rl.mlp_backward(net, Q, dint, saved, dprm, ws)
    torch.cuda.synchronize()
    assert abs(loss[0].item() - tot.item()) <= 1e-3 * tot.item()
    err = _rel(dprm.cpu().double(), g_ref)
    print(f"neural chain: loss {loss[0].item():.6e} vs {tot.item():.6e}, grad rel err {err:.2e}")
    assert err <= 1e-3, err

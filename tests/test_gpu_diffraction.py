"""First-order edge diffraction (Sec. II-E) through the library against the
FP64 oracle: a single wedge with line-of-sight, face reflections and the
diffracted path around its shadow and reflection boundaries; a floor whose
door jambs and pillar corners diffract, alone, with diffuse paths and with a
trainable Tx gain; coefficients, CFR, and both adjoint modes."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import channel as och
from oracle import patterns as opat
from oracle.trace import trace_fields as o_trace, trace_fields_per_id as o_trace_id
from synth.params import Radio, draw_gains, draw_materials, materials_to_raw
from tests.test_oracle_diffraction import _wedge_links

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


def _wedge_case():
    """Rx on two circles around the wedge, across its shadow (phi' + pi) and
    reflection (pi - phi') boundaries, at oblique heights."""
    phi_p = math.radians(60.0)
    tx = (5.0 * math.cos(phi_p), 5.0 * math.sin(phi_p), 0.3)
    rxs = []
    for r, z in ((4.0, 1.2), (9.0, 2.4)):
        for deg in (20, 70, 110, 119, 121, 150, 200, 235, 239.5, 240.5, 250, 265):
            t = math.radians(deg)
            rxs.append((r * math.cos(t), r * math.sin(t), z))
    st = _wedge_links(rxs, tx)
    st.pts = st.pts.astype(np.float32)
    st.nrm = st.nrm.astype(np.float32)
    st.tx_pos = st.tx_pos.astype(np.float32)
    st.rx_pos = st.rx_pos.astype(np.float32)
    raw = np.array([[math.log(5.0 - 1), math.log(0.05), -2.0],
                    [math.log(3.0 - 1), math.log(0.01), -1.0]], np.float32)
    return st, raw


def _floor(with_diffuse):
    from synth import diffuse
    from synth.diffract import add_diffraction
    from synth.floorplan import indoor_floor
    from synth.pathfind import find_store
    plan = indoor_floor(11, width=14.0, depth=10.0, min_room=4.0, max_rooms=2, open_frac=0.6,
                        n_pillars=1, target_tris=400)
    rng = np.random.default_rng(12)
    tx = plan.sample_points(rng, 1, 2.4, 2.6)[0]
    rx = plan.sample_points(rng, 12, 1.0, 2.0)
    st = find_store(plan, tx, rx, 2, n_rays=1 << 15)
    if with_diffuse:
        samples = diffuse.sample_floor(plan, 0.4, rng)
        st = diffuse.add_diffuse(st, tx, samples,
                                 lambda p, e: diffuse.visible_floor(plan, p, e))
    st = add_diffraction(st, plan)
    raw = materials_to_raw(*draw_materials(rng, plan.scene.n_mat, with_scattering=True))
    return st, raw.astype(np.float32)


def _cases():
    out = {}
    for name, fn in (("wedge", _wedge_case), ("floor", lambda: _floor(False)),
                     ("floor_diffuse", lambda: _floor(True))):
        st, raw = fn()
        rng = np.random.default_rng(len(name))
        radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=256, n_elem=4, ula_axis=(1.0, 0.0, 0.0),
                      zeta_tx=0.4, zeta_rx=0.9)
        out[name] = (st, raw, radio, draw_gains(rng, 4))
    return out


CASES = _cases()


def _per_link_rel(x, ref, link_off):
    worst = 0.0
    for l in range(len(link_off) - 1):
        lo, hi = int(link_off[l]), int(link_off[l + 1])
        if hi > lo:
            den = torch.linalg.norm(ref[lo:hi]).item()
            worst = max(worst, torch.linalg.norm(x[lo:hi] - ref[lo:hi]).item() / den)
    return worst


def test_cases_have_diffraction_paths():
    for name, (st, _, _, _) in CASES.items():
        assert np.count_nonzero(st.kind[:st.n_paths] == 2) >= 10, name


@pytest.mark.parametrize("case", list(CASES))
def test_trace_fields_diffraction(rl, case):
    st, raw, radio, _ = CASES[case]
    P = st.n_paths
    say(f"trace_fields diffraction {case}: {P} paths, "
        f"{int(np.count_nonzero(st.kind[:P] == 2))} diffracted")
    dp = rl.DevicePaths(st)
    a = torch.full((P,), float("nan"), dtype=torch.complex64, device="cuda")
    psi = torch.empty(P, dtype=torch.float32, device="cuda")
    rl.trace_fields(rl.radio_from(radio), dp, rl.materials_per_id(torch.tensor(raw, device="cuda")),
                    a, psi)
    torch.cuda.synchronize()
    a_ref, psi_ref = o_trace_id(st, torch.tensor(raw, dtype=f64), radio.fc,
                                zeta_tx=radio.zeta_tx, zeta_rx=radio.zeta_rx,
                                ula_axis=radio.ula_axis)
    a64 = a.cpu().to(c128)
    dmask = torch.tensor(st.kind[:P] == 2)
    err_d = (torch.linalg.norm(a64[dmask] - a_ref[dmask]) / torch.linalg.norm(a_ref[dmask])).item()
    err = _per_link_rel(a64, a_ref, st.link_off)
    say(f"  per-link relative error {err:.2e}, diffracted paths alone {err_d:.2e}")
    assert err <= 1e-5 and err_d <= 1e-5, (err, err_d)
    assert (psi.cpu().double() - psi_ref).abs().max().item() <= 2e-6


@pytest.mark.parametrize("case", list(CASES))
def test_cfr_diffraction_end_to_end(rl, case):
    st, raw, radio, g = CASES[case]
    say(f"cfr diffraction {case}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    a = torch.empty(st.n_paths, dtype=torch.complex64, device="cuda")
    psi = torch.empty(st.n_paths, dtype=torch.float32, device="cuda")
    rl.trace_fields(rc, dp, rl.materials_per_id(torch.tensor(raw, device="cuda")), a, psi)
    H = torch.empty((st.n_links, radio.n_elem, radio.n_sc), dtype=torch.complex64, device="cuda")
    rl.cfr(rc, dp, a, psi, torch.tensor(g, device="cuda"), H)
    torch.cuda.synchronize()
    a_ref, psi_ref = o_trace_id(st, torch.tensor(raw, dtype=f64), radio.fc, zeta_tx=radio.zeta_tx,
                                zeta_rx=radio.zeta_rx, ula_axis=radio.ula_axis)
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    H_ref = och.cfr(st.link_off, st.tau, a_ref, psi_ref, torch.tensor(g, dtype=c128), f)
    num = torch.linalg.norm((H.cpu().to(c128) - H_ref).reshape(st.n_links, -1), dim=1)
    den = torch.linalg.norm(H_ref.reshape(st.n_links, -1), dim=1)
    err = (num / den).max().item()
    say(f"  max per-link CFR error {err:.2e}")
    assert err <= 1e-5, err


@pytest.mark.parametrize("case", list(CASES))
def test_trace_fields_adjoint_diffraction_per_id(rl, case):
    st, raw, radio, _ = CASES[case]
    rng = np.random.default_rng(51)
    P = st.n_paths
    dLda = torch.tensor((rng.normal(size=P) + 1j * rng.normal(size=P)).astype(np.complex64))
    raw64 = torch.tensor(raw, dtype=f64, requires_grad=True)
    a_ref, _ = o_trace_id(st, raw64, radio.fc, zeta_tx=radio.zeta_tx, zeta_rx=radio.zeta_rx,
                          ula_axis=radio.ula_axis)
    (g_ref,) = torch.autograd.grad(a_ref, raw64, grad_outputs=dLda.to(c128))
    say(f"trace_fields_adjoint diffraction per-id {case}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    n_mat = raw.shape[0]
    ws = rl.workspace(rl.RTC_OP_TRACE_FIELDS_ADJOINT, rc, st.n_links, P, n_mat)
    draw = torch.full((n_mat, 3), float("nan"), dtype=torch.float32, device="cuda")
    rl.trace_fields_adjoint(rc, dp, rl.materials_per_id(torch.tensor(raw, device="cuda")),
                            dLda.cuda(), draw, None, ws)
    torch.cuda.synchronize()
    err = (torch.linalg.norm(draw.cpu().double() - g_ref) / torch.linalg.norm(g_ref)).item()
    say(f"  dL/draw error {err:.2e}")
    assert err <= 1e-4, err


def test_adjoint_diffraction_only_face_materials(rl):
    """Only diffracted paths (dL/da zero elsewhere): the gradient reaches
    eps_r and sigma of both faces' materials and never S."""
    st, raw, radio, _ = CASES["wedge"]
    P = st.n_paths
    dmask = st.kind[:P] == 2
    rng = np.random.default_rng(52)
    g = (rng.normal(size=P) + 1j * rng.normal(size=P)) * dmask
    dLda = torch.tensor(g.astype(np.complex64))
    raw64 = torch.tensor(raw, dtype=f64, requires_grad=True)
    a_ref, _ = o_trace_id(st, raw64, radio.fc, zeta_tx=radio.zeta_tx, zeta_rx=radio.zeta_rx,
                          ula_axis=radio.ula_axis)
    (g_ref,) = torch.autograd.grad(a_ref, raw64, grad_outputs=dLda.to(c128))
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    ws = rl.workspace(rl.RTC_OP_TRACE_FIELDS_ADJOINT, rc, st.n_links, P, 2)
    draw = torch.zeros((2, 3), dtype=torch.float32, device="cuda")
    rl.trace_fields_adjoint(rc, dp, rl.materials_per_id(torch.tensor(raw, device="cuda")),
                            dLda.cuda(), draw, None, ws)
    torch.cuda.synchronize()
    got = draw.cpu().double()
    assert torch.all(got[:, 2] == 0) and torch.all(g_ref[:, 2] == 0)
    assert torch.all(g_ref[:, :2].abs() > 0)
    err = (torch.linalg.norm(got - g_ref) / torch.linalg.norm(g_ref)).item()
    say(f"  face-material gradient error {err:.2e}")
    assert err <= 1e-4, err


@pytest.mark.parametrize("case", list(CASES))
def test_trace_fields_adjoint_diffraction_per_interaction(rl, case):
    st, raw, radio, _ = CASES[case]
    rng = np.random.default_rng(53)
    P, D = st.n_paths, st.max_depth
    e32 = torch.tensor(rng.uniform(2, 8, (D, P)), dtype=torch.float32)
    s32 = torch.tensor(10 ** rng.uniform(-3, 0, (D, P)), dtype=torch.float32)
    S32 = torch.tensor(rng.uniform(0.05, 0.6, (D, P)), dtype=torch.float32)
    e64, s64, S64 = (x.double().requires_grad_(True) for x in (e32, s32, S32))
    a_ref, _ = o_trace(st, e64, s64, S64, radio.fc, zeta_tx=radio.zeta_tx,
                       zeta_rx=radio.zeta_rx, ula_axis=radio.ula_axis)
    dLda = torch.tensor((rng.normal(size=P) + 1j * rng.normal(size=P)).astype(np.complex64))
    ge, gs, gS = torch.autograd.grad(a_ref, (e64, s64, S64), grad_outputs=dLda.to(c128))
    say(f"trace per-interaction diffraction {case}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    per = torch.stack([e32, s32, S32]).reshape(3, D * P).contiguous().cuda()
    a = torch.empty(P, dtype=torch.complex64, device="cuda")
    rl.trace_fields(rc, dp, rl.materials_per_interaction(per), a, None)
    dint = torch.full((3, D * P), float("nan"), dtype=torch.float32, device="cuda")
    rl.trace_fields_adjoint(rc, dp, rl.materials_per_interaction(per), dLda.cuda(), None, dint,
                            None)
    torch.cuda.synchronize()
    assert _per_link_rel(a.cpu().to(c128), a_ref.detach(), st.link_off) <= 1e-5
    got = dint.cpu().double().reshape(3, D, P)
    mask = torch.arange(D)[:, None] < torch.tensor(st.depth.astype(np.int64))[None, :]
    for c, ref in enumerate((ge, gs, gS)):
        den = torch.linalg.norm(ref[mask])
        err = (torch.linalg.norm(got[c][mask] - ref[mask]) / den).item()
        say(f"  row {c}: error {err:.2e}")
        assert err <= 1e-4, (c, err)


def test_diffraction_with_tx_gain(rl):
    """The trainable Tx gain multiplies diffracted paths too; dL/dtx_raw
    against the oracle."""
    st, raw, radio, _ = CASES["floor_diffuse"]
    rng = np.random.default_rng(54)
    P, n_vmf = st.n_paths, 2
    tx = np.concatenate([[0.7], rng.normal(size=2), np.log([3.0, 7.0]),
                         rng.normal(size=6)]).astype(np.float32)
    dLda = torch.tensor((rng.normal(size=P) + 1j * rng.normal(size=P)).astype(np.complex64))
    tx64 = torch.tensor(tx, dtype=f64, requires_grad=True)
    raw64 = torch.tensor(raw, dtype=f64, requires_grad=True)
    a_ref, _ = o_trace_id(st, raw64, radio.fc, zeta_tx=radio.zeta_tx, zeta_rx=radio.zeta_rx,
                          ula_axis=radio.ula_axis, tx_raw=tx64, n_vmf=n_vmf)
    g_raw, g_tx = torch.autograd.grad(a_ref, (raw64, tx64), grad_outputs=dLda.to(c128))
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    mats = rl.materials_per_id(torch.tensor(raw, device="cuda"))
    pats = rl.patterns(n_vmf, torch.tensor(tx, device="cuda"), None)
    a = torch.empty(P, dtype=torch.complex64, device="cuda")
    rl.trace_fields_pat(rc, dp, mats, pats, a, None)
    ws = rl.workspace(rl.RTC_OP_TRACE_FIELDS_ADJOINT_PAT, rc, st.n_links, P, raw.shape[0])
    draw = torch.zeros(raw.shape, dtype=torch.float32, device="cuda")
    dtx = torch.zeros(tx.shape, dtype=torch.float32, device="cuda")
    rl.trace_fields_adjoint_pat(rc, dp, mats, pats, dLda.cuda(), draw, None, dtx, None, ws)
    torch.cuda.synchronize()
    assert _per_link_rel(a.cpu().to(c128), a_ref.detach(), st.link_off) <= 1e-5
    for name, got, ref in (("raw", draw, g_raw), ("tx", dtx, g_tx)):
        err = (torch.linalg.norm(got.cpu().double() - ref) / torch.linalg.norm(ref)).item()
        say(f"  dL/d{name} error {err:.2e}")
        assert err <= 1e-4, (name, err)
    _ = opat  # the oracle's gain model is exercised through trace_fields_per_id

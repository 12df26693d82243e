"""Diffuse reflections through the library (trace_fields, its adjoint, the
CFR) against the FP64 oracle: single-bounce Lambertian paths of a box room
and of a small floor, and specular paths whose last interaction is made
diffuse."""
import sys

import numpy as np
import pytest
import torch

from oracle import channel as och
from oracle.trace import trace_fields as o_trace, trace_fields_per_id as o_trace_id
from synth import diffuse
from synth.params import Radio, draw_gains, draw_materials, materials_to_raw
from tests.helpers import multi_material_box, multi_material_box_scene

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


def _box_diffuse():
    """Depth-2 specular paths of the three-material box plus every sample
    point of its walls as a single-bounce diffuse path (a convex room sees
    all of its surfaces)."""
    st, raw = multi_material_box(seed=8, n_rx=12, max_depth=2)
    samples = diffuse.sample_triangles(multi_material_box_scene(), 3, np.random.default_rng(8))
    st = diffuse.add_diffuse(st, st.tx_pos[0].astype(np.float64), samples,
                             lambda p, e: np.ones(len(p), bool))
    return st, raw


def _spec_then_diffuse():
    """Specular paths of the multi-material box with the last interaction of
    every depth-2 path turned diffuse (dA = 0.05 m^2)."""
    st, raw = multi_material_box(seed=9, n_rx=10, max_depth=2)
    kind = st.kind.copy()
    dA = st.dA.copy()
    P = st.n_paths
    last = np.nonzero(st.depth == 2)[0] + P  # slot 1 of depth-2 paths
    kind[last] = 1
    dA[last] = 0.05
    st.kind, st.dA = kind, dA
    return st, raw


def _floor_diffuse():
    from synth.floorplan import indoor_floor
    from synth.pathfind import find_store
    plan = indoor_floor(11, width=14.0, depth=10.0, min_room=4.0, max_rooms=2, open_frac=0.6,
                        n_pillars=1, target_tris=400)
    rng = np.random.default_rng(12)
    tx = plan.sample_points(rng, 1, 2.4, 2.6)[0]
    rx = plan.sample_points(rng, 12, 1.0, 2.0)
    spec = find_store(plan, tx, rx, 3, n_rays=1 << 15)
    samples = diffuse.sample_floor(plan, 0.4, rng)
    st = diffuse.add_diffuse(spec, tx, samples, lambda p, e: diffuse.visible_floor(plan, p, e))
    raw = materials_to_raw(*draw_materials(rng, plan.scene.n_mat, with_scattering=True))
    return st, raw


def _cases():
    out = {}
    for name, fn in (("box_diffuse", _box_diffuse), ("spec_then_diffuse", _spec_then_diffuse),
                     ("floor_diffuse", _floor_diffuse)):
        st, raw = fn()
        rng = np.random.default_rng(len(name))
        radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=256, n_elem=4, ula_axis=(1.0, 0.0, 0.0))
        out[name] = (st, raw.astype(np.float32), radio, draw_gains(rng, 4))
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


def test_cases_have_diffuse_paths():
    for name, (st, _, _, _) in CASES.items():
        assert np.count_nonzero(st.kind) > 0, name


@pytest.mark.parametrize("case", list(CASES))
def test_trace_fields_diffuse(rl, case):
    st, raw, radio, g = CASES[case]
    say(f"trace_fields diffuse {case}: {st.n_paths} paths, {np.count_nonzero(st.kind)} diffuse")
    dp = rl.DevicePaths(st)
    a = torch.full((st.n_paths,), float("nan"), dtype=torch.complex64, device="cuda")
    psi = torch.empty(st.n_paths, dtype=torch.float32, device="cuda")
    rl.trace_fields(rl.radio_from(radio), dp, rl.materials_per_id(torch.tensor(raw, device="cuda")),
                    a, psi)
    torch.cuda.synchronize()
    a_ref, psi_ref = o_trace_id(st, torch.tensor(raw, dtype=f64), radio.fc, ula_axis=radio.ula_axis)
    err = _per_link_rel(a.cpu().to(c128), a_ref, st.link_off)
    say(f"  per-link relative error {err:.2e}")
    assert err <= 1e-5, err
    assert (psi.cpu().double() - psi_ref).abs().max().item() <= 2e-6


@pytest.mark.parametrize("case", list(CASES))
def test_cfr_diffuse_end_to_end(rl, case):
    st, raw, radio, g = CASES[case]
    say(f"cfr diffuse {case}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    a = torch.empty(st.n_paths, dtype=torch.complex64, device="cuda")
    psi = torch.empty(st.n_paths, dtype=torch.float32, device="cuda")
    rl.trace_fields(rc, dp, rl.materials_per_id(torch.tensor(raw, device="cuda")), a, psi)
    H = torch.empty((st.n_links, radio.n_elem, radio.n_sc), dtype=torch.complex64, device="cuda")
    rl.cfr(rc, dp, a, psi, torch.tensor(g, device="cuda"), H)
    torch.cuda.synchronize()
    a_ref, psi_ref = o_trace_id(st, torch.tensor(raw, dtype=f64), radio.fc, ula_axis=radio.ula_axis)
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    H_ref = och.cfr(st.link_off, st.tau, a_ref, psi_ref, torch.tensor(g, dtype=c128), f)
    num = torch.linalg.norm((H.cpu().to(c128) - H_ref).reshape(st.n_links, -1), dim=1)
    den = torch.linalg.norm(H_ref.reshape(st.n_links, -1), dim=1)
    err = (num / den).max().item()
    say(f"  max per-link CFR error {err:.2e}")
    assert err <= 1e-5, err


@pytest.mark.parametrize("case", list(CASES))
def test_trace_fields_adjoint_diffuse_per_id(rl, case):
    st, raw, radio, g = CASES[case]
    rng = np.random.default_rng(41)
    P = st.n_paths
    dLda = torch.tensor((rng.normal(size=P) + 1j * rng.normal(size=P)).astype(np.complex64))
    raw64 = torch.tensor(raw, dtype=f64, requires_grad=True)
    a_ref, _ = o_trace_id(st, raw64, radio.fc, ula_axis=radio.ula_axis)
    (draw_ref,) = torch.autograd.grad(a_ref, raw64, grad_outputs=dLda.to(c128))
    say(f"trace_fields_adjoint per-id diffuse {case}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    n_mat = raw.shape[0]
    ws = rl.workspace(rl.RTC_OP_TRACE_FIELDS_ADJOINT, rc, st.n_links, P, n_mat)
    draw = torch.full((n_mat, 3), float("nan"), dtype=torch.float32, device="cuda")
    rl.trace_fields_adjoint(rc, dp, rl.materials_per_id(torch.tensor(raw, device="cuda")),
                            dLda.cuda(), draw, None, ws)
    torch.cuda.synchronize()
    err = (torch.linalg.norm(draw.cpu().double() - draw_ref) / torch.linalg.norm(draw_ref)).item()
    say(f"  dL/draw error {err:.2e}")
    assert err <= 1e-4, err


@pytest.mark.parametrize("case", list(CASES))
def test_trace_fields_adjoint_diffuse_per_interaction(rl, case):
    st, raw, radio, g = CASES[case]
    rng = np.random.default_rng(42)
    P, D = st.n_paths, st.max_depth
    e32 = torch.tensor(rng.uniform(2, 8, (D, P)), dtype=torch.float32)
    s32 = torch.tensor(10 ** rng.uniform(-3, 0, (D, P)), dtype=torch.float32)
    S32 = torch.tensor(rng.uniform(0.05, 0.6, (D, P)), dtype=torch.float32)
    e64, s64, S64 = (x.double().requires_grad_(True) for x in (e32, s32, S32))
    a_ref, _ = o_trace(st, e64, s64, S64, radio.fc, ula_axis=radio.ula_axis)
    dLda = torch.tensor((rng.normal(size=P) + 1j * rng.normal(size=P)).astype(np.complex64))
    ge, gs, gS = torch.autograd.grad(a_ref, (e64, s64, S64), grad_outputs=dLda.to(c128))
    say(f"trace per-interaction diffuse {case}")
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    per = torch.stack([e32, s32, S32]).reshape(3, D * P).contiguous().cuda()
    a = torch.empty(P, dtype=torch.complex64, device="cuda")
    rl.trace_fields(rc, dp, rl.materials_per_interaction(per), a, None)
    buf = torch.full((4, D * P), float("nan"), dtype=torch.float32, device="cuda")
    dint = buf[:3]
    rl.trace_fields_adjoint(rc, dp, rl.materials_per_interaction(per), dLda.cuda(), None, dint,
                            None)
    torch.cuda.synchronize()
    assert _per_link_rel(a.cpu().to(c128), a_ref.detach(), st.link_off) <= 1e-5
    assert torch.isnan(buf[3]).all(), "write past the end of the per-interaction rows"
    got = dint.cpu().double().reshape(3, D, P)
    depth = torch.tensor(st.depth.astype(np.int64))
    mask = torch.arange(D)[:, None] < depth[None, :]
    for c, ref in enumerate((ge, gs, gS)):
        assert torch.all(got[c][~mask] == 0)
        err = (torch.linalg.norm(got[c][mask] - ref[mask]) / torch.linalg.norm(ref[mask])).item()
        say(f"  row {c}: error {err:.2e}")
        assert err <= 1e-4, (c, err)

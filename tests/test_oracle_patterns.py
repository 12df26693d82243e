"""Pins of the oracle's patterns (Sec. II-B Eq. atenna_normalization and
polarization_model, Sec. III-A trainable Tx gain, Sec. II-D-2 Eq.
backscattering_model, Sec. III-B Eqs. trainable_scattering_pattern and
normalization_hemisphere) and of cross-polarisation in the diffuse field,
each against numerical quadrature on the sphere or hemisphere, closed
forms, or central differences."""
import math

import numpy as np
import pytest
import torch

from oracle import patterns as pt
from oracle.trace import trace_fields, trace_fields_per_id
from synth.store import KIND_DIFFUSE, pack

f64 = torch.float64
FC = 3.5e9


def sphere_grid(n_t=720, n_p=1440):
    """Midpoint grid on the unit sphere: directions [n, 3], weights [n]."""
    t = (torch.arange(n_t, dtype=f64) + 0.5) * math.pi / n_t
    ph = (torch.arange(n_p, dtype=f64) + 0.5) * 2 * math.pi / n_p
    T, P = torch.meshgrid(t, ph, indexing="ij")
    r = torch.stack([torch.sin(T) * torch.cos(P), torch.sin(T) * torch.sin(P), torch.cos(T)], -1)
    wgt = torch.sin(T) * (math.pi / n_t) * (2 * math.pi / n_p)
    return r.reshape(-1, 3), wgt.reshape(-1)


def hemisphere_grid(n_t=600, n_p=1200):
    """Midpoint grid on the upper hemisphere about +z."""
    t = (torch.arange(n_t, dtype=f64) + 0.5) * (math.pi / 2) / n_t
    ph = (torch.arange(n_p, dtype=f64) + 0.5) * 2 * math.pi / n_p
    T, P = torch.meshgrid(t, ph, indexing="ij")
    r = torch.stack([torch.sin(T) * torch.cos(P), torch.sin(T) * torch.sin(P), torch.cos(T)], -1)
    wgt = torch.sin(T) * ((math.pi / 2) / n_t) * (2 * math.pi / n_p)
    return r.reshape(-1, 3), wgt.reshape(-1)


def incidence(theta):
    """Propagation direction arriving at the plane z = 0 from above at polar
    angle theta, and the normal +z."""
    k_in = torch.tensor([math.sin(theta), 0.0, -math.cos(theta)], dtype=f64)
    return k_in, torch.tensor([0.0, 0.0, 1.0], dtype=f64)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vmf_gain_integrates_to_4pi_eta(seed):
    rng = np.random.default_rng(seed)
    M = 3
    raw = torch.tensor(np.concatenate([[rng.normal()], rng.normal(size=M),
                                       np.log(rng.uniform(0.5, 15.0, M)),
                                       rng.normal(size=3 * M)]))
    eta, w, lam, mu = pt.vmf_from_raw(raw, M)
    r, wgt = sphere_grid()
    G = pt.vmf_gain(r, eta, w, lam, mu)
    assert (G >= 0).all()
    total = (G * wgt).sum().item()
    assert abs(total - 4 * math.pi * eta.item()) <= 1e-5 * 4 * math.pi


def test_vmf_single_lobe_closed_forms():
    # one lobe: at the mean direction G = 4 pi eta e^lam / a = 2 eta lam /
    # (1 - e^{-2 lam}); opposite it G = 2 eta lam e^{-2 lam} / (1 - e^{-2 lam})
    lam = 4.0
    raw = torch.tensor([0.7, 0.0, math.log(lam), 0.0, 0.0, 2.0], dtype=f64)
    eta, w, lam_t, mu = pt.vmf_from_raw(raw, 1)
    G = pt.vmf_gain(torch.tensor([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]], dtype=f64), eta, w, lam_t,
                    mu)
    e = eta.item()
    ref = 2 * e * lam / (1 - math.exp(-2 * lam))
    assert abs(G[0].item() - ref) <= 1e-12 * ref
    assert abs(G[1].item() - ref * math.exp(-2 * lam)) <= 1e-12 * ref
    # a nearly flat lobe is the isotropic gain eta
    raw0 = torch.tensor([0.7, 0.0, math.log(1e-6), 0.3, -0.2, 0.9], dtype=f64)
    G0 = pt.vmf_gain(torch.tensor([[0.6, 0.0, 0.8]], dtype=f64), *pt.vmf_from_raw(raw0, 1))
    assert abs(G0.item() - e) <= 1e-5


@pytest.mark.parametrize("lam", [0.5, 2.0, 8.0, 30.0])
def test_hemispherical_normaliser_exact_points_and_accuracy(lam):
    lam_t = torch.tensor(lam, dtype=f64)
    r, wgt = sphere_grid(1440, 2880)
    up = r[:, 2] >= 0
    e = math.exp(-lam)
    A = 2 * math.pi / lam * (1 - e)  # exact integral at cos(beta) = +1
    worst_rel, worst_s = 0.0, 0.0
    for cb in [-1.0, -0.6, -0.2, 0.0, 0.15, 0.3, 0.5, 0.7, 0.9, 1.0]:
        axis = torch.tensor([math.sqrt(max(0.0, 1 - cb * cb)), 0.0, cb], dtype=f64)
        num = ((torch.exp(lam_t * (r @ axis - 1.0)) * wgt)[up]).sum().item()
        approx = pt.hemi_norm_shifted(lam_t, torch.tensor(cb, dtype=f64)).item()
        rel = abs(approx / num - 1.0)
        if cb in (-1.0, 0.0, 1.0):
            assert rel <= 2e-4, (cb, rel)  # exact there (quadrature error only)
        # the fraction of the lobe above the surface, everywhere
        worst_s = max(worst_s, abs(approx - num) / (A * (1 - e)))
        if cb >= 0.0:  # the range the scattering lobes use (cos(beta) = cos(theta_i))
            worst_rel = max(worst_rel, rel)
    assert worst_s <= 0.012, worst_s
    assert worst_rel <= 0.015, worst_rel


@pytest.mark.parametrize("theta", [0.1, 0.7, 1.3])
def test_trainable_pattern_integrates_to_about_one(theta):
    k_in, n = incidence(theta)
    r, wgt = hemisphere_grid()
    w = torch.tensor([0.2, 0.3, 0.5], dtype=f64)
    f = pt.trainable_pattern(k_in.expand_as(r), r, n.expand_as(r), w.expand(len(r), 3),
                             torch.tensor(6.0, dtype=f64), torch.tensor(12.0, dtype=f64))
    total = (f * wgt).sum().item()
    assert abs(total - 1.0) <= 0.05, total
    # the Lambertian lobe alone integrates to exactly one
    f1 = pt.trainable_pattern(k_in.expand_as(r), r, n.expand_as(r),
                              torch.tensor([1.0, 0.0, 0.0], dtype=f64).expand(len(r), 3),
                              torch.tensor(6.0, dtype=f64), torch.tensor(12.0, dtype=f64))
    assert abs((f1 * wgt).sum().item() - 1.0) <= 1e-5


@pytest.mark.parametrize("theta,alpha", [(0.0, 1), (0.5, 5), (1.2, 8), (0.9, 3)])
def test_backscatter_lobe_integral_closed_form(theta, alpha):
    cos_t = torch.tensor(math.cos(theta), dtype=f64)
    axis = torch.tensor([math.sin(theta), 0.0, math.cos(theta)], dtype=f64)
    r, wgt = hemisphere_grid(1200, 2400)
    num = ((((1.0 + r @ axis) / 2.0) ** alpha) * wgt).sum().item()
    assert abs(pt._lobe_hemi_integral(alpha, cos_t).item() / num - 1.0) <= 1e-5


@pytest.mark.parametrize("theta", [0.2, 0.8, 1.4])
def test_backscatter_pattern_normalised_and_lobes(theta):
    k_in, n = incidence(theta)
    r, wgt = hemisphere_grid()
    f = pt.backscatter_pattern(k_in.expand_as(r), r, n.expand_as(r), 5, 8,
                               torch.tensor(0.8, dtype=f64))
    assert abs((f * wgt).sum().item() - 1.0) <= 1e-5
    # specular and backscatter directions are the lobe maxima
    k_r = k_in - 2 * (k_in @ n) * n
    k_b = -k_in
    fr = pt.backscatter_pattern(k_in, k_r, n, 5, 8, torch.tensor(1.0, dtype=f64))
    fb = pt.backscatter_pattern(k_in, k_b, n, 5, 8, torch.tensor(0.0, dtype=f64))
    for other in (torch.tensor([0.0, 0.6, 0.8], dtype=f64),):
        assert pt.backscatter_pattern(k_in, other, n, 5, 8, torch.tensor(1.0, dtype=f64)) < fr
        assert pt.backscatter_pattern(k_in, other, n, 5, 8, torch.tensor(0.0, dtype=f64)) < fb


def _single_diffuse_store(tx, rx, s, dA, normal=(0.0, 0.0, 1.0)):
    L = np.linalg.norm(s - tx) + np.linalg.norm(rx - s)
    rec = dict(points=s[None], normals=np.asarray(normal)[None], mats=[0], faces=[0],
               kinds=[KIND_DIFFUSE], dA=[dA], length=L)
    return pack([[rec]], [tx], [rx], 1, geom_dtype=np.float64)


def test_kx_splits_power_between_polarisations():
    tx = np.array([0.0, 0.0, 2.5])
    rx = np.array([3.0, 1.0, 1.5])
    st = _single_diffuse_store(tx, rx, np.array([1.2, -0.4, 0.0]), 0.02)
    mats = [torch.full((1, 1), v, dtype=f64) for v in (5.0, 0.05, 0.4)]
    powers = {}
    for kx in (0.0, 0.3):
        kxt = torch.full((1, 1), kx, dtype=f64)
        pv = abs(complex(trace_fields(st, *mats, FC, zeta_rx=0.0, kx=kxt)[0][0])) ** 2
        ph = abs(complex(trace_fields(st, *mats, FC, zeta_rx=math.pi / 2, kx=kxt)[0][0])) ** 2
        powers[kx] = (pv, ph)
    tot0 = sum(powers[0.0])
    tot3 = sum(powers[0.3])
    assert abs(tot3 / tot0 - 1.0) <= 1e-12  # K_x moves power, it does not change it


def test_tx_gain_scales_amplitude_by_sqrt_g():
    tx = np.array([0.0, 0.0, 2.5])
    rx = np.array([3.0, 1.0, 1.5])
    st = _single_diffuse_store(tx, rx, np.array([1.2, -0.4, 0.0]), 0.02)
    raw = torch.tensor([[math.log(4.0), math.log(0.05), 0.0]], dtype=f64)
    a0, _ = trace_fields_per_id(st, raw, FC)
    M = 2
    tx_raw = torch.tensor([0.3, 0.1, -0.2, math.log(2.0), math.log(5.0), 0.0, 0.3, 1.0,
                           1.0, 0.0, -0.2], dtype=f64)
    a1, _ = trace_fields_per_id(st, raw, FC, tx_raw=tx_raw, n_vmf=M)
    s = np.array([1.2, -0.4, 0.0])
    k1 = torch.tensor((s - tx) / np.linalg.norm(s - tx), dtype=f64)
    G = pt.vmf_gain(k1[None], *pt.vmf_from_raw(tx_raw, M)).item()
    assert abs(complex(a1[0]) / complex(a0[0]) - math.sqrt(G)) <= 1e-12 * math.sqrt(G)


def test_pattern_parameter_gradients_match_central_differences():
    tx = np.array([0.0, 0.5, 2.5])
    rxs = [np.array([3.0, 1.0, 1.5]), np.array([-2.0, 2.0, 1.0])]
    recs = []
    for rx, spts in zip(rxs, [[np.array([1.2, -0.4, 0.0]), np.array([0.5, 1.5, 0.0])],
                              [np.array([-1.0, 0.7, 0.0])]]):
        recs.append([dict(points=p[None], normals=np.array([[0.0, 0.0, 1.0]]), mats=[0],
                          faces=[0], kinds=[KIND_DIFFUSE], dA=[0.03],
                          length=np.linalg.norm(p - tx) + np.linalg.norm(rx - p))
                     for p in spts])
    st = pack(recs, [tx, tx], rxs, 1, geom_dtype=np.float64)
    raw = torch.tensor([[math.log(3.0), math.log(0.1), 0.2]], dtype=f64)
    tx_raw = torch.tensor([0.3, 0.1, -0.2, math.log(2.0), math.log(5.0), 0.0, 0.3, 1.0,
                           1.0, 0.0, -0.2], dtype=f64, requires_grad=True)
    pat = torch.tensor([[-0.5, 0.2, -0.1, 0.4, math.log(3.0), math.log(7.0)]], dtype=f64,
                       requires_grad=True)
    g = torch.tensor(np.random.default_rng(4).normal(size=(st.n_paths, 2)), dtype=f64)

    def loss(txr, pr):
        a, _ = trace_fields_per_id(st, raw, FC, tx_raw=txr, n_vmf=2, pat_raw=pr, zeta_rx=0.4)
        return (a.real * g[:, 0] + a.imag * g[:, 1]).sum()

    gt, gp = torch.autograd.grad(loss(tx_raw, pat), (tx_raw, pat))
    for x, gx, k in ((tx_raw, gt, 0), (pat, gp, 1)):
        flat = x.detach().reshape(-1)
        for i in range(flat.numel()):
            h = 1e-6
            xp, xm = flat.clone(), flat.clone()
            xp[i] += h
            xm[i] -= h
            args_p = [tx_raw.detach(), pat.detach()]
            args_m = [tx_raw.detach(), pat.detach()]
            args_p[k] = xp.reshape(x.shape)
            args_m[k] = xm.reshape(x.shape)
            fd = (float(loss(*args_p)) - float(loss(*args_m))) / (2 * h)
            an = float(gx.reshape(-1)[i])
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-9) + 1e-13, (k, i, fd, an)

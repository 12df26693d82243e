"""Pins of the oracle's diffuse reflection (Sec. II-D-2, Eq. scattered_field
with the Lambertian pattern), each against something the oracle does not
compute itself: a hemisphere integral, the closed-form power scattered by a
perfectly conducting Lambertian disc, the Brewster zero of the TM
reflection, scaling laws, and central differences."""
import math

import numpy as np
import pytest
import torch

from oracle.em import fresnel, lambertian_pattern, permittivity, wavelength
from oracle.trace import trace_fields
from synth.store import KIND_DIFFUSE, KIND_SPECULAR, pack

f64 = torch.float64
FC = 3.5e9


def _diffuse_store(tx, rx_list, pts_per_link, dA_per_link, normal=(0.0, 0.0, 1.0)):
    links = []
    for rx, pts, dAs in zip(rx_list, pts_per_link, dA_per_link):
        recs = []
        for s, dA in zip(pts, dAs):
            s = np.asarray(s, np.float64)
            L = np.linalg.norm(s - tx) + np.linalg.norm(np.asarray(rx) - s)
            recs.append(dict(points=s[None], normals=np.asarray(normal)[None], mats=[0],
                             faces=[0], kinds=[KIND_DIFFUSE], dA=[dA], length=L))
        links.append(recs)
    return pack(links, [tx] * len(rx_list), rx_list, 1, geom_dtype=np.float64)


def _mats(P, eps, sig, S, D=1):
    return (torch.full((D, P), eps, dtype=f64), torch.full((D, P), sig, dtype=f64),
            torch.full((D, P), S, dtype=f64))


def test_lambertian_pattern_integrates_to_one():
    # midpoint rule in (cos theta, phi); the back hemisphere contributes 0
    n = 4000
    mu = -1.0 + (np.arange(n) + 0.5) * (2.0 / n)
    f = lambertian_pattern(torch.tensor(mu, dtype=f64)).numpy()
    total = 2.0 * math.pi * f.sum() * (2.0 / n)
    assert abs(total - 1.0) < 1e-6


def test_pec_lambertian_disc_closed_form():
    """Tx and Rx at the same point, height h above a perfectly conducting
    disc of radius Rd with S = 1: the power summed over the disc's area
    elements and both receive polarisations tends to
    (lambda/4pi)^2 * integral of cos_i cos_s / (pi d1^2 d2^2) dA
      = (lambda/4pi)^2 [1/(2 h^2) - h^2 / (2 (h^2 + Rd^2)^2)]."""
    h, Rd = 2.0, 6.0
    nr, ns = 600, 48
    # equal-area rings, midpoints
    r_mid = Rd * np.sqrt((np.arange(nr) + 0.5) / nr)
    ph = (np.arange(ns) + 0.5) * 2 * np.pi / ns
    rr, pp = np.meshgrid(r_mid, ph, indexing="ij")
    pts = np.stack([rr * np.cos(pp), rr * np.sin(pp), np.zeros_like(rr)], -1).reshape(-1, 3)
    dA = np.full(len(pts), np.pi * Rd * Rd / (nr * ns))
    tx = np.array([0.0, 0.0, h])
    st = _diffuse_store(tx, [tx.copy()], [pts], [dA])
    eps, sig, S = _mats(st.n_paths, 4.0, 1e12, 1.0)
    a_v, _ = trace_fields(st, eps, sig, S, FC, zeta_rx=0.0)
    a_h, _ = trace_fields(st, eps, sig, S, FC, zeta_rx=math.pi / 2)
    power = float((a_v.abs() ** 2 + a_h.abs() ** 2).sum())
    lam = wavelength(FC)
    ref = (lam / (4 * math.pi)) ** 2 * (1.0 / (2 * h * h) - h * h / (2 * (h * h + Rd * Rd) ** 2))
    assert abs(power / ref - 1.0) < 2e-4, power / ref


@pytest.mark.parametrize("eps_r", [2.5, 6.0])
def test_diffuse_gamma_is_te_or_tm_fresnel(eps_r):
    """Tx above the plane z = 0, diffuse point in the x-z plane: the Tx's
    phi_hat field is purely perpendicular to the plane of incidence (TE),
    theta_hat purely parallel (TM).  The amplitude relative to a perfect
    conductor is then |r_perp| or |r_par|; at the Brewster angle the TM one
    vanishes."""
    h = 3.0
    thb = math.atan(math.sqrt(eps_r))
    s = np.array([h * math.tan(thb), 0.0, 0.0])
    tx = np.array([0.0, 0.0, h])
    rx = np.array([s[0] + 1.0, 0.7, 2.0])
    st = _diffuse_store(tx, [rx], [[s]], [[0.01]])

    def power(eps, sig, zeta_tx):
        m = _mats(1, eps, sig, 0.5)
        tot = 0.0
        for zr in (0.0, math.pi / 2):
            a, _ = trace_fields(st, *m, FC, zeta_tx=zeta_tx, zeta_rx=zr)
            tot += float(a.abs() ** 2)
        return tot

    cos_i = math.cos(thb)
    r_perp, r_par = fresnel(permittivity(torch.tensor(eps_r, dtype=f64),
                                         torch.tensor(0.0, dtype=f64), FC),
                            torch.tensor(cos_i, dtype=f64))
    te = power(eps_r, 0.0, math.pi / 2) / power(eps_r, 1e20, math.pi / 2)
    tm = power(eps_r, 0.0, 0.0) / power(eps_r, 1e20, 0.0)
    assert abs(math.sqrt(te) - abs(complex(r_perp))) < 1e-8
    assert abs(r_par) < 1e-12 and tm < 1e-20


def test_diffuse_scales_with_S_and_sqrt_dA():
    tx = np.array([0.0, 0.0, 2.5])
    rx = np.array([3.0, 1.0, 1.5])
    s = np.array([1.2, -0.4, 0.0])
    a = {}
    for dA in (0.01, 0.04):
        st = _diffuse_store(tx, [rx], [[s]], [[dA]])
        for S in (0.3, 0.6):
            a[(dA, S)] = complex(trace_fields(st, *_mats(1, 5.0, 0.01, S), FC)[0][0])
    assert abs(a[(0.01, 0.6)] / a[(0.01, 0.3)] - 2.0) < 1e-12
    assert abs(a[(0.04, 0.3)] / a[(0.01, 0.3)] - 2.0) < 1e-12


def test_diffuse_behind_surface_is_zero():
    tx = np.array([0.0, 0.0, 2.5])
    rx = np.array([3.0, 1.0, -1.5])  # below the plane z = 0
    st = _diffuse_store(tx, [rx], [[np.array([1.0, 0.0, 0.0])]], [[0.02]])
    a, _ = trace_fields(st, *_mats(1, 5.0, 0.01, 0.5), FC)
    assert abs(complex(a[0])) == 0.0


def _specular_then_diffuse_store():
    """Two-interaction paths whose second interaction is diffuse: first a
    reflection on the wall x = 0, then a diffuse point on the floor."""
    tx = np.array([2.0, 1.0, 2.5])
    links = []
    rxs = [np.array([3.0, 2.0, 1.2]), np.array([4.5, -1.0, 1.7])]
    for rx in rxs:
        recs = []
        for s2 in (np.array([1.5, 0.5, 0.0]), np.array([2.5, 3.0, 0.0])):
            # reflection point on x = 0 between the Tx and the floor point
            img = np.array([-tx[0], tx[1], tx[2]])
            t = (0.0 - img[0]) / (s2[0] - img[0])
            s1 = img + t * (s2 - img)
            L = np.linalg.norm(s1 - tx) + np.linalg.norm(s2 - s1) + np.linalg.norm(rx - s2)
            recs.append(dict(points=np.stack([s1, s2]), normals=np.array([[1.0, 0, 0], [0, 0, 1.0]]),
                             mats=[0, 1], faces=[0, 1], kinds=[KIND_SPECULAR, KIND_DIFFUSE],
                             dA=[0.0, 0.05], length=L))
        links.append(recs)
    return pack(links, [tx] * len(rxs), rxs, 2, geom_dtype=np.float64)


def test_diffuse_gradients_match_central_differences():
    st = _specular_then_diffuse_store()
    P = st.n_paths
    g = torch.tensor(np.random.default_rng(3).normal(size=(P, 2)), dtype=f64)

    def loss(eps, sig, S):
        a, _ = trace_fields(st, eps, sig, S, FC, zeta_tx=0.3)
        return (a.real * g[:, 0] + a.imag * g[:, 1]).sum()

    eps = torch.tensor([[4.0] * P, [6.5] * P], dtype=f64, requires_grad=True)
    sig = torch.tensor([[0.02] * P, [0.3] * P], dtype=f64, requires_grad=True)
    S = torch.tensor([[0.3] * P, [0.45] * P], dtype=f64, requires_grad=True)
    ge, gs, gS = torch.autograd.grad(loss(eps, sig, S), (eps, sig, S))
    for x, gx, k in ((eps, ge, 0), (sig, gs, 1), (S, gS, 2)):
        for d in range(2):
            for p in range(P):
                h = 1e-4 * abs(float(x.detach()[d, p]))
                xp = x.detach().clone()
                xm = x.detach().clone()
                xp[d, p] += h
                xm[d, p] -= h
                args_p = [eps.detach(), sig.detach(), S.detach()]
                args_m = [eps.detach(), sig.detach(), S.detach()]
                args_p[k], args_m[k] = xp, xm
                fd = (float(loss(*args_p)) - float(loss(*args_m))) / (2 * h)
                assert abs(fd - float(gx[d, p])) <= 1e-6 * max(abs(fd), 1e-12) + 1e-14, (k, d, p)

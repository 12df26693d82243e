"""Pins of the oracle's electromagnetic building blocks against closed forms
and physical invariants (Sec. II-D of the paper)."""
import math

import numpy as np
import pytest
import torch

from oracle import em
from oracle.trace import specular_step

f64 = torch.float64


def test_brewster_angle_zero_tm_reflection():
    # lossless dielectric: r_par vanishes at tan(theta_B) = sqrt(eps_r)
    for eps in (1.5, 2.0, 4.0, 9.7):
        th = math.atan(math.sqrt(eps))
        eta = em.permittivity(torch.tensor(eps, dtype=f64), torch.tensor(0.0, dtype=f64), 3.5e9)
        r_perp, r_par = em.fresnel(eta, torch.tensor(math.cos(th), dtype=f64))
        assert abs(r_par.item()) < 1e-14
        assert abs(r_perp.item()) > 0.05


def test_normal_incidence():
    # r_par = -r_perp = (sqrt(eta) - 1) / (sqrt(eta) + 1)
    eta = torch.tensor(5.0 - 0.7j, dtype=torch.complex128)
    r_perp, r_par = em.fresnel(eta, torch.tensor(1.0, dtype=f64))
    ref = (np.sqrt(5.0 - 0.7j) - 1) / (np.sqrt(5.0 - 0.7j) + 1)
    assert abs(r_par.item() - ref) < 1e-15
    assert abs(r_perp.item() + ref) < 1e-15


def test_grazing_incidence():
    eta = torch.tensor(3.3 - 0.2j, dtype=torch.complex128)
    r_perp, r_par = em.fresnel(eta, torch.tensor(0.0, dtype=f64))
    assert abs(r_perp.item() + 1) < 1e-15
    assert abs(r_par.item() + 1) < 1e-15


def test_pec_limit():
    # |eta| -> infinity: r_perp -> -1, r_par -> +1
    eta = em.permittivity(torch.tensor(1.0, dtype=f64), torch.tensor(1e12, dtype=f64), 3.5e9)
    for c in (0.2, 0.5, 0.9):
        r_perp, r_par = em.fresnel(eta, torch.tensor(c, dtype=f64))
        assert abs(r_perp.item() + 1) < 1e-5
        assert abs(r_par.item() - 1) < 1e-5


def test_passive_media_reflect_at_most_unity():
    rng = np.random.default_rng(0)
    eps = torch.tensor(rng.uniform(1, 80, 2000), dtype=f64)
    sig = torch.tensor(10 ** rng.uniform(-4, 3, 2000), dtype=f64)
    c = torch.tensor(rng.uniform(0, 1, 2000), dtype=f64)
    eta = em.permittivity(eps, sig, 3.5e9)
    assert (eta.imag <= 0).all()
    r_perp, r_par = em.fresnel(eta, c)
    assert (r_perp.abs() <= 1 + 1e-12).all()
    assert (r_par.abs() <= 1 + 1e-12).all()


def test_fresnel_derivatives_closed_form():
    # dr_perp/deta = -c/(s (c+s)^2),  dr_par/deta = c (eta - 2 sin^2)/(s (eta c + s)^2)
    rng = np.random.default_rng(1)
    for _ in range(20):
        eta0 = complex(rng.uniform(1.5, 20), -rng.uniform(0.01, 5))
        c = rng.uniform(0.05, 0.99)
        s = np.sqrt(eta0 - (1 - c * c))
        d_perp = -c / (s * (c + s) ** 2)
        d_par = c * (eta0 - 2 * (1 - c * c)) / (s * (eta0 * c + s) ** 2)
        h = 1e-6
        for d_ref, idx in ((d_perp, 0), (d_par, 1)):
            fp = em.fresnel(torch.tensor(eta0 + h, dtype=torch.complex128), torch.tensor(c, dtype=f64))[idx]
            fm = em.fresnel(torch.tensor(eta0 - h, dtype=torch.complex128), torch.tensor(c, dtype=f64))[idx]
            d_fd = (fp - fm).item() / (2 * h)
            assert abs(d_fd - d_ref) < 1e-7 * max(1, abs(d_ref))


def test_permittivity_value():
    # eta = eps_r - j sigma / (eps0 * 2 pi f)
    eta = em.permittivity(torch.tensor(4.0, dtype=f64), torch.tensor(0.1947138, dtype=f64), 3.5e9)
    # eps0 * omega at 3.5 GHz = 0.19471384... S/m, so the imaginary part is ~ -1
    assert abs(eta.real.item() - 4.0) < 1e-15
    assert abs(eta.imag.item() + 1.0) < 1e-6


def test_material_transforms_match_library_routines():
    raw = torch.tensor([[0.3, -2.0, 0.7], [-1.0, 1.0, -3.0]], dtype=f64)
    eps_r, sigma, s = em.materials_from_raw(raw)
    assert torch.allclose(eps_r, 1 + torch.exp(raw[:, 0]))
    assert torch.allclose(s, torch.sigmoid(raw[:, 2]), atol=0, rtol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_pec_tangential_field_vanishes(seed):
    """Basis-free pin: on a perfect conductor the tangential part of
    (incident + reflected) field at the reflection point is zero."""
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    k = rng.normal(size=3)
    k /= np.linalg.norm(k)
    if k @ n > 0:
        k = -k
    # an arbitrary transverse basis for the incoming field
    p = np.cross(k, rng.normal(size=3))
    p /= np.linalg.norm(p)
    q = np.cross(k, p)
    E = torch.tensor(rng.normal(size=2) + 1j * rng.normal(size=2), dtype=torch.complex128)
    eta = em.permittivity(torch.tensor(1.0, dtype=f64), torch.tensor(1e14, dtype=f64), 3.5e9)
    t = lambda x: torch.tensor(x, dtype=f64)
    E_out, e_perp, e_par_in, e_par_out, k_r, _ = specular_step(
        E, t(p), t(q), t(k), t(n), eta, torch.tensor(1.0, dtype=f64))
    e_in = E[0] * t(p).to(torch.complex128) + E[1] * t(q).to(torch.complex128)
    e_ref = E_out[0] * e_perp.to(torch.complex128) + E_out[1] * e_par_out.to(torch.complex128)
    tot = (e_in + e_ref).numpy()
    tang = tot - (tot @ n) * n
    assert np.linalg.norm(tang) < 1e-6 * np.linalg.norm(e_in.numpy())
    # reflected field is transverse to the reflected direction
    assert abs(np.vdot(k_r.numpy(), e_ref.numpy())) < 1e-12
    # reflected direction is the mirror image
    assert np.allclose(k_r.numpy(), k - 2 * (k @ n) * n)

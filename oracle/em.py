"""Electromagnetic building blocks (oracle, FP64).  Test infrastructure only.

Sources in the paper:
  * complex relative permittivity: Sec. II-D (eta = eps_r - j sigma/(eps0 w))
  * Fresnel coefficients: Sec. II-D-1, Eqs. (fresnel-1), (fresnel-2)
  * material parametrisation: Sec. III-C, Eqs. (trainable_materials_1-4)
  * antenna field components in the spherical basis: Sec. II-B
"""
import math

import torch

# Speed of light (exact, SI) and vacuum permittivity (CODATA 2018).
C0 = 299792458.0
EPS0 = 8.8541878128e-12

f64 = torch.float64
c128 = torch.complex128


def materials_from_raw(raw):
    """Sec. III-C with one-dimensional embeddings and unit read-out vector:
    eps_r = 1 + exp(u0), sigma = exp(u1), S = logistic(u2).

    raw: float64 [..., 3].  Returns (eps_r, sigma, S)."""
    raw = torch.as_tensor(raw, dtype=f64)
    eps_r = 1.0 + torch.exp(raw[..., 0])
    sigma = torch.exp(raw[..., 1])
    s = 1.0 / (1.0 + torch.exp(-raw[..., 2]))
    return eps_r, sigma, s


def embedding_readout(v, W):
    """Sec. III-C: the scalars v . w_j of every material and embedding.
    v [L] is the read-out vector shared by all materials, W [n_mat, 4, L]
    holds each material's embeddings w_1 .. w_4.  Returns u [n_mat, 4]."""
    return torch.as_tensor(W, dtype=f64) @ torch.as_tensor(v, dtype=f64)


def materials_from_embeddings(v, W):
    """Eqs. trainable_materials_1-4: sigma = exp(v.w_1), eps_r = 1 +
    exp(v.w_2), S = logistic(v.w_3), K_x = logistic(v.w_4).  Returns
    (eps_r, sigma, S, K_x), each [n_mat]."""
    u = embedding_readout(v, W)
    sigma = torch.exp(u[:, 0])
    eps_r = 1.0 + torch.exp(u[:, 1])
    s = 1.0 / (1.0 + torch.exp(-u[:, 2]))
    kx = 1.0 / (1.0 + torch.exp(-u[:, 3]))
    return eps_r, sigma, s, kx


def specular_amplitude(s):
    """R = sqrt(1 - S^2): the specularly reflected amplitude fraction
    (Sec. II-D)."""
    return torch.sqrt(1.0 - s * s)


def permittivity(eps_r, sigma, freq):
    """eta = eps_r - j sigma / (eps0 * omega), omega = 2 pi f (Sec. II-D).

    The carrier frequency is used for every subcarrier (path coefficients
    are frozen at the carrier; only the delay phase varies with f)."""
    omega = 2.0 * math.pi * freq
    eps_r = torch.as_tensor(eps_r, dtype=f64)
    sigma = torch.as_tensor(sigma, dtype=f64)
    return torch.complex(eps_r, -sigma / (EPS0 * omega))


def fresnel(eta, cos_theta):
    """TE/TM Fresnel reflection coefficients, Eqs. (fresnel-1/-2):

        r_perp = (cos t - sqrt(eta - sin^2 t)) / (cos t + sqrt(eta - sin^2 t))
        r_par  = (eta cos t - sqrt(eta - sin^2 t)) / (eta cos t + sqrt(...))

    with the principal square root (Re >= 0).  cos_theta is the cosine of
    the angle between the incident direction and the (flipped) normal."""
    eta = torch.as_tensor(eta).to(c128)
    c = torch.as_tensor(cos_theta, dtype=f64).to(c128)
    sin2 = 1.0 - c * c
    root = torch.sqrt(eta - sin2)
    r_perp = (c - root) / (c + root)
    r_par = (eta * c - root) / (eta * c + root)
    return r_perp, r_par


def spherical_basis(k):
    """Unit vectors theta_hat, phi_hat at the direction k (float64 [...,3],
    unit norm), from the spherical angles theta = acos(k_z),
    phi = atan2(k_y, k_x)."""
    theta = torch.acos(torch.clamp(k[..., 2], -1.0, 1.0))
    phi = torch.atan2(k[..., 1], k[..., 0])
    ct, st = torch.cos(theta), torch.sin(theta)
    cp, sp = torch.cos(phi), torch.sin(phi)
    theta_hat = torch.stack([ct * cp, ct * sp, -st], dim=-1)
    phi_hat = torch.stack([-sp, cp, torch.zeros_like(cp)], dim=-1)
    return theta_hat, phi_hat


def pattern_isotropic(zeta):
    """Antenna field pattern C = [cos(zeta) sqrt(G), sin(zeta) sqrt(G)] with
    G = 1 (isotropic, radiation efficiency 1), Sec. II-B polarisation
    model.  Returned as a complex128 2-vector in the (theta_hat, phi_hat)
    basis."""
    return torch.tensor([math.cos(zeta), math.sin(zeta)], dtype=c128)


def wavelength(freq):
    return C0 / freq


def lambertian_pattern(cos_s):
    """Scattering pattern of a purely diffuse (Lambertian) surface, the first
    term of Eq. (trainable_scattering_pattern): f_s = cos(theta_s) / pi on
    the hemisphere of the incidence side, 0 behind the surface.  Its
    integral over that hemisphere is 1."""
    cos_s = torch.as_tensor(cos_s, dtype=f64)
    return torch.clamp(cos_s, min=0.0) / math.pi

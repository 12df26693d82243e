"""Antenna and scattering patterns and cross-polarisation (oracle, FP64).
Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library path.

  * trainable Tx gain (Sec. III-A): a mixture of M spherical Gaussians,
        G(r) = 4 pi eta_rad sum_i (w_i / a_i) exp(lambda_i mu_i . r),
        a_i = (2 pi / lambda_i) (exp(lambda_i) - exp(-lambda_i)),
    and the pattern C = sqrt(G) [cos zeta, sin zeta] (Eq. polarization_model)
  * trainable scattering pattern (Sec. III-B, Eq.
    trainable_scattering_pattern): a Lambertian lobe and two hemispherical
    Gaussians about the backscatter and the specular directions, each
    normalised by the approximation of Eq. normalization_hemisphere
  * backscattering-lobe pattern (Sec. II-D-2, Eq. backscattering_model):
    Lambda ((1 + k_r.k_s)/2)^alpha_r + (1 - Lambda) ((1 + k_b.k_s)/2)^alpha_s
    over its exact hemispherical integral
  * cross-polarisation K_x of a diffuse reflection: the scattered field is
    |E_s| [sqrt(1 - K_x), sqrt(K_x)] in its outgoing basis (Eq.
    scattered_field, chi = 0)

Readings (each listed with the design notes):
  * the factor 4 pi in G: each lobe exp(lambda mu.r)/a integrates to one over
    the sphere, so the mixture as printed integrates to eta_rad, while Eq.
    atenna_normalization asks for 4 pi eta_rad (an isotropic antenna has
    unit gain); the factor restores it;
  * the lobes' "incident direction" points from the surface back to the
    source, k_b = -k_in, which makes the second lobe the backscatter lobe the
    models are named for; k_r = k_in - 2 (n . k_in) n is the specular
    direction of the propagation direction k_in;
  * the hemispherical normaliser of a lobe with axis v uses cos(beta) =
    v . n (the part of the lobe above the surface), not the scattered
    direction; it interpolates between the exact hemispherical integrals
    at cos(beta) = -1 and +1 with the fraction s of Eq.
    normalization_hemisphere, which also makes it exact at cos(beta) = 0;
  * raw parametrisations: eta_rad = logistic, mixture weights = softmax of
    logits, concentrations = exp, mean directions = normalised 3-vectors;
    pattern lobe weights = softmax, lambda_2, lambda_3 = exp; K_x = logistic.
"""
import math

import torch

from .em import f64


def _dot(a, b):
    return (a * b).sum(-1)


# ------------------------------------------------------------ Tx gain
def vmf_from_raw(tx_raw, M):
    """[1 + 5M] raw vector -> (eta_rad, w [M], lam [M], mu [M, 3])."""
    tx_raw = torch.as_tensor(tx_raw, dtype=f64)
    eta = torch.sigmoid(tx_raw[0])
    w = torch.softmax(tx_raw[1:1 + M], 0)
    lam = torch.exp(tx_raw[1 + M:1 + 2 * M])
    m = tx_raw[1 + 2 * M:1 + 5 * M].reshape(M, 3)
    mu = m / torch.linalg.norm(m, dim=-1, keepdim=True)
    return eta, w, lam, mu


def vmf_gain(r, eta, w, lam, mu):
    """G(r) for unit directions r [..., 3] (Sec. III-A, with the factor 4 pi
    of Eq. atenna_normalization)."""
    c = r @ mu.T                                           # [..., M]
    # 4 pi (w/a) e^{lam c} = 2 w lam e^{lam (c - 1)} / (1 - e^{-2 lam})
    g = 2.0 * w * lam * torch.exp(lam * (c - 1.0)) / (1.0 - torch.exp(-2.0 * lam))
    return eta * g.sum(-1)


# --------------------------------------------------- scattering patterns
def meder_fraction(lam, cos_beta):
    """s of Eq. normalization_hemisphere: the approximate fraction of a
    spherical Gaussian of concentration lam whose axis makes cos_beta with
    the normal that lies above the surface (0 at -1, 1/2 at 0, 1 at +1)."""
    t = torch.sqrt(lam) * (1.6988 * lam ** 2 + 10.8438 * lam) / (lam ** 2 + 6.2201 * lam + 10.2415)
    return (1.0 - torch.exp(-t * (1.0 + cos_beta))) / (
        (1.0 - torch.exp(-t)) * (1.0 + torch.exp(-t * cos_beta)))


def hemi_norm_shifted(lam, cos_beta):
    """Approximate integral over the hemisphere of exp(lam (v.axis - 1)):
    (2 pi / lam) (1 - e^-lam) (e^-lam + s (1 - e^-lam)), the exact values
    (2 pi / lam)(1 - e^-lam) e^-lam at cos_beta = -1 and
    (2 pi / lam)(1 - e^-lam) at +1 joined by the fraction s."""
    e = torch.exp(-lam)
    s = meder_fraction(lam, cos_beta)
    return (2.0 * math.pi / lam) * (1.0 - e) * (e + s * (1.0 - e))


def pattern_from_raw(pat_raw):
    """[..., 6] raw per-material values -> (K_x, w [...,3], lam2, lam3)."""
    kx = torch.sigmoid(pat_raw[..., 0])
    w = torch.softmax(pat_raw[..., 1:4], -1)
    return kx, w, torch.exp(pat_raw[..., 4]), torch.exp(pat_raw[..., 5])


def trainable_pattern(k_in, k_s, n, w, lam2, lam3):
    """f_s(k_i, k_s, n) of Eq. trainable_scattering_pattern with n on the
    incidence side (n . k_in < 0).  w [..., 3], lam2, lam3 [...]."""
    k_b = -k_in
    k_r = k_in - 2.0 * _dot(k_in, n)[..., None] * n
    cos_s = _dot(k_s, n)
    cos_i = -_dot(k_in, n)
    lobe2 = torch.exp(lam2 * (_dot(k_s, k_b) - 1.0)) / hemi_norm_shifted(lam2, cos_i)
    lobe3 = torch.exp(lam3 * (_dot(k_s, k_r) - 1.0)) / hemi_norm_shifted(lam3, cos_i)
    f = w[..., 0] * cos_s / math.pi + w[..., 1] * lobe2 + w[..., 2] * lobe3
    return torch.where(cos_s > 0, f, torch.zeros_like(f))


def _lobe_hemi_integral(alpha, cos_t):
    """Exact integral over the hemisphere n.v >= 0 of ((1 + v.a)/2)^alpha
    for an axis a with a.n = cos_t (integer alpha >= 0): the binomial
    expansion in (a.v)^k, each integrated in closed form
        int (a.v)^k = sum_{j even} C(k, j) sin^j cos^{k-j} 2pi (j-1)!!/j!!
                      * B((j + 2)/2, (k - j + 1)/2) / 2."""
    sin_t = torch.sqrt(torch.clamp(1.0 - cos_t ** 2, min=0.0))
    total = torch.zeros_like(cos_t)
    for k in range(alpha + 1):
        ik = torch.zeros_like(cos_t)
        for j in range(0, k + 1, 2):
            dfac = 1.0
            for q in range(j - 1, 0, -2):
                dfac *= q
            for q in range(j, 0, -2):
                dfac /= q
            beta = math.exp(math.lgamma((j + 2) / 2) + math.lgamma((k - j + 1) / 2)
                            - math.lgamma((k + 3) / 2))
            ik = ik + (math.comb(k, j) * sin_t ** j * cos_t ** (k - j)
                       * 2.0 * math.pi * dfac * 0.5 * beta)
        total = total + math.comb(alpha, k) * ik
    return total / 2.0 ** alpha


def backscatter_pattern(k_in, k_s, n, alpha_r, alpha_s, Lam):
    """Eq. backscattering_model with its exact normaliser; integer alpha_r,
    alpha_s; n on the incidence side."""
    k_b = -k_in
    k_r = k_in - 2.0 * _dot(k_in, n)[..., None] * n
    cos_i = -_dot(k_in, n)
    cos_s = _dot(k_s, n)
    num = (Lam * ((1.0 + _dot(k_r, k_s)) / 2.0) ** alpha_r
           + (1.0 - Lam) * ((1.0 + _dot(k_b, k_s)) / 2.0) ** alpha_s)
    # both axes make cos_i with the normal
    F = Lam * _lobe_hemi_integral(alpha_r, cos_i) + (1.0 - Lam) * _lobe_hemi_integral(alpha_s, cos_i)
    f = num / F
    return torch.where(cos_s > 0, f, torch.zeros_like(f))

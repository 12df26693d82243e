"""First-order edge diffraction (oracle, FP64).  Test infrastructure only:
imported by tests, the smoke check and the CPU baseline of the benchmark,
never by the library path.

Sec. II-E models diffraction by the uniform theory of diffraction (UTD) of
Kouyoumjian and Pathak in an edge-fixed coordinate system, differentiable in
the materials of both faces of the wedge, and prints no formula for the
diffraction matrix.  Written here from that published method, with the
finite-conductivity form of Luebbers:

  * wedge of exterior angle n pi (0 < n <= 2); face 0 and face n; unit edge
    direction e oriented so that t0 = n0 x e points from the edge into face 0
    (n0 the normal of face 0 on the free-space side); the angle of a
    direction d about the edge is atan2(d_t . n0, d_t . t0), d_t the part of
    d normal to e, so that free space is 0 < phi < n pi
  * incidence: s' the propagation direction of the incident ray, phi' the
    angle of -s' (towards the source); diffraction: s the direction to the
    observer, phi its angle; cos(beta0) = s'.e = s.e (Keller's cone)
  * D_{s,h} = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0) *
        [ cot((pi + b-)/2n) F(k L a+(b-)) + cot((pi - b-)/2n) F(k L a-(b-))
          + R0 cot((pi - b+)/2n) F(k L a-(b+)) + Rn cot((pi + b+)/2n) F(k L a+(b+)) ]
    b- = phi - phi', b+ = phi + phi', a+-(b) = 2 cos^2((2 n pi N+- - b)/2)
    with N+- the integers closest to (b +- pi) / (2 n pi);
    a perfect conductor has R = -1 (soft) and +1 (hard); for a finite
    conductivity R0 and Rn are the Fresnel coefficients r_perp (soft) and
    r_par (hard) of face 0 at the grazing angle of the incident ray and of
    face n at the grazing angle of the diffracted ray
  * transition function F(x) = 2 j sqrt(x) e^{jx} int_{sqrt(x)}^inf e^{-j t^2} dt
  * L = s s' sin^2(beta0) / (s + s') for a spherical wave, spreading
    sqrt(s' / (s (s + s'))) and phase e^{-j k s} after the edge
  * E^d = -D_s E^i_beta beta_hat - D_h E^i_phi phi_hat with the edge-fixed
    bases phi_hat' = -(e x s')/|e x s'|, beta_hat' = phi_hat' x s' of the
    incident ray and phi_hat = (e x s)/|e x s|, beta_hat = phi_hat x s of the
    diffracted one.

Readings (each listed with the design notes): the grazing angles of the
finite-conductivity coefficients in three dimensions are taken from the
rays, cos(theta0) = sin(beta0) |sin phi'| and cos(thetan) = sin(beta0)
|sin(n pi - phi)| (Luebbers' angles phi' and n pi - phi at normal incidence);
the scattering coefficient S does not enter diffraction; in per-interaction
mode both faces take the interaction's values.  Luebbers' coefficients act
on the edge-fixed (soft, hard) components, which are the face's (TE, TM)
components only at normal incidence on the edge: for oblique rays on lossy
faces the total field keeps a small jump at the reflection boundaries (the
heuristic's own, pinned in the tests).
"""
import math

import numpy as np
import torch
from scipy.special import fresnel as _scipy_fresnel

from .em import c128, f64, fresnel


def _unit(v):
    return v / torch.linalg.norm(v, dim=-1, keepdim=True)


def _dot(a, b):
    return (a * b).sum(-1)


def transition_function(x):
    """F(x) for real x >= 0 (complex128 tensor), from the Fresnel integrals
    C(u), S(u) = int_0^u cos, sin(pi t^2 / 2) dt of scipy:
    int_a^inf e^{-j t^2} dt = sqrt(pi/2) [(1/2 - C(u)) - j (1/2 - S(u))],
    u = a sqrt(2/pi)."""
    x = np.asarray(torch.as_tensor(x, dtype=f64).detach().numpy(), np.float64)
    a = np.sqrt(x)
    s_u, c_u = _scipy_fresnel(a * math.sqrt(2.0 / math.pi))
    tail = math.sqrt(math.pi / 2.0) * ((0.5 - c_u) - 1j * (0.5 - s_u))
    return torch.tensor(2j * a * np.exp(1j * x) * tail, dtype=c128)


def _a_pm(beta, n, sign):
    """a+ (sign = +1) or a- (sign = -1) of the wedge at angle beta."""
    N = torch.round((beta + sign * math.pi) / (2.0 * n * math.pi))
    return 2.0 * torch.cos((2.0 * n * math.pi * N - beta) / 2.0) ** 2


def utd_coefficients(phi, phi_p, beta0, L, n, k, R0, Rn):
    """D for one polarisation: R0, Rn the face coefficients (complex,
    may require grad), phi, phi_p, beta0, L, n float64 tensors (geometry),
    k the wavenumber.  Returns complex128."""
    phi, phi_p, beta0, L, n = (torch.as_tensor(t, dtype=f64) for t in (phi, phi_p, beta0, L, n))
    bm = phi - phi_p
    bp = phi + phi_p
    kL = k * L

    def term(b, sign_cot, sign_a):
        cot = 1.0 / torch.tan((math.pi + sign_cot * b) / (2.0 * n))
        return cot.to(c128) * transition_function(kL * _a_pm(b, n, sign_a))

    pre = (-np.exp(-1j * math.pi / 4.0)
           / (2.0 * n * torch.sqrt(torch.as_tensor(2.0 * math.pi * k, dtype=f64)) * torch.sin(beta0)))
    return pre.to(c128) * (term(bm, +1.0, +1.0) + term(bm, -1.0, -1.0)
                           + R0 * term(bp, -1.0, -1.0) + Rn * term(bp, +1.0, +1.0))


def gtd_coefficients(phi, phi_p, beta0, n, k, R0, Rn):
    """Keller's geometrical-theory coefficient, the limit of D far from the
    shadow and reflection boundaries (F -> 1), summed in closed form:
    cot((pi + b)/2n) + cot((pi - b)/2n) = 2 sin(pi/n) / (cos(b/n) - cos(pi/n))."""
    phi, phi_p, beta0 = (torch.as_tensor(t, dtype=f64) for t in (phi, phi_p, beta0))
    pre = -np.exp(-1j * math.pi / 4.0) / (2.0 * n * math.sqrt(2.0 * math.pi * k)
                                          * torch.sin(beta0))
    s = math.sin(math.pi / n)
    c = math.cos(math.pi / n)
    inc = 2.0 * s / (torch.cos((phi - phi_p) / n) - c)
    # with distinct R0, Rn the reflected pair no longer sums in closed form
    cp = 1.0 / torch.tan((math.pi - (phi + phi_p)) / (2.0 * n))
    cn = 1.0 / torch.tan((math.pi + (phi + phi_p)) / (2.0 * n))
    return pre.to(c128) * (inc.to(c128) + R0 * cp.to(c128) + Rn * cn.to(c128))


def wedge_angle(d, e, n0):
    """Angle of direction d about the edge e, measured from face 0 (t0 =
    n0 x e) towards n0, in [0, 2 pi)."""
    t0 = torch.cross(n0, e, dim=-1)
    dt = d - _dot(d, e)[..., None] * e
    ang = torch.atan2(_dot(dt, n0), _dot(dt, t0))
    return torch.remainder(ang, 2.0 * math.pi)


def edge_geometry(src, q, obs, e, n0):
    """Incidence and diffraction geometry at the edge point q.  Returns a
    dict of s_in, s_out (unit propagation directions), s_p, s (distances),
    beta0, phi_p, phi, and the edge-fixed unit vectors beta_in, phi_in,
    beta_out, phi_out."""
    s_in = _unit(q - src)
    s_out = _unit(obs - q)
    phi_in = -_unit(torch.cross(e, s_in, dim=-1))
    beta_in = torch.cross(phi_in, s_in, dim=-1)
    phi_out = _unit(torch.cross(e, s_out, dim=-1))
    beta_out = torch.cross(phi_out, s_out, dim=-1)
    return dict(s_in=s_in, s_out=s_out, s_p=torch.linalg.norm(q - src, dim=-1),
                s=torch.linalg.norm(obs - q, dim=-1),
                beta0=torch.acos(torch.clamp(_dot(s_out, e), -1.0, 1.0)),
                phi_p=wedge_angle(-s_in, e, n0), phi=wedge_angle(s_out, e, n0),
                beta_in=beta_in, phi_in=phi_in, beta_out=beta_out, phi_out=phi_out)


def face_coefficients(eta0, eta_n, geo, n):
    """Luebbers' face coefficients (R0s, R0h, Rns, Rnh): Fresnel r_perp
    (soft) and r_par (hard) of face 0 at cos(theta0) = sin(beta0)|sin phi'|
    and of face n at cos(thetan) = sin(beta0)|sin(n pi - phi)|."""
    sb = torch.sin(geo["beta0"])
    c0 = sb * torch.abs(torch.sin(geo["phi_p"]))
    cn = sb * torch.abs(torch.sin(n * math.pi - geo["phi"]))
    r0s, r0h = fresnel(eta0, c0)
    rns, rnh = fresnel(eta_n, cn)
    return r0s, r0h, rns, rnh


def diffraction_step(E, p_out, q_out, geo, n, k, eta0, eta_n):
    """The field after the edge in the basis (beta_out, phi_out), without
    spreading and phase: E [..., 2] in the basis (p_out, q_out) of the
    incident ray.  Returns (E_out, D_s, D_h)."""
    L = geo["s"] * geo["s_p"] * torch.sin(geo["beta0"]) ** 2 / (geo["s"] + geo["s_p"])
    r0s, r0h, rns, rnh = face_coefficients(eta0, eta_n, geo, n)
    Ds = utd_coefficients(geo["phi"], geo["phi_p"], geo["beta0"], L, n, k, r0s, rns)
    Dh = utd_coefficients(geo["phi"], geo["phi_p"], geo["beta0"], L, n, k, r0h, rnh)
    yb = _dot(geo["beta_in"], p_out) * E[..., 0] + _dot(geo["beta_in"], q_out) * E[..., 1]
    yp = _dot(geo["phi_in"], p_out) * E[..., 0] + _dot(geo["phi_in"], q_out) * E[..., 1]
    return torch.stack([-Ds * yb, -Dh * yp], dim=-1), Ds, Dh

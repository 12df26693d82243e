"""Per-path field computation (oracle, FP64).  Test infrastructure only.

Follows Sec. II-C (transfer function), Sec. II-D-1 (specular reflection) and
Eq. (cfr_cont) of the paper, evaluated path by path (vectorised over paths,
one interaction slot at a time):

  E <- C_T(k_1) in the (theta_hat, phi_hat) basis of the departure direction
  for each reflection j:   E <- diag(R r_perp, R r_par) D_j E
  at the receiver:         E <- D_{Q+1} E in the Rx (theta_hat, phi_hat) basis
  a = lambda/(4 pi) * C_R^H E / (c tau)

A diffuse reflection (Sec. II-D-2, Eq. scattered_field) may end a path
(store kind 1 at its last interaction; elsewhere the kind is ignored and
the interaction is specular):

  y = D_Q E in the incidence basis, Gamma |E| = |diag(r_perp, r_par) y|,
  |E_s|^2 = |E|^2 cos(theta_i) dA S^2 Gamma^2 f_s,  f_s = cos(theta_s)/pi,
  E <- [|E_s|, 0] in the outgoing basis (K_x = 0, chi_1 = chi_2 = 0),
  a = lambda/(4 pi) * C_R^H D_{Q+1} E / (rho_Q d_{Q+1})

with rho_Q the unfolded length from the Tx to the diffuse point (the
incoming wave's spreading) and d_{Q+1} the distance to the Rx (the
scattered spherical wave's).

A first-order edge diffraction (Sec. II-E; store kind 2, the path's only
interaction, the stored normal that of face 0 on the free-space side) takes
the incident field into the edge-fixed basis, applies diag(-D_s, -D_h) of
oracle.diffraction with the face materials of the interaction (face 0) and
of the store's face-n id, and ends in the diffracted edge-fixed basis:

  a = lambda/(4 pi) * C_R^H D_2 E / sqrt(s' s (s + s'))

(the incident spherical wave's 1/s' times the spreading sqrt(s'/(s(s+s')))).

Readings (the paper is silent or cites without printing):
  * spreading: planar reflectors and a point source give A^r = rho/(rho+d),
    whose product with 1/d_1 telescopes to 1/(total length) = 1/(c tau);
    tau is taken from the path store, not recomputed from FP32 points.
  * reflection bases: e_perp = k_i x n / |k_i x n|, e_par_in = e_perp x k_i,
    e_par_out = e_perp x k_r, components ordered (perp, par) as in
    diag(r_perp, r_par).
  * the stored normal may face either way; it is flipped per interaction so
    that cos(theta_i) = -k_i . n > 0.
  * normal incidence (|k_i x n| < 1e-7): e_perp is the incoming field
    basis' first vector made orthogonal to k_i (the result does not depend
    on the choice there because r_par = -r_perp).
  * both antenna ends use the spherical basis of the direction pointing away
    from the antenna along the path: k_1 at the Tx, -k_{Q+1} at the Rx.
  * coefficients are evaluated at the carrier: lambda_c, eta(omega_c).
  * array phase: element m of a half-wavelength ULA along u, centred on the
    Tx, sees psi_i (m - (M-1)/2) with psi_i = pi k_1 . u (carrier only).
  * diffuse reflection: the scattered field takes the outgoing basis
    e_perp = k_s x n / |k_s x n|, e_par = e_perp x k_s (built from the
    scattered direction and the normal as for a reflection; if k_s is along
    n, e_perp is the incidence e_perp made orthogonal to k_s); with K_x = 0
    all of |E_s| is in e_perp.  Its phase is the propagation delay alone
    (chi = 0; the phase of the incoming field does not carry over, only its
    norm does), and the Rx behind the surface (cos theta_s <= 0) gets 0.
"""
import math

import numpy as np
import torch

from .em import (C0, c128, f64, fresnel, lambertian_pattern, materials_from_raw,
                 pattern_isotropic, permittivity, spherical_basis, specular_amplitude,
                 wavelength)


def _unit(v):
    return v / torch.linalg.norm(v, dim=-1, keepdim=True)


def _dot(a, b):
    return (a * b).sum(-1)


def specular_step(E, p_out, q_out, k_in, n, eta, R):
    """One specular reflection (Eqs. rel1, basis_transform, rel2,
    specular_reflection).

    E: complex [...,2] field in the outgoing basis (p_out, q_out) of the
    previous process; k_in: incident unit direction; n: stored unit normal;
    eta: complex permittivity; R: specular amplitude fraction.
    Returns (E_out, e_perp, e_par_in, e_par_out, k_r, cos_theta)."""
    flip = _dot(k_in, n) > 0
    n = torch.where(flip[..., None], -n, n)
    cos_t = -_dot(k_in, n)
    cr = torch.cross(k_in, n, dim=-1)
    crn = torch.linalg.norm(cr, dim=-1, keepdim=True)
    # normal incidence fallback
    alt = p_out - _dot(p_out, k_in)[..., None] * k_in
    alt = alt / torch.linalg.norm(alt, dim=-1, keepdim=True)
    small = crn < 1e-7
    e_perp = torch.where(small, alt, cr / torch.where(small, torch.ones_like(crn), crn))
    e_par_in = torch.cross(e_perp, k_in, dim=-1)
    k_r = k_in - 2.0 * _dot(k_in, n)[..., None] * n
    e_par_out = torch.cross(e_perp, k_r, dim=-1)
    # basis change D: rows = new incoming basis, columns = previous outgoing
    d00 = _dot(e_perp, p_out)
    d01 = _dot(e_perp, q_out)
    d10 = _dot(e_par_in, p_out)
    d11 = _dot(e_par_in, q_out)
    e0 = d00 * E[..., 0] + d01 * E[..., 1]
    e1 = d10 * E[..., 0] + d11 * E[..., 1]
    r_perp, r_par = fresnel(eta, cos_t)
    E_out = torch.stack([R * r_perp * e0, R * r_par * e1], dim=-1)
    return E_out, e_perp, e_par_in, e_par_out, k_r, cos_t


def _sqrt0(x):
    """sqrt with a zero (not NaN) gradient at x <= 0."""
    pos = x > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, x, torch.ones_like(x))),
                       torch.zeros_like(x))


def diffuse_step(E, p_out, q_out, k_in, n, eta, S, dA, k_s, pattern=None, kx=None):
    """One diffuse reflection (Eq. scattered_field, chi = 0), without the
    spreading factors (the caller divides by rho_Q d_{Q+1}).

    E: complex [...,2] field in the outgoing basis (p_out, q_out) of the
    previous process; k_in: incident direction; n: stored unit normal;
    eta: complex permittivity; S: scattering coefficient; dA: area element;
    k_s: scattered direction; pattern: f_s(k_in, k_s, n) with n on the
    incidence side, or None for the Lambertian cos(theta_s)/pi; kx: K_x, or
    None for 0.  Returns (E_out, e_perp_s, e_par_s)."""
    flip = _dot(k_in, n) > 0
    n = torch.where(flip[..., None], -n, n)
    cos_i = -_dot(k_in, n)
    cos_s = _dot(k_s, n)
    f_s = lambertian_pattern(cos_s) if pattern is None else pattern(k_in, k_s, n)
    cr = torch.cross(k_in, n, dim=-1)
    crn = torch.linalg.norm(cr, dim=-1, keepdim=True)
    alt = p_out - _dot(p_out, k_in)[..., None] * k_in
    alt = alt / torch.linalg.norm(alt, dim=-1, keepdim=True)
    small = crn < 1e-7
    e_perp = torch.where(small, alt, cr / torch.where(small, torch.ones_like(crn), crn))
    e_par_in = torch.cross(e_perp, k_in, dim=-1)
    y0 = _dot(e_perp, p_out) * E[..., 0] + _dot(e_perp, q_out) * E[..., 1]
    y1 = _dot(e_par_in, p_out) * E[..., 0] + _dot(e_par_in, q_out) * E[..., 1]
    r_perp, r_par = fresnel(eta, cos_i)
    # Gamma |E_in| = |diag(r_perp, r_par) y|
    g_norm = _sqrt0(torch.abs(r_perp * y0) ** 2 + torch.abs(r_par * y1) ** 2)
    amp = S * g_norm * _sqrt0(torch.clamp(cos_i, min=0.0) * dA * f_s)
    # outgoing basis from (k_s, n)
    cs = torch.cross(k_s, n, dim=-1)
    csn = torch.linalg.norm(cs, dim=-1, keepdim=True)
    alt_s = e_perp - _dot(e_perp, k_s)[..., None] * k_s
    alt_s = alt_s / torch.linalg.norm(alt_s, dim=-1, keepdim=True)
    small_s = csn < 1e-7
    e_perp_s = torch.where(small_s, alt_s, cs / torch.where(small_s, torch.ones_like(csn), csn))
    e_par_s = torch.cross(e_perp_s, k_s, dim=-1)
    if kx is None:
        E_out = torch.stack([amp.to(c128), torch.zeros_like(amp).to(c128)], dim=-1)
    else:
        E_out = torch.stack([(amp * _sqrt0(1.0 - kx)).to(c128), (amp * _sqrt0(kx)).to(c128)],
                            dim=-1)
    return E_out, e_perp_s, e_par_s


def _gather_paths(store, sel):
    P_all = int(store.n_paths)
    D = int(store.max_depth)
    link_of = np.repeat(np.arange(store.n_links), np.diff(store.link_off))[sel]
    tx = torch.tensor(store.tx_pos[link_of], dtype=f64)
    rx = torch.tensor(store.rx_pos[link_of], dtype=f64)
    depth = torch.tensor(store.depth[sel].astype(np.int64))
    pts, nrm, mat, kind, dA = [], [], [], [], []
    for k in range(D):
        idx = k * P_all + sel
        pts.append(torch.tensor(store.pts[:, idx].T, dtype=f64))
        nrm.append(torch.tensor(store.nrm[:, idx].T, dtype=f64))
        mat.append(torch.tensor(store.mat[idx].astype(np.int64)))
        kind.append(torch.tensor(store.kind[idx].astype(np.int64)))
        dA.append(torch.tensor(store.dA[idx], dtype=f64))
    tau = torch.tensor(store.tau[sel], dtype=f64)
    return tx, rx, depth, pts, nrm, mat, tau, kind, dA


def departure_direction(store, sel=None):
    """k_1, the unit direction leaving the Tx, per path (float64 [P,3])."""
    sel = np.arange(store.n_paths) if sel is None else np.asarray(sel)
    tx, rx, depth, pts, _, _, _, _, _ = _gather_paths(store, sel)
    first = torch.where((depth > 0)[:, None], pts[0], rx) if store.max_depth > 0 else rx
    return _unit(first - tx)


def _gather_edges(store, sel):
    """Edge direction [P,3], wedge n [P] and face-n material [P] of the
    selected paths (zeros where the store has no diffraction paths)."""
    if store.edge is None:
        P = len(sel)
        return (torch.zeros((P, 3), dtype=f64), torch.zeros(P, dtype=f64),
                torch.zeros(P, dtype=torch.int64))
    e = torch.tensor(store.edge[:3, sel].T, dtype=f64)
    return e, torch.tensor(store.edge[3, sel], dtype=f64), torch.tensor(
        store.mat_n[sel].astype(np.int64))


def trace_fields(store, eps_r, sigma, s, fc, zeta_tx=0.0, zeta_rx=0.0,
                 ula_axis=(1.0, 0.0, 0.0), sel=None, tx_gain=None, kx=None, pattern=None,
                 eps_n=None, sigma_n=None):
    """Path coefficients a_i and array phase steps psi_i.

    eps_r, sigma, s: per-interaction material values, float64 tensors of
    shape [max_depth, P] (P = len(sel)), may require grad.  Slots beyond a
    path's depth are ignored.  Optional: tx_gain, a callable r -> G(r) on
    unit departure directions (Sec. III-A; isotropic if None); kx [D, P]
    K_x per interaction; pattern(k, k_in, k_s, n) -> f_s for interaction
    slot k (Lambertian if None); eps_n, sigma_n [P]: the material of face n
    of a diffracting wedge (default: the interaction's own, slot 0).
    Returns (a complex128 [P], psi float64 [P])."""
    sel = np.arange(store.n_paths) if sel is None else np.asarray(sel)
    tx, rx, depth, pts, nrm, _, tau, kind, dA = _gather_paths(store, sel)
    P = len(sel)
    D = int(store.max_depth)
    lam = wavelength(fc)
    first = torch.where((depth > 0)[:, None], pts[0], rx) if D > 0 else rx
    k1 = _unit(first - tx)
    p_out, q_out = spherical_basis(k1)
    E = pattern_isotropic(zeta_tx).expand(P, 2).clone()
    if tx_gain is not None:
        # C = sqrt(G) [cos zeta, sin zeta] (Eq. polarization_model)
        E = E * _sqrt0(tx_gain(k1)).to(c128)[:, None]
    prev = tx
    rho = torch.zeros(P, dtype=f64)  # unfolded length from the Tx
    diffuse_end = torch.zeros(P, dtype=torch.bool)
    diffracted = torch.zeros(P, dtype=torch.bool)
    spread_d = torch.ones(P, dtype=f64)
    up = torch.tensor([0.0, 0.0, 1.0], dtype=f64).expand(P, 3)
    xhat = torch.tensor([1.0, 0.0, 0.0], dtype=f64).expand(P, 3)
    for k in range(D):
        act = depth > k
        # inactive slots get a harmless stand-in geometry so that no NaN
        # enters the graph; their results are discarded below
        s_k = torch.where(act[:, None], pts[k], prev + up)
        n_k = torch.where(act[:, None], nrm[k], xhat)
        k_in = _unit(s_k - prev)
        eta = permittivity(eps_r[k], sigma[k], fc)
        R = specular_amplitude(s[k])
        E_new, e_perp, _, e_par_out, _, _ = specular_step(E, p_out, q_out, k_in, n_k, eta, R)
        # a diffuse reflection is honoured at a path's last interaction
        dif = act & (kind[k] == 1) & (depth == k + 1)
        if bool(dif.any()):
            # stand-in geometry for the other lanes keeps the graph finite
            rx_k = torch.where(dif[:, None], rx, s_k + 2.0 * n_k + up)
            k_s = _unit(rx_k - s_k)
            s_dif = torch.where(dif, s[k], torch.zeros_like(s[k]))
            pat_k = None if pattern is None else (lambda a, b, c, k=k: pattern(k, a, b, c))
            E_d, ep_d, eq_d = diffuse_step(E, p_out, q_out, k_in, n_k, eta, s_dif,
                                           torch.where(dif, dA[k], torch.ones_like(dA[k])), k_s,
                                           pattern=pat_k, kx=None if kx is None else kx[k])
            E_new = torch.where(dif[:, None], E_d, E_new)
            e_perp = torch.where(dif[:, None], ep_d, e_perp)
            e_par_out = torch.where(dif[:, None], eq_d, e_par_out)
            diffuse_end = diffuse_end | dif
        # first-order edge diffraction (Sec. II-E): the path's one interaction
        dfr = (act & (kind[k] == 2) & (depth == 1)
               if k == 0 and store.edge is not None else None)
        if dfr is not None and bool(dfr.any()):
            from . import diffraction as odf
            e_all, n_all, _ = _gather_edges(store, sel)
            # stand-in wedge geometry for the other lanes keeps the graph finite
            sd = lambda v, alt: torch.where(dfr[:, None], v, torch.tensor(alt, dtype=f64))  # noqa: E731
            geo = odf.edge_geometry(sd(prev, [-3.0, 4.0, 0.4]), sd(s_k, [0.0, 0.0, 0.0]),
                                    sd(rx, [-2.0, -1.5, 1.1]), sd(e_all, [0.0, 0.0, 1.0]),
                                    sd(n_k, [0.0, 1.0, 0.0]))
            n_w = torch.where(dfr, n_all, torch.full_like(n_all, 1.5))
            eta_n = eta if eps_n is None else permittivity(eps_n, sigma_n, fc)
            E_w, _, _ = odf.diffraction_step(E, p_out, q_out, geo, n_w, 2.0 * math.pi / lam,
                                             eta, eta_n)
            E_new = torch.where(dfr[:, None], E_w, E_new)
            e_perp = torch.where(dfr[:, None], geo["beta_out"], e_perp)
            e_par_out = torch.where(dfr[:, None], geo["phi_out"], e_par_out)
            # spherical-wave spreading: (1/s') sqrt(s' / (s (s + s')))
            sp = geo["s_p"]
            so = geo["s"]
            spread_d = torch.where(dfr, torch.sqrt(sp * so * (sp + so)), spread_d)
            diffracted = diffracted | dfr
        E = torch.where(act[:, None], E_new, E)
        p_out = torch.where(act[:, None], e_perp, p_out)
        q_out = torch.where(act[:, None], e_par_out, q_out)
        rho = torch.where(act, rho + torch.linalg.norm(s_k - prev, dim=-1), rho)
        prev = torch.where(act[:, None], s_k, prev)
    k_last = _unit(rx - prev)
    t_r, p_r = spherical_basis(-k_last)
    e0 = _dot(t_r, p_out) * E[:, 0] + _dot(t_r, q_out) * E[:, 1]
    e1 = _dot(p_r, p_out) * E[:, 0] + _dot(p_r, q_out) * E[:, 1]
    c_r = pattern_isotropic(zeta_rx)
    received = c_r[0].conj() * e0 + c_r[1].conj() * e1
    # spreading: 1/(total length) along specular chains; 1/(rho_Q d_{Q+1})
    # for a path ending in a diffuse reflection
    d_last = torch.linalg.norm(rx - prev, dim=-1)
    length = torch.where(diffuse_end, rho * d_last, C0 * tau)
    length = torch.where(diffracted, spread_d, length)
    a = (lam / (4.0 * math.pi)) * received / length
    u = torch.tensor(ula_axis, dtype=f64)
    psi = math.pi * _dot(k1, u.expand(P, 3))
    return a, psi


def per_interaction_from_ids(store, table, sel=None):
    """Gather a per-material table [n_mat] onto interaction slots -> [D, P]."""
    sel = np.arange(store.n_paths) if sel is None else np.asarray(sel)
    P_all = int(store.n_paths)
    rows = []
    for k in range(int(store.max_depth)):
        ids = torch.tensor(store.mat[k * P_all + sel].astype(np.int64))
        rows.append(table[ids])
    if not rows:
        return torch.zeros((0, len(sel)), dtype=table.dtype)
    return torch.stack(rows)


def trace_fields_per_id(store, raw, fc, sel=None, tx_raw=None, n_vmf=0, pat_raw=None,
                        backscatter=None, **kw):
    """Per-material-id mode: raw [n_mat, 3] -> (eps_r, sigma, S) by the
    Sec. III-C transforms, gathered per interaction, then trace_fields.

    Optional: tx_raw [1 + 5 n_vmf], the raw trainable Tx gain (Sec. III-A);
    pat_raw [n_mat, 6], per material the raw K_x and trainable scattering
    pattern (Sec. III-B); or backscatter = (kx [n_mat], alpha_r, alpha_s,
    Lam [n_mat]), the backscattering-lobe pattern (Eq.
    backscattering_model) with its K_x, for ground truth."""
    from . import patterns as pt
    eps_r, sigma, s = materials_from_raw(raw)
    gather = lambda t: per_interaction_from_ids(store, t, sel)  # noqa: E731
    if tx_raw is not None:
        eta, w, lam, mu = pt.vmf_from_raw(tx_raw, n_vmf)
        kw["tx_gain"] = lambda r: pt.vmf_gain(r, eta, w, lam, mu)
    if pat_raw is not None:
        kx, w3, lam2, lam3 = pt.pattern_from_raw(torch.as_tensor(pat_raw, dtype=f64))
        kx_i, w_i = gather(kx), torch.stack([gather(w3[:, c]) for c in range(3)], -1)
        l2_i, l3_i = gather(lam2), gather(lam3)
        kw["kx"] = kx_i
        kw["pattern"] = lambda k, k_in, k_s, n: pt.trainable_pattern(k_in, k_s, n, w_i[k],
                                                                     l2_i[k], l3_i[k])
    elif backscatter is not None:
        kx, a_r, a_s, Lam = backscatter
        kw["kx"] = gather(torch.as_tensor(kx, dtype=f64))
        Lam_i = gather(torch.as_tensor(Lam, dtype=f64))
        kw["pattern"] = lambda k, k_in, k_s, n: pt.backscatter_pattern(k_in, k_s, n, a_r, a_s,
                                                                       Lam_i[k])
    if store.edge is not None:
        sel_ = np.arange(store.n_paths) if sel is None else np.asarray(sel)
        mn = torch.tensor(store.mat_n[sel_].astype(np.int64))
        kw["eps_n"], kw["sigma_n"] = eps_r[mn], sigma[mn]
    return trace_fields(store, gather(eps_r), gather(sigma), gather(s), fc, sel=sel, **kw)

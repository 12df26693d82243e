"""Channel synthesis and losses (oracle, FP64).  Test infrastructure only.

  * CFR as a sum over paths, Eq. (cfr_cont): H(f) = sum_i a_i e^{-j 2 pi f tau_i}
  * discrete OFDM CFR, Sec. II-A: H[n] = H(f_c + n df), n = -N/2 .. N/2-1,
    stored at index n + N/2 (odd N: n = -(N-1)/2 .. (N-1)/2)
  * CIR by the centred N-point IDFT with 1/sqrt(N), Sec. II-A; the power
    delay profile p_l = |h[l]|^2 (Eq. delay_spread's p_l)
  * workload loss: coherent NMSE + power-delay-profile NMSE, each normalised
    by the target energy over the whole batch, unit weights by default.
"""
import math

import numpy as np
import torch

from .em import c128, f64


def subcarrier_freqs(fc, bandwidth, n_sc):
    """f_n = fc + (n - floor(N/2)) * W/N for storage index n = 0..N-1 (for
    the even N of Sec. II-A, n - N/2 = -N/2 .. N/2-1; for odd N the carrier
    is the middle subcarrier)."""
    n = torch.arange(n_sc, dtype=f64)
    return fc + (n - (n_sc // 2)) * (bandwidth / n_sc)


def array_coefficients(a, psi, g):
    """b[i, m] = a_i g_m exp(j psi_i (m - (M-1)/2)): the per-element path
    coefficient of a centred ULA (phase taken at the carrier)."""
    M = g.shape[0]
    m = torch.arange(M, dtype=f64) - (M - 1) / 2.0
    phase = psi[:, None] * m[None, :]
    return a[:, None] * g[None, :] * torch.exp(1j * phase.to(c128))


def cfr(link_off, tau, a, psi, g, freqs, links=None):
    """H[l, m, n] = sum_{i in link l} b[i, m] exp(-j 2 pi f_n tau_i).

    The exponentials are evaluated directly in float64 from f_n * tau_i (no
    recurrence); the sum over paths is a plain complex matrix product per
    link.  a, psi, tau are indexed by global path id; returns complex128
    [len(links), M, N]."""
    link_off = np.asarray(link_off)
    links = range(len(link_off) - 1) if links is None else links
    tau = torch.as_tensor(tau, dtype=f64)
    out = []
    b_all = array_coefficients(a, psi, g)
    for l in links:
        lo, hi = int(link_off[l]), int(link_off[l + 1])
        ph = -2.0 * math.pi * freqs[None, :] * tau[lo:hi, None]
        e = torch.exp(1j * ph.to(c128))              # [P_l, N]
        out.append(b_all[lo:hi].transpose(0, 1) @ e)  # [M, N]
    if not out:
        return torch.zeros((0, g.shape[0], freqs.shape[0]), dtype=c128)
    return torch.stack(out)


def cir(H):
    """Centred IDFT with 1/sqrt(N) over the last axis.  Returns h with the
    delay index l = -N/2..N/2-1 stored at l + N/2."""
    N = H.shape[-1]
    n = torch.arange(N, dtype=f64) - N / 2
    ell = torch.arange(N, dtype=f64) - N / 2
    kern = torch.exp(1j * (2.0 * math.pi / N) * (n[:, None] * ell[None, :]).to(c128))
    return (H @ kern) / math.sqrt(N)


def pdp(H):
    """Power delay profile p_l = |h[l]|^2 via the library inverse FFT:
    p = N |ifft(H)|^2 (the centring only reorders the taps and multiplies by
    a unit-modulus factor, neither of which changes |.|^2 up to ordering)."""
    N = H.shape[-1]
    return N * torch.abs(torch.fft.ifft(H, dim=-1)) ** 2


def cfr_loss_sums(H, H_tgt):
    """The four sums of the workload loss over a batch [B, M, N]:
    (sum |H - H*|^2, sum |H*|^2, sum (p - p*)^2, sum (p*)^2)."""
    p = pdp(H)
    pt = pdp(H_tgt)
    return (torch.sum(torch.abs(H - H_tgt) ** 2), torch.sum(torch.abs(H_tgt) ** 2),
            torch.sum((p - pt) ** 2), torch.sum(pt ** 2))


def cfr_loss(H, H_tgt, w_coh=1.0, w_pdp=1.0):
    """Coherent + incoherent CFR loss over a batch [B, M, N]:

        L_coh = sum |H - H*|^2 / sum |H*|^2
        L_pdp = sum (p - p*)^2 / sum (p*)^2
        L = w_coh L_coh + w_pdp L_pdp

    Returns (L, L_coh, L_pdp) as float64 scalars."""
    e_coh, z_coh, e_pdp, z_pdp = cfr_loss_sums(H, H_tgt)
    coh = e_coh / z_coh
    inc = e_pdp / z_pdp
    return w_coh * coh + w_pdp * inc, coh, inc


def nmse(H, H_tgt):
    """Held-out CFR NMSE = sum|H - H*|^2 / sum|H*|^2."""
    return torch.sum(torch.abs(H - H_tgt) ** 2) / torch.sum(torch.abs(H_tgt) ** 2)

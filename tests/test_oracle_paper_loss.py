"""Pins of the oracle's paper loss (Sec. III-E Eqs. loss, smape,
delay_spread, channel_gain; Sec. III-F Eqs. scaling_param, alpha_hat;
Sec. IV-C ALE/RAE), each against something the oracle does not compute
itself: closed forms of spike and flat delay profiles, a library weighted
variance, Parseval, invariances, a least-squares solver and central
differences."""
import math

import numpy as np
import pytest
import torch

from oracle import paper_loss as pl

f64 = torch.float64
c128 = torch.complex128


def spikes(N, taps, amps):
    """CFR rows (storage order, subcarrier n at offset n - N/2) of paths at
    integer tap delays: H[n] = sum_i a_i exp(-j 2 pi (n - N/2) l_i / N).
    Their CIR is a_i sqrt(N) at tap l_i and exactly zero elsewhere."""
    n = np.arange(N) - N // 2
    H = np.zeros(N, np.complex128)
    for l, a in zip(taps, amps):
        H += a * np.exp(-2j * np.pi * n * l / N)
    return torch.tensor(H)


def random_cfr(rng, rows, N, n_paths=12, max_tap=40.0):
    """Rows of fractional-delay multipath CFRs (leakage over every tap)."""
    n = np.arange(N) - N // 2
    out = np.zeros((rows, N), np.complex128)
    for b in range(rows):
        d = rng.uniform(0.0, max_tap, n_paths)
        a = (rng.normal(size=n_paths) + 1j * rng.normal(size=n_paths)) * np.exp(-d / 10.0)
        out[b] = (a[:, None] * np.exp(-2j * np.pi * n[None, :] * d[:, None] / N)).sum(0)
    return torch.tensor(out)


W = 50e6


@pytest.mark.parametrize("N", [64, 1024])
def test_two_spikes_closed_form(N):
    a1, a2 = 0.7 * np.exp(0.3j), 1.9 * np.exp(-2.0j)
    l1, l2 = 3, 17
    H = spikes(N, [l1, l2], [a1, a2])
    P, tau = pl.gain_and_delay_spread(H[None], W)
    e1, e2 = abs(a1) ** 2, abs(a2) ** 2
    assert abs(P.item() - N * (e1 + e2)) <= 1e-12 * N * (e1 + e2)
    w1, w2 = e1 / (e1 + e2), e2 / (e1 + e2)
    ref = abs(l1 - l2) * math.sqrt(w1 * w2) / W
    assert abs(tau.item() - ref) <= 1e-12 * ref


def test_negative_taps_are_early_delays():
    # a spike at tap -5 (wrapped) and one at +5: mean 0, spread 5 taps
    N = 128
    H = spikes(N, [-5, 5], [1.0, 1.0])
    _, tau = pl.gain_and_delay_spread(H[None], W)
    assert abs(tau.item() - 5.0 / W) <= 1e-12 * 5.0 / W


@pytest.mark.parametrize("N", [16, 256])
def test_flat_profile_closed_form(N):
    # one occupied subcarrier -> |h[l]|^2 = |c|^2 / N on every tap: the
    # discrete uniform distribution on N consecutive integers
    c = 0.3 - 1.1j
    H = torch.zeros(N, dtype=c128)
    H[5] = c
    P, tau = pl.gain_and_delay_spread(H[None], W)
    assert abs(P.item() - abs(c) ** 2) <= 1e-13
    ref = math.sqrt((N * N - 1) / 12.0) / W
    assert abs(tau.item() - ref) <= 1e-12 * ref


def test_spread_matches_library_weighted_variance():
    rng = np.random.default_rng(3)
    N = 256
    taps = rng.choice(np.arange(-60, 100), 5, replace=False)
    amps = rng.normal(size=5) + 1j * rng.normal(size=5)
    _, tau = pl.gain_and_delay_spread(spikes(N, taps, amps)[None], W)
    var = np.cov(taps.astype(np.float64), aweights=np.abs(amps) ** 2, bias=True)
    assert abs(tau.item() - math.sqrt(var) / W) <= 1e-12 * tau.item()


def test_gain_is_cfr_energy():
    # Parseval for the unitary IDFT
    H = random_cfr(np.random.default_rng(4), 6, 512)
    P, _ = pl.gain_and_delay_spread(H, W)
    ref = (H.abs() ** 2).sum(-1)
    assert torch.allclose(P, ref, rtol=1e-12, atol=0)


def test_invariances():
    rng = np.random.default_rng(5)
    H = random_cfr(rng, 4, 256)
    P, tau = pl.gain_and_delay_spread(H, W)
    # a complex scale leaves the spread and multiplies the gain by |c|^2
    c = 2.5 * np.exp(0.7j)
    P2, tau2 = pl.gain_and_delay_spread(H * c, W)
    assert torch.allclose(tau2, tau, rtol=1e-12, atol=0)
    assert torch.allclose(P2, P * abs(c) ** 2, rtol=1e-12, atol=0)
    # a delay by an integer number of taps shifts spike profiles rigidly
    N = 256
    taps, amps = [2, 9, 30], [1.0, 0.5j, -0.8]
    n = torch.arange(N, dtype=f64) - N // 2
    sh = torch.exp(-2j * math.pi * n * 11 / N)
    _, t0 = pl.gain_and_delay_spread(spikes(N, taps, amps)[None], W)
    _, t1 = pl.gain_and_delay_spread((spikes(N, taps, amps) * sh)[None], W)
    assert abs(t1.item() - t0.item()) <= 1e-12 * t0.item()
    # the conversion to seconds is 1 / W
    _, t3 = pl.gain_and_delay_spread(H, 2 * W)
    assert torch.allclose(t3 * 2, tau, rtol=1e-14, atol=0)


def test_zero_row_and_single_tap():
    N = 64
    H = torch.zeros((2, N), dtype=c128)
    H[1] = spikes(N, [7], [2.0])
    P, tau = pl.gain_and_delay_spread(H, W)
    assert P[0].item() == 0.0 and tau[0].item() == 0.0
    assert abs(P[1].item() - 4.0 * N) <= 1e-12 * N and tau[1].item() < 1e-9 / W


def test_smape_values():
    x = torch.tensor([1.0, 3.0, 2.0, 0.0, 0.0, 5.0], dtype=f64)
    y = torch.tensor([1.0, 1.0, 0.0, 0.0, 4.0, 15.0], dtype=f64)
    ref = torch.tensor([0.0, 0.5, 1.0, 0.0, 1.0, 0.5], dtype=f64)
    assert torch.equal(pl.smape(x, y), ref)
    assert torch.equal(pl.smape(y, x), ref)


def test_alpha_hat_least_squares():
    rng = np.random.default_rng(6)
    P = rng.uniform(0.1, 2.0, 50)
    P_hat = 0.37 * P * rng.uniform(0.8, 1.2, 50)
    sol = np.linalg.lstsq(P[:, None], P_hat, rcond=None)[0][0]
    assert abs(pl.alpha_hat(P, P_hat) - sol) <= 1e-13 * abs(sol)
    assert abs(pl.alpha_hat(P, 3.0 * P) - 3.0) <= 1e-15


def test_alpha_ema_sequence():
    # alpha_0 = alpha^_1, so alpha_1 = alpha^_1; then the moving average
    seq, a = [], None
    for i, ah in enumerate([2.0, 4.0, 6.0]):
        a = pl.alpha_ema(a, ah, 0.5, i == 0)
        seq.append(a)
    assert seq == [2.0, 3.0, 4.5]
    assert pl.alpha_ema(7.0, 1.0, 0.0, False) == 1.0


def test_ale_rae():
    P_m = torch.tensor([1.0, 3.0, 2.0, 2.0], dtype=f64)   # two points, two antennas
    t_m = torch.tensor([10e-9, 30e-9, 4e-9, 8e-9], dtype=f64)
    P_p = torch.tensor([20.0, 20.0, 2.0, 2.0], dtype=f64)
    t_p = torch.tensor([30e-9, 30e-9, 3e-9, 3e-9], dtype=f64)
    ale, rae = pl.ale_rae(P_m, t_m, P_p, t_p, 2)
    assert abs(ale[0].item() - 10.0) <= 1e-12 and abs(ale[1].item()) <= 1e-12
    assert abs(rae[0].item() - 0.5) <= 1e-12 and abs(rae[1].item() - 0.5) <= 1e-12
    ale_s, _ = pl.ale_rae(P_m, t_m, P_p, t_p, 2, scale=10.0)
    assert abs(ale_s[0].item()) <= 1e-12


def test_loss_zero_at_truth_and_bounded():
    rng = np.random.default_rng(7)
    H = random_cfr(rng, 8, 128)
    P, tau = pl.gain_and_delay_spread(H, W)
    L, lt, lg = pl.batch_loss(H, P, tau, W)
    assert L.item() == 0.0
    # every SMAPE is in [0, 1], so the loss is in [0, 2]
    L2, lt2, lg2 = pl.batch_loss(random_cfr(rng, 8, 128), P, tau, W)
    assert 0.0 < lt2.item() < 1.0 and 0.0 < lg2.item() < 1.0
    assert abs(L2.item() - lt2.item() - lg2.item()) <= 1e-15
    # scaled measurements: alpha P against the prediction
    L3, _, lg3 = pl.batch_loss(H * math.sqrt(3.0), P, tau, W, alpha=3.0)
    assert lg3.item() <= 1e-15


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(8)
    N = 64
    Ht = random_cfr(rng, 3, N, max_tap=12.0)
    P_t, tau_t = pl.gain_and_delay_spread(Ht, W)
    H = random_cfr(rng, 3, N, max_tap=12.0).requires_grad_(True)
    L, _, _ = pl.batch_loss(H, P_t, tau_t, W, alpha=1.3, w_tau=0.7, w_gain=1.1)
    (g,) = torch.autograd.grad(L, H)
    H0 = H.detach()
    for b, n in [(0, 0), (0, 17), (1, 40), (2, 63)]:
        for part in (1.0, 1j):
            h = 1e-6 * H0.abs().max().item()
            Hp, Hm = H0.clone(), H0.clone()
            Hp[b, n] += h * part
            Hm[b, n] -= h * part
            fd = (pl.batch_loss(Hp, P_t, tau_t, W, 1.3, 0.7, 1.1)[0].item() -
                  pl.batch_loss(Hm, P_t, tau_t, W, 1.3, 0.7, 1.1)[0].item()) / (2 * h)
            an = g[b, n].real.item() if part == 1.0 else g[b, n].imag.item()
            assert abs(fd - an) <= 1e-6 * g.abs().max().item(), (b, n, part, fd, an)

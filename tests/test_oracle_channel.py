"""Pins of the oracle's channel synthesis, CIR / power-delay profile, loss
and reference gradients (Sec. II-A of the paper, workload loss)."""
import math

import numpy as np
import pytest
import torch

from oracle import channel, em
from oracle.adam import adam_step
from oracle.trace import trace_fields_per_id
from tests.helpers import single_path_store, tiny_workload

f64 = torch.float64
c128 = torch.complex128


def _freqs(radio):
    return channel.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)


def test_subcarrier_grid():
    f = channel.subcarrier_freqs(3.5e9, 50e6, 256)
    assert f[128].item() == 3.5e9
    assert abs(f[0].item() - (3.5e9 - 25e6)) < 1e-3
    assert abs((f[1] - f[0]).item() - 195312.5) < 1e-6


def test_single_path_cfr_closed_form():
    """One path: |H[n]| constant, phase exactly -2 pi f_n tau."""
    st = single_path_store(np.zeros((0, 3)), [0, 0, 1.0], [37.0, 11.0, 2.0], np.zeros((0, 3)))
    a = torch.tensor([0.3 - 0.2j], dtype=c128)
    psi = torch.zeros(1, dtype=f64)
    g = torch.ones(1, dtype=c128)
    f = channel.subcarrier_freqs(3.5e9, 50e6, 1024)
    H = channel.cfr(st.link_off, st.tau, a, psi, g, f)[0, 0]
    assert torch.allclose(H.abs(), torch.full_like(H.abs(), abs(0.3 - 0.2j)), rtol=1e-13)
    ref = (0.3 - 0.2j) * np.exp(-2j * np.pi * (f.numpy() * st.tau[0]))
    assert np.max(np.abs(H.numpy() - ref)) < 1e-12


def test_array_phase_progression():
    """One path into a ULA: |H| equal over elements, phase step psi."""
    a = torch.tensor([1.0 + 0.5j], dtype=c128)
    psi = torch.tensor([0.77], dtype=f64)
    g = torch.ones(8, dtype=c128)
    b = channel.array_coefficients(a, psi, g)[0]
    assert torch.allclose(b.abs(), torch.full((8,), abs(1 + 0.5j), dtype=f64))
    steps = torch.angle(b[1:] / b[:-1])
    assert torch.allclose(steps, torch.full((7,), 0.77, dtype=f64), atol=1e-14)
    # centred: elements m and M-1-m have conjugate array phases
    assert abs(torch.angle(b[0] / a[0]).item() + torch.angle(b[7] / a[0]).item()) < 1e-14


def test_cir_explicit_idft_matches_fft_route():
    """The explicit centred IDFT (Sec. II-A) and the FFT route of pdp()
    give the same power profile once the taps are re-centred."""
    rng = np.random.default_rng(0)
    H = torch.tensor(rng.normal(size=(3, 64)) + 1j * rng.normal(size=(3, 64)), dtype=c128)
    h = channel.cir(H)
    p_fft = channel.pdp(H)
    # centred tap l (index l + N/2) sits at fft index l mod N
    p_c = torch.roll(p_fft, shifts=32, dims=-1)
    assert torch.allclose(h.abs() ** 2, p_c, rtol=1e-12)


def test_parseval():
    rng = np.random.default_rng(1)
    H = torch.tensor(rng.normal(size=(5, 256)) + 1j * rng.normal(size=(5, 256)), dtype=c128)
    p = channel.pdp(H)
    assert torch.allclose(p.sum(-1), (H.abs() ** 2).sum(-1), rtol=1e-12)


def test_single_path_pdp_peaks_at_delay_bin():
    """A single path's PDP is a Dirichlet kernel centred at tau*W."""
    for dist in (3.0, 17.3, 55.0):
        st = single_path_store(np.zeros((0, 3)), [0, 0, 0.0], [dist, 0.0, 0.0], np.zeros((0, 3)))
        f = channel.subcarrier_freqs(3.5e9, 50e6, 256)
        H = channel.cfr(st.link_off, st.tau, torch.ones(1, dtype=c128), torch.zeros(1, dtype=f64),
                        torch.ones(1, dtype=c128), f)[0, 0]
        p = channel.pdp(H)
        # ifft index l sees e^{+j 2 pi n l / N}; the path contributes
        # e^{-j 2 pi n df tau}, so the peak is at l = tau W (mod N)
        peak = int(torch.argmax(p))
        assert peak == int(round(st.tau[0] * 50e6)) % 256


def test_loss_zero_at_target_and_gradient_zero():
    _, st, raw, radio, g = tiny_workload()
    f = _freqs(radio)
    raw_t = torch.tensor(raw, dtype=f64, requires_grad=True)
    a, psi = trace_fields_per_id(st, raw_t, radio.fc)
    H = channel.cfr(st.link_off, st.tau, a, psi, torch.tensor(g, dtype=c128), f)
    Ht = H.detach().clone()
    L, coh, inc = channel.cfr_loss(H, Ht)
    assert L.item() == 0.0
    (grad,) = torch.autograd.grad(L, raw_t)
    assert torch.all(grad == 0)


def _loss_of(st, radio, raw, g, Ht, sel_links=None):
    f = _freqs(radio)
    a, psi = trace_fields_per_id(st, raw, radio.fc)
    H = channel.cfr(st.link_off, st.tau, a, psi, g, f)
    return channel.cfr_loss(H, Ht)[0]


def test_reference_gradient_matches_central_differences():
    """The FP64 autograd gradient of the loss w.r.t. the raw material
    parameters and the element gains equals central finite differences
    with a relative step of 1e-4."""
    _, st, raw, radio, _ = tiny_workload()
    st = st.subset_links(range(8))
    rng = np.random.default_rng(3)
    M = 4
    radio = type(radio)(fc=radio.fc, bandwidth=radio.bandwidth, n_sc=64, n_elem=M)
    g_t = torch.tensor(rng.uniform(0.8, 1.2, M) * np.exp(1j * rng.uniform(-0.7, 0.7, M)), dtype=c128)
    raw_gt = torch.tensor(raw, dtype=f64)
    raw_gt[0, 2] = -1.0  # S = 0.27 in the target
    f = _freqs(radio)
    a, psi = trace_fields_per_id(st, raw_gt, radio.fc)
    Ht = channel.cfr(st.link_off, st.tau, a, psi, g_t, f).detach()
    # evaluate at a perturbed point
    raw0 = raw_gt + torch.tensor([[0.3, -0.5, 0.4]], dtype=f64)
    g0 = g_t * torch.tensor(rng.uniform(0.9, 1.1, M) * np.exp(1j * rng.uniform(-0.2, 0.2, M)), dtype=c128)
    rr = raw0.clone().requires_grad_(True)
    gg = g0.clone().requires_grad_(True)
    L = _loss_of(st, radio, rr, gg, Ht)
    d_raw, d_g = torch.autograd.grad(L, (rr, gg))
    for j in range(3):
        h = 1e-4 * max(abs(raw0[0, j].item()), 1e-2)
        e = torch.zeros_like(raw0)
        e[0, j] = h
        fd = (_loss_of(st, radio, raw0 + e, g0, Ht) - _loss_of(st, radio, raw0 - e, g0, Ht)).item() / (2 * h)
        assert abs(fd - d_raw[0, j].item()) < 1e-6 * max(abs(fd), 1e-3), (j, fd, d_raw[0, j].item())
    # complex gains: torch convention dL/dg = dL/dRe g + j dL/dIm g
    for m in range(M):
        for part, unit in ((0, 1.0), (1, 1j)):
            h = 1e-4 * abs(g0[m].item())
            e = torch.zeros_like(g0)
            e[m] = h * unit
            fd = (_loss_of(st, radio, raw0, g0 + e, Ht) - _loss_of(st, radio, raw0, g0 - e, Ht)).item() / (2 * h)
            an = d_g[m].real.item() if part == 0 else d_g[m].imag.item()
            assert abs(fd - an) < 1e-6 * max(abs(fd), 1e-3), (m, part, fd, an)


def test_two_ray_permittivity_derivative_closed_form():
    """dH/d eps_r of the ground path equals lam/(4 pi d2) R dr_par/deta
    times the delay phase (vertical polarisation)."""
    from tests.test_oracle_trace import _two_ray_store
    st = _two_ray_store(2.0, 1.5, 10.0)
    eps = torch.tensor(5.0, dtype=f64, requires_grad=True)
    sig = torch.tensor(0.05, dtype=f64)
    from oracle.trace import trace_fields
    D, P = st.max_depth, st.n_paths
    a, psi = trace_fields(st, eps.expand(D, P), sig.expand(D, P), torch.zeros(D, P, dtype=f64), 3.5e9)
    (da_re,) = torch.autograd.grad(a[1].real, eps, retain_graph=True)
    (da_im,) = torch.autograd.grad(a[1].imag, eps)
    d2 = math.hypot(10.0, 3.5)
    c = 3.5 / d2
    eta = 5.0 - 1j * 0.05 / (em.EPS0 * 2 * math.pi * 3.5e9)
    s = np.sqrt(eta - (1 - c * c))
    d_par = c * (eta - 2 * (1 - c * c)) / (s * (eta * c + s) ** 2)
    lam = em.C0 / 3.5e9
    ref = lam / (4 * math.pi * d2) * d_par
    assert abs(complex(da_re.item(), da_im.item()) - ref) < 1e-6 * abs(ref)


def test_adam_matches_library_optimizer():
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=17)
    pt = torch.tensor(p0.copy(), dtype=f64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(17), np.zeros(17)
    for t in range(1, 30):
        gr = rng.normal(size=17) * (1 + t)
        pt.grad = torch.tensor(gr, dtype=f64)
        opt.step()
        p, m, v = adam_step(p, gr, m, v, t)
        assert np.allclose(p, pt.detach().numpy(), rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------------------------
# Values of the workload loss and the held-out NMSE, fixed by hand.
#
# A row H*[n] = A exp(-j 2 pi n k / N) is one path at integer tap k: the
# centred IDFT with 1/sqrt(N) of Sec. II-A puts all of its energy N|A|^2 in
# one tap, so p* is N|A|^2 at one tap and 0 elsewhere.  These rows make every
# sum of the loss a closed form: a normaliser taken from the prediction,
# per row instead of over the batch, or without the squares would change
# the values below.

def _tap_row(N, amp, k):
    n = torch.arange(N, dtype=f64)
    return amp * torch.exp(-2j * math.pi * n * k / N).to(c128)


def test_loss_scaled_target_closed_form():
    """H = c H*: L_coh = |c - 1|^2 and L_pdp = (|c|^2 - 1)^2 for any H*."""
    rng = np.random.default_rng(11)
    Ht = torch.tensor(rng.normal(size=(3, 2, 64)) + 1j * rng.normal(size=(3, 2, 64)), dtype=c128)
    for c in (1.0, 0.5, 1.7 - 0.4j, -1.0, 1j, 0.0):
        L, coh, inc = channel.cfr_loss(c * Ht, Ht)
        assert abs(coh.item() - abs(c - 1) ** 2) < 1e-13
        assert abs(inc.item() - (abs(c) ** 2 - 1) ** 2) < 1e-12
        assert abs(L.item() - (abs(c - 1) ** 2 + (abs(c) ** 2 - 1) ** 2)) < 1e-12
        assert abs(channel.nmse(c * Ht, Ht).item() - abs(c - 1) ** 2) < 1e-13
    # weights multiply the two terms
    L, coh, inc = channel.cfr_loss(0.5 * Ht, Ht, w_coh=3.0, w_pdp=0.25)
    assert abs(L.item() - (3.0 * 0.25 + 0.25 * 0.75 ** 2)) < 1e-13


def test_loss_zero_prediction_is_one_plus_one():
    rng = np.random.default_rng(12)
    Ht = torch.tensor(rng.normal(size=(2, 3, 32)) + 1j * rng.normal(size=(2, 3, 32)), dtype=c128)
    L, coh, inc = channel.cfr_loss(torch.zeros_like(Ht), Ht)
    assert abs(coh.item() - 1.0) < 1e-15 and abs(inc.item() - 1.0) < 1e-15
    assert abs(L.item() - 2.0) < 1e-15
    assert abs(channel.nmse(torch.zeros_like(Ht), Ht).item() - 1.0) < 1e-15


def test_loss_single_tap_rows_by_hand():
    """A spurious second path B at tap k1 next to the target's path A at
    tap k0: sum|H - H*|^2 = N|B|^2 against sum|H*|^2 = N|A|^2, and the PDPs
    differ by N|B|^2 at tap k1 only, against sum (p*)^2 = (N|A|^2)^2."""
    N = 128
    A, B = 0.8 - 0.3j, 0.25 + 0.1j
    Ht = _tap_row(N, A, 9).reshape(1, 1, N)
    H = Ht + _tap_row(N, B, 40).reshape(1, 1, N)
    # the PDP itself: N |A|^2 at tap 9, N |B|^2 at tap 40
    p = channel.pdp(H)[0, 0]
    assert abs(p[9].item() - N * abs(A) ** 2) < 1e-12 and abs(p[40].item() - N * abs(B) ** 2) < 1e-12
    assert torch.sum(p).item() == pytest.approx(N * (abs(A) ** 2 + abs(B) ** 2), rel=1e-14)
    L, coh, inc = channel.cfr_loss(H, Ht)
    assert coh.item() == pytest.approx(abs(B) ** 2 / abs(A) ** 2, rel=1e-13)
    # normalised by the target's sum (p*)^2: |B|^4/|A|^4 (the prediction's
    # sum p^2 would give |B|^4/(|A|^4 + |B|^4))
    assert inc.item() == pytest.approx(abs(B) ** 4 / abs(A) ** 4, rel=1e-12)
    assert channel.nmse(H, Ht).item() == pytest.approx(abs(B) ** 2 / abs(A) ** 2, rel=1e-13)


def test_loss_normalised_over_the_batch():
    """Two rows of unequal target energy: each term is one ratio of sums
    over the whole batch, not a mean of per-row ratios."""
    N = 64
    A0, A1 = 2.0, 0.5 + 0.5j          # target energies N*4 and N*0.5
    c0, c1 = 1.1, 0.6j                # H = c H* row by row
    Ht = torch.stack([_tap_row(N, A0, 3), _tap_row(N, A1, 20)]).reshape(2, 1, N)
    H = torch.stack([c0 * Ht[0], c1 * Ht[1]])
    E0, E1 = N * abs(A0) ** 2, N * abs(A1) ** 2          # sum |H*|^2 per row
    Q0, Q1 = (N * abs(A0) ** 2) ** 2, (N * abs(A1) ** 2) ** 2  # sum (p*)^2 per row
    coh_ref = (abs(c0 - 1) ** 2 * E0 + abs(c1 - 1) ** 2 * E1) / (E0 + E1)
    inc_ref = ((abs(c0) ** 2 - 1) ** 2 * Q0 + (abs(c1) ** 2 - 1) ** 2 * Q1) / (Q0 + Q1)
    L, coh, inc = channel.cfr_loss(H, Ht)
    assert coh.item() == pytest.approx(coh_ref, rel=1e-13)
    assert inc.item() == pytest.approx(inc_ref, rel=1e-12)
    assert L.item() == pytest.approx(coh_ref + inc_ref, rel=1e-12)
    # the per-row mean differs markedly here
    per_row = 0.5 * (abs(c0 - 1) ** 2 + abs(c1 - 1) ** 2)
    assert abs(per_row - coh_ref) > 0.1
    assert channel.nmse(H, Ht).item() == pytest.approx(coh_ref, rel=1e-13)

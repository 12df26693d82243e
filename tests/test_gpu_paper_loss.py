"""The paper's loss through the library (rtc_cir_stats, rtc_paper_loss,
rtc_eval_ale_rae) against the FP64 oracle: per-row gain and delay spread,
the batch loss, dL/dH, the scale estimate over successive calls and the
ALE/RAE metrics, over the one-wave (N <= 1024) and the workgroup (N > 1024)
kernels, ragged row counts, and degenerate rows (all zero, a single tap,
one occupied subcarrier).  The last test runs the full 16,384 x 32 x 1,024
batch and checks sampled rows."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import paper_loss as opl

pytestmark = pytest.mark.gpu

c128 = torch.complex128
f64 = torch.float64


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


def multipath_rows(rng, rows, N, n_paths=10, max_tap=None, decay=8.0):
    """CFR rows (storage order, subcarrier offset n - N/2) of random paths
    at fractional tap delays d with complex gains decaying in d."""
    max_tap = max_tap if max_tap is not None else max(1.0, N / 8)
    n = np.arange(N) - N // 2
    out = np.zeros((rows, N), np.complex128)
    for b in range(rows):
        d = rng.uniform(0.0, max_tap, n_paths)
        a = (rng.normal(size=n_paths) + 1j * rng.normal(size=n_paths)) * np.exp(-d / decay)
        out[b] = (a[:, None] * np.exp(-2j * np.pi * n[None, :] * d[:, None] / N)).sum(0)
    return out * 1e-4


def degenerate_rows(N):
    """All zero, a single integer-tap path, one occupied subcarrier."""
    n = np.arange(N) - N // 2
    z = np.zeros(N, np.complex128)
    spike = 3e-4 * np.exp(-2j * np.pi * n * (1 % N) / N)
    flat = np.zeros(N, np.complex128)
    flat[N // 2 - 1] = 2e-4 + 1e-4j
    return np.stack([z, spike, flat])


def make_batch(seed, n_links, n_elem, N, degenerate=True):
    rng = np.random.default_rng(seed)
    R = n_links * n_elem
    H = multipath_rows(rng, R, N)
    if degenerate and R >= 6:
        H[1:4] = degenerate_rows(N)
    return H.reshape(n_links, n_elem, N)


def radio(rl, N, n_elem, bw=50e6):
    return rl.make_radio(3.5e9, bw / N, N, n_elem)


def to_dev(H):
    return torch.tensor(H.astype(np.complex64), device="cuda")


CASES = [(2, 5, 3), (16, 7, 2), (256, 37, 3), (1024, 11, 4), (2048, 5, 3), (4096, 3, 2)]


@pytest.mark.parametrize("N,L,M", CASES)
def test_cir_stats(rl, N, L, M):
    say(f"cir_stats N={N} rows={L * M}")
    H = make_batch(1 + N, L, M, N)
    Hd = to_dev(H)
    stats = torch.full((L * M, 2), float("nan"), dtype=f64, device="cuda")
    rl.cir_stats(radio(rl, N, M), L, Hd, stats)
    torch.cuda.synchronize()
    H32 = torch.tensor(H.astype(np.complex64)).to(c128).reshape(L * M, N)
    P, tau = opl.gain_and_delay_spread(H32, 50e6)
    got = stats.cpu()
    assert torch.isfinite(got).all()
    assert torch.allclose(got[:, 0], P, rtol=2e-6, atol=0), (got[:, 0], P)
    # delay spread: relative, with an absolute floor for rows whose spread is
    # near zero.  There the FP32 transform's noise sets the value: taps of
    # relative amplitude ~ eps sqrt(log2 N / N) spread over +-N/2 give a
    # spread of ~ N eps sqrt(log2 N / 12) taps; the floor is 8x that.
    err = (got[:, 1] - tau).abs()
    floor = 8.0 * N * 2.0 ** -24 * math.sqrt(max(1.0, math.log2(N)) / 12.0)
    tol = 2e-5 * tau + floor / 50e6
    assert bool((err <= tol).all()), (err / tol).max().item()
    if L * M >= 6 and N >= 4:
        assert got[1, 0].item() == 0.0 and got[1, 1].item() == 0.0  # zero row
        flat = math.sqrt((N * N - 1) / 12.0) / 50e6
        assert abs(got[3, 1].item() - flat) <= 1e-5 * flat


def _oracle_loss(H32, P_t, tau_t, alpha, w_tau, w_gain, bw=50e6):
    H = H32.clone().requires_grad_(True)
    L, lt, lg = opl.batch_loss(H, P_t, tau_t, bw, alpha=alpha, w_tau=w_tau, w_gain=w_gain)
    (g,) = torch.autograd.grad(L, H)
    return L.item(), lt.item(), lg.item(), g


@pytest.mark.parametrize("N,L,M", CASES)
def test_paper_loss_and_gradient(rl, N, L, M):
    say(f"paper_loss N={N} rows={L * M}")
    H = make_batch(100 + N, L, M, N)
    Ht = make_batch(200 + N, L, M, N, degenerate=False)
    R = L * M
    H32 = torch.tensor(H.astype(np.complex64)).to(c128).reshape(R, N)
    Ht32 = torch.tensor(Ht.astype(np.complex64)).to(c128).reshape(R, N)
    P_t, tau_t = opl.gain_and_delay_spread(Ht32, 50e6)
    w_tau, w_gain, alpha = 0.75, 1.25, 1.7
    Lr, ltr, lgr, g_ref = _oracle_loss(H32, P_t, tau_t, alpha, w_tau, w_gain)
    rc = radio(rl, N, M)
    tgt = torch.stack([P_t, tau_t], 1).contiguous().cuda()
    al = torch.tensor([alpha, 0.0], dtype=f64, device="cuda")
    loss = torch.full((3,), float("nan"), dtype=f64, device="cuda")
    pred = torch.full((R, 2), float("nan"), dtype=f64, device="cuda")
    Hd = to_dev(H)
    dLdH = torch.full_like(Hd, float("nan"))
    ws = rl.workspace(rl.RTC_OP_PAPER_LOSS, rc, L, 0)
    rl.paper_loss(rc, L, Hd, tgt, al, loss, dLdH, ws, update_alpha=False, w_tau=w_tau,
                  w_gain=w_gain, pred_stats=pred)
    torch.cuda.synchronize()
    got = loss.cpu().tolist()
    say(f"  loss {got} oracle {[Lr, ltr, lgr]}")
    assert abs(got[0] - Lr) <= 1e-5 and abs(got[1] - ltr) <= 1e-5 and abs(got[2] - lgr) <= 1e-5
    assert al.cpu().tolist() == [alpha, 0.0]  # not updated
    # the statistics written beside the loss are those of rtc_cir_stats
    stats = torch.empty((R, 2), dtype=f64, device="cuda")
    rl.cir_stats(rc, L, Hd, stats)
    assert torch.allclose(pred, stats, rtol=1e-12, atol=0)
    g = dLdH.cpu().to(c128).reshape(R, N)
    assert torch.isfinite(g.real).all() and torch.isfinite(g.imag).all()
    worst = 0.0
    for b in range(R):
        if b == 2 and R >= 6:
            # the single-tap row sits on the kink of sqrt at zero variance:
            # both gradients there are set by rounding noise of the taps
            continue
        den = torch.linalg.norm(g_ref[b]).item()
        num = torch.linalg.norm(g[b] - g_ref[b]).item()
        if den == 0.0:
            assert num == 0.0, b
        else:
            worst = max(worst, num / den)
    say(f"  dL/dH max per-row relative error {worst:.2e}")
    assert worst <= 1e-4, worst
    # in place: dL/dH written over H gives the same result
    Hin = Hd.clone()
    rl.paper_loss(rc, L, Hin, tgt, al, loss, Hin, ws, update_alpha=False, w_tau=w_tau,
                  w_gain=w_gain)
    torch.cuda.synchronize()
    assert torch.equal(Hin, dLdH)


def test_scale_estimate_over_calls(rl):
    """alpha_0 = alpha^_1, then the moving average with delta; each call's
    loss uses the alpha of that call."""
    N, L, M = 256, 20, 4
    R = L * M
    rng = np.random.default_rng(9)
    Ht = make_batch(300, L, M, N, degenerate=False)
    Ht32 = torch.tensor(Ht.astype(np.complex64)).to(c128).reshape(R, N)
    P_t, tau_t = opl.gain_and_delay_spread(Ht32, 50e6)
    rc = radio(rl, N, M)
    tgt = torch.stack([P_t, tau_t], 1).contiguous().cuda()
    # the stored value is replaced by alpha^ on the first update
    al = torch.tensor([123.0, 0.0], dtype=f64, device="cuda")
    loss = torch.empty(3, dtype=f64, device="cuda")
    ws = rl.workspace(rl.RTC_OP_PAPER_LOSS, rc, L, 0)
    delta = 0.8
    a_ref = None
    for i in range(3):
        # predictions: a scaled and perturbed copy of the measurements
        H = Ht * math.sqrt(0.3 + 0.2 * i) * (1 + 0.05 * rng.normal(size=Ht.shape))
        H32 = torch.tensor(H.astype(np.complex64)).to(c128).reshape(R, N)
        P_hat, _ = opl.gain_and_delay_spread(H32, 50e6)
        a_ref = opl.alpha_ema(a_ref, opl.alpha_hat(P_t, P_hat), delta, i == 0)
        rl.paper_loss(rc, L, to_dev(H), tgt, al, loss, None, ws, update_alpha=True, delta=delta)
        torch.cuda.synchronize()
        a_got, n_got = al.cpu().tolist()
        say(f"  call {i}: alpha {a_got:.9f} oracle {a_ref:.9f}")
        assert n_got == i + 1
        assert abs(a_got - a_ref) <= 2e-6 * a_ref
        Lr, _, _ = opl.batch_loss(H32, P_t, tau_t, 50e6, alpha=a_got)
        assert abs(loss[0].item() - Lr.item()) <= 1e-5


def test_loss_zero_at_truth(rl):
    N, L, M = 1024, 9, 4
    H = make_batch(400, L, M, N, degenerate=False)
    R = L * M
    rc = radio(rl, N, M)
    Hd = to_dev(H)
    stats = torch.empty((R, 2), dtype=f64, device="cuda")
    al = torch.tensor([1.0, 0.0], dtype=f64, device="cuda")
    loss = torch.empty(3, dtype=f64, device="cuda")
    ws = rl.workspace(rl.RTC_OP_PAPER_LOSS, rc, L, 0)
    dummy = torch.ones((R, 2), dtype=f64, device="cuda")
    rl.paper_loss(rc, L, Hd, dummy, al, loss, None, ws, pred_stats=stats)
    dLdH = torch.empty_like(Hd)
    rl.paper_loss(rc, L, Hd, stats, al, loss, dLdH, ws)
    torch.cuda.synchronize()
    # targets are the kernel's own statistics of the same rows: loss and
    # gradient exactly zero
    assert loss.cpu().tolist() == [0.0, 0.0, 0.0]
    assert torch.count_nonzero(dLdH).item() == 0


def test_ale_rae(rl):
    L, M = 33, 4
    rng = np.random.default_rng(11)
    meas = torch.tensor(np.stack([rng.uniform(1e-9, 1e-7, L * M), rng.uniform(5e-9, 9e-8, L * M)],
                                 1))
    pred = torch.tensor(np.stack([rng.uniform(1e-9, 1e-7, L * M), rng.uniform(5e-9, 9e-8, L * M)],
                                 1))
    out = torch.empty((L, 2), dtype=f64, device="cuda")
    scale = torch.tensor([0.6], dtype=f64, device="cuda")
    rl.eval_ale_rae(L, M, meas.cuda(), pred.cuda(), out, scale=scale)
    torch.cuda.synchronize()
    ale, rae = opl.ale_rae(meas[:, 0], meas[:, 1], pred[:, 0], pred[:, 1], M, scale=0.6)
    got = out.cpu()
    assert torch.allclose(got[:, 0], ale, rtol=1e-12, atol=1e-12)
    assert torch.allclose(got[:, 1], rae, rtol=1e-12, atol=0)


def test_full_scale_sampled_rows(rl):
    """16,384 links x 32 elements x 1,024 subcarriers, the launch the
    benchmark times: sampled rows' statistics and gradients against the
    oracle, the mean loss against the mean of the per-row statistics."""
    L, M, N = 16384, 32, 1024
    R = L * M
    say(f"paper_loss full scale: {R} rows x {N}")
    gen = torch.Generator(device="cuda").manual_seed(5)
    # random multipath rows: white taps shaped by a decaying delay profile
    taps = torch.randn((R, N), dtype=torch.complex64, device="cuda", generator=gen)
    prof = torch.exp(-torch.arange(N, device="cuda", dtype=torch.float32) / 24.0)
    H = torch.fft.fft(taps * prof, dim=-1) * 1e-4
    gen2 = torch.Generator(device="cuda").manual_seed(6)
    tgt = torch.stack([torch.rand(R, dtype=f64, device="cuda", generator=gen2) * 2e-6 + 1e-7,
                       torch.rand(R, dtype=f64, device="cuda", generator=gen2) * 4e-7 + 1e-8],
                      1).contiguous()
    rc = radio(rl, N, M)
    al = torch.tensor([1.0, 0.0], dtype=f64, device="cuda")
    loss = torch.empty(3, dtype=f64, device="cuda")
    pred = torch.empty((R, 2), dtype=f64, device="cuda")
    dLdH = torch.empty_like(H)
    ws = rl.workspace(rl.RTC_OP_PAPER_LOSS, rc, L, 0)
    rl.paper_loss(rc, L, H, tgt, al, loss, dLdH, ws, update_alpha=True, delta=0.9,
                  pred_stats=pred)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(12).choice(R, 24, replace=False))
    ri = torch.tensor(rows, device="cuda")
    H32 = H[ri].cpu().to(c128)
    P_t, tau_t = tgt[ri, 0].cpu(), tgt[ri, 1].cpu()
    P_ref, tau_ref = opl.gain_and_delay_spread(H32, 50e6)
    got = pred[ri].cpu()
    assert torch.allclose(got[:, 0], P_ref, rtol=2e-6, atol=0)
    assert torch.allclose(got[:, 1], tau_ref, rtol=2e-5, atol=0)
    a = al[0].item()
    assert al[1].item() == 1.0
    # alpha^ from the kernel's own per-row gains (Parseval) in FP64
    Pp = pred[:, 0].double()
    a_ref = ((tgt[:, 0] * Pp).sum() / (tgt[:, 0] ** 2).sum()).item()
    assert abs(a - a_ref) <= 1e-5 * abs(a_ref)
    # each sampled row's gradient is that of its own term, divided by R
    Hs = H32.clone().requires_grad_(True)
    Ph, th = opl.gain_and_delay_spread(Hs, 50e6)
    tot, _, _ = opl.example_losses(P_t, tau_t, Ph, th, alpha=a)
    (g_ref,) = torch.autograd.grad(tot.sum() / R, Hs)
    g = dLdH[ri].cpu().to(c128)
    err = (torch.linalg.norm(g - g_ref, dim=1) / torch.linalg.norm(g_ref, dim=1)).max().item()
    say(f"  sampled rows: dL/dH max relative error {err:.2e}, alpha {a:.6e}")
    assert err <= 1e-4
    # the batch loss is the mean of the per-row SMAPE terms of the kernel's
    # own statistics
    lt = opl.smape(tgt[:, 1].cpu(), pred[:, 1].cpu()).mean().item()
    lg = opl.smape(a * tgt[:, 0].cpu(), pred[:, 0].cpu()).mean().item()
    got_l = loss.cpu().tolist()
    assert abs(got_l[1] - lt) <= 1e-9 and abs(got_l[2] - lg) <= 1e-9
    assert abs(got_l[0] - (lt + lg)) <= 1e-9

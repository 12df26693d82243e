"""The allocation-free loss entry point (rtc_cfr_loss_noalloc) against the
workspace one (rtc_cfr_loss) through the C ABI: the same kernels, so the
loss terms and dL/dH agree bit for bit, over consecutive calls of falling
size that share the library's fixed scratch, and the first against the
oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import channel as och

pytestmark = pytest.mark.gpu
c128 = torch.complex128


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


def _rows(rng, L, M, N):
    """Seeded CFR batch with a few dominant taps per row plus noise."""
    H = rng.normal(size=(L, M, N)) + 1j * rng.normal(size=(L, M, N))
    return (H * rng.uniform(0.1, 10.0, size=(L, M, 1))).astype(np.complex64)


def _pair(rl, rc, L, H, Ht, tgt_stats=None, p_tgt=None, w=(1.0, 1.0)):
    """(loss, dL/dH) from both entry points on the same inputs."""
    dev = "cuda"
    ws = rl.workspace(rl.RTC_OP_CFR_LOSS, rc, L, 0)
    loss_ref = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
    g_ref = torch.full_like(H, float("nan"))
    rl.cfr_loss(rc, L, H, Ht, tgt_stats, w[0], w[1], loss_ref, g_ref, ws, p_tgt=p_tgt)
    loss = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
    g = torch.full_like(H, float("nan"))
    rl.cfr_loss_noalloc(rc, L, H, Ht, tgt_stats, w[0], w[1], loss, g, p_tgt=p_tgt)
    torch.cuda.synchronize()
    return loss.cpu(), g.cpu(), loss_ref.cpu(), g_ref.cpu()


def test_noalloc_matches_workspace_entry_point(rl):
    rng = np.random.default_rng(31)
    # call 1: 256 links x 32 elements x 1,024 subcarriers, targets' statistics
    # computed inside the call (both scratch regions in use)
    L, M, N = 256, 32, 1024
    say(f"noalloc loss call 1: L={L} M={M} N={N}")
    rc = rl.make_radio(3.5e9, 50e6 / N, N, M)
    Hh, Hth = _rows(rng, L, M, N), _rows(rng, L, M, N)
    H, Ht = torch.tensor(Hh, device="cuda"), torch.tensor(Hth, device="cuda")
    loss, g, loss_ref, g_ref = _pair(rl, rc, L, H, Ht, w=(0.7, 1.3))
    assert torch.equal(loss, loss_ref), (loss, loss_ref)
    assert torch.equal(g, g_ref)
    # and the oracle on the same inputs (FP64)
    Hd = torch.tensor(Hh, dtype=c128).requires_grad_(True)
    tot, coh, inc = och.cfr_loss(Hd, torch.tensor(Hth, dtype=c128), w_coh=0.7, w_pdp=1.3)
    (gd,) = torch.autograd.grad(tot, Hd)
    for got, ref in zip(loss.tolist(), (tot.item(), coh.item(), inc.item())):
        assert abs(got - ref) <= 1e-5 * abs(ref), (got, ref)
    err = (torch.linalg.norm(g.to(c128) - gd) / torch.linalg.norm(gd)).item()
    assert err <= 1e-4, err

    # call 2: a smaller batch right after, with precomputed target statistics
    # and PDP; the scratch keeps call 1's values, none of which may be read
    L, M, N = 7, 4, 256
    say(f"noalloc loss call 2: L={L} M={M} N={N}")
    rc = rl.make_radio(3.5e9, 50e6 / N, N, M)
    H = torch.tensor(_rows(rng, L, M, N), device="cuda")
    Ht = torch.tensor(_rows(rng, L, M, N), device="cuda")
    stats = torch.empty(2, dtype=torch.float64, device="cuda")
    p_tgt = torch.empty(L * M * N, dtype=torch.float32, device="cuda")
    rl.cfr_target_stats(rc, L, Ht, stats, rl.workspace(rl.RTC_OP_CFR_TARGET_STATS, rc, L, 0),
                        p_tgt=p_tgt)
    loss, g, loss_ref, g_ref = _pair(rl, rc, L, H, Ht, tgt_stats=stats, p_tgt=p_tgt)
    assert torch.equal(loss, loss_ref), (loss, loss_ref)
    assert torch.equal(g, g_ref)
    # loss only (no dL/dH)
    loss2 = torch.empty(3, dtype=torch.float64, device="cuda")
    rl.cfr_loss_noalloc(rc, L, H, Ht, None, 1.0, 1.0, loss2, None)
    torch.cuda.synchronize()
    assert torch.equal(loss2.cpu(), loss_ref)


def test_noalloc_at_its_row_limit(rl):
    """Exactly the maximum number of rows (two-subcarrier rows keep it
    small), then one link more is refused."""
    max_rows = rl.cfr_loss_noalloc_max_rows()
    M, N = 32, 2
    L = max_rows // M
    say(f"noalloc loss at the limit: L={L} M={M} N={N}")
    rc = rl.make_radio(3.5e9, 1e6, N, M)
    rng = np.random.default_rng(5)
    H = torch.tensor(_rows(rng, L, M, N), device="cuda")
    Ht = torch.tensor(_rows(rng, L, M, N), device="cuda")
    loss, g, loss_ref, g_ref = _pair(rl, rc, L, H, Ht)
    assert torch.equal(loss, loss_ref) and torch.equal(g, g_ref)
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="exceed"):
        rl.cfr_loss_noalloc(rc, L + 1, H, Ht, None, 1.0, 1.0, loss, None)

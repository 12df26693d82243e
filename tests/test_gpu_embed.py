"""Material embeddings (Sec. III-C) through the library: rtc_embed_readout
and its backward against the FP64 oracle and its autograd."""
import math

import numpy as np
import pytest
import torch

from oracle.em import embedding_readout

pytestmark = pytest.mark.gpu
f64 = torch.float64

# raw column fed by embedding j (paper order sigma, eps_r, S); K_x -> pattern
RAW_COL = (1, 0, 2)


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


def _draw(seed, n_mat, L):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=L).astype(np.float32)
    W = (rng.normal(size=(n_mat, 4, L)) / math.sqrt(L)).astype(np.float32)
    return v, W


@pytest.mark.parametrize("n_mat,L", [(1, 1), (3, 30), (7, 5), (300, 30), (4096, 64), (2, 1024)])
def test_readout(rl, n_mat, L):
    v, W = _draw(n_mat + L, n_mat, L)
    raw = torch.full((n_mat, 3), float("nan"), device="cuda")
    pat = torch.full((n_mat, 6), float("nan"), device="cuda")
    rl.embed_readout(torch.tensor(v, device="cuda"), torch.tensor(W, device="cuda"), raw, pat)
    torch.cuda.synchronize()
    u = embedding_readout(torch.tensor(v, dtype=f64), torch.tensor(W, dtype=f64))
    scale = torch.tensor(np.abs(W).astype(np.float64) @ np.abs(v).astype(np.float64))
    for j, c in enumerate(RAW_COL):
        err = (raw.cpu().double()[:, c] - u[:, j]).abs()
        assert torch.all(err <= 1e-7 * scale[:, j] + 1e-30), (j, err.max().item())
    assert torch.all((pat.cpu().double()[:, 0] - u[:, 3]).abs() <= 1e-7 * scale[:, 3] + 1e-30)
    assert torch.isnan(pat[:, 1:]).all(), "columns other than K_x were written"


def test_readout_without_pattern_rows(rl):
    v, W = _draw(9, 5, 30)
    raw = torch.zeros((5, 3), device="cuda")
    rl.embed_readout(torch.tensor(v, device="cuda"), torch.tensor(W, device="cuda"), raw, None)
    torch.cuda.synchronize()
    u = embedding_readout(torch.tensor(v, dtype=f64), torch.tensor(W, dtype=f64))
    assert torch.allclose(raw.cpu().double()[:, 0], u[:, 1], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("n_mat,L,with_pat", [(3, 30, True), (3, 30, False), (257, 17, True),
                                               (1, 1024, True)])
def test_backward(rl, n_mat, L, with_pat):
    v, W = _draw(100 + L, n_mat, L)
    rng = np.random.default_rng(L)
    g_raw = rng.normal(size=(n_mat, 3)).astype(np.float32)
    g_pat = rng.normal(size=(n_mat, 6)).astype(np.float32)
    v64 = torch.tensor(v, dtype=f64, requires_grad=True)
    W64 = torch.tensor(W, dtype=f64, requires_grad=True)
    u = embedding_readout(v64, W64)
    gu = torch.zeros((n_mat, 4), dtype=f64)
    for j, c in enumerate(RAW_COL):
        gu[:, j] = torch.tensor(g_raw[:, c], dtype=f64)
    if with_pat:
        gu[:, 3] = torch.tensor(g_pat[:, 0], dtype=f64)
    gv, gW = torch.autograd.grad(u, (v64, W64), grad_outputs=gu)
    dv = torch.full((L,), float("nan"), device="cuda")
    dW = torch.full((n_mat, 4, L), float("nan"), device="cuda")
    rl.embed_readout_backward(torch.tensor(v, device="cuda"), torch.tensor(W, device="cuda"),
                              torch.tensor(g_raw, device="cuda"),
                              torch.tensor(g_pat, device="cuda") if with_pat else None, dv, dW)
    torch.cuda.synchronize()
    # dW: one product each, rounded once
    assert torch.all((dW.cpu().double() - gW).abs() <= 6e-8 * gW.abs() + 1e-30)
    # dv: FP64 sums rounded once
    bound = torch.tensor(np.abs(W).astype(np.float64).transpose(2, 0, 1).reshape(L, -1)
                         @ gu.abs().reshape(-1).numpy())
    assert torch.all((dv.cpu().double() - gv).abs() <= 1e-7 * bound + 1e-30)


def test_outputs_optional(rl):
    v, W = _draw(3, 2, 4)
    g = torch.ones((2, 3), device="cuda")
    dv = torch.zeros(4, device="cuda")
    rl.embed_readout_backward(torch.tensor(v, device="cuda"), torch.tensor(W, device="cuda"), g,
                              None, dv, None)
    torch.cuda.synchronize()
    assert torch.isfinite(dv).all() and dv.abs().sum() > 0

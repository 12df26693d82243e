"""Pins of the oracle's material embeddings (Sec. III-C, Eqs.
trainable_materials_1-4): brute-force sums, the one-dimensional special
case, the invariances of the over-parametrisation, ranges and central
differences."""
import math

import numpy as np
import torch

from oracle.em import embedding_readout, materials_from_embeddings, materials_from_raw

f64 = torch.float64


def _draw(seed, n_mat=3, L=30):
    rng = np.random.default_rng(seed)
    return (torch.tensor(rng.normal(size=L), dtype=f64),
            torch.tensor(rng.normal(size=(n_mat, 4, L)) / math.sqrt(L), dtype=f64))


def test_readout_brute_force():
    v, W = _draw(1, n_mat=4, L=7)
    u = embedding_readout(v, W)
    for m in range(4):
        for j in range(4):
            s = 0.0
            for l in range(7):
                s += float(v[l]) * float(W[m, j, l])
            assert abs(float(u[m, j]) - s) <= 1e-14 * (1 + abs(s))


def test_one_dimensional_case_is_the_raw_transform():
    """L = 1 and v = 1: the embeddings are the raw scalars themselves, in
    the paper's order (w_1 -> sigma, w_2 -> eps_r, w_3 -> S)."""
    rng = np.random.default_rng(2)
    raw = torch.tensor(rng.normal(size=(5, 3)), dtype=f64)  # (eps, sigma, S) order
    W = torch.stack([raw[:, 1], raw[:, 0], raw[:, 2], torch.zeros(5, dtype=f64)], 1)[..., None]
    eps, sig, s, kx = materials_from_embeddings(torch.ones(1, dtype=f64), W)
    e0, s0, S0 = materials_from_raw(raw)
    assert torch.allclose(eps, e0, rtol=1e-15) and torch.allclose(sig, s0, rtol=1e-15)
    assert torch.allclose(s, S0, rtol=1e-15)
    assert torch.allclose(kx, torch.full_like(kx, 0.5))


def test_known_values():
    """Table I materials reached through chosen embeddings."""
    table = [(5.24, 0.121, 0.3, 0.2), (2.73, 0.027, 0.5, 0.4), (1.48, 0.004, 0.8, 0.3)]
    L = 3
    v = torch.tensor([2.0, -1.0, 0.5], dtype=f64)
    W = torch.zeros((3, 4, L), dtype=f64)
    for m, (e, sg, S, K) in enumerate(table):
        target = [math.log(sg), math.log(e - 1.0), math.log(S / (1 - S)), math.log(K / (1 - K))]
        for j, t in enumerate(target):
            W[m, j, 0] = t / 2.0  # only the first coordinate carries the value
    eps, sig, s, kx = materials_from_embeddings(v, W)
    for m, (e, sg, S, K) in enumerate(table):
        assert abs(eps[m].item() - e) < 1e-12 and abs(sig[m].item() - sg) < 1e-14
        assert abs(s[m].item() - S) < 1e-14 and abs(kx[m].item() - K) < 1e-14


def test_invariances_of_the_overparametrisation():
    """u = v.w is unchanged by v -> c v, w -> w / c and by a rotation
    applied to v and to every w."""
    v, W = _draw(3)
    u = embedding_readout(v, W)
    assert torch.allclose(embedding_readout(3.7 * v, W / 3.7), u, rtol=1e-13, atol=1e-14)
    Q, _ = torch.linalg.qr(torch.tensor(np.random.default_rng(4).normal(size=(30, 30)),
                                        dtype=f64))
    assert torch.allclose(embedding_readout(Q @ v, W @ Q.T), u, rtol=1e-12, atol=1e-13)


def test_ranges():
    v, W = _draw(5, n_mat=50)
    eps, sig, s, kx = materials_from_embeddings(3.0 * v, W)
    assert torch.all(eps > 1) and torch.all(sig > 0)
    assert torch.all((s > 0) & (s < 1)) and torch.all((kx > 0) & (kx < 1))


def test_gradients_central_differences():
    v, W = _draw(6, n_mat=2, L=5)
    wts = torch.tensor([0.3, -1.1, 0.7, 0.4], dtype=f64)

    def f(v, W):
        return sum(w * t.sum() for w, t in zip(wts, materials_from_embeddings(v, W)))

    v1, W1 = v.clone().requires_grad_(True), W.clone().requires_grad_(True)
    gv, gW = torch.autograd.grad(f(v1, W1), (v1, W1))
    h = 1e-6
    for l in range(5):
        e = torch.zeros(5, dtype=f64)
        e[l] = h
        fd = (f(v + e, W) - f(v - e, W)) / (2 * h)
        assert abs(fd.item() - gv[l].item()) <= 1e-7 * (1 + abs(fd.item()))
    for idx in [(0, 0, 1), (1, 1, 4), (0, 2, 2), (1, 3, 0)]:
        e = torch.zeros_like(W)
        e[idx] = h
        fd = (f(v, W + e) - f(v, W - e)) / (2 * h)
        assert abs(fd.item() - gW[idx].item()) <= 1e-7 * (1 + abs(fd.item()))

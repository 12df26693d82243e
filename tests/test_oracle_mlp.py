"""Pins of the neural-material oracle (Sec. III-D): the encoding's
definition, the forward against torch.nn layers, the hand-written backward
against autograd and central differences."""
import math

import numpy as np
import torch

from oracle import mlp
from synth.params import mlp_init

f64 = torch.float64


def test_param_count():
    assert mlp.N_PARAMS == 56579 and mlp.N_IN == 51


def test_encoding_at_origin_and_values():
    pb = torch.zeros(2, 3, dtype=f64)
    x = mlp.encode(pb)
    assert x.shape == (2, 51)
    assert torch.all(x[:, :3] == 0)
    assert torch.allclose(x[:, 3::2], torch.zeros_like(x[:, 3::2]), atol=1e-15)  # sines
    assert torch.allclose(x[:, 4::2], torch.ones_like(x[:, 4::2]))               # cosines
    pb = torch.tensor([[0.1, -0.3, 0.45]], dtype=f64)
    x = mlp.encode(pb)
    # coordinate c, frequency k: sin(2^k pi p) at 3 + 16 c + 2 (k - 1)
    for c in range(3):
        for k in range(1, 9):
            assert abs(x[0, 3 + 16 * c + 2 * (k - 1)].item() - math.sin(2 ** k * math.pi * pb[0, c].item())) < 1e-12
            assert abs(x[0, 4 + 16 * c + 2 * (k - 1)].item() - math.cos(2 ** k * math.pi * pb[0, c].item())) < 1e-12
    # the exact-reduction form of the BF16 mode gives the same values for
    # the same (FP32) coordinates
    pb32 = pb.float().double()
    assert torch.allclose(mlp.encode(pb32, "bf16"), mlp.encode(pb32), atol=1e-12)


def _setup(seed=0, q=50):
    rng = np.random.default_rng(seed)
    params = torch.tensor(mlp_init(rng, out_bias=(1.0, -2.0, -1.0)), dtype=f64)
    pts = torch.tensor(rng.uniform([0, 0, 0], [60, 40, 3], (q, 3)), dtype=f64)
    return params, pts, np.array([30.0, 20.0, 1.5]), 1.0 / 60.0


def test_forward_matches_torch_nn_layers():
    params, pts, c, inv = _setup()
    (eps, sig, S), _ = mlp.forward(params, pts, c, inv)
    net = torch.nn.Sequential(*[m for (o, i) in mlp.SHAPES
                                for m in (torch.nn.Linear(i, o).double(), torch.nn.ReLU())][:-1])
    lin = [m for m in net if isinstance(m, torch.nn.Linear)]
    with torch.no_grad():
        for m, (W, b) in zip(lin, mlp.unpack(params)):
            m.weight.copy_(W)
            m.bias.copy_(b)
    x = mlp.encode((pts - torch.tensor(c)) * inv)
    o = net(x)
    assert torch.allclose(eps, 1 + torch.nn.functional.softplus(o[:, 0]), rtol=1e-13)
    assert torch.allclose(sig, torch.nn.functional.softplus(o[:, 1]), rtol=1e-13)
    assert torch.allclose(S, torch.sigmoid(o[:, 2]), rtol=1e-13)


def test_manual_backward_equals_autograd():
    params, pts, c, inv = _setup(1)
    rng = np.random.default_rng(2)
    g = [torch.tensor(rng.normal(size=len(pts)), dtype=f64) for _ in range(3)]
    p = params.clone().requires_grad_(True)
    (eps, sig, S), inter = mlp.forward(p, pts, c, inv)
    L = (g[0] * eps + g[1] * sig + g[2] * S).sum()
    (auto,) = torch.autograd.grad(L, p)
    (eps, sig, S), inter = mlp.forward(params, pts, c, inv)
    man = mlp.backward(params, inter, *g)
    assert torch.allclose(man, auto, rtol=1e-10, atol=1e-14)


def test_gradient_central_differences():
    params, pts, c, inv = _setup(3, q=8)
    rng = np.random.default_rng(4)
    g = [torch.tensor(rng.normal(size=len(pts)), dtype=f64) for _ in range(3)]

    def L(p):
        (eps, sig, S), _ = mlp.forward(p, pts, c, inv)
        return (g[0] * eps + g[1] * sig + g[2] * S).sum().item()
    _, inter = mlp.forward(params, pts, c, inv)
    man = mlp.backward(params, inter, *g)
    for idx in rng.choice(mlp.N_PARAMS, 40, replace=False):
        h = 1e-4 * max(abs(params[idx].item()), 1e-2)
        e = torch.zeros_like(params)
        e[idx] = h
        fd = (L(params + e) - L(params - e)) / (2 * h)
        assert abs(fd - man[idx].item()) < 1e-6 * max(1.0, abs(fd)), (idx, fd, man[idx].item())


def test_bf16_mode_is_close_to_fp64():
    params, pts, c, inv = _setup(5, q=200)
    (e1, s1, S1), _ = mlp.forward(params, pts, c, inv)
    (e2, s2, S2), _ = mlp.forward(params, pts, c, inv, mode="bf16")
    for a, b in ((e1, e2), (s1, s2), (S1, S2)):
        rel = (torch.linalg.norm(a - b) / torch.linalg.norm(a)).item()
        assert 1e-5 < rel < 3e-2

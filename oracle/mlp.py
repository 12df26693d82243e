"""Neural materials (oracle).  Test infrastructure only.

Sec. III-D: a small MLP maps each interaction point to material parameters.
Positional encoding (Eq. pos_encoding) applied per coordinate to the point
normalised by the scene's axis-aligned bounding box, p_bar = (p - b)/Delta_b.

Readings: Delta_b is the longest edge of the bounding box; the input is
[p_bar, then per coordinate and k = 1..8: sin(2^k pi p_bar), cos(2^k pi p_bar)]
(51 features); 4 hidden ReLU layers of 128; outputs eps_r = 1 + softplus(o0),
sigma = softplus(o1), S = logistic(o2).

Two modes:
  'fp64'  everything in float64 (the method as defined)
  'bf16'  the rounding points of a BF16 implementation: weights and every
          layer input (the encoding and each hidden activation) rounded to
          BF16 (nearest even, through FP32), accumulation in float64; in the
          backward the deltas that feed the next product are rounded the
          same way.  The encoding is evaluated exactly as such an
          implementation would: p_bar in FP32 arithmetic,
          sin(2 pi frac(2^(k-1) p_bar)).
"""
import math

import torch

f64 = torch.float64
N_FREQ = 8
WIDTH = 128
N_IN = 3 + 6 * N_FREQ
N_OUT = 3
SHAPES = [(WIDTH, N_IN), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (N_OUT, WIDTH)]
N_PARAMS = sum(o * i + o for o, i in SHAPES)


def unpack(params):
    """Flat vector -> [(W [out, in], b [out])] in the packing W0, b0, W1, ..."""
    out, off = [], 0
    for o, i in SHAPES:
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    return out


def bf16(x):
    """Round to BF16 (nearest even) through FP32, return float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(f64)


def normalise(points, center, inv_extent, mode="fp64"):
    if mode == "bf16":
        p = torch.as_tensor(points, dtype=torch.float32)
        c = torch.as_tensor(center, dtype=torch.float32)
        return ((p - c) * torch.tensor(inv_extent, dtype=torch.float32)).to(f64)
    return (torch.as_tensor(points, dtype=f64) - torch.as_tensor(center, dtype=f64)) * inv_extent


def encode(pbar, mode="fp64"):
    """[Q, 3] -> [Q, 51]: p_bar, then for each coordinate and k = 1..8 the
    pair sin(2^k pi p_bar), cos(2^k pi p_bar)."""
    feats = [pbar]
    for c in range(3):
        for k in range(1, N_FREQ + 1):
            if mode == "bf16":
                x = pbar[:, c].to(torch.float32) * (2.0 ** (k - 1))  # exact
                fr = (x - torch.floor(x)).to(f64)
                arg = 2.0 * math.pi * fr
            else:
                arg = (2.0 ** k) * math.pi * pbar[:, c]
            feats.append(torch.stack([torch.sin(arg), torch.cos(arg)], dim=1))
    return torch.cat(feats, dim=1)


def forward(params, points, center, inv_extent, mode="fp64"):
    """Returns (eps_r, sigma, S) [Q] each, and the intermediates
    (x0, [h1..h4], o) for the manual backward."""
    layers = unpack(params)
    x = encode(normalise(points, center, inv_extent, mode), mode)
    rnd = bf16 if mode == "bf16" else (lambda t: t)
    x0 = rnd(x)
    hs = []
    h = x0
    for W, b in layers[:-1]:
        h = rnd(torch.relu(h @ rnd(W).T + b))
        hs.append(h)
    W4, b4 = layers[-1]
    o = h @ rnd(W4).T + b4
    eps = 1.0 + torch.nn.functional.softplus(o[:, 0])
    sig = torch.nn.functional.softplus(o[:, 1])
    S = torch.sigmoid(o[:, 2])
    return (eps, sig, S), (x0, hs, o)


def backward(params, inter, d_eps, d_sig, d_S, mode="fp64"):
    """Gradient of the parameters for output gradients dL/d(eps_r, sigma, S)
    [Q] each, written out layer by layer (reverse mode of forward)."""
    layers = unpack(params)
    rnd = bf16 if mode == "bf16" else (lambda t: t)
    x0, hs, o = inter
    d_o = torch.stack([d_eps * torch.sigmoid(o[:, 0]),
                       d_sig * torch.sigmoid(o[:, 1]),
                       d_S * torch.sigmoid(o[:, 2]) * (1.0 - torch.sigmoid(o[:, 2]))], dim=1)
    d = rnd(d_o)
    grads = [None] * 5
    inputs = [x0] + hs
    for l in range(4, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ inputs[l], d.sum(0))
        if l > 0:
            d = rnd((d @ rnd(W)) * (inputs[l] > 0).to(f64))
    flat = []
    for dW, db in grads:
        flat += [dW.reshape(-1), db]
    return torch.cat(flat)

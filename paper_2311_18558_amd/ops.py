"""torch.autograd.Function wrappers over the C ABI.

Each forward calls one library entry point; each backward calls the matching
hand-written adjoint.  torch's complex-gradient convention (dL/dRe z +
j dL/dIm z for a real loss) is the library's, so gradients pass through
unchanged.

These Functions are the composable face of the library: a caller builds a
loss from them and calls backward().  The calibration driver (pipeline.py,
calibrate.py) issues the same entry points itself, over buffers it allocates
once, so that a step can be recorded into a HIP graph.

    params --MaterialMLP--> (eps_r, sigma, S) per interaction
           --TraceFieldsPerInteraction--> (a, psi)
    raw    --TraceFields--> (a, psi)
    (a, psi, g) --CFR--> H --CFRLoss(H*)--> L
"""
import torch

from . import lib


def _ws(op, radio_c, n_links, n_paths, n_mat=1, device="cuda"):
    return lib.workspace(op, radio_c, n_links, n_paths, n_mat, device)


class TraceFields(torch.autograd.Function):
    """raw material parameters [n_mat, 3] -> (a c64 [P], psi f32 [P]).

    psi (the array phase step of each path) depends on the geometry alone
    and is not differentiable."""

    @staticmethod
    def forward(ctx, raw, paths, radio_c):
        raw = raw.contiguous()
        a = torch.empty(paths.n_paths, dtype=torch.complex64, device=raw.device)
        psi = torch.empty(paths.n_paths, dtype=torch.float32, device=raw.device)
        lib.trace_fields(radio_c, paths, lib.materials_per_id(raw), a, psi)
        ctx.save_for_backward(raw)
        ctx.paths, ctx.radio = paths, radio_c
        ctx.mark_non_differentiable(psi)
        return a, psi

    @staticmethod
    def backward(ctx, ga, _gpsi):
        (raw,) = ctx.saved_tensors
        if ga is None:
            return torch.zeros_like(raw), None, None
        draw = torch.empty_like(raw)
        ws = _ws(lib.RTC_OP_TRACE_FIELDS_ADJOINT, ctx.radio, ctx.paths.n_links,
                 ctx.paths.n_paths, raw.shape[0], raw.device)
        lib.trace_fields_adjoint(ctx.radio, ctx.paths, lib.materials_per_id(raw),
                                 ga.contiguous(), draw, None, ws)
        return draw, None, None


class TraceFieldsPerInteraction(torch.autograd.Function):
    """per-interaction (eps_r, sigma, S) rows [3, D*P] -> (a, psi)."""

    @staticmethod
    def forward(ctx, per_inter, paths, radio_c):
        per_inter = per_inter.contiguous()
        a = torch.empty(paths.n_paths, dtype=torch.complex64, device=per_inter.device)
        psi = torch.empty(paths.n_paths, dtype=torch.float32, device=per_inter.device)
        lib.trace_fields(radio_c, paths, lib.materials_per_interaction(per_inter), a, psi)
        ctx.save_for_backward(per_inter)
        ctx.paths, ctx.radio = paths, radio_c
        ctx.mark_non_differentiable(psi)
        return a, psi

    @staticmethod
    def backward(ctx, ga, _gpsi):
        (per_inter,) = ctx.saved_tensors
        if ga is None:
            return torch.zeros_like(per_inter), None, None
        d = torch.empty_like(per_inter)
        lib.trace_fields_adjoint(ctx.radio, ctx.paths, lib.materials_per_interaction(per_inter),
                                 ga.contiguous(), None, d, None)
        return d, None, None


class MaterialMLP(torch.autograd.Function):
    """Neural materials: MLP parameters (FP32 master vector) and points
    [3, Q] -> per-interaction (eps_r, sigma, S) rows [3, Q].

    The forward keeps the BF16 activations the backward needs (the
    library's saved buffer); the backward returns dL/dparams.  Points are
    not differentiable (the geometry is fixed)."""

    @staticmethod
    def forward(ctx, params, points, aabb_min, aabb_max):
        params = params.contiguous()
        points = points.contiguous()
        Q = int(points.shape[1])
        net = lib.make_mlp(params, aabb_min, aabb_max)
        out = torch.empty((3, Q), dtype=torch.float32, device=params.device)
        saved = lib.mlp_saved(Q, params.device)
        ws = lib.mlp_workspace(Q, params.device)
        lib.mlp_forward(net, Q, points[0], points[1], points[2], out, saved, ws)
        ctx.save_for_backward(params)
        ctx.net, ctx.Q, ctx.saved, ctx.ws = net, Q, saved, ws
        return out

    @staticmethod
    def backward(ctx, gout):
        (params,) = ctx.saved_tensors
        if gout is None:
            return torch.zeros_like(params), None, None, None
        dparams = torch.empty_like(params)
        lib.mlp_backward(ctx.net, ctx.Q, gout.contiguous(), ctx.saved, dparams, ctx.ws)
        return dparams, None, None, None


class CFR(torch.autograd.Function):
    """(a, psi, g) -> H c64 [L, M, N]."""

    @staticmethod
    def forward(ctx, a, psi, g, paths, radio_c):
        a, psi, g = a.contiguous(), psi.contiguous(), g.contiguous()
        H = torch.empty((paths.n_links, radio_c.n_elem, radio_c.n_sc), dtype=torch.complex64,
                        device=a.device)
        lib.cfr(radio_c, paths, a, psi, g, H)
        ctx.save_for_backward(a, psi, g)
        ctx.paths, ctx.radio = paths, radio_c
        return H

    @staticmethod
    def backward(ctx, gH):
        a, psi, g = ctx.saved_tensors
        dLda = torch.empty_like(a)
        dLdg = torch.empty_like(g)
        ws = _ws(lib.RTC_OP_CFR_ADJOINT, ctx.radio, ctx.paths.n_links, ctx.paths.n_paths,
                 1, a.device)
        lib.cfr_adjoint(ctx.radio, ctx.paths, a, psi, g, gH.contiguous(), dLda, dLdg, ws)
        return dLda, None, dLdg, None, None


class CFRLoss(torch.autograd.Function):
    """(H, H*) -> (total loss, terms): the total a float64 scalar, terms the
    float64 [3] vector {total, coherent, PDP} (not differentiable).  dL/dH
    comes out of the same kernel pass and is kept for backward; a gradient
    flowing into the total scales it."""

    @staticmethod
    def forward(ctx, H, H_tgt, radio_c, tgt_stats=None, w_coh=1.0, w_pdp=1.0):
        n_links = H.shape[0]
        terms = torch.empty(3, dtype=torch.float64, device=H.device)
        dLdH = torch.empty_like(H) if ctx.needs_input_grad[0] else None
        ws = _ws(lib.RTC_OP_CFR_LOSS, radio_c, n_links, 0, 1, H.device)
        lib.cfr_loss(radio_c, n_links, H.contiguous(), H_tgt.contiguous(), tgt_stats, w_coh,
                     w_pdp, terms, dLdH, ws)
        ctx.dLdH = dLdH
        total = terms[0].clone()
        ctx.mark_non_differentiable(terms)
        return total, terms

    @staticmethod
    def backward(ctx, g_total, _g_terms):
        if ctx.dLdH is None or g_total is None:
            return None, None, None, None, None, None
        return ctx.dLdH * g_total.to(torch.float32), None, None, None, None, None

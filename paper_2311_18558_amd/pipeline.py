"""One calibration step of the hot path with preallocated device buffers.

    trace_fields -> cfr -> loss (dL/dH in place) -> cfr_adjoint
                 -> trace_fields_adjoint -> Adam

With the workload loss at shapes the fused pass takes (up to 32 elements,
256 to 1,024 subcarriers) cfr, loss and cfr_adjoint are one library call,
rtc_cfr_loss_adjoint, and H and dL/dH never leave the chip (fused=False keeps
the three calls).

(Algorithm 1 of the paper, per-material-id mode.)  The loss is either the
workload loss (coherent + power-delay-profile NMSE, loss="workload") or the
paper's own (loss="paper": SMAPE of RMS delay spread and gain per CIR row,
Sec. III-E, with the moving-average measurement scale of Sec. III-F when
update_alpha is set).
Every step runs in the library's kernels; this module only owns buffers,
workspaces and the order of calls, all on one stream.
"""
import numpy as np
import torch

from . import lib


class Pipeline:
    def __init__(self, store, radio, raw0, g0, device="cuda", stream=None, loss="workload",
                 update_alpha=False, delta=0.99, fused=True, targets="cir"):
        if loss not in ("workload", "paper"):
            raise ValueError(loss)
        if targets not in ("cir", "cfr"):
            raise ValueError(targets)
        # the targets as their transforms X* ("cir": the fused pass and the
        # separate loss read X*) or as H* ("cfr": with the target PDP stored
        # for the fused pass, formed per row by the separate loss); the same
        # loss either way
        self.targets = targets
        self.loss_kind = loss
        self.update_alpha, self.delta = update_alpha, delta
        self.dev = torch.device(device)
        self.stream = stream
        self.paths = store if isinstance(store, lib.DevicePaths) else lib.DevicePaths(store, self.dev)
        self.radio = lib.radio_from(radio)
        L, P = self.paths.n_links, self.paths.n_paths
        M, N = self.radio.n_elem, self.radio.n_sc
        self.L, self.P, self.M, self.N = L, P, M, N
        self.fused = bool(fused) and loss == "workload" and lib.fused_supported(self.radio)
        self.raw = torch.tensor(np.asarray(raw0, np.float32), device=self.dev)
        self.g = torch.tensor(np.asarray(g0, np.complex64), device=self.dev)
        self.n_mat = self.raw.shape[0]
        self.a = torch.empty(P, dtype=torch.complex64, device=self.dev)
        self.psi = torch.empty(P, dtype=torch.float32, device=self.dev)
        # H (and dL/dH in place) only exists outside the fused pass; the fused
        # step keeps a buffer for forward evaluations (targets, metrics)
        self.H = torch.empty((L, M, N), dtype=torch.complex64, device=self.dev)
        self.ws_fused = (lib.workspace(lib.RTC_OP_CFR_LOSS_ADJOINT, self.radio, L, P, 1, self.dev)
                         if self.fused else None)
        self.loss = torch.zeros(3, dtype=torch.float64, device=self.dev)
        self.dLda = torch.empty(P, dtype=torch.complex64, device=self.dev)
        self.dLdg = torch.empty(M, dtype=torch.complex64, device=self.dev)
        self.draw = torch.empty_like(self.raw)
        op = lib.RTC_OP_CFR_LOSS if loss == "workload" else lib.RTC_OP_PAPER_LOSS
        self.ws_loss = lib.workspace(op, self.radio, L, P, 1, self.dev)
        # measurement scale state {alpha, updates} (paper loss)
        self.alpha = torch.tensor([1.0, 0.0], dtype=torch.float64, device=self.dev)
        self.ws_adj = lib.workspace(lib.RTC_OP_CFR_ADJOINT, self.radio, L, P, 1, self.dev)
        self.ws_tr = lib.workspace(lib.RTC_OP_TRACE_FIELDS_ADJOINT, self.radio, L, P,
                                   self.n_mat, self.dev)
        self.mats = lib.materials_per_id(self.raw)
        # Adam state (float32), materials and gains (as interleaved reals)
        self.m_raw = torch.zeros_like(self.raw)
        self.v_raw = torch.zeros_like(self.raw)
        self.g_real = torch.view_as_real(self.g)
        self.dLdg_real = torch.view_as_real(self.dLdg)
        self.m_g = torch.zeros_like(self.g_real)
        self.v_g = torch.zeros_like(self.g_real)
        self.t = 0
        self.H_tgt = None
        self.tgt_stats = None
        self.p_tgt = self.X_tgt = None

    # individual stages (each one library call)
    def trace(self):
        lib.trace_fields(self.radio, self.paths, self.mats, self.a, self.psi, self.stream)

    def cfr(self, out=None):
        lib.cfr(self.radio, self.paths, self.a, self.psi, self.g,
                self.H if out is None else out, self.stream)

    def set_target(self, H_tgt):
        """Targets for the loss; what the loss needs of them is computed once
        here (they do not change while calibrating on this batch): energies
        and power delay profiles (workload loss) or per-row gain and RMS
        delay spread (paper loss)."""
        self.H_tgt = H_tgt
        if self.loss_kind == "paper":
            self.tgt_stats = torch.empty((self.L * self.M, 2), dtype=torch.float64,
                                         device=self.dev)
            lib.cir_stats(self.radio, self.L, H_tgt, self.tgt_stats, self.stream)
            self.alpha.copy_(torch.tensor([1.0, 0.0], dtype=torch.float64))
            return
        # targets as X* (targets="cir"): the fused pass reads 8 B per tap of
        # them, the separate loss runs two transforms per row; as H*
        # (targets="cfr"): the fused pass takes H* and a stored p* (12 B per
        # tap), the separate loss forms p* from H* by one more transform per
        # row (24 B per tap instead of 28 with a stored p*, and faster)
        self.tgt_stats = torch.empty(2, dtype=torch.float64, device=self.dev)
        self.p_tgt = self.X_tgt = None
        if self.targets == "cir":
            self.X_tgt = torch.empty((self.L, self.M, self.N), dtype=torch.complex64,
                                     device=self.dev)
            lib.cfr_target_cir(self.radio, self.L, H_tgt, self.tgt_stats, self.X_tgt,
                               self.ws_loss, self.stream)
            return
        if self.fused:
            self.p_tgt = torch.empty((self.L, self.M, self.N), dtype=torch.float32,
                                     device=self.dev)
        lib.cfr_target_stats(self.radio, self.L, H_tgt, self.tgt_stats, self.ws_loss, self.stream,
                             p_tgt=self.p_tgt)

    def loss_and_grad(self):
        if self.loss_kind == "paper":
            lib.paper_loss(self.radio, self.L, self.H, self.tgt_stats, self.alpha, self.loss,
                           self.H, self.ws_loss, update_alpha=self.update_alpha,
                           delta=self.delta, stream=self.stream)
            return
        if self.X_tgt is not None:
            lib.cfr_loss_cir(self.radio, self.L, self.H, self.X_tgt, self.tgt_stats, 1.0, 1.0,
                             self.loss, self.H, self.ws_loss, self.stream)
            return
        lib.cfr_loss(self.radio, self.L, self.H, self.H_tgt, self.tgt_stats, 1.0, 1.0,
                     self.loss, self.H, self.ws_loss, self.stream, p_tgt=self.p_tgt)

    def cfr_loss_adjoint(self):
        if self.X_tgt is not None:
            lib.cfr_loss_adjoint_cir(self.radio, self.paths, self.a, self.psi, self.g, self.X_tgt,
                                     self.tgt_stats, 1.0, 1.0, self.loss, self.dLda, self.dLdg,
                                     self.ws_fused, self.stream)
            return
        lib.cfr_loss_adjoint(self.radio, self.paths, self.a, self.psi, self.g, self.H_tgt,
                             self.tgt_stats, self.p_tgt, 1.0, 1.0, self.loss, self.dLda,
                             self.dLdg, self.ws_fused, self.stream)

    def cfr_adjoint(self):
        lib.cfr_adjoint(self.radio, self.paths, self.a, self.psi, self.g, self.H, self.dLda,
                        self.dLdg, self.ws_adj, self.stream)

    def trace_adjoint(self):
        lib.trace_fields_adjoint(self.radio, self.paths, self.mats, self.dLda, self.draw, None,
                                 self.ws_tr, self.stream)

    def adam(self, lr=0.01, train_gains=True):
        self.t += 1
        lib.adam_step(self.raw, self.draw, self.m_raw, self.v_raw, self.t, lr=lr,
                      stream=self.stream)
        if train_gains:
            lib.adam_step(self.g_real, self.dLdg_real, self.m_g, self.v_g, self.t, lr=lr,
                          stream=self.stream)

    @property
    def stages(self):
        if self.fused:
            return ("trace_fields", "cfr_loss_adjoint", "trace_fields_adjoint", "adam")
        loss = "cfr_loss" if self.loss_kind == "workload" else "paper_loss"
        return ("trace_fields", "cfr", loss, "cfr_adjoint", "trace_fields_adjoint", "adam")

    def step(self, lr=0.01, events=None):
        """One full calibration step.  `events`, if given, maps stage name
        to a list that receives (start, end) CUDA events per stage."""
        if self.fused:
            fns = (self.trace, self.cfr_loss_adjoint, self.trace_adjoint, lambda: self.adam(lr))
        else:
            fns = (self.trace, self.cfr, self.loss_and_grad, self.cfr_adjoint, self.trace_adjoint,
                   lambda: self.adam(lr))
        for name, fn in zip(self.stages, fns):
            if events is None:
                fn()
            else:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                events.setdefault(name, []).append((e0, e1))

"""One calibration step streamed over Rx batches, for scenes whose CFRs do
not fit the device at once (the large-scene configuration: 4 Tx x 65,536 Rx,
~2,000 paths per link, 4,096 subcarriers, 32 elements: 3.4e10 CFR taps).

The path store stays resident on the device as a list of link batches; the
targets are the paper's per-CIR-row statistics (Sec. III-E: gain and RMS
delay spread, two doubles per row), so no target CFR is kept.  One optimiser
step runs, batch by batch,

    [neural materials forward] -> trace_fields -> cfr -> paper loss
    -> cfr_adjoint -> trace_fields_adjoint -> [neural materials backward]

with the loss of every batch weighted by its share of the CIR rows (the
batch losses then sum to the mean over all rows, as one unstreamed step over
the whole scene would compute it) and the parameter gradients accumulated in
device memory; Adam runs once after the last batch.  Every stage is a
library kernel; buffers are sized once for the largest batch.  The
measurement scale is fixed (alpha = 1, synthetic targets as in Sec. IV-B).
"""
import numpy as np
import torch

from . import lib


class StreamedCalibration:
    def __init__(self, batches, radio, mode, raw0=None, mlp_params0=None, aabb=None, g0=None,
                 lr=0.01, lr_mlp=1e-4, device="cuda"):
        if mode not in ("per_id", "neural"):
            raise ValueError(mode)
        self.dev = torch.device(device)
        self.batches = list(batches)
        self.radio = lib.radio_from(radio)
        self.mode = mode
        M, N = self.radio.n_elem, self.radio.n_sc
        self.g = torch.tensor(np.ones(M, np.complex64) if g0 is None else g0, device=self.dev)
        self.rows_total = sum(b.n_links for b in self.batches) * M
        Lmax = max(b.n_links for b in self.batches)
        Pmax = max(b.n_paths for b in self.batches)
        # neural materials are evaluated at the used interaction slots only
        self.compact = ([lib.compact_interactions(b) for b in self.batches]
                        if mode == "neural" else None)
        Qmax = max(c[1] for c in self.compact) if self.compact else 0
        self.a = torch.empty(Pmax, dtype=torch.complex64, device=self.dev)
        self.psi = torch.empty(Pmax, dtype=torch.float32, device=self.dev)
        self.dLda = torch.empty(Pmax, dtype=torch.complex64, device=self.dev)
        self.H = torch.empty(Lmax * M * N, dtype=torch.complex64, device=self.dev)
        self.alpha = torch.tensor([1.0, 0.0], dtype=torch.float64, device=self.dev)
        self.loss_rows = torch.zeros((len(self.batches), 3), dtype=torch.float64,
                                     device=self.dev)
        n_ws = max(lib.workspace_size(op, self.radio, Lmax, Pmax, 1)
                   for op in (lib.RTC_OP_PAPER_LOSS, lib.RTC_OP_CFR_ADJOINT))
        self.ws = torch.empty(max(n_ws, 8), dtype=torch.uint8, device=self.dev)
        if mode == "per_id":
            self.params = torch.tensor(np.asarray(raw0, np.float32), device=self.dev)
            self.mats = lib.materials_per_id(self.params)
            n_tr = lib.workspace_size(lib.RTC_OP_TRACE_FIELDS_ADJOINT, self.radio, Lmax, Pmax,
                                      self.params.shape[0])
            self.ws_tr = torch.empty(max(n_tr, 8), dtype=torch.uint8, device=self.dev)
            self.lr = lr
        else:
            self.params = torch.tensor(np.asarray(mlp_params0, np.float32), device=self.dev)
            self.net = lib.make_mlp(self.params, *aabb)
            # per-interaction rows of a batch are packed with its own row length
            self.per = torch.empty(3 * Qmax, dtype=torch.float32, device=self.dev)
            self.dint = torch.empty(3 * Qmax, dtype=torch.float32, device=self.dev)
            self.saved = lib.mlp_saved(Qmax, self.dev)
            self.mlp_ws = lib.mlp_workspace(Qmax, self.dev)
            self.lr = lr_mlp
        self.grad = torch.zeros_like(self.params)
        self.grad_b = torch.empty_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.targets = None

    # ----------------------------------------------------------- targets
    def set_targets(self, gt_raw):
        """Per-row targets (P, tau_RMS) of every batch from hidden per-id
        ground-truth materials (the method's own CFRs at the truth)."""
        raw = torch.tensor(np.asarray(gt_raw, np.float32), device=self.dev)
        mats = lib.materials_per_id(raw)
        M, N = self.radio.n_elem, self.radio.n_sc
        self.targets = []
        for b in self.batches:
            H = self.H[:b.n_links * M * N]
            lib.trace_fields(self.radio, b, mats, self.a, self.psi)
            lib.cfr(self.radio, b, self.a, self.psi, self.g, H)
            t = torch.empty((b.n_links * M, 2), dtype=torch.float64, device=self.dev)
            lib.cir_stats(self.radio, b.n_links, H, t)
            self.targets.append(t)

    # ------------------------------------------------------------- step
    def _materials(self, i):
        if self.mode == "per_id":
            return self.mats, None
        idx, Q, pts = self.compact[i]
        per = self.per[:3 * Q].view(3, Q)
        lib.mlp_forward(self.net, Q, pts[0], pts[1], pts[2], per, self.saved, self.mlp_ws)
        return lib.materials_per_interaction(per, (idx, Q)), Q

    def batch_step(self, i, events=None):
        """Forward, weighted paper loss and reverse pass of batch i; the
        parameter gradient is added to self.grad.  events: a dict that
        collects (start, end) CUDA events per stage, or None."""
        b = self.batches[i]
        M, N = self.radio.n_elem, self.radio.n_sc
        H = self.H[:b.n_links * M * N]
        w = float(b.n_links * M) / self.rows_total
        mark = _Marks(events)
        mark("materials")
        mats, Q = self._materials(i)
        mark("trace_fields")
        lib.trace_fields(self.radio, b, mats, self.a, self.psi)
        mark("cfr")
        lib.cfr(self.radio, b, self.a, self.psi, self.g, H)
        mark("paper_loss")
        lib.paper_loss(self.radio, b.n_links, H, self.targets[i], self.alpha, self.loss_rows[i],
                       H, self.ws, update_alpha=False, w_tau=w, w_gain=w)
        mark("cfr_adjoint")
        lib.cfr_adjoint(self.radio, b, self.a, self.psi, self.g, H, self.dLda, None, self.ws)
        mark("trace_fields_adjoint")
        if self.mode == "per_id":
            lib.trace_fields_adjoint(self.radio, b, mats, self.dLda, self.grad_b, None,
                                     self.ws_tr)
        else:
            dint = self.dint[:3 * Q].view(3, Q)
            lib.trace_fields_adjoint(self.radio, b, mats, self.dLda, None, dint, None)
            mark("materials_backward")
            lib.mlp_backward(self.net, Q, dint, self.saved, self.grad_b, self.mlp_ws)
        mark("axpy")
        lib.axpy(self.grad, self.grad_b)
        mark(None)

    def step(self, update=True, events=None):
        """One optimiser step over every batch; returns the loss L (device
        scalar: the sum of the batches' weighted losses)."""
        self.grad.zero_()
        for i in range(len(self.batches)):
            self.batch_step(i, events)
        if update:
            lib.adam_step_dev(self.params, self.grad, self.m, self.v, self.step_dev, True,
                              lr=self.lr)
        return self.loss_rows[:, 0].sum()


class _Marks:
    """Stage timing on the current stream: mark(name) closes the open stage
    and opens `name` (None closes only); events[name] collects (start, end)
    pairs."""

    def __init__(self, events):
        self.events = events
        self.open = None

    def __call__(self, name):
        if self.events is None:
            return
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        if self.open is not None:
            self.events.setdefault(self.open[0], []).append((self.open[1], e))
        self.open = None if name is None else (name, e)


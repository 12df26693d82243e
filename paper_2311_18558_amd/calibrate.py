"""Gradient-based scene calibration (Algorithm 1 of the paper, with Adam as
in Sec. IV-B) on fixed paths, in two parametrisations:

  'per_id'  trainable materials per class (Sec. III-C, one-dimensional
            embeddings): raw [n_mat, 3] plus the complex element gains
  'neural'  neural materials (Sec. III-D): MLP weights plus the gains
  'embed'   material embeddings of dimension L with a shared read-out
            vector (Sec. III-C, Eqs. trainable_materials_1-4)

Optionally (per_id and embed) the trainable Tx gain (Sec. III-A) and the
trainable scattering pattern with K_x per material (Sec. III-B) are
calibrated with the materials; in embed mode K_x comes from the fourth
embedding.

The loss is the workload loss (coherent + power-delay-profile NMSE) or, with
loss="paper", the paper's own (Sec. III-E: SMAPE of RMS delay spread and gain
per CIR row, against measurements scaled by the moving-average estimate of
Sec. III-F when update_alpha is set).

Every step of the method runs in librtcal; this module draws batches,
stages their inputs (device gathers of the fixed path store and targets) and
sequences the library calls on one stream.
"""
import math

import numpy as np
import torch

from . import lib

# prior mid-points used to initialise (eps_r in U[2, 10], sigma in
# logU[1e-3, 1], S = 0.1)
INIT_EPS, INIT_SIG, INIT_S = 5.5, 10 ** -1.5, 0.1


def raw_prior(n_mat):
    u = np.array([math.log(INIT_EPS - 1.0), math.log(INIT_SIG), math.log(INIT_S / (1 - INIT_S))])
    return np.tile(u, (n_mat, 1)).astype(np.float32)


def mlp_out_bias():
    """Output biases that map to the prior mid-points through
    eps_r = 1 + softplus, sigma = softplus, S = logistic."""
    inv_softplus = lambda y: math.log(math.expm1(y))
    return (inv_softplus(INIT_EPS - 1.0), inv_softplus(INIT_SIG), math.log(INIT_S / (1 - INIT_S)))


class Calibrator:
    def __init__(self, dp, radio, H_all, mode, raw0=None, mlp_params0=None, g0=None,
                 aabb=None, lr=0.01, lr_mlp=1e-3, lr_gain=None, device="cuda", loss="workload",
                 update_alpha=False, delta=0.99, embed0=None, n_vmf=0, tx_raw0=None,
                 pat_raw0=None, fused=True):
        """embed0 = (v [L], W [n_mat, 4, L]) for mode 'embed'; n_vmf, tx_raw0
        [1 + 5 n_vmf] the initial raw Tx gain; pat_raw0 [n_mat, 6] the
        initial raw scattering patterns (see rtc_patterns).  fused: with the
        workload loss at shapes the fused pass takes, each step runs CFR,
        loss and CFR adjoint as one library call on the batch's targets in
        the delay domain (rtc_cfr_target_cir, rtc_cfr_loss_adjoint_cir);
        fused=False keeps the three separate calls."""
        if loss not in ("workload", "paper"):
            raise ValueError(loss)
        if mode not in ("per_id", "neural", "embed"):
            raise ValueError(mode)
        if mode == "neural" and pat_raw0 is not None:
            raise ValueError("scattering patterns are calibrated per material (per_id, embed)")
        self.dev = torch.device(device)
        self.loss_kind, self.update_alpha, self.delta = loss, update_alpha, delta
        self.fused = bool(fused) and loss == "workload" and lib.fused_supported(
            lib.radio_from(radio))
        self.alpha = torch.tensor([1.0, 0.0], dtype=torch.float64, device=self.dev)
        self.dp = dp
        self.radio = lib.radio_from(radio)
        self.H_all = H_all
        self.mode = mode
        M = self.radio.n_elem
        self.g = torch.tensor(np.ones(M, np.complex64) if g0 is None else g0, device=self.dev)
        self.g_real = torch.view_as_real(self.g)
        self.m_g = torch.zeros_like(self.g_real)
        self.v_g = torch.zeros_like(self.g_real)
        self.lr, self.lr_mlp = lr, lr_mlp
        self.lr_gain = lr if lr_gain is None else lr_gain
        self.t = 0
        # Adam's step count lives on the device so that a recorded graph
        # advances it on replay
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self._none = torch.zeros(0, dtype=torch.float32, device=self.dev)
        # one flat FP32 parameter vector: [materials or MLP | patterns | Tx gain]
        segs = []
        if mode == "per_id":
            segs.append(("raw", np.asarray(raw0, np.float32)))
        elif mode == "embed":
            segs += [("v", np.asarray(embed0[0], np.float32)),
                     ("W", np.asarray(embed0[1], np.float32))]
        else:
            segs.append(("mlp", np.asarray(mlp_params0, np.float32)))
        self.n_main = sum(a.size for _, a in segs)
        if pat_raw0 is not None:
            segs.append(("pat", np.asarray(pat_raw0, np.float32)))
        self.n_vmf = int(n_vmf)
        if self.n_vmf:
            segs.append(("tx", np.asarray(tx_raw0, np.float32)))
        flat = np.concatenate([a.reshape(-1) for _, a in segs])
        self.params = torch.tensor(flat, device=self.dev)
        self.dparams = torch.zeros_like(self.params)
        self.P, self.G = {}, {}
        o = 0
        for name, a in segs:
            self.P[name] = self.params[o:o + a.size].view(a.shape)
            self.G[name] = self.dparams[o:o + a.size].view(a.shape)
            o += a.size
        self.m_p = torch.zeros_like(self.params)
        self.v_p = torch.zeros_like(self.params)
        if mode == "per_id":
            self.raw = self.P["raw"]
        elif mode == "embed":
            self.raw = torch.empty((self.P["W"].shape[0], 3), dtype=torch.float32,
                                   device=self.dev)
            self.draw = torch.empty_like(self.raw)
        if mode != "neural":
            self.mats = lib.materials_per_id(self.raw)
        else:
            self.net = lib.make_mlp(self.P["mlp"], *aabb)
        self.with_patterns = pat_raw0 is not None or self.n_vmf > 0
        self.pats = (lib.patterns(self.n_vmf, self.P.get("tx"), self.P.get("pat"))
                     if self.with_patterns else None)
        self._bufs = {}
        if loss == "paper":
            # per-row gain and RMS delay spread of every measured CFR, once
            La = H_all.shape[0]
            self.tgt_all = torch.empty((La * M, 2), dtype=torch.float64, device=self.dev)
            lib.cir_stats(self.radio, La, H_all, self.tgt_all)
            self.tgt_all = self.tgt_all.view(La, M, 2)

    def _buf(self, name, shape, dtype):
        b = self._bufs.get(name)
        n = int(np.prod(shape))
        if b is None or b.numel() < n or b.dtype != dtype:
            b = torch.empty(max(n, 1), dtype=dtype, device=self.dev)
            self._bufs[name] = b
        return b[:n].view(shape)

    def _ws(self, op, L, P, n_mat=1):
        n = lib.workspace_size(op, self.radio, L, P, n_mat)
        return self._buf(f"ws{op}", (max(n, 8),), torch.uint8)

    def _materials(self, b):
        """Per-interaction materials of batch paths b (neural mode) or the
        per-id descriptor."""
        if self.mode == "embed":
            lib.embed_readout(self.P["v"], self.P["W"], self.raw, self.P.get("pat"))
        if self.mode != "neural":
            return self.mats, None
        # the network is evaluated at the batch's used interaction slots only
        comp = getattr(b, "compact", None)
        if comp is None:
            comp = b.compact = lib.compact_interactions(b)
        idx, Q, pts = comp
        per = self._buf("per", (3, Q), torch.float32)
        saved = self._buf("saved", (int(lib.load().rtc_mlp_saved_size(Q)),), torch.uint8)
        ws = self._buf("mlpws", (int(lib.load().rtc_mlp_workspace_size(Q)),), torch.uint8)
        lib.mlp_forward(self.net, Q, pts[0], pts[1], pts[2], per, saved, ws)
        return lib.materials_per_interaction(per, (idx, Q)), (Q, saved, ws)

    def forward(self, b, H_out):
        mats, aux = self._materials(b)
        P = b.n_paths
        a = self._buf("a", (P,), torch.complex64)
        psi = self._buf("psi", (P,), torch.float32)
        lib.trace_fields_pat(self.radio, b, mats, self.pats, a, psi)
        lib.cfr(self.radio, b, a, psi, self.g, H_out)
        return mats, aux, a, psi

    def step(self, links, update=True, batch=None):
        """One iteration of Algorithm 1 on the batch `links`; returns the
        loss terms as a device float64 [3] tensor.  With update=False only
        the loss and the gradients (self.dparams, self.dLdg) are formed.
        batch: the gathered paths of `links` (lib.subset_links), if the
        caller has them (no host synchronisation is left then)."""
        b = lib.subset_links(self.dp, links)[0] if batch is None else batch
        L, P = b.n_links, b.n_paths
        M, N = self.radio.n_elem, self.radio.n_sc
        loss = self._buf("loss", (3,), torch.float64)
        dLda = self._buf("dLda", (P,), torch.complex64)
        dLdg = self._buf("dLdg", (M,), torch.complex64)
        if self.fused:
            # the batch's targets as X* with their statistics (one transform
            # per row, as the separate loss forms p* from H*), then CFR, loss
            # and CFR adjoint in one pass: H and dL/dH stay on chip
            Xt = self._buf("Xt", (L, M, N), torch.complex64)
            tstats = self._buf("tstats", (2,), torch.float64)
            lib.cfr_target_cir(self.radio, L, self.H_all[links], tstats, Xt,
                               self._ws(lib.RTC_OP_CFR_TARGET_STATS, L, P))
            mats, aux = self._materials(b)
            a = self._buf("a", (P,), torch.complex64)
            psi = self._buf("psi", (P,), torch.float32)
            lib.trace_fields_pat(self.radio, b, mats, self.pats, a, psi)
            lib.cfr_loss_adjoint_cir(self.radio, b, a, psi, self.g, Xt, tstats, 1.0, 1.0, loss,
                                     dLda, dLdg, self._ws(lib.RTC_OP_CFR_LOSS_ADJOINT, L, P))
            return self._backward_and_update(b, mats, aux, dLda, dLdg, loss, update)
        H = self._buf("H", (L, M, N), torch.complex64)
        mats, aux, a, psi = self.forward(b, H)
        if self.loss_kind == "paper":
            tgt = self.tgt_all[links].reshape(-1, 2)
            lib.paper_loss(self.radio, L, H, tgt, self.alpha, loss, H,
                           self._ws(lib.RTC_OP_PAPER_LOSS, L, P), update_alpha=self.update_alpha,
                           delta=self.delta)
        else:
            lib.cfr_loss(self.radio, L, H, self.H_all[links], None, 1.0, 1.0, loss, H,
                         self._ws(lib.RTC_OP_CFR_LOSS, L, P))
        lib.cfr_adjoint(self.radio, b, a, psi, self.g, H, dLda, dLdg,
                        self._ws(lib.RTC_OP_CFR_ADJOINT, L, P))
        return self._backward_and_update(b, mats, aux, dLda, dLdg, loss, update)

    def _backward_and_update(self, b, mats, aux, dLda, dLdg, loss, update):
        """From dL/da and dL/dg of the batch to the parameter gradients
        (trace adjoint, MLP or embedding backward) and, with update, one
        Adam step."""
        L, P = b.n_links, b.n_paths
        op = (lib.RTC_OP_TRACE_FIELDS_ADJOINT_PAT if self.with_patterns
              else lib.RTC_OP_TRACE_FIELDS_ADJOINT)
        if self.mode != "neural":
            draw = self.G["raw"] if self.mode == "per_id" else self.draw
            lib.trace_fields_adjoint_pat(self.radio, b, mats, self.pats, dLda, draw, None,
                                         self.G.get("tx"), self.G.get("pat"),
                                         self._ws(op, L, P, self.raw.shape[0]))
            if self.mode == "embed":
                lib.embed_readout_backward(self.P["v"], self.P["W"], self.draw, self.G.get("pat"),
                                           self.G["v"], self.G["W"])
        else:
            Q, saved, ws = aux
            dint = self._buf("dint", (3, Q), torch.float32)
            lib.trace_fields_adjoint_pat(self.radio, b, mats, self.pats, dLda, None, dint,
                                         self.G.get("tx"), None,
                                         self._ws(op, L, P) if self.n_vmf else None)
            lib.mlp_backward(self.net, Q, dint, saved, self.G["mlp"], ws)
        self.dLdg = dLdg
        if not update:
            return loss
        self.t += 1
        n = self.n_main
        lr = self.lr_mlp if self.mode == "neural" else self.lr
        lib.adam_step_dev(self.params[:n], self.dparams[:n], self.m_p[:n], self.v_p[:n],
                          self.step_dev, False, lr=lr)
        if self.params.numel() > n:
            lib.adam_step_dev(self.params[n:], self.dparams[n:], self.m_p[n:], self.v_p[n:],
                              self.step_dev, False, lr=self.lr)
        if self.lr_gain > 0:
            lib.adam_step_dev(self.g_real, torch.view_as_real(dLdg), self.m_g, self.v_g,
                              self.step_dev, False, lr=self.lr_gain)
        # one optimiser step: advance the shared step count once
        lib.adam_step_dev(self._none, self._none, self._none, self._none, self.step_dev, True)
        return loss

    def save(self, path):
        """Checkpoint: parameters, Adam moments and step count, element
        gains and their moments, the measurement scale, to an .npz file
        (plain arrays; load() restores them bit for bit)."""
        host = {k: t.detach().cpu().numpy() for k, t in
                zip(("params", "m_p", "v_p", "g_real", "m_g", "v_g", "step_dev", "alpha"),
                    self._state())}
        np.savez(path, t=np.array(self.t), mode=np.array(self.mode), **host)

    def load(self, path):
        """Restore a checkpoint written by save() into a calibrator built
        with the same configuration (shapes are checked)."""
        z = np.load(path, allow_pickle=False)
        if str(z["mode"]) != self.mode:
            raise ValueError(f"checkpoint of mode {z['mode']}, calibrator of mode {self.mode}")
        for name, dst in zip(("params", "m_p", "v_p", "g_real", "m_g", "v_g", "step_dev", "alpha"),
                             self._state()):
            src = torch.from_numpy(z[name])
            if src.shape != dst.shape:
                raise ValueError(f"{name}: checkpoint shape {tuple(src.shape)}, "
                                 f"calibrator {tuple(dst.shape)}")
            dst.copy_(src.to(dst.device))
        self.t = int(z["t"])

    def _state(self):
        return [self.params, self.m_p, self.v_p, self.g_real, self.m_g, self.v_g, self.step_dev,
                self.alpha]

    def record(self, links, warmup=2):
        """One step on the fixed batch `links` recorded into a HIP graph
        (torch.cuda.CUDAGraph): every stage is a library kernel launched on
        the capture stream, with no host synchronisation, allocation or
        memset inside.  `warmup` eager steps on a side stream first (buffers
        and workspaces are allocated there); the parameters and optimiser
        state are then restored, so replay k of the graph is step k of the
        calibration.  Returns (graph, loss) with loss the device tensor each
        replay overwrites."""
        links = torch.as_tensor(links, device=self.dev)
        batch = lib.subset_links(self.dp, links)[0]
        if self.mode == "neural":
            batch.compact = lib.compact_interactions(batch)
        saved = [t.clone() for t in self._state()]
        t0 = self.t
        side = torch.cuda.Stream(device=self.dev)
        side.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.step(links, batch=batch)
        torch.cuda.current_stream(self.dev).wait_stream(side)
        torch.cuda.synchronize(self.dev)
        for dst, src in zip(self._state(), saved):
            dst.copy_(src)
        self.t = t0
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            loss = self.step(links, batch=batch)
        self.t = t0  # recording ran no step
        self._graph_keep = (batch, links)
        return graph, loss

    def learned(self):
        """Current materials, patterns and Tx gain as host values: dict with
        eps_r, sigma, S [n_mat] (per_id, embed), K_x, w [n_mat, 3], lam2,
        lam3 (with patterns) and eta, w_tx, lam_tx, mu_tx (with a Tx gain).
        Only host arithmetic on copies of the device parameters."""
        out = {}
        if self.mode == "embed":
            lib.embed_readout(self.P["v"], self.P["W"], self.raw, self.P.get("pat"))
        if self.mode != "neural":
            r = self.raw.double().cpu().numpy()
            out.update(eps_r=1.0 + np.exp(r[:, 0]), sigma=np.exp(r[:, 1]),
                       S=1.0 / (1.0 + np.exp(-r[:, 2])))
        if "pat" in self.P:
            q = self.P["pat"].double().cpu().numpy()
            e = np.exp(q[:, 1:4] - q[:, 1:4].max(1, keepdims=True))
            out.update(K_x=1.0 / (1.0 + np.exp(-q[:, 0])), w=e / e.sum(1, keepdims=True),
                       lam2=np.exp(q[:, 4]), lam3=np.exp(q[:, 5]))
        if self.n_vmf:
            t = self.P["tx"].double().cpu().numpy()
            K = self.n_vmf
            e = np.exp(t[1:1 + K] - t[1:1 + K].max())
            mu = t[1 + 2 * K:1 + 5 * K].reshape(K, 3)
            out.update(eta=1.0 / (1.0 + np.exp(-t[0])), w_tx=e / e.sum(),
                       lam_tx=np.exp(t[1 + K:1 + 2 * K]),
                       mu_tx=mu / np.linalg.norm(mu, axis=1, keepdims=True))
        return out

    def nmse(self, links, chunk=512):
        """Held-out CFR NMSE = sum|H - H*|^2 / sum|H*|^2 over `links`."""
        num, den = 0.0, 0.0
        M, N = self.radio.n_elem, self.radio.n_sc
        for i in range(0, len(links), chunk):
            ls = links[i:i + chunk]
            b, _ = lib.subset_links(self.dp, ls)
            H = self._buf("Hn", (b.n_links, M, N), torch.complex64)
            self.forward(b, H)
            H_t = self.H_all[ls]
            ws = self._ws(lib.RTC_OP_CFR_LOSS, b.n_links, b.n_paths)
            stats = self._buf("stats", (2,), torch.float64)
            lib.cfr_target_stats(self.radio, b.n_links, H_t, stats, ws)
            loss = self._buf("lossn", (3,), torch.float64)
            lib.cfr_loss(self.radio, b.n_links, H, H_t, stats, 1.0, 0.0, loss, None, ws)
            zc = stats[0].item()
            num += loss[1].item() * zc
            den += zc
        return num / den


    def paper_metrics(self, links, chunk=512):
        """Held-out paper loss (current alpha, no update) and the Sec. IV-C
        metrics: mean ALE (dB) and mean RAE over `links`; requires
        loss="paper"."""
        M, N = self.radio.n_elem, self.radio.n_sc
        tot = {"loss": 0.0, "ale": 0.0, "rae": 0.0}
        n = 0
        for i in range(0, len(links), chunk):
            ls = links[i:i + chunk]
            b, _ = lib.subset_links(self.dp, ls)
            H = self._buf("Hn", (b.n_links, M, N), torch.complex64)
            self.forward(b, H)
            tgt = self.tgt_all[ls].reshape(-1, 2)
            pred = self._buf("pred", (b.n_links * M, 2), torch.float64)
            loss = self._buf("lossn", (3,), torch.float64)
            lib.paper_loss(self.radio, b.n_links, H, tgt, self.alpha, loss, None,
                           self._ws(lib.RTC_OP_PAPER_LOSS, b.n_links, b.n_paths),
                           pred_stats=pred)
            m = self._buf("metrics", (b.n_links, 2), torch.float64)
            lib.eval_ale_rae(b.n_links, M, tgt, pred, m,
                             scale=self.alpha[:1] if self.update_alpha else None)
            k = b.n_links
            tot["loss"] += loss[0].item() * k
            tot["ale"] += m[:, 0].sum().item()
            tot["rae"] += m[:, 1].sum().item()
            n += k
        return {k: v / n for k, v in tot.items()}


def targets(dp, radio, raw=None, per_inter=None, g=None, device="cuda", chunk=2048):
    """Ground-truth CFRs of every link, computed by the library itself."""
    rc = lib.radio_from(radio)
    L, M, N = dp.n_links, rc.n_elem, rc.n_sc
    H = torch.empty((L, M, N), dtype=torch.complex64, device=device)
    g_d = torch.tensor(g, device=device)
    if raw is not None:
        raw_d = torch.tensor(raw, device=device)
        mats = lib.materials_per_id(raw_d)
        a = torch.empty(dp.n_paths, dtype=torch.complex64, device=device)
        psi = torch.empty(dp.n_paths, dtype=torch.float32, device=device)
        lib.trace_fields(rc, dp, mats, a, psi)
        lib.cfr(rc, dp, a, psi, g_d, H)
    else:
        per = torch.tensor(per_inter, device=device)
        a = torch.empty(dp.n_paths, dtype=torch.complex64, device=device)
        psi = torch.empty(dp.n_paths, dtype=torch.float32, device=device)
        lib.trace_fields(rc, dp, lib.materials_per_interaction(per), a, psi)
        lib.cfr(rc, dp, a, psi, g_d, H)
    return H


def _run(cal, train, held, max_steps, batch, eval_every, rng, stop_at=None, log=None):
    """Steps until max_steps (or held-out NMSE <= stop_at); returns
    (steps done, seconds spent in steps, NMSE history [(step, nmse)])."""
    import time
    hist = [(0, cal.nmse(held))]
    t_steps, s = 0.0, 0
    while s < max_steps:
        n = min(eval_every, max_steps - s)
        idx = [torch.tensor(rng.choice(len(train), batch, replace=False), device=cal.dev)
               for _ in range(n)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            cal.step(train[idx[i]])
        torch.cuda.synchronize()
        t_steps += time.perf_counter() - t0
        s += n
        nm = cal.nmse(held)
        hist.append((s, nm))
        if log:
            log(f"{cal.mode} step {s} held-out NMSE {nm:.4e}")
        if stop_at is not None and nm <= stop_at:
            break
    return s, t_steps, hist


def compare_learned_vs_plain(dp, radio, H_all, n_mat, aabb, train, held, plain_steps=3000,
                             learned_max_steps=3000, batch=512, eval_every=100, lr=0.01,
                             lr_mlp=1e-4, seed=0, log=None):
    """The plain per-material-id calibration for `plain_steps` gives
    NMSE_plain; the neural-material calibration then runs until its held-out
    NMSE reaches NMSE_plain (or `learned_max_steps`).  Steps/s of both at the
    same batch size, steps and step-time to equal NMSE."""
    from synth.params import mlp_init
    rng = np.random.default_rng(seed)
    tr = torch.as_tensor(train, device="cuda")
    he = torch.as_tensor(held, device="cuda")
    plain = Calibrator(dp, radio, H_all, "per_id", raw0=raw_prior(n_mat), lr=lr)
    ps, pt, ph = _run(plain, tr, he, plain_steps, batch, eval_every, rng, log=log)
    nmse_plain = ph[-1][1]
    neural = Calibrator(dp, radio, H_all, "neural",
                        mlp_params0=mlp_init(np.random.default_rng(seed + 5), mlp_out_bias()),
                        aabb=aabb, lr=lr, lr_mlp=lr_mlp)
    ls, lt, lh = _run(neural, tr, he, learned_max_steps, batch, eval_every, rng,
                      stop_at=nmse_plain, log=log)
    reached = lh[-1][1] <= nmse_plain
    # continue to the plain method's step count to report what the network gains
    ls2, lt2, lh2 = _run(neural, tr, he, max(0, plain_steps - ls), batch, eval_every, rng, log=log)
    return {
        "batch": batch,
        "plain_steps": ps, "plain_steps_per_s": round(ps / pt, 2),
        "plain_heldout_nmse": nmse_plain,
        "learned_steps_per_s": round((ls + ls2) / (lt + lt2), 2),
        "learned_reached_plain_nmse": bool(reached),
        "learned_steps_to_plain_nmse": ls if reached else None,
        "learned_seconds_to_plain_nmse": round(lt, 3) if reached else None,
        "learned_heldout_nmse_at_plain_steps": (lh2[-1][1] if ls2 else lh[-1][1]),
        "lr": lr, "lr_mlp": lr_mlp,
    }

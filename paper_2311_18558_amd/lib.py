"""ctypes binding of librtcal (argument marshalling only).

Every function here forwards device pointers of torch tensors to the C ABI
declared in include/rtcal.h and raises RuntimeError with the library's
message on a non-zero status.  There is no fallback: if the shared library
is not built, load() raises.

torch is imported before the library is opened so that librtcal binds to the
HIP runtime torch already loaded (one runtime per process).
"""
import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtcal.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_f32 = ctypes.c_float
c_f64 = ctypes.c_double
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t

RTC_OP_CFR_LOSS = 1
RTC_OP_CFR_ADJOINT = 2
RTC_OP_TRACE_FIELDS_ADJOINT = 3
RTC_OP_CFR_TARGET_STATS = 4
RTC_OP_PAPER_LOSS = 5
RTC_OP_TRACE_FIELDS_ADJOINT_PAT = 6
RTC_OP_CFR_LOSS_ADJOINT = 8


class Radio(ctypes.Structure):
    _fields_ = [("fc_hz", c_f64), ("df_hz", c_f64), ("n_sc", c_i32), ("n_elem", c_i32),
                ("ula_axis", c_f32 * 3), ("zeta_tx", c_f32), ("zeta_rx", c_f32)]


class Paths(ctypes.Structure):
    _fields_ = [("n_links", c_i32), ("n_paths", c_i32), ("max_depth", c_i32),
                ("link_off", c_vp), ("tx_pos", c_vp), ("rx_pos", c_vp), ("depth", c_vp),
                ("kind", c_vp), ("px", c_vp), ("py", c_vp), ("pz", c_vp), ("nx", c_vp),
                ("ny", c_vp), ("nz", c_vp), ("dA", c_vp), ("mat", c_vp), ("tau", c_vp),
                ("edge", c_vp), ("mat_n", c_vp)]


class Materials(ctypes.Structure):
    _fields_ = [("n_mat", c_i32), ("raw", c_vp), ("per_inter", c_vp), ("inter_idx", c_vp),
                ("n_inter", c_i64)]


class Patterns(ctypes.Structure):
    _fields_ = [("n_vmf", c_i32), ("tx_raw", c_vp), ("mat_raw", c_vp)]


class Mlp(ctypes.Structure):
    _fields_ = [("params", c_vp), ("aabb_center", c_f32 * 3), ("inv_extent", c_f32),
                ("n_freq", c_i32), ("width", c_i32), ("n_hidden", c_i32)]


# name -> (restype, argtypes)
_SIGS = {
    "rtc_abi_version": (ctypes.c_int, []),
    "rtc_last_error": (ctypes.c_char_p, []),
    "rtc_workspace_size": (c_size, [ctypes.c_int, ctypes.POINTER(Radio), c_i32, c_i32, c_i32]),
    "rtc_trace_fields": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths),
                                        ctypes.POINTER(Materials), c_vp, c_vp, c_vp]),
    "rtc_trace_fields_pat": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths),
                                            ctypes.POINTER(Materials), ctypes.POINTER(Patterns),
                                            c_vp, c_vp, c_vp]),
    "rtc_embed_readout": (ctypes.c_int, [c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rtc_embed_readout_backward": (ctypes.c_int, [c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp,
                                                  c_vp, c_vp]),
    "rtc_trace_fields_adjoint_pat": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths),
                                                    ctypes.POINTER(Materials),
                                                    ctypes.POINTER(Patterns), c_vp, c_vp, c_vp,
                                                    c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_cfr": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths), c_vp, c_vp, c_vp,
                               c_vp, c_vp]),
    "rtc_cfr_target_stats": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp,
                                            c_vp, c_size, c_vp]),
    "rtc_cfr_target_cir": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp, c_vp,
                                          c_size, c_vp]),
    "rtc_cfr_loss": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp, c_vp, c_f32,
                                    c_f32, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_cfr_loss_cir": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp, c_f32,
                                        c_f32, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_cfr_loss_noalloc": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp,
                                            c_vp, c_f32, c_f32, c_vp, c_vp, c_vp]),
    "rtc_cfr_loss_noalloc_max_rows": (c_i64, []),
    "rtc_cir_stats": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp]),
    "rtc_paper_loss": (ctypes.c_int, [ctypes.POINTER(Radio), c_i32, c_vp, c_vp, c_vp, c_i32, c_f64,
                                      c_f32, c_f32, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_eval_ale_rae": (ctypes.c_int, [c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rtc_cfr_adjoint": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths), c_vp, c_vp,
                                       c_vp, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_cfr_loss_adjoint": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths), c_vp,
                                            c_vp, c_vp, c_vp, c_vp, c_vp, c_f32, c_f32, c_vp,
                                            c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_cfr_loss_adjoint_cir": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths),
                                                c_vp, c_vp, c_vp, c_vp, c_vp, c_f32, c_f32, c_vp,
                                                c_vp, c_vp, c_vp, c_size, c_vp]),
    "rtc_trace_fields_adjoint": (ctypes.c_int, [ctypes.POINTER(Radio), ctypes.POINTER(Paths),
                                                ctypes.POINTER(Materials), c_vp, c_vp, c_vp,
                                                c_vp, c_size, c_vp]),
    "rtc_adam_step": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, c_f32, c_f32, c_f32,
                                     c_f32, c_vp]),
    "rtc_adam_step_dev": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_i32, c_f32,
                                         c_f32, c_f32, c_f32, c_vp]),
    "rtc_axpy": (ctypes.c_int, [c_vp, c_vp, c_f32, c_i64, c_vp]),
    "rtc_validate_paths": (ctypes.c_int, [ctypes.POINTER(Paths), c_i32, c_vp, c_vp, c_size,
                                          c_vp]),
    "rtc_mlp_n_params": (c_i32, []),
    "rtc_mlp_saved_size": (c_size, [c_i64]),
    "rtc_mlp_workspace_size": (c_size, [c_i64]),
    "rtc_mlp_forward": (ctypes.c_int, [ctypes.POINTER(Mlp), c_i64, c_vp, c_vp, c_vp, c_vp, c_vp,
                                       c_size, c_vp, c_size, c_vp]),
    "rtc_mlp_backward": (ctypes.c_int, [ctypes.POINTER(Mlp), c_i64, c_vp, c_vp, c_vp, c_vp,
                                        c_size, c_vp]),
}

_lib = None


def load():
    """Open librtcal.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2311_18558_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_names():
    return list(_SIGS)


def _check(status, fn):
    if status != 0:
        msg = load().rtc_last_error().decode(errors="replace")
        raise RuntimeError(f"{fn} failed with status {status}: {msg}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_radio(fc, df, n_sc, n_elem, ula_axis=(1.0, 0.0, 0.0), zeta_tx=0.0, zeta_rx=0.0):
    r = Radio()
    r.fc_hz = float(fc)
    r.df_hz = float(df)
    r.n_sc = int(n_sc)
    r.n_elem = int(n_elem)
    for i in range(3):
        r.ula_axis[i] = float(ula_axis[i])
    r.zeta_tx = float(zeta_tx)
    r.zeta_rx = float(zeta_rx)
    return r


def radio_from(radio):
    """Radio struct from an object with fc, df, n_sc, n_elem, ula_axis,
    zeta_tx, zeta_rx attributes."""
    return make_radio(radio.fc, radio.df, radio.n_sc, radio.n_elem, radio.ula_axis,
                      radio.zeta_tx, radio.zeta_rx)


class DevicePaths:
    """A path store uploaded to device memory, with its C descriptor."""

    def __init__(self, store, device="cuda"):
        d = torch.device(device)
        t = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to(dtype=dt, device=d)
        self.n_links = int(store.n_links)
        self.n_paths = int(store.n_paths)
        self.max_depth = int(store.max_depth)
        self.link_off = t(store.link_off, torch.int64)
        self.tx_pos = t(store.tx_pos.reshape(-1), torch.float32)
        self.rx_pos = t(store.rx_pos.reshape(-1), torch.float32)
        self.depth = t(store.depth, torch.uint8)
        self.pts = t(store.pts, torch.float32)
        self.nrm = t(store.nrm, torch.float32)
        self.mat = t(store.mat.astype(np.int16), torch.int16)
        self.tau = t(store.tau, torch.float64)
        has_diffuse = bool(np.any(store.kind != 0))
        self.kind = t(store.kind, torch.uint8) if has_diffuse else None
        self.dA = t(store.dA, torch.float32) if has_diffuse else None
        has_edge = getattr(store, "edge", None) is not None
        self.edge = t(store.edge, torch.float32) if has_edge else None
        self.mat_n = t(store.mat_n.astype(np.int16), torch.int16) if has_edge else None
        s = Paths()
        s.n_links, s.n_paths, s.max_depth = self.n_links, self.n_paths, self.max_depth
        s.link_off = self.link_off.data_ptr()
        s.tx_pos = self.tx_pos.data_ptr()
        s.rx_pos = self.rx_pos.data_ptr()
        s.depth = self.depth.data_ptr()
        s.kind = self.kind.data_ptr() if self.kind is not None else None
        s.dA = self.dA.data_ptr() if self.dA is not None else None
        DP = self.max_depth * self.n_paths
        base_p = self.pts.data_ptr()
        base_n = self.nrm.data_ptr()
        s.px, s.py, s.pz = base_p, base_p + 4 * DP, base_p + 8 * DP
        s.nx, s.ny, s.nz = base_n, base_n + 4 * DP, base_n + 8 * DP
        s.mat = self.mat.data_ptr()
        s.tau = self.tau.data_ptr()
        s.edge = self.edge.data_ptr() if has_edge else None
        s.mat_n = self.mat_n.data_ptr() if has_edge else None
        self.c = s
        if os.environ.get("RTCAL_DEBUG", "0") not in ("", "0"):
            check_paths(self)


RTC_OP_VALIDATE_PATHS = 7
VALIDATE_NAMES = ("link_off", "depth", "material id", "kind", "tau", "unit vector",
                  "non-finite coordinate", "dA or wedge n")


def validate_paths(paths, n_mat=0, stream=None):
    """Violation counts per category (host dict) of a device path store
    (rtc_validate_paths; synchronises the stream)."""
    dev = paths.link_off.device
    counts = torch.zeros(8, dtype=torch.int64, device=dev)
    n = int(load().rtc_workspace_size(RTC_OP_VALIDATE_PATHS, None, 0, 0, 0))
    ws = torch.empty(max(n, 8), dtype=torch.uint8, device=dev)
    _check(load().rtc_validate_paths(ctypes.byref(paths.c), int(n_mat), _ptr(counts), _ptr(ws),
                                     ws.numel(), _stream(stream)), "rtc_validate_paths")
    return dict(zip(VALIDATE_NAMES, counts.cpu().tolist()))


def check_paths(paths, n_mat=0):
    """Raise if the device-side check finds violations (RTCAL_DEBUG=1 runs it
    on every DevicePaths upload)."""
    bad = {k: v for k, v in validate_paths(paths, n_mat).items() if v}
    if bad:
        raise RuntimeError(f"invalid path store: {bad}")


def materials_per_id(raw):
    """Descriptor for per-id mode; keeps a reference to `raw` so the device
    memory outlives the descriptor."""
    m = Materials()
    m.n_mat = int(raw.shape[0])
    m.raw = raw.data_ptr()
    m.per_inter = None
    m._keep = raw
    return m


def materials_per_interaction(per_inter, compact=None):
    """per_inter: float32 [3, R] rows eps_r, sigma, S.  compact: the
    (inter_idx, n_inter) of compact_interactions for rows of used slots
    only, or None for rows indexed like the path slots."""
    m = Materials()
    m.n_mat = 1
    m.raw = None
    m.per_inter = per_inter.data_ptr()
    if compact is not None:
        m.inter_idx = compact[0].data_ptr()
        m.n_inter = int(compact[1])
    m._keep = (per_inter, compact)
    return m


def compact_interactions(dp):
    """Rows for the used interaction slots (k < depth[p]) of a DevicePaths,
    in slot order: returns (inter_idx int32 [D*P] with -1 for unused slots,
    n_inter, points float32 [3, n_inter]).  Input staging (index operations
    on the fixed geometry, once per path set)."""
    D, P = dp.max_depth, dp.n_paths
    used = (torch.arange(D, device=dp.depth.device)[:, None]
            < dp.depth.to(torch.int64)[None, :]).reshape(-1)
    n_inter = int(used.sum().item())
    idx = torch.full((D * P,), -1, dtype=torch.int32, device=used.device)
    idx[used] = torch.arange(n_inter, dtype=torch.int32, device=used.device)
    pts = dp.pts[:, used].contiguous()
    return idx, n_inter, pts


def workspace_size(op, radio, n_links, n_paths, n_mat=1):
    rp = None if radio is None else ctypes.byref(radio)
    return int(load().rtc_workspace_size(op, rp, n_links, n_paths, n_mat))


def workspace(op, radio, n_links, n_paths, n_mat=1, device="cuda"):
    n = max(workspace_size(op, radio, n_links, n_paths, n_mat), 8)
    return torch.empty(n, dtype=torch.uint8, device=device)


# ------------------------------------------------------------ entry points
def trace_fields(radio, paths, mats, a, psi, stream=None):
    _check(load().rtc_trace_fields(ctypes.byref(radio), ctypes.byref(paths.c), ctypes.byref(mats),
                                   _ptr(a), _ptr(psi), _stream(stream)), "rtc_trace_fields")


def patterns(n_vmf=0, tx_raw=None, mat_raw=None):
    """Descriptor of the trainable patterns (keeps references to the
    device tensors)."""
    p = Patterns()
    p.n_vmf = int(n_vmf)
    p.tx_raw = None if tx_raw is None else tx_raw.data_ptr()
    p.mat_raw = None if mat_raw is None else mat_raw.data_ptr()
    p._keep = (tx_raw, mat_raw)
    return p


def trace_fields_pat(radio, paths, mats, pats, a, psi, stream=None):
    _check(load().rtc_trace_fields_pat(ctypes.byref(radio), ctypes.byref(paths.c),
                                       ctypes.byref(mats),
                                       None if pats is None else ctypes.byref(pats), _ptr(a),
                                       _ptr(psi), _stream(stream)), "rtc_trace_fields_pat")


def trace_fields_adjoint_pat(radio, paths, mats, pats, dLda, dLd_raw, dLd_inter, dLd_tx, dLd_pat,
                             ws, stream=None):
    _check(load().rtc_trace_fields_adjoint_pat(
        ctypes.byref(radio), ctypes.byref(paths.c), ctypes.byref(mats),
        None if pats is None else ctypes.byref(pats), _ptr(dLda), _ptr(dLd_raw), _ptr(dLd_inter),
        _ptr(dLd_tx), _ptr(dLd_pat), _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream)),
        "rtc_trace_fields_adjoint_pat")


def embed_readout(v, W, raw, pat_raw=None, stream=None):
    """v float32 [L], W float32 [n_mat, 4, L] -> raw [n_mat, 3] (and column 0
    of pat_raw [n_mat, 6], the K_x logit)."""
    n_mat, _, L = W.shape
    _check(load().rtc_embed_readout(n_mat, L, _ptr(v), _ptr(W), _ptr(raw), _ptr(pat_raw),
                                    _stream(stream)), "rtc_embed_readout")


def embed_readout_backward(v, W, dLd_raw, dLd_pat, dLd_v, dLd_W, stream=None):
    n_mat, _, L = W.shape
    _check(load().rtc_embed_readout_backward(n_mat, L, _ptr(v), _ptr(W), _ptr(dLd_raw),
                                             _ptr(dLd_pat), _ptr(dLd_v), _ptr(dLd_W),
                                             _stream(stream)), "rtc_embed_readout_backward")


def cfr(radio, paths, a, psi, g, H, stream=None):
    _check(load().rtc_cfr(ctypes.byref(radio), ctypes.byref(paths.c), _ptr(a), _ptr(psi), _ptr(g),
                          _ptr(H), _stream(stream)), "rtc_cfr")


def cfr_target_stats(radio, n_links, H_tgt, stats, ws, stream=None, p_tgt=None):
    """p_tgt: optional float32 [n_links*n_elem*n_sc] receiving the target PDP."""
    _check(load().rtc_cfr_target_stats(ctypes.byref(radio), n_links, _ptr(H_tgt), _ptr(stats),
                                       _ptr(p_tgt), _ptr(ws), ws.numel(), _stream(stream)),
           "rtc_cfr_target_stats")


def cfr_target_cir(radio, n_links, H_tgt, stats, X_tgt, ws, stream=None):
    """X_tgt: complex64 [n_links, n_elem, n_sc] receiving the targets'
    transforms X*_k = sum_n H*[n] exp(+j 2 pi n k / N) (for cfr_loss_adjoint_cir)."""
    _check(load().rtc_cfr_target_cir(ctypes.byref(radio), n_links, _ptr(H_tgt), _ptr(stats),
                                     _ptr(X_tgt), _ptr(ws), ws.numel(), _stream(stream)),
           "rtc_cfr_target_cir")


def cfr_loss(radio, n_links, H, H_tgt, tgt_stats, w_coh, w_pdp, loss, dLdH, ws, stream=None,
             p_tgt=None):
    """p_tgt: optional target PDP from cfr_target_stats for the same H_tgt."""
    _check(load().rtc_cfr_loss(ctypes.byref(radio), n_links, _ptr(H), _ptr(H_tgt), _ptr(tgt_stats),
                               _ptr(p_tgt), float(w_coh), float(w_pdp), _ptr(loss), _ptr(dLdH),
                               _ptr(ws), ws.numel(), _stream(stream)), "rtc_cfr_loss")


def cfr_loss_cir(radio, n_links, H, X_tgt, tgt_stats, w_coh, w_pdp, loss, dLdH, ws,
                 stream=None):
    """cfr_loss with the targets as their transforms X* and stats from
    cfr_target_cir (the same loss and gradient, two transforms per row)."""
    _check(load().rtc_cfr_loss_cir(ctypes.byref(radio), n_links, _ptr(H), _ptr(X_tgt),
                                   _ptr(tgt_stats), float(w_coh), float(w_pdp), _ptr(loss),
                                   _ptr(dLdH), _ptr(ws), ws.numel(), _stream(stream)),
           "rtc_cfr_loss_cir")


def cfr_loss_noalloc(radio, n_links, H, H_tgt, tgt_stats, w_coh, w_pdp, loss, dLdH,
                     stream=None, p_tgt=None):
    """rtc_cfr_loss without a workspace (the library's fixed per-GPU
    scratch; calls on one GPU must not overlap)."""
    _check(load().rtc_cfr_loss_noalloc(ctypes.byref(radio), n_links, _ptr(H), _ptr(H_tgt),
                                       _ptr(tgt_stats), _ptr(p_tgt), float(w_coh), float(w_pdp),
                                       _ptr(loss), _ptr(dLdH), _stream(stream)),
           "rtc_cfr_loss_noalloc")


def cfr_loss_noalloc_max_rows():
    return int(load().rtc_cfr_loss_noalloc_max_rows())


def cir_stats(radio, n_links, H, stats, stream=None):
    """stats: float64 [n_links*n_elem, 2] receiving {P, tau_RMS} per CIR row."""
    _check(load().rtc_cir_stats(ctypes.byref(radio), n_links, _ptr(H), _ptr(stats),
                                _stream(stream)), "rtc_cir_stats")


def paper_loss(radio, n_links, H, tgt_stats, alpha, loss, dLdH, ws, update_alpha=False,
               delta=0.99, w_tau=1.0, w_gain=1.0, pred_stats=None, stream=None):
    """alpha: float64 [2] device state {alpha, updates}; loss: float64 [3]."""
    _check(load().rtc_paper_loss(ctypes.byref(radio), n_links, _ptr(H), _ptr(tgt_stats),
                                 _ptr(alpha), int(bool(update_alpha)), float(delta), float(w_tau),
                                 float(w_gain), _ptr(loss), _ptr(pred_stats), _ptr(dLdH),
                                 _ptr(ws), ws.numel(), _stream(stream)), "rtc_paper_loss")


def eval_ale_rae(n_links, n_elem, meas, pred, out, scale=None, stream=None):
    """out: float64 [n_links, 2] receiving {ALE (dB), RAE} per link."""
    _check(load().rtc_eval_ale_rae(int(n_links), int(n_elem), _ptr(meas), _ptr(pred), _ptr(scale),
                                   _ptr(out), _stream(stream)), "rtc_eval_ale_rae")


def cfr_adjoint(radio, paths, a, psi, g, dLdH, dLda, dLdg, ws, stream=None):
    _check(load().rtc_cfr_adjoint(ctypes.byref(radio), ctypes.byref(paths.c), _ptr(a), _ptr(psi),
                                  _ptr(g), _ptr(dLdH), _ptr(dLda), _ptr(dLdg), _ptr(ws),
                                  0 if ws is None else ws.numel(), _stream(stream)),
           "rtc_cfr_adjoint")


def fused_supported(radio):
    """Shapes rtc_cfr_loss_adjoint takes (others: the three separate calls)."""
    return 1 <= radio.n_elem <= 32 and radio.n_sc in (256, 512, 1024)


def cfr_loss_adjoint(radio, paths, a, psi, g, H_tgt, tgt_stats, p_tgt, w_coh, w_pdp, loss,
                     dLda, dLdg, ws, stream=None):
    """CFR, workload loss and CFR adjoint in one pass per link (H and dL/dH
    stay on chip); tgt_stats and p_tgt from cfr_target_stats of H_tgt."""
    _check(load().rtc_cfr_loss_adjoint(ctypes.byref(radio), ctypes.byref(paths.c), _ptr(a),
                                       _ptr(psi), _ptr(g), _ptr(H_tgt), _ptr(tgt_stats),
                                       _ptr(p_tgt), float(w_coh), float(w_pdp), _ptr(loss),
                                       _ptr(dLda), _ptr(dLdg), _ptr(ws),
                                       0 if ws is None else ws.numel(), _stream(stream)),
           "rtc_cfr_loss_adjoint")


def cfr_loss_adjoint_cir(radio, paths, a, psi, g, X_tgt, tgt_stats, w_coh, w_pdp, loss, dLda,
                         dLdg, ws, stream=None):
    """cfr_loss_adjoint with the targets as their transforms X* and stats
    from cfr_target_cir (the same loss and gradient)."""
    _check(load().rtc_cfr_loss_adjoint_cir(ctypes.byref(radio), ctypes.byref(paths.c), _ptr(a),
                                           _ptr(psi), _ptr(g), _ptr(X_tgt), _ptr(tgt_stats),
                                           float(w_coh), float(w_pdp), _ptr(loss), _ptr(dLda),
                                           _ptr(dLdg), _ptr(ws), 0 if ws is None else ws.numel(),
                                           _stream(stream)), "rtc_cfr_loss_adjoint_cir")


def trace_fields_adjoint(radio, paths, mats, dLda, dLd_raw, dLd_inter, ws, stream=None):
    _check(load().rtc_trace_fields_adjoint(ctypes.byref(radio), ctypes.byref(paths.c),
                                           ctypes.byref(mats), _ptr(dLda), _ptr(dLd_raw),
                                           _ptr(dLd_inter), _ptr(ws),
                                           0 if ws is None else ws.numel(), _stream(stream)),
           "rtc_trace_fields_adjoint")


def adam_step(param, grad, m, v, step, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().rtc_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(),
                                int(step), float(lr), float(beta1), float(beta2), float(eps),
                                _stream(stream)), "rtc_adam_step")


def adam_step_dev(param, grad, m, v, step, advance, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8,
                  stream=None):
    """step: int32 device counter of updates made (see rtc_adam_step_dev)."""
    _check(load().rtc_adam_step_dev(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(),
                                    _ptr(step), int(bool(advance)), float(lr), float(beta1),
                                    float(beta2), float(eps), _stream(stream)),
           "rtc_adam_step_dev")


def axpy(y, x, alpha=1.0, stream=None):
    """y += alpha x (float32 device tensors of equal size)."""
    assert y.numel() == x.numel()
    _check(load().rtc_axpy(_ptr(y), _ptr(x), float(alpha), y.numel(), _stream(stream)), "rtc_axpy")


def replicate_paths(dp, device=None):
    """A device copy of a DevicePaths (its own memory): input staging for
    stores made of repeated link sets."""
    b = DevicePaths.__new__(DevicePaths)
    for k in ("n_links", "n_paths", "max_depth"):
        setattr(b, k, getattr(dp, k))
    for k in ("link_off", "tx_pos", "rx_pos", "depth", "pts", "nrm", "mat", "tau", "kind", "dA",
              "edge", "mat_n"):
        v = getattr(dp, k, None)
        setattr(b, k, None if v is None else v.clone())
    s = Paths()
    s.n_links, s.n_paths, s.max_depth = b.n_links, b.n_paths, b.max_depth
    s.link_off, s.tx_pos, s.rx_pos = (b.link_off.data_ptr(), b.tx_pos.data_ptr(),
                                      b.rx_pos.data_ptr())
    s.depth = b.depth.data_ptr()
    s.kind = None if b.kind is None else b.kind.data_ptr()
    s.dA = None if b.dA is None else b.dA.data_ptr()
    DP = b.max_depth * b.n_paths
    bp, bn = b.pts.data_ptr(), b.nrm.data_ptr()
    s.px, s.py, s.pz = bp, bp + 4 * DP, bp + 8 * DP
    s.nx, s.ny, s.nz = bn, bn + 4 * DP, bn + 8 * DP
    s.mat = b.mat.data_ptr()
    s.tau = b.tau.data_ptr()
    s.edge = None if b.edge is None else b.edge.data_ptr()
    s.mat_n = None if b.mat_n is None else b.mat_n.data_ptr()
    b.c = s
    return b


# ------------------------------------------------------------ neural materials
def make_mlp(params, aabb_min, aabb_max):
    """Descriptor of the neural-material MLP: params is the FP32 master
    vector (device); the normalisation uses the scene AABB's centre and
    longest edge."""
    lo = np.asarray(aabb_min, np.float64)
    hi = np.asarray(aabb_max, np.float64)
    m = Mlp()
    m.params = params.data_ptr()
    c = 0.5 * (lo + hi)
    for i in range(3):
        m.aabb_center[i] = float(c[i])
    m.inv_extent = float(1.0 / np.max(hi - lo))
    m.n_freq, m.width, m.n_hidden = 8, 128, 4
    m._keep = params
    return m


def mlp_n_params():
    return int(load().rtc_mlp_n_params())


def mlp_saved(n_points, device="cuda"):
    return torch.empty(max(int(load().rtc_mlp_saved_size(n_points)), 8), dtype=torch.uint8,
                       device=device)


def mlp_workspace(n_points, device="cuda"):
    return torch.empty(max(int(load().rtc_mlp_workspace_size(n_points)), 8), dtype=torch.uint8,
                       device=device)


def mlp_forward(net, n_points, px, py, pz, out, saved, ws, stream=None):
    _check(load().rtc_mlp_forward(ctypes.byref(net), int(n_points), _ptr(px), _ptr(py), _ptr(pz),
                                  _ptr(out), _ptr(saved), 0 if saved is None else saved.numel(),
                                  _ptr(ws), ws.numel(), _stream(stream)), "rtc_mlp_forward")


def mlp_backward(net, n_points, dLdout, saved, dLdparams, ws, stream=None):
    _check(load().rtc_mlp_backward(ctypes.byref(net), int(n_points), _ptr(dLdout), _ptr(saved),
                                   _ptr(dLdparams), _ptr(ws), ws.numel(), _stream(stream)),
           "rtc_mlp_backward")


def subset_links(dp, links):
    """Device-side batch: a DevicePaths holding only `links` (int64 device
    tensor), gathered with index operations (input staging; no method
    arithmetic).  Returns (DevicePaths, slot_index) where slot_index [D*Pb]
    maps the batch's interaction slots to the full store's slots."""
    dev = dp.link_off.device
    links = links.to(device=dev, dtype=torch.int64)
    start = dp.link_off[links]
    cnt = dp.link_off[links + 1] - start
    off = torch.zeros(len(links) + 1, dtype=torch.int64, device=dev)
    off[1:] = torch.cumsum(cnt, 0)
    Pb = int(off[-1].item())
    rep = torch.repeat_interleave(torch.arange(len(links), device=dev), cnt, output_size=Pb)
    idx = start[rep] + (torch.arange(Pb, device=dev) - off[:-1][rep])
    D, P = dp.max_depth, dp.n_paths
    slot = (torch.arange(D, device=dev)[:, None] * P + idx[None, :]).reshape(-1)
    b = DevicePaths.__new__(DevicePaths)
    b.n_links, b.n_paths, b.max_depth = len(links), Pb, D
    b.link_off = off
    b.tx_pos = dp.tx_pos.view(-1, 3)[links].reshape(-1).contiguous()
    b.rx_pos = dp.rx_pos.view(-1, 3)[links].reshape(-1).contiguous()
    b.depth = dp.depth[idx].contiguous()
    b.pts = dp.pts[:, slot].contiguous()
    b.nrm = dp.nrm[:, slot].contiguous()
    b.mat = dp.mat[slot].contiguous()
    b.tau = dp.tau[idx].contiguous()
    b.kind = dp.kind[slot].contiguous() if dp.kind is not None else None
    b.dA = dp.dA[slot].contiguous() if dp.dA is not None else None
    b.edge = dp.edge[:, idx].contiguous() if dp.edge is not None else None
    b.mat_n = dp.mat_n[idx].contiguous() if dp.mat_n is not None else None
    s = Paths()
    s.n_links, s.n_paths, s.max_depth = b.n_links, Pb, D
    s.link_off = b.link_off.data_ptr()
    s.tx_pos = b.tx_pos.data_ptr()
    s.rx_pos = b.rx_pos.data_ptr()
    s.depth = b.depth.data_ptr()
    s.kind = b.kind.data_ptr() if b.kind is not None else None
    s.dA = b.dA.data_ptr() if b.dA is not None else None
    DPb = D * Pb
    bp, bn = b.pts.data_ptr(), b.nrm.data_ptr()
    s.px, s.py, s.pz = bp, bp + 4 * DPb, bp + 8 * DPb
    s.nx, s.ny, s.nz = bn, bn + 4 * DPb, bn + 8 * DPb
    s.mat = b.mat.data_ptr()
    s.tau = b.tau.data_ptr()
    s.edge = b.edge.data_ptr() if b.edge is not None else None
    s.mat_n = b.mat_n.data_ptr() if b.mat_n is not None else None
    b.c = s
    return b, slot

"""Benchmark of the calibration hot path on one MI355X.

One step = trace_fields -> cfr_loss_adjoint (CFR, workload loss and CFR
adjoint in one pass per link, H and dL/dH on chip) -> trace_fields_adjoint
-> Adam, over the whole `scale` workload (indoor floor, 16,384 Rx links x 32
Tx elements x 1,024 subcarriers, specular paths up to fifth order, ~186
paths per link), inputs resident in HBM.  The same step with cfr, cfr_loss
and cfr_adjoint as separate calls is reported beside it.

Prints ONE JSON line (rank 0):
  value          CFR taps/s (taps = links x elements x subcarriers per step)
  roofline       dominant kernel's algorithmic FLOP/s (8 M N P per launch) from
                 HIP events on the launch stream, against the published dense
                 FP16 matrix-core peak the contraction runs on (2.5 PFLOP/s);
                 beside it the ceiling of the two-way FP16 split (three partial
                 products per real product) and the issued MFMA rate
  cpu_baseline   the FP64 oracle on a bounded sample of links, on all of
                 torch's host threads and on one
  paper_loss_step  the same step with the paper's own loss (SMAPE of RMS
                 delay spread and gain, moving-average measurement scale)
  large_scene    the streamed step on the urban block (4 Tx x 2,048 outdoor
                 Rx, real specular + diffuse paths, ~2,000 per link, 4,096
                 subcarriers, neural materials, the paper's loss); --config5
                 runs it at full size, 4 Tx x 65,536 Rx
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --copy-probe ...      also runs a 2 GiB device copy
                                             first (HBM counter calibration)
       python bench.py --traffic FETCH.csv WRITE.csv
                                             rocprofv3 --pmc FETCH_SIZE /
                                             WRITE_SIZE results of a
                                             --copy-probe run -> traffic.json
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

PEAK_FP32_MATRIX_TFLOPS = 157.3  # MI355X dense FP32 MFMA
PEAK_F16_MATRIX_TFLOPS = 2500.0  # MI355X dense FP16 / BF16 MFMA
SPLIT_PRODUCTS = 3  # FP16 partial products per real product (two-way split)
PEAK_SPLIT_TFLOPS = PEAK_F16_MATRIX_TFLOPS / SPLIT_PRODUCTS
PEAK_HBM_GBS = 8000.0
# the arithmetic of the CFR contraction: FP32 operands split into two FP16
# parts each, three FP16 products per real product, FP32 accumulation
# (~3 * 2^-22 relative error per product); FP64 phase reduction
DTYPE = "fp16x2-split/fp32-acc"
COPY_PROBE_BYTES = 2 << 30
# sources whose change invalidates the committed HBM counter figures
HOT_SOURCES = ["cfr.hip", "fused.hip", "cfr_common.h", "split_f16.h", "dev_common.h",
               "api_common.h", "loss.hip", "paper_loss.hip", "fft_wave.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload():
    from synth import workloads
    t0 = time.time()
    w = workloads.scale()
    log(f"workload scale: {w.store.n_links} links, {w.store.n_paths} paths "
        f"({w.store.n_paths / w.store.n_links:.1f}/link), {w.meta['tris']} triangles, "
        f"generated in {time.time() - t0:.1f}s")
    return w


def kernel_work(name, L, M, N, P, D):
    """Algorithmic work per launch: (flops, bytes)."""
    taps = L * M * N
    if name in ("cfr", "cfr_adjoint"):
        return 8.0 * M * N * P, 8.0 * taps + 20.0 * P
    if name == "cfr_loss":
        # H and H* in (the target PDP formed from H*), dL/dH out
        return 0.0, 24.0 * taps
    if name == "cfr_loss_adjoint":
        # forward and adjoint contractions; the targets' transforms X* in
        # (8 B per tap), the path data in and dL/da out
        return 16.0 * M * N * P, 8.0 * taps + 28.0 * P
    if name == "cfr_loss_adjoint_cfr":
        # the same with the targets as H* and the stored target PDP (12 B per tap)
        return 16.0 * M * N * P, 12.0 * taps + 28.0 * P
    if name in ("trace_fields", "trace_fields_adjoint"):
        # per interaction: point, normal (24 B) + material id (2 B); per path
        # depth (1 B) + tau (8 B); out: a (8 B) + psi (4 B) or in: dL/da
        return 0.0, P * (26.0 * D + 9.0 + 12.0)
    return 0.0, 0.0


MFMA_FLOPS = 2 * 32 * 32 * 16  # one v_mfma_f32_32x32x16_f16


def mfma_issued(name, link_off, M, N):
    """FP16 MFMA instructions one launch of the CFR kernels issues: 12 per
    (16 paths, 32 subcarrier pairs, 32 elements) in the forward product and
    per (32 paths, 16 pairs, 32 elements) in the adjoint; the forward wave
    covers 4 pair tiles, padding included."""
    cnt = np.diff(np.asarray(link_off, np.int64))
    mblk = -(-M // 32)
    Q = (N + 1) // 2
    if name == "cfr":
        qchunks = -(-Q // 128)
        return int((-(-cnt // 16)).sum()) * mblk * qchunks * 4 * 12
    if name == "cfr_adjoint":
        return int((-(-cnt // 32)).sum()) * mblk * (-(-Q // 16)) * 12
    if name in ("cfr_loss_adjoint", "cfr_loss_adjoint_cfr"):
        # the fused pass runs both products in the same tilings
        return mfma_issued("cfr", link_off, M, N) + mfma_issued("cfr_adjoint", link_off, M, N)
    return 0


def diffuse_bench(steps=3, warmup=1):
    """The same calibration step on the diffuse workload (specular up to
    fifth order + single-bounce Lambertian paths, ~2,000 paths per link,
    2,048 Rx x 32 elements x 4,096 subcarriers)."""
    from synth import workloads
    from paper_2311_18558_amd.pipeline import Pipeline
    t0 = time.time()
    w = workloads.diffuse()
    st, radio = w.store, w.radio
    n_dif = int(np.count_nonzero(st.kind))
    log(f"workload diffuse: {st.n_links} links, {st.n_paths} paths ({st.n_paths / st.n_links:.1f}"
        f"/link, {n_dif} diffuse), generated in {time.time() - t0:.1f}s")
    L, M, N, P = st.n_links, radio.n_elem, radio.n_sc, st.n_paths
    rng = np.random.default_rng(8)
    raw0 = (w.raw + rng.normal(scale=0.3, size=w.raw.shape)).astype(np.float32)
    pipe = Pipeline(st, radio, w.raw, w.g)
    H_tgt = torch.empty_like(pipe.H)
    pipe.trace()
    pipe.cfr(out=H_tgt)
    pipe.set_target(H_tgt)
    pipe.raw.copy_(torch.tensor(raw0, device=pipe.dev))
    for _ in range(warmup):
        pipe.step()
    torch.cuda.synchronize()
    events = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pipe.step(events=events)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per = {k: round(float(np.mean([a.elapsed_time(b) for a, b in v])), 4)
           for k, v in events.items()}
    log("diffuse per-stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in per.items()))
    fl = 8.0 * M * N * P
    out = {"workload": "scale floor, 2,048 Rx, specular up to 5th order + single-bounce "
                       "Lambertian diffuse, 4,096 subcarriers over 100 MHz, 32-element ULA",
           "links": L, "paths": P, "paths_per_link": round(P / L, 1), "diffuse_paths": n_dif,
           "subcarriers": N, "elements": M, "steps": steps, "ms_per_step": round(ms, 3),
           "taps_per_s": round(L * M * N / (ms * 1e-3), 1), "kernels_ms": per,
           "cfr_tflops": round(fl / (per["cfr"] * 1e-3) / 1e12, 2),
           "cfr_adjoint_tflops": round(fl / (per["cfr_adjoint"] * 1e-3) / 1e12, 2),
           "trace_fields_paths_per_s": round(P / (per["trace_fields"] * 1e-3), 1),
           "trace_fields_adjoint_paths_per_s": round(P / (per["trace_fields_adjoint"] * 1e-3), 1)}
    del pipe, H_tgt
    torch.cuda.empty_cache()
    return out


def separate_calls_step(st, radio, w, raw0, H_tgt, steps, warmup=1, label="separate-calls",
                        **pipe_kw):
    """The same step with cfr, cfr_loss and cfr_adjoint as three library
    calls (H and dL/dH through HBM) instead of the fused pass (or, with
    pipe_kw, another variant of the step)."""
    from paper_2311_18558_amd.pipeline import Pipeline
    pipe = Pipeline(st, radio, w.raw, w.g, **(pipe_kw or {"fused": False}))
    pipe.set_target(H_tgt)
    pipe.raw.copy_(torch.tensor(raw0, device=pipe.dev))
    for _ in range(warmup):
        pipe.step()
    torch.cuda.synchronize()
    events = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pipe.step(events=events)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per = {k: round(float(np.mean([a.elapsed_time(b) for a, b in v])), 4)
           for k, v in events.items()}
    res = {"steps": steps, "ms_per_step": round(ms, 4), "kernels_ms": per}
    log(f"{label} step: {res}")
    del pipe
    torch.cuda.empty_cache()
    return res


def paper_loss_step(st, radio, w, raw0, H_tgt, steps, warmup=1):
    """The same step with the paper's own loss (SMAPE of RMS delay spread and
    gain per CIR row) and the moving-average measurement scale in place of
    the workload loss: per-stage times over `steps` steps."""
    from paper_2311_18558_amd.pipeline import Pipeline
    pipe = Pipeline(st, radio, w.raw, w.g, loss="paper", update_alpha=True, delta=0.99)
    pipe.set_target(H_tgt)
    pipe.raw.copy_(torch.tensor(raw0, device=pipe.dev))
    for _ in range(warmup):
        pipe.step()
    torch.cuda.synchronize()
    events = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pipe.step(events=events)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per = {k: round(float(np.mean([a.elapsed_time(b) for a, b in v])), 4)
           for k, v in events.items()}
    L, M, N = st.n_links, radio.n_elem, radio.n_sc
    # the gain pass for the scale estimate reads H once, the loss pass reads
    # H and writes dL/dH: 24 bytes per tap
    gbs = 24.0 * L * M * N / (per["paper_loss"] * 1e-3) / 1e9
    res = {"steps": steps, "ms_per_step": round(ms, 4),
           "taps_per_s": round(L * M * N / (ms * 1e-3), 1), "kernels_ms": per,
           "paper_loss_gbs": round(gbs, 1), "loss": pipe.loss.cpu().tolist(),
           "alpha": pipe.alpha[0].item()}
    log(f"paper-loss step: {res}")
    del pipe
    torch.cuda.empty_cache()
    return res


def recovery_bench(steps=200, warmup=5):
    """Step rate of the synthetic recovery experiment's calibration step
    (Sec. IV-B shape on the stand-in hallway: 256 Tx, 1 Rx antenna, specular
    up to third order + single-bounce diffuse paths, 1,024 subcarriers):
    trainable L = 30 embeddings, scattering patterns and an M = 3 Tx gain,
    the paper's loss, Adam, every link per step.  The targets here are the
    library's own forward at other parameters (only the time is reported)."""
    import math
    from paper_2311_18558_amd import lib as rl
    from paper_2311_18558_amd.calibrate import Calibrator
    from synth import workloads
    t0 = time.time()
    w = workloads.recovery()
    st = w.store
    log(f"workload recovery: {st.n_links} links, {st.n_paths} paths, "
        f"generated in {time.time() - t0:.1f}s")
    dp = rl.DevicePaths(st)
    rng = np.random.default_rng(0)
    L = 30
    v0 = rng.normal(size=L)
    W0 = rng.normal(size=(3, 4, L)) * 0.1 / math.sqrt(L)
    pat0 = np.zeros((3, 6))
    pat0[:, 4:] = math.log(5.0)
    tx0 = np.concatenate([[0.0], np.zeros(3), np.zeros(3), rng.normal(size=9)])
    # targets: the same model at the ground-truth materials and Tx gain
    gt_pat = np.zeros((3, 6), np.float32)
    gt_pat[:, 0] = np.log(w.meta["kx"] / (1 - w.meta["kx"]))
    raw_d = torch.tensor(w.raw, device="cuda")
    a = torch.empty(st.n_paths, dtype=torch.complex64, device="cuda")
    psi = torch.empty(st.n_paths, dtype=torch.float32, device="cuda")
    H = torch.empty((st.n_links, 1, w.radio.n_sc), dtype=torch.complex64, device="cuda")
    rc = rl.radio_from(w.radio)
    pats = rl.patterns(3, torch.tensor(w.meta["tx_raw"], device="cuda"),
                       torch.tensor(gt_pat, device="cuda"))
    rl.trace_fields_pat(rc, dp, rl.materials_per_id(raw_d), pats, a, psi)
    rl.cfr(rc, dp, a, psi, torch.ones(1, dtype=torch.complex64, device="cuda"), H)
    cal = Calibrator(dp, w.radio, H, "embed", embed0=(v0, W0), n_vmf=3, tx_raw0=tx0,
                     pat_raw0=pat0, lr=0.01, lr_gain=0.0, loss="paper")
    links = torch.arange(st.n_links, device="cuda")
    for _ in range(warmup):
        cal.step(links)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        cal.step(links)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the same step recorded into a HIP graph and replayed
    graph, _ = cal.record(links)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_g = e0.elapsed_time(e1) / steps
    out = {"workload": "stand-in hallway 24 x 6 x 3 m with a pillar, 256 Tx, 1 Rx antenna, "
                       "specular up to 3rd order + single-bounce diffuse + first-order "
                       "diffraction, 1,024 subcarriers over 50 MHz",
           "links": st.n_links, "paths": st.n_paths, "steps": steps, "ms_per_step": round(ms, 3),
           "steps_per_s": round(1e3 / ms, 1),
           "graph_ms_per_step": round(ms_g, 3), "graph_steps_per_s": round(1e3 / ms_g, 1),
           "seconds_for_3000_steps": round(3.0 * min(ms, ms_g), 2)}
    log(f"recovery step: {out}")
    del cal, H, dp
    torch.cuda.empty_cache()
    return out


def large_scene_bench(n_rx=2048, batch=2048, steps=2, warmup=1):
    """The large-scene configuration, streamed: the urban block (~100,000
    triangles, 16 material classes), 4 Tx with 32-element ULAs, n_rx outdoor
    Rx at 1.5 m per Tx, specular paths up to fifth order plus single-bounce
    diffuse (real paths, generated batch by batch on the host and kept
    resident on the device), 4,096 subcarriers over 100 MHz, neural
    materials, the paper's loss; one batch per `batch` Rx of one Tx.  The
    default is the bounded sample of 4 x 2,048 links; n_rx=65,536 is the
    full configuration (262,144 links)."""
    from paper_2311_18558_amd import lib as rl
    from paper_2311_18558_amd.calibrate import mlp_out_bias
    from paper_2311_18558_amd.stream import StreamedCalibration
    from synth import workloads
    from synth.params import mlp_init
    t0 = time.time()
    w = workloads.urban(n_rx=n_rx, batch=batch, lazy=True)
    radio = w.radio
    nb = w.meta["n_batches"]
    batches = []
    for i in range(nb):
        batches.append(rl.DevicePaths(w.meta["batch"](i)))
        if (i + 1) % 16 == 0 or i + 1 == nb:
            log(f"large scene: {i + 1}/{nb} batches resident, "
                f"{torch.cuda.memory_allocated() / 1e9:.1f} GB, {time.time() - t0:.0f}s")
    gen_s = time.time() - t0
    L = sum(b.n_links for b in batches)
    P = sum(b.n_paths for b in batches)
    cal = StreamedCalibration(batches, radio, "neural",
                              mlp_params0=mlp_init(np.random.default_rng(5), mlp_out_bias()),
                              aabb=w.aabb, g0=w.g)
    cal.set_targets(w.raw)
    torch.cuda.synchronize()
    log(f"large scene: targets ready, {torch.cuda.memory_allocated() / 1e9:.1f} GB allocated")
    for _ in range(warmup):
        cal.step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        loss = cal.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # stage split from one more step with events between the stages
    events = {}
    cal.step(events=events)
    torch.cuda.synchronize()
    stages = {k: round(sum(a.elapsed_time(b) for a, b in v), 2) for k, v in events.items()}
    M, N = radio.n_elem, radio.n_sc
    out = {"workload": f"large scene: urban block 400 x 400 m ({w.meta['tris']:,} triangles, "
                       f"{w.meta['n_mat']} material classes), 4 Tx x {n_rx:,} outdoor Rx at 1.5 m, "
                       "real specular paths up to 5th order + single-bounce diffuse, 32-element "
                       "ULA, 4,096 subcarriers over 100 MHz, neural materials, paper loss, "
                       f"streamed in {batch:,}-Rx batches",
           "links": L, "paths": P, "paths_per_link": round(P / L, 1), "batches": nb,
           "taps": L * M * N, "steps": steps, "ms_per_step": round(ms, 1),
           "taps_per_s": round(L * M * N / (ms * 1e-3), 1),
           "stage_ms": stages, "host_generation_s": round(gen_s, 1),
           "peak_hbm_gb": round(torch.cuda.max_memory_allocated() / 1e9, 1),
           "loss": loss.item()}
    log(f"large scene: {out}")
    del cal, batches
    torch.cuda.empty_cache()
    return out


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform's."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def _oracle_links(w, budget_s, max_links, seed):
    """The FP64 oracle (forward, loss, reverse-mode gradient) on whole links
    of the workload until budget_s of wall time is spent: (links, seconds)."""
    from oracle import channel as och
    from oracle.trace import trace_fields_per_id
    st, radio = w.store, w.radio
    f = och.subcarrier_freqs(radio.fc, radio.bandwidth, radio.n_sc)
    rng = np.random.default_rng(seed)
    raw_gt = torch.tensor(w.raw, dtype=torch.float64)
    g = torch.tensor(w.g, dtype=torch.complex128)
    raw0 = raw_gt + torch.tensor(rng.normal(scale=0.3, size=w.raw.shape))
    order = rng.permutation(st.n_links)
    done, t_used = 0, 0.0
    for l in order[:max_links]:
        sub = st.subset_links([l])
        a_t, p_t = trace_fields_per_id(sub, raw_gt, radio.fc, ula_axis=radio.ula_axis)
        Ht = och.cfr(sub.link_off, sub.tau, a_t, p_t, g, f)
        t0 = time.perf_counter()
        rr = raw0.clone().requires_grad_(True)
        gg = g.clone().requires_grad_(True)
        a, psi = trace_fields_per_id(sub, rr, radio.fc, ula_axis=radio.ula_axis)
        H = och.cfr(sub.link_off, sub.tau, a, psi, gg, f)
        L, _, _ = och.cfr_loss(H, Ht)
        torch.autograd.grad(L, (rr, gg))
        t_used += time.perf_counter() - t0
        done += 1
        if t_used >= budget_s:
            break
    return done, t_used


def cpu_baseline(w, budget_s=12.0, budget_1_s=8.0, max_links=8192):
    """The oracle timed on the host: once with all of torch's intra-op
    threads (the reported value) and once on one thread."""
    radio = w.radio
    n_thr = torch.get_num_threads()
    done, t_used = _oracle_links(w, budget_s, max_links, seed=0)
    torch.set_num_threads(1)
    try:
        done1, t1 = _oracle_links(w, budget_1_s, max_links, seed=1)
    finally:
        torch.set_num_threads(n_thr)
    per_link = radio.n_elem * radio.n_sc
    return {"value": done * per_link / t_used, "unit": "taps/s", "cores": n_thr,
            "kind": "oracle",
            "sample": f"{done} whole links of the scale workload (forward, loss and FP64 "
                      f"autograd gradient; targets precomputed), {t_used:.1f}s on {n_thr} "
                      f"threads",
            "single_thread": {"value": done1 * per_link / t1, "unit": "taps/s", "cores": 1,
                              "sample": f"{done1} whole links, {t1:.1f}s"},
            "host_cpu": cpu_model(), "host_cpus_visible": os.cpu_count()}


def calib_compare(w, steps):
    """Plain (per-material-id) vs learned (neural materials) calibration on
    the scale scene with a spatially varying hidden material field and
    hidden element gains: batch 512 Rx, Adam; 14,336 training / 2,048
    held-out Rx."""
    from paper_2311_18558_amd import lib as rl
    from paper_2311_18558_amd.calibrate import compare_learned_vs_plain, targets
    from synth import workloads
    wl = workloads.learned(geometry=(w.meta["plan"], w.store))
    dp = rl.DevicePaths(wl.store)
    H_all = targets(dp, wl.radio, per_inter=wl.meta["per_inter"], g=wl.g)
    log(f"calibration comparison: {steps} plain steps, learned up to {steps}")
    res = compare_learned_vs_plain(dp, wl.radio, H_all, wl.meta["n_mat"], wl.aabb,
                                   wl.meta["train"], wl.meta["heldout"], plain_steps=steps,
                                   learned_max_steps=steps, log=log)
    log(f"calib: {res}")
    del H_all, dp
    torch.cuda.empty_cache()
    return res


def hot_source_sha():
    import hashlib
    h = hashlib.sha1()
    for f in HOT_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_18558_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic():
    """HBM bytes per launch of the CFR kernels from the committed rocprofv3
    counter summary; empty when absent or taken on other kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return {}
    try:
        t = json.load(open(p))
    except Exception:
        return {}
    if t.get("source_sha") != hot_source_sha():
        return {}
    return {k: v["traffic_bytes"] for k, v in t.get("kernels", {}).items()}


def summarize_traffic(fetch_csv, write_csv):
    """HBM traffic per launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch)
    of a --copy-probe run: each counter is scaled by what it reads for the
    2 GiB device copy (COPY_PROBE_BYTES read and written).  Writes
    profiles/traffic.json and prints a markdown summary."""
    import csv
    import re

    def per_kernel(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
            vals.setdefault(name, {}).setdefault(int(r["Dispatch_Id"]), 0.0)
            vals[name][int(r["Dispatch_Id"])] += float(r["Counter_Value"]) * 1024.0
        return vals

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    copy_names = [k for k in fetch if "copyBuffer" in k]
    # the probe's copies are the largest copy dispatches
    cf = max(v for k in copy_names for v in fetch[k].values())
    cw = max(v for k in copy_names for v in write.get(k, {0: 0.0}).values())
    sf, sw = cf / COPY_PROBE_BYTES, cw / COPY_PROBE_BYTES
    out = {"source_sha": hot_source_sha(), "copy_probe_bytes": COPY_PROBE_BYTES,
           "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    names = {"rtc::cfr_fused_kernel<10, true>": "cfr_loss_adjoint",
             "rtc::cfr_fused_kernel<10, false>": "cfr_loss_adjoint_cfr",
             "rtc::cfr_kernel": "cfr", "rtc::cfr_adjoint_wave_kernel": "cfr_adjoint",
             "rtc::cfr_adjoint_kernel<8>": "cfr_adjoint_wg",
             "rtc::cfr_loss_wave_kernel<10, 2>": "cfr_loss",
             "rtc::paper_loss_wave_kernel<10, true>": "paper_loss",
             "rtc::gain_products_kernel": "gain_products"}
    lines = ["| kernel | dispatches | FETCH_SIZE (GB) | WRITE_SIZE (GB) | HBM read (GB) "
             "| HBM write (GB) |", "|---|---:|---:|---:|---:|---:|"]
    for k, short in names.items():
        if k not in fetch:
            continue
        f = float(np.mean(list(fetch[k].values())))
        w = float(np.mean(list(write.get(k, {0: 0.0}).values())))
        rb, wb = f / sf, w / sw
        out["kernels"][short] = {"fetch_bytes": rb, "write_bytes": wb, "traffic_bytes": rb + wb}
        lines.append(f"| `{k}` | {len(fetch[k])} | {f / 1e9:.3f} | {w / 1e9:.3f} | "
                     f"{rb / 1e9:.3f} | {wb / 1e9:.3f} |")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"copy probe: {COPY_PROBE_BYTES / 2**30:.0f} GiB read + written; FETCH_SIZE reads "
          f"{sf:.3f}x, WRITE_SIZE {sw:.3f}x the bytes moved\n")
    print("\n".join(lines))


def summarize_counters(*csvs):
    """Per-kernel VALU / MFMA / LDS figures from rocprofv3 --pmc csv files
    (any split of the counters over runs), averaged over the dispatches of
    each (kernel, grid size); prints a markdown table.  GRBM_GUI_ACTIVE is
    summed over the 8 XCDs (cycles = GRBM_GUI_ACTIVE / 8); a wave64 VALU
    instruction takes 4 cycles of a 16-lane SIMD; 1,024 SIMDs."""
    import collections
    import csv
    import re
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    count = collections.Counter()
    for path in csvs:
        disp = collections.defaultdict(dict)
        meta = {}
        for r in csv.DictReader(open(path)):
            d = int(r["Dispatch_Id"])
            disp[d][r["Counter_Name"]] = disp[d].get(r["Counter_Name"], 0.0) + float(
                r["Counter_Value"])
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
            meta[d] = (name, int(r["Grid_Size"]))
        seen = collections.Counter(meta.values())
        for key, n in seen.items():
            count[key] = max(count[key], n)
        for d, c in disp.items():
            for k, v in c.items():
                per[meta[d]][k].append(v)
    simds = 1024
    peak_per_cycle = PEAK_F16_MATRIX_TFLOPS * 1e12 / 2.4e9  # dense FP16 flops per clock
    lines = ["| kernel | grid | dispatches | cycles (M) | VALU busy | MFMA busy | "
             "MFMA flops issued / peak per cycle | VALU instr / wave | LDS instr / wave | "
             "LDS bank-conflict cycles / LDS active |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for (name, grid), c in sorted(per.items(), key=lambda kv: -np.mean(kv[1].get(
            "GRBM_GUI_ACTIVE", [0]))):
        a = {k: float(np.mean(v)) for k, v in c.items()}
        cyc = a.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        if cyc < 1e5:
            continue
        waves = a.get("SQ_WAVES", 0.0)
        valu = 4.0 * a.get("SQ_INSTS_VALU", 0.0) / (simds * cyc)
        mfma = a.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (simds * cyc)
        mops = (a.get("SQ_INSTS_VALU_MFMA_MOPS_F16", 0.0)
                + a.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)) * 512.0
        lds_act = a.get("SQ_ACTIVE_INST_LDS", 0.0)
        conf = a.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds_act if lds_act else 0.0
        lines.append(f"| `{name}` | {grid} | {count[(name, grid)]} | {cyc / 1e6:.2f} | "
                     f"{valu:.2f} | {mfma:.2f} | {mops / cyc / peak_per_cycle:.3f} | "
                     f"{a.get('SQ_INSTS_VALU', 0.0) / max(waves, 1):.0f} | "
                     f"{a.get('SQ_INSTS_LDS', 0.0) / max(waves, 1):.0f} | {conf:.2f} |")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-calib", action="store_true",
                    help="skip the learned-vs-plain calibration comparison")
    ap.add_argument("--calib-steps", type=int, default=3000)
    ap.add_argument("--no-diffuse", action="store_true",
                    help="skip the diffuse-scattering workload line")
    ap.add_argument("--no-recovery", action="store_true",
                    help="skip the synthetic-recovery step-rate line")
    ap.add_argument("--no-large-scene", action="store_true",
                    help="skip the bounded large-scene line (4 Tx x 2,048 urban Rx)")
    ap.add_argument("--config5", action="store_true",
                    help="run the large-scene line at full size, 4 Tx x 65,536 Rx (~5 min)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="start with a 2 GiB device copy (counter calibration)")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE results and exit")
    ap.add_argument("--counters", nargs="+", metavar="PMC_CSV",
                    help="summarise rocprofv3 --pmc VALU / MFMA / LDS counters and exit")
    args = ap.parse_args()
    if args.traffic:
        summarize_traffic(*args.traffic)
        return
    if args.counters:
        summarize_counters(*args.counters)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the hot path here is the one-GPU share of the "
              "workload; sharding across GPUs is described in the design notes but not built.",
              file=sys.stderr)
        sys.exit(2)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2311_18558_amd import lib as rl
    from paper_2311_18558_amd.pipeline import Pipeline
    rl.load()
    if args.copy_probe:
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy probe: 3 x {COPY_PROBE_BYTES} bytes")

    w = build_workload()
    st, radio = w.store, w.radio
    L, M, N, P, D = st.n_links, radio.n_elem, radio.n_sc, st.n_paths, st.max_depth
    rng = np.random.default_rng(7)
    raw0 = (w.raw + rng.normal(scale=0.3, size=w.raw.shape)).astype(np.float32)
    pipe = Pipeline(st, radio, w.raw, w.g)
    # targets from the ground truth, then start from perturbed parameters
    H_tgt = torch.empty_like(pipe.H)
    pipe.trace()
    pipe.cfr(out=H_tgt)
    pipe.set_target(H_tgt)
    pipe.raw.copy_(torch.tensor(raw0, device=pipe.dev))
    torch.cuda.synchronize()
    log("targets ready")

    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()
    events = {}
    t0 = time.perf_counter()
    e_start = torch.cuda.Event(enable_timing=True)
    e_end = torch.cuda.Event(enable_timing=True)
    e_start.record()
    for _ in range(args.steps):
        pipe.step(events=events)
    e_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e_start.elapsed_time(e_end)
    ms_step = total_ms / args.steps
    per_kernel = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in events.items()}
    log("per-stage ms: " + ", ".join(f"{k} {v:.3f}" for k, v in per_kernel.items()))
    loss = pipe.loss.cpu().tolist()

    taps = L * M * N
    value = taps / (ms_step * 1e-3)
    if pipe.fused:
        hot = "cfr_loss_adjoint"
    else:
        hot = max(("cfr", "cfr_adjoint"), key=lambda k: per_kernel[k])
    fl, _ = kernel_work(hot, L, M, N, P, D)
    achieved = fl / (per_kernel[hot] * 1e-3) / 1e12
    traffic = load_traffic().get(hot)
    # the contraction runs on the FP16 matrix cores: frac is taken against
    # their published dense peak; the ceiling of the split arithmetic (three
    # FP16 products per real product) and what the matrix cores actually
    # issue (the conjugate-pair form issues half the products of the direct
    # sum) are reported beside it
    roofline = {"bound": "mfma", "kernel": hot, "achieved": round(achieved, 2),
                "peak": PEAK_F16_MATRIX_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_F16_MATRIX_TFLOPS, 4), "traffic": traffic,
                "peak_basis": f"MI355X dense FP16 matrix peak {PEAK_F16_MATRIX_TFLOPS:.0f} "
                              f"TFLOP/s; algorithmic work "
                              f"{'16' if hot == 'cfr_loss_adjoint' else '8'} M N P flops "
                              f"per launch",
                "split_ceiling_tflops": round(PEAK_SPLIT_TFLOPS, 1),
                "split_ceiling_frac": round(achieved / PEAK_SPLIT_TFLOPS, 4),
                "fp32_matrix_peak_frac": round(achieved / PEAK_FP32_MATRIX_TFLOPS, 4)}
    issued = mfma_issued(hot, st.link_off, M, N) * MFMA_FLOPS / (per_kernel[hot] * 1e-3) / 1e12
    roofline["mfma_issued_tflops"] = round(issued, 1)
    roofline["mfma_issued_frac"] = round(issued / PEAK_F16_MATRIX_TFLOPS, 4)
    kernels = {}
    for k, ms in per_kernel.items():
        fl_k, by_k = kernel_work(k, L, M, N, P, D)
        ent = {"ms": round(ms, 4)}
        if fl_k:
            ent["tflops"] = round(fl_k / (ms * 1e-3) / 1e12, 2)
        if by_k:
            ent["gbs"] = round(by_k / (ms * 1e-3) / 1e9, 1)
        kernels[k] = ent
    fwd_adj_flops = 16.0 * M * N * P
    out = {
        "metric": "CFR taps/s fwd+adjoint",
        "value": round(value, 1),
        "unit": "taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": "scale: procedural indoor floor (~5,000 triangles, 10 material "
                               "classes), 1 Tx with a 32-element ULA, 16,384 Rx, specular paths "
                               "up to 5th order, 1,024 subcarriers over 50 MHz at 3.5 GHz",
                   "links": L, "elements": M, "subcarriers": N, "paths": P,
                   "paths_per_link": round(P / L, 1), "max_depth": D},
        "roofline": roofline,
        "hot_path_tflops": round(fwd_adj_flops / (
            (per_kernel["cfr_loss_adjoint"] if pipe.fused
             else per_kernel["cfr"] + per_kernel["cfr_adjoint"]) * 1e-3) / 1e12, 2),
        "kernels": kernels,
        "loss": loss[0],
        "wall_s": round(wall, 3),
    }
    if pipe.fused:
        out["separate_calls_step"] = separate_calls_step(st, radio, w, raw0, H_tgt,
                                                         min(args.steps, 5))
        # the fused pass with the targets as H* and the stored target PDP
        out["fused_cfr_targets_step"] = separate_calls_step(
            st, radio, w, raw0, H_tgt, min(args.steps, 5), label="fused (H*, p* targets)",
            targets="cfr")
    out["paper_loss_step"] = paper_loss_step(st, radio, w, raw0, H_tgt, min(args.steps, 5))
    del pipe, H_tgt
    torch.cuda.empty_cache()
    if not args.no_diffuse:
        out["diffuse"] = diffuse_bench()
    if not args.no_recovery:
        out["recovery"] = recovery_bench()
    if args.config5:
        out["large_scene"] = large_scene_bench(n_rx=65536, steps=1)
    elif not args.no_large_scene:
        out["large_scene"] = large_scene_bench()
    if not args.no_calib:
        out["calib"] = calib_compare(w, args.calib_steps)
    if not args.no_cpu_baseline:
        log("timing the oracle on a sample (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(w)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""The synthetic recovery experiment of Sec. IV-B on a stand-in hallway.

Ground truth: FP64 oracle CFRs for Table I's materials with the
backscattering-lobe pattern (alpha_r = 5, alpha_s = 8, Lambda = 0.8) and a
three-lobe Tx gain.  The library then calibrates, from generic initial
values, L = 30 material embeddings, per-material scattering patterns and an
M = 3 Tx gain by Adam (lr 0.01) on every link per step, and the recovered
materials are compared with Table I."""
import math
import sys
import time

import numpy as np
import pytest
import torch

from oracle import channel as och
from oracle.trace import trace_fields_per_id
from synth.workloads import RECOVERY_LOBES, TABLE_I, recovery

pytestmark = pytest.mark.gpu

STEPS = 3000
L_EMBED = 30


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def experiment(gpu_lib):
    t0 = time.perf_counter()
    w = recovery()
    st, m = w.store, w.meta
    a_r, a_s, lam = RECOVERY_LOBES
    a, psi = trace_fields_per_id(st, torch.tensor(w.raw, dtype=torch.float64), w.radio.fc,
                                 tx_raw=torch.tensor(m["tx_raw"], dtype=torch.float64),
                                 n_vmf=m["n_vmf"],
                                 backscatter=(m["kx"], a_r, a_s, np.full(3, lam)))
    f = och.subcarrier_freqs(w.radio.fc, w.radio.bandwidth, w.radio.n_sc)
    H = och.cfr(st.link_off, st.tau, a, psi, torch.ones(1, dtype=torch.complex128), f)
    say(f"recovery targets: {st.n_links} links, {st.n_paths} paths, "
        f"{time.perf_counter() - t0:.1f} s")
    return w, H.to(torch.complex64)


def initial_state(seed=0):
    """Generic start: embeddings near zero (eps_r ~ 2, sigma ~ 1 S/m, S ~ K_x ~
    0.5), equal pattern weights with lam_2 = lam_3 = 5, an isotropic-like Tx
    gain (eta 0.5, equal weights, lam = 1, random axes)."""
    rng = np.random.default_rng(seed)
    v0 = rng.normal(size=L_EMBED)
    W0 = rng.normal(size=(3, 4, L_EMBED)) * 0.1 / math.sqrt(L_EMBED)
    pat0 = np.zeros((3, 6))
    pat0[:, 4:] = math.log(5.0)
    tx0 = np.concatenate([[0.0], np.zeros(3), np.zeros(3), rng.normal(size=9)])
    return v0, W0, pat0, tx0


def calibrate(w, H, loss, steps):
    from paper_2311_18558_amd import lib
    from paper_2311_18558_amd.calibrate import Calibrator
    v0, W0, pat0, tx0 = initial_state()
    dp = lib.DevicePaths(w.store)
    cal = Calibrator(dp, w.radio, H.cuda(), "embed", embed0=(v0, W0), n_vmf=3, tx_raw0=tx0,
                     pat_raw0=pat0, lr=0.01, lr_gain=0.0, loss=loss)
    links = torch.arange(w.store.n_links, device="cuda")
    first = cal.step(links)[0].item()
    for s in range(2, steps + 1):
        out = cal.step(links)
        if s % 500 == 0:
            r = cal.learned()
            say(f"  [{loss}] step {s}: loss {out[0].item():.3e} eps_r {np.round(r['eps_r'], 3)} "
                f"sigma {np.round(r['sigma'], 4)} S {np.round(r['S'], 3)} "
                f"K_x {np.round(r['K_x'], 3)}")
    torch.cuda.synchronize()
    return cal, first, out[0].item()


@pytest.mark.parametrize("loss", ["paper", "workload"])
def test_recovers_table_i(experiment, loss):
    """After 3,000 Adam steps the materials match Table I: eps_r within 2 %,
    S and K_x within 0.03, sigma within 10 % for floor and walls.  The
    ceiling's sigma (0.004 S/m at eps_r = 1.48: sigma/(eps0 w) ~ 0.02) hardly
    changes any field, so only its order of magnitude is asked for."""
    w, H = experiment
    t0 = time.perf_counter()
    cal, first, last = calibrate(w, H, loss, STEPS)
    el = time.perf_counter() - t0
    r = cal.learned()
    say(f"[{loss}] {STEPS} steps in {el:.1f} s, loss {first:.3e} -> {last:.3e}")
    say(f"  eps_r {r['eps_r']}, sigma {r['sigma']}, S {r['S']}, K_x {r['K_x']}, eta {r['eta']}")
    assert last < first / 50
    assert np.all(np.abs(r["eps_r"] / TABLE_I[:, 0] - 1) <= 0.02)
    assert np.all(np.abs(r["sigma"][:2] / TABLE_I[:2, 1] - 1) <= 0.10)
    assert 0.002 <= r["sigma"][2] <= 0.008
    assert np.all(np.abs(r["S"] - TABLE_I[:, 2]) <= 0.03)
    assert np.all(np.abs(r["K_x"] - TABLE_I[:, 3]) <= 0.03)


def test_recovers_tx_gain(experiment):
    """The learned Tx gain matches the ground truth's lobes (matched by
    their mean directions): weights within 0.03, concentrations within 10 %,
    axes within 3 degrees, efficiency within 0.02."""
    from synth.workloads import RECOVERY_TX
    w, H = experiment
    cal, _, _ = calibrate(w, H, "paper", STEPS)
    r = cal.learned()
    mu_gt = np.asarray(RECOVERY_TX["mu"], np.float64)
    mu_gt /= np.linalg.norm(mu_gt, axis=1, keepdims=True)
    match = np.argmax(mu_gt @ r["mu_tx"].T, axis=1)
    assert sorted(match.tolist()) == [0, 1, 2]
    ang = np.degrees(np.arccos(np.clip(np.sum(mu_gt * r["mu_tx"][match], 1), -1, 1)))
    say(f"  Tx: eta {r['eta']:.4f} w {r['w_tx'][match]} lam {r['lam_tx'][match]} "
        f"axis error {ang} deg")
    assert abs(r["eta"] - RECOVERY_TX["eta"]) <= 0.02
    assert np.all(np.abs(r["w_tx"][match] - np.asarray(RECOVERY_TX["w"])) <= 0.03)
    assert np.all(np.abs(r["lam_tx"][match] / np.asarray(RECOVERY_TX["lam"]) - 1) <= 0.10)
    assert np.all(ang <= 3.0)

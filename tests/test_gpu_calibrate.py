"""Calibration (Algorithm 1 with Adam) through the library on a reduced
scale scene: plain per-material-id calibration recovers method-generated
targets, and the neural-material field beats it on a spatially varying
hidden field (what the network gains)."""
import sys

import numpy as np
import pytest
import torch

from synth import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small():
    return workloads.learned(n_rx=1024, n_heldout=128, n_sc=256, n_elem=8)


def test_plain_calibration_recovers_per_id_targets(gpu_lib, small):
    from paper_2311_18558_amd import lib
    from paper_2311_18558_amd.calibrate import Calibrator, raw_prior, targets
    w = small
    say("plain calibration on per-id targets")
    dp = lib.DevicePaths(w.store)
    H = targets(dp, w.radio, raw=w.raw, g=w.g)
    cal = Calibrator(dp, w.radio, H, "per_id", raw0=raw_prior(w.meta["n_mat"]))
    held = torch.tensor(w.meta["heldout"], device="cuda")
    train = torch.tensor(w.meta["train"], device="cuda")
    n0 = cal.nmse(held)
    rng = np.random.default_rng(0)
    for _ in range(400):
        cal.step(train[torch.tensor(rng.choice(len(train), 128, replace=False), device="cuda")])
    n1 = cal.nmse(held)
    print(f"held-out NMSE {n0:.3e} -> {n1:.3e}")
    assert n1 < 1e-2 * n0
    # the loss at the ground truth is zero
    cal_gt = Calibrator(dp, w.radio, H, "per_id", raw0=w.raw, g0=w.g)
    assert cal_gt.nmse(held) < 1e-10


def test_learned_field_beats_plain(gpu_lib, small):
    from paper_2311_18558_amd import lib
    from paper_2311_18558_amd.calibrate import compare_learned_vs_plain, targets
    w = small
    say("learned vs plain on a spatial field")
    dp = lib.DevicePaths(w.store)
    H = targets(dp, w.radio, per_inter=w.meta["per_inter"], g=w.g)
    res = compare_learned_vs_plain(dp, w.radio, H, w.meta["n_mat"], w.aabb, w.meta["train"],
                                   w.meta["heldout"], plain_steps=600, learned_max_steps=600,
                                   batch=128, eval_every=100, lr_mlp=3e-4)
    print(res)
    assert res["learned_reached_plain_nmse"]
    assert res["learned_heldout_nmse_at_plain_steps"] < res["plain_heldout_nmse"]

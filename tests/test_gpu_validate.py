"""Device-side path-store check (rtc_validate_paths): zero counts for valid
stores, and for each planted defect exactly the planted count in its
category (the check reads every array within its bounds, whatever the
values); RTCAL_DEBUG=1 makes every upload raise on a defective store."""
import copy
import math

import numpy as np
import pytest
import torch

from tests.test_gpu_diffraction import CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


@pytest.mark.parametrize("case", list(CASES))
def test_valid_stores_have_no_violations(rl, case):
    st, raw, _, _ = CASES[case]
    counts = rl.validate_paths(rl.DevicePaths(st), n_mat=raw.shape[0])
    assert not any(counts.values()), counts


def _planted(st, what):
    s = copy.deepcopy(st)
    P, D = s.n_paths, s.max_depth
    d1 = np.nonzero(s.depth >= 1)[0][:3]       # three paths with a first slot
    if what == "link_off":
        s.link_off = s.link_off.copy()
        s.link_off[2] = s.link_off[3] + 1      # breaks l=2 and l=3 monotonicity
        return s, {"link_off": 1}
    if what == "depth":
        # on paths of full depth, so that no unused (zero) slot becomes used
        full = np.nonzero(s.depth == D)[0][:3]
        s.depth = s.depth.copy()
        s.depth[full] = D + 1
        return s, {"depth": 3}
    if what == "material id":
        s.mat = s.mat.copy()
        s.mat[d1] = 999
        return s, {"material id": 3}
    if what == "kind":
        s.kind = s.kind.copy()
        s.kind[d1] = 7
        return s, {"kind": 3}
    if what == "tau":
        s.tau = s.tau.copy()
        s.tau[:2] = [float("nan"), -1.0]
        return s, {"tau": 2}
    if what == "unit vector":
        s.nrm = s.nrm.copy()
        s.nrm[:, d1] *= 1.5
        return s, {"unit vector": 3}
    if what == "non-finite coordinate":
        s.pts = s.pts.copy()
        s.pts[0, d1[:2]] = float("inf")
        return s, {"non-finite coordinate": 2}
    raise ValueError(what)


@pytest.mark.parametrize("what", ["link_off", "depth", "material id", "kind", "tau",
                                  "unit vector", "non-finite coordinate"])
def test_planted_defects_are_counted(rl, what):
    st, raw, _, _ = CASES["floor_diffuse"]
    bad, expect = _planted(st, what)
    counts = rl.validate_paths(rl.DevicePaths(bad), n_mat=raw.shape[0])
    for k, v in counts.items():
        assert v == expect.get(k, 0), (what, counts)


def test_wedge_range_and_debug_switch(rl, monkeypatch):
    st, raw, _, _ = CASES["wedge"]
    s = copy.deepcopy(st)
    dfr = np.nonzero(s.kind[:s.n_paths] == 2)[0][:2]
    s.edge = s.edge.copy()
    s.edge[3, dfr] = 2.5
    counts = rl.validate_paths(rl.DevicePaths(s), n_mat=raw.shape[0])
    assert counts["dA or wedge n"] == 2 and sum(counts.values()) == 2
    monkeypatch.setenv("RTCAL_DEBUG", "1")
    rl.DevicePaths(st)  # a valid store passes
    with pytest.raises(RuntimeError, match="wedge n"):
        rl.DevicePaths(s)
    _ = math

"""Per-interaction materials in compact rows (used slots only) against the
slot-indexed rows: identical coefficients and identical gradients at the
used slots, on a store of mixed depths with diffuse and diffraction paths."""
import numpy as np
import pytest
import torch

from tests.test_gpu_diffraction import CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl(gpu_lib):
    from paper_2311_18558_amd import lib
    return lib


@pytest.mark.parametrize("case", ["floor_diffuse", "wedge"])
def test_compact_rows_match_slot_rows(rl, case):
    st, _, radio, _ = CASES[case]
    rng = np.random.default_rng(61)
    P, D = st.n_paths, st.max_depth
    dp = rl.DevicePaths(st)
    rc = rl.radio_from(radio)
    full = torch.tensor(np.stack([rng.uniform(2, 8, D * P), 10 ** rng.uniform(-3, 0, D * P),
                                  rng.uniform(0.05, 0.6, D * P)]).astype(np.float32),
                        device="cuda")
    idx, n_inter, pts = rl.compact_interactions(dp)
    used = idx >= 0
    assert int(used.sum()) == n_inter == int(st.depth.astype(np.int64).sum())
    comp = full[:, used].contiguous()
    assert torch.equal(pts, dp.pts[:, used])
    a_full = torch.empty(P, dtype=torch.complex64, device="cuda")
    a_comp = torch.empty(P, dtype=torch.complex64, device="cuda")
    m_full = rl.materials_per_interaction(full)
    m_comp = rl.materials_per_interaction(comp, (idx, n_inter))
    rl.trace_fields(rc, dp, m_full, a_full, None)
    rl.trace_fields(rc, dp, m_comp, a_comp, None)
    dLda = torch.tensor((rng.normal(size=P) + 1j * rng.normal(size=P)).astype(np.complex64),
                        device="cuda")
    g_full = torch.full((3, D * P), float("nan"), device="cuda")
    rl.trace_fields_adjoint(rc, dp, m_full, dLda, None, g_full, None)
    g_c = torch.full((3, n_inter), float("nan"), device="cuda")
    rl.trace_fields_adjoint(rc, dp, m_comp, dLda, None, g_c, None)
    torch.cuda.synchronize()
    assert torch.equal(a_full, a_comp)
    assert torch.equal(g_full[:, used], g_c)
    assert torch.all(g_full[:, ~used] == 0)

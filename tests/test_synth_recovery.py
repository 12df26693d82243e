"""The recovery workload's geometry: without its pillar a convex hallway, so
every link has all 1 + 6 + 18 + 38 specular images up to third order and
every surface sample as a diffuse path; per-link Tx positions in the
diffuse delays; the Table I ground truth in the raw layout; with the pillar,
blocked paths and first-order diffraction at its corners."""
import numpy as np
import pytest

from synth.store import KIND_DIFFUSE
from synth.workloads import TABLE_I, recovery, vmf_to_raw

C0 = 299792458.0


@pytest.fixture(scope="module")
def small():
    return recovery(seed=3, n_tx=6, density=0.25, n_sc=64, pillar=None)


def test_path_counts(small):
    st = small.store
    cnt = np.diff(st.link_off)
    P = st.n_paths
    kind = st.kind.reshape(st.max_depth, P)
    n_dif = (kind == KIND_DIFFUSE).sum(0)
    n_samples = n_dif.sum() // st.n_links
    for l in range(st.n_links):
        lo, hi = st.link_off[l], st.link_off[l + 1]
        spec = (n_dif[lo:hi] == 0)
        assert spec.sum() == 63
        assert np.bincount(st.depth[lo:hi][spec], minlength=4).tolist() == [1, 6, 18, 38]
        assert (~spec).sum() == n_samples
    assert cnt.sum() == P


def test_diffuse_delays_use_each_links_tx(small):
    st = small.store
    P = st.n_paths
    for l in range(st.n_links):
        lo, hi = int(st.link_off[l]), int(st.link_off[l + 1])
        idx = np.arange(lo, hi)
        dif = idx[st.kind[idx] == KIND_DIFFUSE]
        s = st.pts[:, dif].T.astype(np.float64)
        tx = st.tx_pos[l].astype(np.float64)
        rx = st.rx_pos[l].astype(np.float64)
        ref = (np.linalg.norm(s - tx, axis=1) + np.linalg.norm(rx - s, axis=1)) / C0
        assert np.allclose(st.tau[dif], ref, rtol=1e-6)
    assert len(np.unique(st.tx_pos, axis=0)) == st.n_links
    assert len(np.unique(st.rx_pos, axis=0)) == 1
    assert P > 0


def test_materials_and_surfaces(small):
    st = small.store
    dif = st.kind == KIND_DIFFUSE
    z = st.pts[2, dif]
    m = st.mat[dif]
    assert np.all(m[np.isclose(z, 0.0)] == 0) and np.all(m[np.isclose(z, 3.0)] == 2)
    walls = ~np.isclose(z, 0.0) & ~np.isclose(z, 3.0)
    assert np.all(m[walls] == 1)
    raw = small.raw.astype(np.float64)
    assert np.allclose(1 + np.exp(raw[:, 0]), TABLE_I[:, 0], rtol=1e-6)
    assert np.allclose(np.exp(raw[:, 1]), TABLE_I[:, 1], rtol=1e-6)
    assert np.allclose(1 / (1 + np.exp(-raw[:, 2])), TABLE_I[:, 2], rtol=1e-6)


def test_tx_raw_roundtrip():
    t = vmf_to_raw(0.9, (0.6, 0.25, 0.15), (6.0, 2.0, 10.0), np.eye(3))
    assert abs(1 / (1 + np.exp(-t[0])) - 0.9) < 1e-6
    w = np.exp(t[1:4]) / np.exp(t[1:4]).sum()
    assert np.allclose(w, (0.6, 0.25, 0.15), rtol=1e-6)
    assert np.allclose(np.exp(t[4:7]), (6, 2, 10), rtol=1e-6)


def test_pillar_blocks_and_diffracts():
    from synth.store import KIND_DIFFRACTION
    w = recovery(seed=3, n_tx=12, density=0.25, n_sc=64)
    st = w.store
    P = st.n_paths
    kind = st.kind[:P]
    assert (kind == KIND_DIFFRACTION).sum() >= 6
    x0, y0, x1, y1 = w.meta["pillar"]
    d = np.nonzero(kind == KIND_DIFFRACTION)[0]
    q = st.pts[:, d]
    on_corner = (np.isclose(q[0], x0) | np.isclose(q[0], x1)) & (np.isclose(q[1], y0) |
                                                               np.isclose(q[1], y1))
    assert on_corner.all() and np.all(st.mat_n[d] == 1) and np.all(st.mat[d] == 1)
    # fewer specular images than the full set of the empty hallway
    spec = (kind == 0)
    assert spec.sum() < 63 * st.n_links

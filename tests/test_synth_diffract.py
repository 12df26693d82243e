"""Diffraction-path geometry on the floors: diffraction points lie on free
box corners with Keller's equal angles to the edge, both rays in the wedge's
free space (0 < phi, phi' < 3 pi / 2 measured from face 0), delays from the
two legs; merge_links keeps every link's paths in order."""
import math

import numpy as np
import pytest
import torch

from oracle.diffraction import edge_geometry
from synth.diffract import add_diffraction, floor_edges
from synth.floorplan import indoor_floor
from synth.pathfind import find_store
from synth.store import KIND_DIFFRACTION, merge_links

C0 = 299792458.0


@pytest.fixture(scope="module")
def floor():
    plan = indoor_floor(11, width=14.0, depth=10.0, min_room=4.0, max_rooms=2, open_frac=0.6,
                        n_pillars=1, target_tris=400)
    rng = np.random.default_rng(12)
    tx = plan.sample_points(rng, 1, 2.4, 2.6)[0]
    rx = plan.sample_points(rng, 12, 1.0, 2.0)
    spec = find_store(plan, tx, rx, 2, n_rays=1 << 14)
    return plan, spec, add_diffraction(spec, plan)


def test_edges_are_free_corners(floor):
    plan, _, _ = floor
    E = floor_edges(plan)
    assert len(E) > 0
    for cx, cy, n0x, n0y, ez, *_ in E:
        # a corner of some box and inside no other
        hits = [(abs(cx - b[0]) < 1e-9 or abs(cx - b[2]) < 1e-9) and
                (abs(cy - b[1]) < 1e-9 or abs(cy - b[3]) < 1e-9) for b in plan.boxes]
        assert sum(hits) == 1
        assert abs(n0x) + abs(n0y) == 1 and abs(ez) == 1


def test_diffraction_paths_geometry(floor):
    plan, spec, st = floor
    P = st.n_paths
    d = np.nonzero(st.kind[:P] == KIND_DIFFRACTION)[0]
    assert len(d) > 10
    link = st.link_of_path()
    for p in d:
        q = st.pts[:, p].astype(np.float64)
        tx = st.tx_pos[link[p]].astype(np.float64)
        rx = st.rx_pos[link[p]].astype(np.float64)
        e = st.edge[:3, p].astype(np.float64)
        n0 = st.nrm[:, p].astype(np.float64)
        assert st.depth[p] == 1 and st.edge[3, p] == np.float32(1.5)
        assert abs(st.tau[p] * C0 - (np.linalg.norm(q - tx) + np.linalg.norm(rx - q))) < 1e-5
        g = edge_geometry(torch.tensor(tx), torch.tensor(q), torch.tensor(rx), torch.tensor(e),
                          torch.tensor(n0))
        # Keller's cone (to the float32 rounding of the stored point)
        assert abs(float(g["s_in"] @ torch.tensor(e)) - float(g["s_out"] @ torch.tensor(e))) < 1e-5
        assert 0 < g["phi_p"].item() < 1.5 * math.pi and 0 < g["phi"].item() < 1.5 * math.pi
        # face 0 lies along n0 x e from the corner
        t0 = np.cross(n0, e)
        assert abs(abs(t0[0]) + abs(t0[1]) - 1) < 1e-6 and abs(t0[2]) < 1e-6
        assert st.mat[p] == st.mat_n[p]


def test_merge_links_keeps_order(floor):
    _, spec, st = floor
    assert st.n_links == spec.n_links
    for l in range(spec.n_links):
        a0, a1 = spec.link_off[l], spec.link_off[l + 1]
        b0 = st.link_off[l]
        n = a1 - a0
        assert np.array_equal(st.tau[b0:b0 + n], spec.tau[a0:a1])
        assert np.array_equal(st.depth[b0:b0 + n], spec.depth[a0:a1])
        for k in range(spec.max_depth):
            assert np.array_equal(st.pts[:, k * st.n_paths + b0:k * st.n_paths + b0 + n],
                                  spec.pts[:, k * spec.n_paths + a0:k * spec.n_paths + a1])
    m = merge_links(spec, spec)
    assert m.n_paths == 2 * spec.n_paths and m.edge is None

"""The urban block and its open-sky path and visibility search.

The large-scene workload is a procedural block (box buildings on a
tessellated ground, Tx at street crossings below every roof).  The native
finder treats it as a 2.5-D plan under open sky; these tests check that
reading against exhaustive 3-D geometry on small blocks: every specular path
of the image method over the full triangle scene (roofs included), and the
exact 3-D segment tests for the diffuse samples."""
import numpy as np
import pytest

from synth import imagemethod
from synth.diffuse import _same_side, visible_triangles
from synth.pathfind import find_store, visible_samples
from synth.urban import outdoor_rx, rx_grid, sample_surfaces, transmitters, urban_block


def _small_block(seed):
    # one city block of a few buildings, a single ground quad (target_tris=0)
    return urban_block(seed, size=60.0, street_w=(8.0, 10.0), block=(20.0, 30.0),
                       min_lot=10.0, target_tris=0)


def _path_set(st, link):
    out = set()
    P = st.n_paths
    for p in range(st.link_off[link], st.link_off[link + 1]):
        q = int(st.depth[p])
        faces = tuple(int(st.face[k * P + p]) for k in range(q))
        out.add((q, faces, round(float(st.tau[p]) * 299792458.0, 6)))
    return out


def test_urban_block_recipe():
    plan = urban_block(11)
    assert abs(plan.scene.n_tri - 100_000) <= 1000
    assert plan.scene.n_mat == 16
    assert len(np.unique(plan.scene.face_mat)) == 16
    assert plan.width == plan.depth == 400.0
    assert plan.box_height.min() >= 15.0 and plan.box_height.max() <= 45.0
    # buildings do not overlap and stay inside the block
    b = plan.boxes
    assert (b[:, 0] >= 0).all() and (b[:, 2] <= 400).all()
    ov = ((b[:, None, 0] < b[None, :, 2]) & (b[None, :, 0] < b[:, None, 2]) &
          (b[:, None, 1] < b[None, :, 3]) & (b[None, :, 1] < b[:, None, 3]))
    assert ov.sum() == len(b)
    tx = transmitters(plan, 4)
    assert tx.shape == (4, 3) and (tx[:, 2] == 10.0).all()
    assert plan.free(tx[:, 0], tx[:, 1], margin=2.0).all()
    assert (tx[:, 2] < plan.box_height.min()).all()
    g = rx_grid(plan)
    assert g.shape == (65_536, 3) and (g[:, 2] == 1.5).all()
    assert np.allclose(np.diff(np.unique(g[:, 0])), 400.0 / 256)
    rx = outdoor_rx(plan, np.random.default_rng(0), 2048)
    assert len(rx) == 2048 and plan.free(rx[:, 0], rx[:, 1], margin=0.3).all()


@pytest.mark.parametrize("seed,depth", [(3, 2), (5, 3)])
def test_open_sky_finder_matches_exhaustive(seed, depth):
    plan = _small_block(seed)
    assert len(plan.boxes) >= 2
    tx = transmitters(plan, 1)[0]
    rx = outdoor_rx(plan, np.random.default_rng(seed), 3)
    st = find_store(plan, tx, rx, depth, n_rays=1 << 16)
    ref = imagemethod.find_store(plan.scene, tx, rx, depth)
    for l in range(len(rx)):
        a, b = _path_set(st, l), _path_set(ref, l)
        assert a == b, (l, sorted(a ^ b)[:5])
    assert st.n_paths == ref.n_paths
    # the block has both ground and facade reflections
    assert (st.depth >= 1).any()


@pytest.mark.parametrize("cell", [1.0, 4.0])
def test_native_diffuse_visibility_matches_3d(cell):
    plan = _small_block(7)
    tx = transmitters(plan, 1)[0]
    rx = outdoor_rx(plan, np.random.default_rng(1), 4)
    pts, nrm, mat, face, dA, seg = sample_surfaces(plan, 0.3, np.random.default_rng(2))
    # facades only up to the Tx height; ground samples are outside every building
    assert pts[seg >= 0, 2].max() <= 10.0
    assert plan.free(pts[seg < 0, 0], pts[seg < 0, 1], margin=0.0).all()
    off, idx = visible_samples(plan, tx, rx, pts, nrm, seg, cell=cell)
    n = len(pts)
    vis_tx = visible_triangles(plan.scene, pts, face, tx)
    total = 0
    for r in range(len(rx)):
        want = (_same_side(pts, nrm, np.repeat(tx[None], n, 0), np.repeat(rx[r][None], n, 0)) &
                (np.einsum("ij,ij->i", tx[None] - pts, nrm) > 0) & vis_tx &
                visible_triangles(plan.scene, pts, face, rx[r]))
        got = np.zeros(n, bool)
        got[idx[off[r]:off[r + 1]]] = True
        assert (got == want).all(), (r, np.nonzero(got != want)[0][:5])
        total += int(want.sum())
    assert total > 100


def test_surface_samples_cover_their_area():
    plan = _small_block(7)
    pts, nrm, mat, face, dA, seg = sample_surfaces(plan, 0.5, np.random.default_rng(0))
    fac = seg >= 0
    want_fac = sum(2 * ((x1 - x0) + (y1 - y0)) * min(h, 10.0)
                   for (x0, y0, x1, y1), h in zip(plan.boxes, plan.box_height))
    assert np.isclose(dA[fac].sum(), want_fac, rtol=1e-12)
    # normals point out of their building; facade samples carry its material
    c = 0.5 * (plan.boxes[:, :2] + plan.boxes[:, 2:])
    b = seg[fac] // 4
    assert (np.einsum("ij,ij->i", pts[fac, :2] - c[b], nrm[fac, :2]) > 0).all()
    assert (mat[fac] == plan.box_mat[b]).all()
    assert (mat[~fac] == 0).all() and (nrm[~fac] == [0, 0, 1]).all()

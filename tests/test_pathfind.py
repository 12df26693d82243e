"""The native 2.5-D path finder returns exactly the specular paths the
exhaustive image method finds (same face sequences, same lengths) on small
floors with interior walls, door gaps and pillars."""
import numpy as np
import pytest

from synth import imagemethod
from synth.floorplan import indoor_floor
from synth.pathfind import find_store


def _path_set(st, link):
    out = set()
    P = st.n_paths
    for p in range(st.link_off[link], st.link_off[link + 1]):
        q = int(st.depth[p])
        faces = tuple(int(st.face[k * P + p]) for k in range(q))
        out.add((q, faces, round(float(st.tau[p]) * 299792458.0, 7)))
    return out


@pytest.mark.parametrize("seed,depth,n_rx", [(4, 2, 6), (5, 3, 2)])
def test_native_finder_matches_exhaustive(seed, depth, n_rx):
    plan = indoor_floor(seed, width=12.0, depth=9.0, min_room=4.0, max_rooms=2,
                        open_frac=0.4, door_w=(1.0, 2.0), n_pillars=1,
                        pillar_w=(0.6, 0.6), target_tris=0)
    rng = np.random.default_rng(seed)
    tx = plan.sample_points(rng, 1, 2.4, 2.6)[0]
    rx = plan.sample_points(rng, n_rx, 1.0, 2.0)
    st = find_store(plan, tx, rx, depth, n_rays=1 << 16)
    ref = imagemethod.find_store(plan.scene, tx, rx, depth)
    for l in range(n_rx):
        a, b = _path_set(st, l), _path_set(ref, l)
        assert a == b, (l, sorted(a ^ b)[:5])
    assert st.n_paths == ref.n_paths


def test_scale_floor_recipe():
    plan = indoor_floor(3, max_rooms=2, open_frac=0.7, n_pillars=0)
    assert abs(plan.scene.n_tri - 5000) <= 100
    assert plan.scene.n_mat == 10
    # walls are 0.2 m thick boxes spanning floor to ceiling
    th = np.minimum(plan.boxes[:, 2] - plan.boxes[:, 0], plan.boxes[:, 3] - plan.boxes[:, 1])
    assert np.allclose(th, 0.2)

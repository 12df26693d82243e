"""Single-bounce diffuse path generation (geometry only)."""
import numpy as np

from synth import diffuse
from synth.floorplan import indoor_floor
from synth.imagemethod import find_store
from synth.scene import box_room, uniform_points_in_box


def test_box_room_every_sample_is_a_path():
    rng = np.random.default_rng(0)
    sc = box_room()
    tx = uniform_points_in_box(rng, 1, sc.aabb_min, sc.aabb_max)[0]
    rxs = uniform_points_in_box(rng, 5, sc.aabb_min, sc.aabb_max)
    spec = find_store(sc, tx, rxs, 2, geom_dtype=np.float64)
    samples = diffuse.sample_triangles(sc, 3, rng)
    st = diffuse.add_diffuse(spec, tx, samples,
                             lambda p, e: diffuse.visible_triangles(sc, p, samples[3], e)
                             if len(p) == len(samples[0]) else np.ones(len(p), bool))
    cnt = st.paths_per_link()
    assert np.all(cnt == spec.paths_per_link() + 36)
    # the total area of the room's surfaces is split over the samples
    area = 2 * (10 * 8 + 10 * 3 + 8 * 3)
    for l in range(st.n_links):
        sel = np.arange(st.link_off[l], st.link_off[l + 1])
        dif = sel[st.kind[sel] == 1]
        assert len(dif) == 36 and np.all(st.depth[dif] == 1)
        assert abs(st.dA[dif].astype(np.float64).sum() - area) < 1e-4  # dA is FP32
        s = st.pts[:, dif].T
        L = np.linalg.norm(s - tx, axis=1) + np.linalg.norm(rxs[l] - s, axis=1)
        assert np.allclose(st.tau[dif] * 299792458.0, L, rtol=1e-14)
    # the specular part is unchanged
    for l in range(st.n_links):
        a = np.arange(spec.link_off[l], spec.link_off[l + 1])
        b = np.arange(st.link_off[l], st.link_off[l] + len(a))
        assert np.array_equal(spec.tau[a], st.tau[b])


def test_floor_footprint_visibility_matches_triangle_test():
    plan = indoor_floor(5, width=20.0, depth=14.0, max_rooms=3, n_pillars=2, target_tris=600)
    rng = np.random.default_rng(1)
    pts, nrm, mat, face, dA = diffuse.sample_floor(plan, 0.3, rng)
    ends = plan.sample_points(rng, 6, 1.0, 2.0)
    sel = rng.choice(len(pts), 150, replace=False)
    for e in ends:
        fast = diffuse.visible_floor(plan, pts[sel], e)
        exact = diffuse.visible_triangles(plan.scene, pts[sel], face[sel], e)
        assert np.array_equal(fast, exact)

"""Pins of the oracle's per-path field computation: Friis free space,
image theory over a perfect ground, the two-ray model, reciprocity and the
box-room image lattice."""
import math

import numpy as np
import pytest
import torch

from oracle import em
from oracle.trace import trace_fields, trace_fields_per_id
from synth import imagemethod
from synth.scene import box_room, uniform_points_in_box
from tests.helpers import ground_plane, single_path_store

f64 = torch.float64
FC = 3.5e9
LAM = 299792458.0 / FC


def _mats(store, eps, sig, s=0.0):
    D, P = store.max_depth, store.n_paths
    mk = lambda v: torch.full((D, P), v, dtype=f64)
    return mk(eps), mk(sig), mk(s)


@pytest.mark.parametrize("zeta,sign", [(0.0, 1.0), (math.pi / 2, -1.0)])
def test_friis_line_of_sight(zeta, sign):
    rng = np.random.default_rng(3)
    for _ in range(10):
        tx = rng.uniform(-5, 5, 3)
        rx = rng.uniform(-5, 5, 3)
        st = single_path_store(np.zeros((0, 3)), tx, rx, np.zeros((0, 3)))
        d = np.linalg.norm(np.float32(rx).astype(np.float64) - np.float32(tx).astype(np.float64))
        a, _ = trace_fields(st, *_mats(st, 2.0, 0.1), FC, zeta_tx=zeta, zeta_rx=zeta)
        # tau is the exact FP64 length / c
        d_tau = st.tau[0] * em.C0
        assert abs(a[0].item() - sign * LAM / (4 * math.pi * d_tau)) < 1e-12 * LAM / d_tau
        assert abs(d - d_tau) < 1e-5


def _two_ray_store(ht, hr, dist, max_depth=1):
    tx = np.array([0.0, 0.0, ht])
    rx = np.array([dist, 0.0, hr])
    scene = ground_plane()
    st = imagemethod.find_store(scene, tx, [rx], max_depth)
    return st


@pytest.mark.parametrize("zeta", [0.0, math.pi / 2])
def test_image_theory_perfect_ground(zeta):
    """Over a perfect conductor the ground acts as an image source:
    a vertically polarised isotropic source has an image of the same
    polarisation, a horizontally polarised one an image of opposite sign.
    With the Rx basis on the arriving direction this gives
    V: lam/4pi (e1/d1 + e2/d2),  H: -lam/4pi (e1/d1 - e2/d2)."""
    for ht, hr, dist in ((2.0, 1.5, 10.0), (7.0, 1.0, 3.0), (1.0, 9.0, 40.0)):
        st = _two_ray_store(ht, hr, dist)
        assert st.n_paths == 2
        a, _ = trace_fields(st, *_mats(st, 1.0, 1e15), FC, zeta_tx=zeta, zeta_rx=zeta)
        d1 = st.tau[0] * em.C0
        d2 = st.tau[1] * em.C0
        assert abs(d2 - math.hypot(dist, ht + hr)) < 1e-9
        if zeta == 0.0:
            ref = [LAM / (4 * math.pi * d1), LAM / (4 * math.pi * d2)]
        else:
            ref = [-LAM / (4 * math.pi * d1), LAM / (4 * math.pi * d2)]
        # sigma = 1e15 leaves r_par - 1 ~ 1e-8, and the stored FP32 points
        # perturb the directions by ~1e-7
        for i in range(2):
            assert abs(a[i].item() - ref[i]) < 1e-6 * abs(ref[i])


def test_two_ray_finite_ground():
    """Two-ray model with a lossy ground: the reflected path carries the TM
    coefficient for vertical and the TE coefficient for horizontal
    polarisation at the grazing geometry's incidence angle."""
    eps, sig = 5.24, 0.121
    for zeta in (0.0, math.pi / 2):
        for ht, hr, dist in ((2.0, 1.5, 10.0), (25.0, 1.5, 200.0)):
            st = _two_ray_store(ht, hr, dist)
            a, _ = trace_fields(st, *_mats(st, eps, sig, 0.3), FC, zeta_tx=zeta, zeta_rx=zeta)
            d2 = math.hypot(dist, ht + hr)
            cos_i = (ht + hr) / d2
            eta = eps - 1j * sig / (em.EPS0 * 2 * math.pi * FC)
            root = np.sqrt(eta - (1 - cos_i ** 2))
            r_perp = (cos_i - root) / (cos_i + root)
            r_par = (eta * cos_i - root) / (eta * cos_i + root)
            R = math.sqrt(1 - 0.3 ** 2)
            if zeta == 0.0:
                ref = LAM / (4 * math.pi * d2) * R * r_par
            else:
                ref = -LAM / (4 * math.pi * d2) * R * r_perp
            # incidence angle from the exact geometry, the oracle's from the
            # FP32-stored reflection point
            assert abs(a[1].item() - ref) < 1e-6 * abs(ref)
            # grazing limit: the ground path tends to minus the direct path
    # (r_par + 1 ~ 2 eta cos / sqrt(eta - 1) ~ 3e-3 at this geometry)
    st = _two_ray_store(0.5, 0.5, 1800.0)
    a, _ = trace_fields(st, *_mats(st, eps, sig), FC)
    assert abs(a[1].item() / a[0].item() + 1) < 5e-3


def _reverse_store(st):
    """Same geometric paths with Tx and Rx swapped (interaction order
    reversed)."""
    from synth.store import pack
    recs = []
    P = st.n_paths
    for p in range(P):
        q = int(st.depth[p])
        idx = [k * P + p for k in range(q)][::-1]
        recs.append(dict(points=st.pts[:, idx].T.astype(np.float64),
                         normals=st.nrm[:, idx].T.astype(np.float64),
                         mats=[int(st.mat[i]) for i in idx], faces=[0] * q,
                         kinds=[0] * q, dA=[0.0] * q, length=st.tau[p] * em.C0))
    return pack([recs], [st.rx_pos[0]], [st.tx_pos[0]], st.max_depth, geom_dtype=np.float64)


@pytest.mark.parametrize("zt,zr", [(0.0, 0.0), (0.3, 1.1), (math.pi / 2, 0.4)])
def test_reciprocity(zt, zr):
    rng = np.random.default_rng(7)
    scene = box_room()
    tx, rx = uniform_points_in_box(rng, 2, scene.aabb_min, scene.aabb_max)
    # exact (float64) geometry: with FP32-rounded points the path is only
    # specular to ~1e-7 and reciprocity holds only to that level
    st = imagemethod.find_store(scene, tx, [rx], 2, geom_dtype=np.float64)
    rev = _reverse_store(st)
    m = _mats(st, 4.1, 0.05, 0.2)
    a_fwd, _ = trace_fields(st, *m, FC, zeta_tx=zt, zeta_rx=zr)
    a_rev, _ = trace_fields(rev, *m, FC, zeta_tx=zr, zeta_rx=zt)
    assert torch.allclose(a_fwd, a_rev, rtol=1e-12, atol=0)


def test_box_room_path_count_and_image_lattice():
    """A convex box at depth <= 2 has 1 + 6 + 18 = 25 paths for a generic
    Tx/Rx pair, and every path length equals the distance from the Rx to
    a point of the reflection lattice of the Tx."""
    rng = np.random.default_rng(11)
    scene = box_room()
    L = np.array([10.0, 8.0, 3.0])
    for _ in range(10):
        tx, rx = uniform_points_in_box(rng, 2, scene.aabb_min, scene.aabb_max)
        st = imagemethod.find_store(scene, tx, [rx], 2)
        assert st.n_paths == 25
        lattice = []
        for ix in range(-2, 3):
            for iy in range(-2, 3):
                for iz in range(-2, 3):
                    orders = abs(ix) + abs(iy) + abs(iz)
                    if orders > 2:
                        continue
                    img = []
                    for ax, i in enumerate((ix, iy, iz)):
                        # reflection lattice of [0, L]: |i| reflections give
                        # x + i L (i even) or (i + 1) L - x (i odd)
                        img.append(tx[ax] + i * L[ax] if i % 2 == 0 else (i + 1) * L[ax] - tx[ax])
                    lattice.append(np.linalg.norm(np.array(img) - rx))
        lengths = np.sort(st.tau * em.C0)
        assert np.allclose(lengths, np.sort(lattice), rtol=0, atol=1e-9)


def test_per_id_mode_equals_explicit_materials():
    rng = np.random.default_rng(5)
    scene = box_room()
    tx, rx = uniform_points_in_box(rng, 2, scene.aabb_min, scene.aabb_max)
    st = imagemethod.find_store(scene, tx, [rx], 2)
    raw = torch.tensor([[1.2, -3.0, -0.5]], dtype=f64)
    a1, _ = trace_fields_per_id(st, raw, FC)
    eps, sig, s = em.materials_from_raw(raw)
    a2, _ = trace_fields(st, *_mats(st, eps.item(), sig.item(), s.item()), FC)
    assert torch.allclose(a1, a2, rtol=1e-14, atol=0)

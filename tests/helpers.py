"""Shared test fixtures: tiny scenes and path stores built from explicit
geometry, and the workload stores of the tiny configuration."""
import functools

import numpy as np

from synth import imagemethod
from synth.params import Radio, draw_gains, draw_materials, materials_to_raw
from synth.scene import SceneBuilder, box_room, uniform_points_in_box
from synth.store import KIND_SPECULAR, pack


def ground_plane(size=1000.0, z=0.0, mat=0):
    b = SceneBuilder()
    s = size
    b.add_quad((-s, -s, z), (s, -s, z), (s, s, z), (-s, s, z), mat=mat)
    return b.build(n_mat=1)


def single_path_store(points, tx, rx, normals, mats=None, max_depth=None):
    """Store with one link holding one path through the given points."""
    points = np.asarray(points, np.float64).reshape(-1, 3)
    q = len(points)
    mats = [0] * q if mats is None else mats
    chain = [np.asarray(tx, np.float64)] + list(points) + [np.asarray(rx, np.float64)]
    length = sum(float(np.linalg.norm(chain[j + 1] - chain[j])) for j in range(len(chain) - 1))
    rec = dict(points=points, normals=np.asarray(normals, np.float64).reshape(-1, 3),
               mats=mats, faces=list(range(q)), kinds=[KIND_SPECULAR] * q,
               dA=[0.0] * q, length=length)
    return pack([[rec]], [tx], [rx], q if max_depth is None else max_depth)


@functools.lru_cache(maxsize=None)
def tiny_workload(seed=1234, n_rx=64, n_sc=256, max_depth=2):
    """Box room 10x8x3 m, one material, Tx at a seeded point, n_rx Rx
    uniform inside (0.5 m margin), specular paths up to max_depth."""
    rng = np.random.default_rng(seed)
    scene = box_room()
    tx = uniform_points_in_box(rng, 1, scene.aabb_min, scene.aabb_max)[0]
    rxs = uniform_points_in_box(rng, n_rx, scene.aabb_min, scene.aabb_max)
    store = imagemethod.find_store(scene, tx, rxs, max_depth)
    eps_r, sigma, s = draw_materials(rng, 1, with_scattering=False)
    raw = materials_to_raw(eps_r, sigma, s)
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=n_sc, n_elem=1)
    g = np.ones(1, np.complex64)
    return scene, store, raw, radio, g

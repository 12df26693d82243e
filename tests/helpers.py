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


def ragged_subset(store, rng, keep_prob=0.7, empty_every=7):
    """Drop paths at random (every `empty_every`-th link loses all of them)
    to make odd and zero path counts; the result is still a valid store."""
    from synth.store import PathStore
    cnt = store.paths_per_link()
    keep_links = []
    sel = []
    for l in range(store.n_links):
        idx = np.arange(store.link_off[l], store.link_off[l + 1])
        if l % empty_every == 3:
            idx = idx[:0]
        else:
            idx = idx[rng.random(len(idx)) < keep_prob]
        sel.append(idx)
    sel_all = np.concatenate(sel)
    off = np.zeros(store.n_links + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in sel])
    P, D = store.n_paths, store.max_depth
    Pn = int(off[-1])
    idx = (np.arange(D)[:, None] * P + sel_all[None, :]).reshape(-1)
    return PathStore(n_links=store.n_links, n_paths=Pn, max_depth=D, link_off=off,
                     tx_pos=store.tx_pos.copy(), rx_pos=store.rx_pos.copy(),
                     depth=store.depth[sel_all].copy(), kind=store.kind[idx].copy(),
                     pts=store.pts[:, idx].copy(), nrm=store.nrm[:, idx].copy(),
                     mat=store.mat[idx].copy(), dA=store.dA[idx].copy(),
                     tau=store.tau[sel_all].copy(), face=store.face[idx].copy())


@functools.lru_cache(maxsize=None)
def array_workload(seed=99, n_rx=48, n_sc=1024, n_elem=32, max_depth=2, n_mat=1):
    """Box room with a Tx ULA: n_elem elements, n_sc subcarriers."""
    rng = np.random.default_rng(seed)
    scene = box_room()
    tx = uniform_points_in_box(rng, 1, scene.aabb_min, scene.aabb_max)[0]
    rxs = uniform_points_in_box(rng, n_rx, scene.aabb_min, scene.aabb_max)
    store = imagemethod.find_store(scene, tx, rxs, max_depth)
    eps_r, sigma, s = draw_materials(rng, n_mat, with_scattering=True)
    raw = materials_to_raw(eps_r, sigma, s)
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=n_sc, n_elem=n_elem,
                  ula_axis=(0.6, 0.8, 0.0))
    g = draw_gains(rng, n_elem)
    return scene, store, raw, radio, g


def multi_material_box_scene(n_mat=3):
    """Box room whose six faces carry material ids f % n_mat."""
    scene = box_room()
    scene.face_mat = (np.arange(scene.n_face) % n_mat).astype(np.int32)
    scene.n_mat = n_mat
    return scene


def multi_material_box(seed=5, n_rx=16, n_mat=3, max_depth=3):
    """Box room whose six faces carry material ids f % n_mat."""
    rng = np.random.default_rng(seed)
    scene = multi_material_box_scene(n_mat)
    tx = uniform_points_in_box(rng, 1, scene.aabb_min, scene.aabb_max)[0]
    rxs = uniform_points_in_box(rng, n_rx, scene.aabb_min, scene.aabb_max)
    store = imagemethod.find_store(scene, tx, rxs, max_depth)
    eps_r, sigma, s = draw_materials(rng, n_mat, with_scattering=True)
    return store, materials_to_raw(eps_r, sigma, s)

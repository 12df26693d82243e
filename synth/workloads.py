"""Named synthetic workloads (seeded).

  tiny      box room 10 x 8 x 3 m, one material, Tx at a seeded point,
            64 Rx, specular depth <= 2, 256 subcarriers over 50 MHz,
            single isotropic Tx antenna
  scale     indoor floor 60 x 40 x 3 m (~5,000 triangles, 10 material
            classes: floor, ceiling, four exterior sides, four interior wall
            types), Tx at 2.5 m near the centre with a 32-element
            half-wavelength ULA along x, 16,384 Rx at 1-2 m height,
            specular depth <= 5, 1,024 subcarriers over 50 MHz at 3.5 GHz
  diffuse   the scale floor with 2,048 Rx: specular paths up to fifth order
            plus single-bounce Lambertian diffuse paths from stratified
            surface samples (~0.35 per m^2), ~2,000 paths per link; 4,096
            subcarriers over 100 MHz at 3.5 GHz, 32-element ULA
  recovery  stand-in for the synthetic dataset of Sec. IV-B: a straight
            hallway 24 x 6 x 3 m (floor, walls and ceiling as three
            materials) with a 1.2 m square pillar of the wall material, one
            Rx antenna near one end at 2 m, 256 Tx at random points;
            specular paths up to third order, single-bounce diffuse paths
            from ~1 sample per m^2 of surface and first-order diffraction at
            the pillar's corners; 1,024
            subcarriers over 50 MHz at 3.438 GHz; ground truth of Table I
            with the backscattering-lobe pattern (alpha_r = 5, alpha_s = 8,
            Lambda = 0.8) and a three-lobe Tx gain
  adjoint   the scale floor and paths with hidden ground truth:
            materials with S ~ U[0, 0.5] and 32 complex element gains;
            14,336 training / 2,048 held-out Rx
  urban     the large-scene configuration's scene: a procedural urban block
            400 x 400 m (~100,000 triangles: box buildings 15-45 m tall on a
            tessellated ground plane, 16 material classes), 4 Tx at street
            crossings at 10 m, each with a 32-element ULA, n_rx Rx at 1.5 m
            (65,536 at full size): outdoor points of a 512 x 512 grid;
            specular paths up to fifth order plus single-bounce Lambertian
            diffuse paths from facade (up to 10 m) and ground samples, ~2,000
            paths per link; 4,096 subcarriers over 100 MHz at 3.5 GHz.  One
            path store per Tx and batch of Rx (the streaming batches).
"""
from dataclasses import dataclass, field

import numpy as np

from . import diffuse as _diffuse
from . import imagemethod
from .floorplan import indoor_floor
from .params import Radio, draw_gains, draw_materials, materials_to_raw
from .pathfind import find_store, visible_samples
from .scene import SceneBuilder, box_room, uniform_points_in_box
from .store import PathStore

# Floor recipe of the scale workload: two rooms with wide openings.  With
# specular paths up to fifth order (the order the paper traces for its
# measured indoor scene) this gives ~185 paths per link on average.
SCALE_FLOOR = dict(max_rooms=2, open_frac=0.7, n_pillars=0)
SCALE_DEPTH = 5


@dataclass
class Workload:
    name: str
    store: PathStore
    radio: Radio
    raw: np.ndarray          # float32 [n_mat, 3] ground-truth raw material parameters
    g: np.ndarray            # complex64 [n_elem] ground-truth element gains
    aabb: tuple = None       # (min [3], max [3]) of the scene
    meta: dict = field(default_factory=dict)


def tiny(seed=1234, n_rx=64, n_sc=256, max_depth=2) -> Workload:
    rng = np.random.default_rng(seed)
    scene = box_room()
    tx = uniform_points_in_box(rng, 1, scene.aabb_min, scene.aabb_max)[0]
    rxs = uniform_points_in_box(rng, n_rx, scene.aabb_min, scene.aabb_max)
    store = imagemethod.find_store(scene, tx, rxs, max_depth)
    raw = materials_to_raw(*draw_materials(rng, 1, with_scattering=False))
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=n_sc, n_elem=1)
    return Workload("tiny", store, radio, raw, np.ones(1, np.complex64),
                    (scene.aabb_min, scene.aabb_max))


def _scale_geometry(seed, n_rx, max_depth, n_rays):
    plan = indoor_floor(seed, **SCALE_FLOOR)
    rng = np.random.default_rng(seed + 1)
    tx = np.array([plan.width / 2, plan.depth / 2, 2.5])
    while not plan.free(tx[0], tx[1], margin=0.3):
        tx[:2] += rng.uniform(-1.0, 1.0, 2)
    rx = plan.sample_points(rng, n_rx, 1.0, 2.0)
    store = find_store(plan, tx, rx, max_depth, n_rays=n_rays)
    return plan, store


def scale(seed=3, n_rx=16384, n_sc=1024, n_elem=32, max_depth=SCALE_DEPTH,
          n_rays=1 << 18) -> Workload:
    plan, store = _scale_geometry(seed, n_rx, max_depth, n_rays)
    rng = np.random.default_rng(seed + 2)
    n_mat = plan.scene.n_mat
    raw = materials_to_raw(*draw_materials(rng, n_mat, with_scattering=False))
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=n_sc, n_elem=n_elem, ula_axis=(1.0, 0.0, 0.0))
    return Workload("scale", store, radio, raw, np.ones(n_elem, np.complex64),
                    (plan.scene.aabb_min, plan.scene.aabb_max),
                    meta=dict(plan=plan, tris=plan.scene.n_tri, n_mat=n_mat))


def diffuse(seed=3, n_rx=2048, n_sc=4096, bandwidth=100e6, n_elem=32, max_depth=SCALE_DEPTH,
            n_rays=1 << 18, density=0.35) -> Workload:
    """Per-link shape of a large scene with diffuse scattering (~2,000 paths
    per link, 4,096 subcarriers) on the scale floor."""
    plan, spec = _scale_geometry(seed, n_rx, max_depth, n_rays)
    rng = np.random.default_rng(seed + 5)
    samples = _diffuse.sample_floor(plan, density, rng)
    tx = spec.tx_pos[0].astype(np.float64)
    store = _diffuse.add_diffuse(spec, tx, samples,
                                 lambda p, e: _diffuse.visible_floor(plan, p, e))
    n_mat = plan.scene.n_mat
    raw = materials_to_raw(*draw_materials(rng, n_mat, with_scattering=True))
    radio = Radio(fc=3.5e9, bandwidth=bandwidth, n_sc=n_sc, n_elem=n_elem,
                  ula_axis=(1.0, 0.0, 0.0))
    return Workload("diffuse", store, radio, raw, draw_gains(rng, n_elem),
                    (plan.scene.aabb_min, plan.scene.aabb_max),
                    meta=dict(plan=plan, n_mat=n_mat, n_samples=len(samples[0])))


def adjoint(seed=3, n_rx=16384, n_sc=1024, n_elem=32, max_depth=SCALE_DEPTH,
            n_rays=1 << 18, n_heldout=2048, geometry=None) -> Workload:
    """`geometry` = (plan, store) of the same seed reuses already traced
    paths (the scale workload's)."""
    plan, store = geometry if geometry is not None else _scale_geometry(seed, n_rx, max_depth,
                                                                        n_rays)
    n_rx = store.n_links
    rng = np.random.default_rng(seed + 3)
    n_mat = plan.scene.n_mat
    raw = materials_to_raw(*draw_materials(rng, n_mat, with_scattering=True))
    g = draw_gains(rng, n_elem)
    radio = Radio(fc=3.5e9, bandwidth=50e6, n_sc=n_sc, n_elem=n_elem, ula_axis=(1.0, 0.0, 0.0))
    perm = rng.permutation(n_rx)
    return Workload("adjoint", store, radio, raw, g, (plan.scene.aabb_min, plan.scene.aabb_max),
                    meta=dict(plan=plan, n_mat=n_mat, train=np.sort(perm[n_heldout:]),
                              heldout=np.sort(perm[:n_heldout])))


def spatial_field(store, plan, raw_base, seed, aabb):
    """Ground-truth per-interaction materials varying in space: per-class
    base values times smooth sinusoidal perturbations of three octaves,
        q(p) = sum_{o=0..2} 2^-o sin(2 pi 2^o 4 (u_o . p_bar) + phi_o)
        eps_r = 1 + (eps_base - 1) e^{0.3 q},  sigma = sigma_base e^{0.5 q},
        S = logistic(logit(S_base) + 0.5 q)
    with seeded unit vectors u_o and phases phi_o drawn independently per
    parameter; p_bar is the point normalised by the scene box.  Returns
    float32 [3, max_depth*n_paths] rows (eps_r, sigma, S)."""
    rng = np.random.default_rng(seed)
    lo, hi = (np.asarray(a, np.float64) for a in aabb)
    pts = store.pts.T.astype(np.float64)
    pbar = (pts - 0.5 * (lo + hi)) / np.max(hi - lo)
    ids = store.mat.astype(np.int64)
    eps_b = 1.0 + np.exp(raw_base[:, 0].astype(np.float64))
    sig_b = np.exp(raw_base[:, 1].astype(np.float64))
    lgt_b = raw_base[:, 2].astype(np.float64)
    qs = []
    for _ in range(3):
        q = np.zeros(len(pbar))
        for o in range(3):
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            phi = rng.uniform(0, 2 * np.pi)
            q += 2.0 ** (-o) * np.sin(2 * np.pi * 2 ** o * 4 * (pbar @ u) + phi)
        qs.append(q)
    eps = 1.0 + (eps_b[ids] - 1.0) * np.exp(0.3 * qs[0])
    sig = sig_b[ids] * np.exp(0.5 * qs[1])
    S = 1.0 / (1.0 + np.exp(-(lgt_b[ids] + 0.5 * qs[2])))
    return np.stack([eps, sig, S]).astype(np.float32)


def learned(seed=3, n_rx=16384, **kw) -> Workload:
    """The adjoint workload with a spatially varying ground-truth field."""
    w = adjoint(seed=seed, n_rx=n_rx, **kw)
    w.name = "learned"
    w.meta["per_inter"] = spatial_field(w.store, w.meta["plan"], w.raw, seed + 11, w.aabb)
    return w


# Table I of the paper: floor (concrete), walls (plasterboard), ceiling
# (ceiling board); columns eps_r, sigma [S/m], S, K_x.
TABLE_I = np.array([[5.24, 0.121, 0.3, 0.2],
                    [2.73, 0.027, 0.5, 0.4],
                    [1.48, 0.004, 0.8, 0.3]])
# Backscattering-lobe pattern of the synthetic dataset: alpha_r, alpha_s, Lambda
RECOVERY_LOBES = (5, 8, 0.8)
# Ground-truth Tx gain, a member of the trainable family (M = 3): radiation
# efficiency 0.9, weights (0.6, 0.25, 0.15), concentrations (6, 2, 10) and
# mean directions along the hallway, upwards and across it.
RECOVERY_TX = dict(eta=0.9, w=(0.6, 0.25, 0.15), lam=(6.0, 2.0, 10.0),
                   mu=((-1.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.6, 0.8, 0.0)))


def vmf_to_raw(eta, w, lam, mu):
    """Raw Tx-gain vector [1 + 5M] (logistic, softmax logits, log, 3-vectors)."""
    w = np.asarray(w, np.float64)
    mu = np.asarray(mu, np.float64)
    return np.concatenate([[np.log(eta / (1.0 - eta))], np.log(w), np.log(lam),
                           mu.reshape(-1)]).astype(np.float32)


def hallway_scene(size=(24.0, 6.0, 3.0), pillar=None):
    """Straight hallway [0,sx]x[0,sy]x[0,sz]: material 0 the floor, 1 the
    four walls, 2 the ceiling; optionally a floor-to-ceiling pillar (x0, y0,
    x1, y1) of the wall material, whose four vertical corners diffract."""
    b = SceneBuilder()
    b.add_box((0.0, 0.0, 0.0), size, 1)
    if pillar is not None:
        x0, y0, x1, y1 = pillar
        b.add_box((x0, y0, 0.0), (x1, y1, size[2]), 1, skip=("-z", "+z"))
    sc = b.build(n_mat=3)
    nz = sc.face_normal[:, 2]
    sc.face_mat = np.where(nz > 0.5, 0, np.where(nz < -0.5, 2, 1)).astype(np.int32)
    return sc


RECOVERY_PILLAR = (11.4, 2.4, 12.6, 3.6)


def recovery(seed=7, n_tx=256, size=(24.0, 6.0, 3.0), density=1.0, max_depth=3, n_sc=1024,
             fc=3.438e9, bandwidth=50e6, pillar=RECOVERY_PILLAR) -> Workload:
    from types import SimpleNamespace
    from . import diffract as _diffract
    rng = np.random.default_rng(seed)
    scene = hallway_scene(size, pillar)
    rx = np.array([1.0, size[1] / 2, 2.0])
    txs = np.stack([rng.uniform(0.5, size[0] - 0.5, n_tx), rng.uniform(0.5, size[1] - 0.5, n_tx),
                    rng.uniform(0.5, 2.5, n_tx)], 1)
    if pillar is not None:
        # no Tx inside or against the pillar
        x0, y0, x1, y1 = pillar
        inside = ((txs[:, 0] > x0 - 0.3) & (txs[:, 0] < x1 + 0.3) &
                  (txs[:, 1] > y0 - 0.3) & (txs[:, 1] < y1 + 0.3))
        txs[inside, 0] = np.where(txs[inside, 0] < 0.5 * (x0 + x1), x0 - 0.6, x1 + 0.6)
    links = [imagemethod.find_paths(scene, t, rx, max_depth) for t in txs]
    spec = imagemethod.pack(links, list(txs), [rx] * n_tx, max_depth)
    samples = _diffuse.sample_triangles_density(scene, density, rng)
    if pillar is None:
        # a convex room: every sample point sees every Tx and the Rx
        store = _diffuse.add_diffuse(spec, None, samples, lambda p, e: np.ones(len(p), bool))
    else:
        # the pillar spans floor to ceiling: a segment between interior points
        # is blocked exactly when its floor-plan projection enters the pillar;
        # its four vertical corners (wall material) diffract.  Its faces are
        # the scene's last four, in the order -x, +x, -y, +y.
        box = SimpleNamespace(boxes=np.asarray([pillar], np.float64), box_mat=np.array([1]),
                              box_face0=np.array([scene.n_face - 4]))
        store = _diffuse.add_diffuse(spec, None, samples,
                                     lambda p, e: _diffuse.visible_floor(box, p, e))
        store = _diffract.add_diffraction(store, box, _diffract.floor_edges(box))
    raw = materials_to_raw(TABLE_I[:, 0], TABLE_I[:, 1], TABLE_I[:, 2])
    radio = Radio(fc=fc, bandwidth=bandwidth, n_sc=n_sc, n_elem=1)
    meta = dict(kx=TABLE_I[:, 3].copy(), lobes=RECOVERY_LOBES, n_vmf=3,
                tx_raw=vmf_to_raw(**RECOVERY_TX), table=TABLE_I.copy(), pillar=pillar)
    return Workload("recovery", store, radio, raw, np.ones(1, np.complex64),
                    (scene.aabb_min, scene.aabb_max), meta)


def urban_store(plan, tx, rx, samples, max_depth=SCALE_DEPTH, n_rays=1 << 18):
    """The path store of one Tx and a set of Rx in the urban block: its
    specular paths, then the single-bounce diffuse paths through the
    surface samples (sample_surfaces' output) both ends see."""
    spec = find_store(plan, tx, rx, max_depth, n_rays=n_rays, cell=4.0)
    off, idx = visible_samples(plan, tx, rx, samples[0], samples[1], samples[5], cell=4.0)
    per_link = [idx[off[l]:off[l + 1]] for l in range(len(rx))]
    return _diffuse.append_diffuse(spec, np.repeat(np.asarray(tx, np.float64)[None], len(rx), 0),
                                   samples[:5], per_link)


def urban(seed=11, n_tx=4, n_rx=2048, n_sc=4096, bandwidth=100e6, n_elem=32,
          max_depth=SCALE_DEPTH, n_rays=1 << 18, density=0.65, grid=512, batch=None,
          lazy=False) -> Workload:
    """The urban block with n_tx transmitters and n_rx receivers, a seeded
    choice of the outdoor points of the grid x grid receiver grid at 1.5 m
    (the same for every Tx).  The links are cut into batches of `batch`
    receivers of one Tx (default: all n_rx), Tx-major.  meta["batch"](i)
    builds batch i's path store; unless lazy, meta["batches"] holds them all
    and store is the first."""
    from . import urban as _urban
    plan = _urban.urban_block(seed)
    tx = _urban.transmitters(plan, n_tx)
    rng = np.random.default_rng(seed + 1)
    rx = _urban.outdoor_rx(plan, rng, n_rx, grid)
    samples = _urban.sample_surfaces(plan, density, np.random.default_rng(seed + 2))
    n_mat = plan.scene.n_mat
    raw = materials_to_raw(*draw_materials(rng, n_mat, with_scattering=True))
    radio = Radio(fc=3.5e9, bandwidth=bandwidth, n_sc=n_sc, n_elem=n_elem,
                  ula_axis=(1.0, 0.0, 0.0))
    B = len(rx) if batch is None else int(batch)
    per_tx = (len(rx) + B - 1) // B

    def make(i):
        t, c = divmod(i, per_tx)
        return urban_store(plan, tx[t], rx[c * B:(c + 1) * B], samples, max_depth, n_rays)

    n_batches = n_tx * per_tx
    batches = None if lazy else [make(i) for i in range(n_batches)]
    return Workload("urban", None if lazy else batches[0], radio, raw, draw_gains(rng, n_elem),
                    (plan.scene.aabb_min, plan.scene.aabb_max),
                    meta=dict(plan=plan, batches=batches, batch=make, n_batches=n_batches,
                              tx=tx, rx=rx, n_mat=n_mat, n_samples=len(samples[0]),
                              tris=plan.scene.n_tri))

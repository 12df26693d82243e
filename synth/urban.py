"""Procedural urban block (2.5-D): seeded box buildings on a ground plane.

The square [0, S]^2 is cut into city blocks by streets along x and y
(seeded widths); every city block is split recursively into lots, each
lot a building separated from its neighbours by narrow alleys.  A building
is a closed box (four facades and a roof, one quad of two triangles each)
of seeded height; the ground is tessellated into tiles (coplanar faces of
the ground material) to make up the triangle budget.  Material classes: 0
the ground, 1 .. n_mat-1 facade types (one per building, its roof alike).

Paths are found by the native 2.5-D finder under open sky: with every
transmitter below the lowest roof, a path's height stays between 0 and the
Tx height (at most one ground reflection), so roofs are never reached and a
building blocks exactly by its footprint.
"""
from dataclasses import dataclass

import numpy as np

from .floorplan import FloorPlan
from .scene import SceneBuilder

GROUND = 0


@dataclass
class UrbanPlan(FloorPlan):
    box_height: np.ndarray = None  # [n_box] building heights (m)
    streets_x: np.ndarray = None   # centre lines of the streets along y (x values)
    streets_y: np.ndarray = None   # centre lines of the streets along x (y values)


def _cuts(rng, size, street_w, block):
    """Street and block intervals along one axis: street, block, street, ...,
    street, scaled to fill [0, size].  Returns (block intervals, street
    centre lines)."""
    parts = [rng.uniform(*street_w)]
    while True:
        b = rng.uniform(*block)
        s = rng.uniform(*street_w)
        if sum(parts) + b + s > size and len(parts) > 1:
            break
        parts += [b, s]
    parts = np.asarray(parts) * (size / sum(parts))
    edges = np.concatenate([[0.0], np.cumsum(parts)])
    blocks = [(edges[i], edges[i + 1]) for i in range(1, len(parts), 2)]
    streets = np.array([0.5 * (edges[i] + edges[i + 1]) for i in range(0, len(parts), 2)])
    return blocks, streets


def _lots(rng, x0, y0, x1, y1, min_lot, depth=0):
    """Recursive split of a city block into lots (rectangles)."""
    w, h = x1 - x0, y1 - y0
    if depth >= 4 or max(w, h) < 2 * min_lot or (depth >= 1 and rng.uniform() < 0.25):
        return [(x0, y0, x1, y1)]
    f = rng.uniform(0.3, 0.7)
    if w >= h:
        xm = x0 + f * w
        return (_lots(rng, x0, y0, xm, y1, min_lot, depth + 1) +
                _lots(rng, xm, y0, x1, y1, min_lot, depth + 1))
    ym = y0 + f * h
    return (_lots(rng, x0, y0, x1, ym, min_lot, depth + 1) +
            _lots(rng, x0, ym, x1, y1, min_lot, depth + 1))


def urban_block(seed, size=400.0, street_w=(10.0, 18.0), block=(40.0, 80.0), alley=(1.5, 3.0),
                min_lot=12.0, height=(15.0, 45.0), n_mat=16, target_tris=100_000) -> UrbanPlan:
    rng = np.random.default_rng(seed)
    bx, sx = _cuts(rng, size, street_w, block)
    by, sy = _cuts(rng, size, street_w, block)
    boxes = []
    for (x0, x1) in bx:
        for (y0, y1) in by:
            for (a0, b0, a1, b1) in _lots(rng, x0, y0, x1, y1, min_lot):
                # alleys: shrink the lot's sides that face another lot
                g = 0.5 * rng.uniform(*alley)
                a0 += g if a0 > x0 else 0.0
                a1 -= g if a1 < x1 else 0.0
                b0 += g if b0 > y0 else 0.0
                b1 -= g if b1 < y1 else 0.0
                boxes.append((a0, b0, a1, b1))
    boxes = np.asarray(boxes, np.float64)
    nb = len(boxes)
    box_mat = rng.integers(1, n_mat, nb).astype(np.int64)
    box_h = rng.uniform(*height, nb)
    # ground tiles to reach the triangle budget (10 triangles per building)
    n_tiles = max(1, (target_tris - 10 * nb) // 2)
    nt = max(1, int(round(np.sqrt(n_tiles))))
    b = SceneBuilder()
    box_face0 = np.zeros(nb, np.int64)
    for i, ((x0, y0, x1, y1), m, h) in enumerate(zip(boxes, box_mat, box_h)):
        box_face0[i] = b.add_quad((x0, y1, 0), (x0, y0, 0), (x0, y0, h), (x0, y1, h), int(m))
        b.add_quad((x1, y0, 0), (x1, y1, 0), (x1, y1, h), (x1, y0, h), int(m))
        b.add_quad((x0, y0, 0), (x1, y0, 0), (x1, y0, h), (x0, y0, h), int(m))
        b.add_quad((x1, y1, 0), (x0, y1, 0), (x0, y1, h), (x1, y1, h), int(m))
        b.add_quad((x0, y0, h), (x1, y0, h), (x1, y1, h), (x0, y1, h), int(m))
    floor_face = None
    for j in range(nt):
        for i in range(nt):
            u0, u1 = size * i / nt, size * (i + 1) / nt
            v0, v1 = size * j / nt, size * (j + 1) / nt
            f = b.add_quad((u0, v0, 0), (u1, v0, 0), (u1, v1, 0), (u0, v1, 0), GROUND)
            if floor_face is None:
                floor_face = f
    scene = b.build(n_mat=n_mat)
    return UrbanPlan(scene=scene, boxes=boxes, box_mat=box_mat, box_face0=box_face0, width=size,
                     depth=size, height=0.0, floor_face=int(floor_face), ceil_face=-1,
                     tiles=(nt, nt), box_height=box_h, streets_x=sx, streets_y=sy)


def transmitters(plan, n_tx=4, z=10.0):
    """Tx at street crossings: the crossing nearest to each of n_tx points
    spread over the block (quadrant centres for four)."""
    k = int(np.ceil(np.sqrt(n_tx)))
    out = []
    for t in range(n_tx):
        gx = plan.width * ((t % k) + 0.5) / k
        gy = plan.depth * ((t // k) + 0.5) / k
        x = plan.streets_x[np.argmin(np.abs(plan.streets_x - gx))]
        y = plan.streets_y[np.argmin(np.abs(plan.streets_y - gy))]
        out.append((x, y, z))
    return np.asarray(out, np.float64)


def rx_grid(plan, n=256, z=1.5):
    """The n x n receiver grid (cell centres) at height z: [n*n, 3]."""
    c = (np.arange(n) + 0.5) * (plan.width / n)
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(n * n, z)], 1)


def outdoor_rx(plan, rng, n_rx, grid=256, z=1.5, margin=0.3):
    """A seeded choice of n_rx grid receivers in free space (outside every
    building, margin m from its walls), in grid order."""
    g = rx_grid(plan, grid, z)
    free = np.nonzero(plan.free(g[:, 0], g[:, 1], margin))[0]
    pick = np.sort(rng.choice(free, min(n_rx, len(free)), replace=False))
    return g[pick]


def sample_surfaces(plan, density, rng, z_max=10.0):
    """Stratified jittered samples on every facade up to height z_max (the
    transmitters' height: every segment from such a point to a Tx or an Rx
    then stays below the lowest roof, so a building blocks it exactly by its
    footprint) and on the free ground, about `density` per square metre.
    Returns (pts, nrm, mat, face, dA, seg): seg is the facade's row in
    plan.wall_segments() (-1 on the ground)."""
    pts, nrm, mat, face, dA, seg = [], [], [], [], [], []

    def rect(origin, u, v, n, m, f, sg):
        lu, lv = np.linalg.norm(u), np.linalg.norm(v)
        nu = max(1, int(round(lu * np.sqrt(density))))
        nv = max(1, int(round(lv * np.sqrt(density))))
        iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
        fu = (iu + rng.uniform(size=iu.shape)) / nu
        fv = (iv + rng.uniform(size=iv.shape)) / nv
        p = origin + fu.reshape(-1, 1) * u + fv.reshape(-1, 1) * v
        pts.append(p)
        nrm.append(np.repeat(np.asarray(n, np.float64)[None], len(p), 0))
        mat.append(np.full(len(p), m))
        face.append(np.full(len(p), f))
        dA.append(np.full(len(p), lu * lv / (nu * nv)))
        seg.append(np.full(len(p), sg))

    for i, ((x0, y0, x1, y1), m, f0, h) in enumerate(zip(plan.boxes, plan.box_mat,
                                                         plan.box_face0, plan.box_height)):
        z = np.array([0.0, 0.0, min(h, z_max)])
        rect(np.array([x0, y0, 0.0]), np.array([0.0, y1 - y0, 0.0]), z, (-1, 0, 0), m, f0, 4 * i)
        rect(np.array([x1, y0, 0.0]), np.array([0.0, y1 - y0, 0.0]), z, (1, 0, 0), m, f0 + 1,
             4 * i + 1)
        rect(np.array([x0, y0, 0.0]), np.array([x1 - x0, 0.0, 0.0]), z, (0, -1, 0), m, f0 + 2,
             4 * i + 2)
        rect(np.array([x0, y1, 0.0]), np.array([x1 - x0, 0.0, 0.0]), z, (0, 1, 0), m, f0 + 3,
             4 * i + 3)
    nx, ny = plan.tiles
    # the ground in strips of tiles (one rect per tile row keeps the count of
    # arrays small); every point gets the tile face it falls in
    for j in range(ny):
        y0, y1 = plan.depth * j / ny, plan.depth * (j + 1) / ny
        rect(np.array([0.0, y0, 0.0]), np.array([plan.width, 0.0, 0.0]),
             np.array([0.0, y1 - y0, 0.0]), (0, 0, 1), GROUND, -1, -1)
    pts = np.concatenate(pts)
    nrm, mat, face, dA, seg = (np.concatenate(x) for x in (nrm, mat, face, dA, seg))
    g = face < 0
    face[g] = plan.tile_face(pts[g, 0], pts[g, 1], np.zeros(int(g.sum()), bool))
    # ground points under a building are not surfaces
    keep = ~g | plan.free(pts[:, 0], pts[:, 1], margin=0.0)
    return (pts[keep], nrm[keep], mat[keep].astype(np.int64), face[keep].astype(np.int64),
            dA[keep], seg[keep].astype(np.int32))

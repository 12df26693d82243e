"""Procedural indoor floor (2.5-D): seeded recursive rectangular rooms.

The floor plan [0, W] x [0, D] is closed by exterior wall boxes and split
recursively into rooms by interior walls: boxes spanning floor to ceiling,
cut by door gaps.  Square pillars stand in the rooms.  Every box is 12
triangles; floor and ceiling are tessellated into tiles (coplanar faces of
one material) to make up the triangle budget.

Material classes: 0 floor, 1 ceiling, 2..5 the four exterior wall sides,
6.. interior wall types (drawn per wall piece and per pillar).
"""
import heapq
from dataclasses import dataclass

import numpy as np

from .scene import Scene, SceneBuilder

FLOOR, CEILING, EXTERIOR = 0, 1, 2
N_EXTERIOR = 4


@dataclass
class FloorPlan:
    scene: Scene
    boxes: np.ndarray      # [n_box, 4] x0, y0, x1, y1
    box_mat: np.ndarray    # [n_box]
    box_face0: np.ndarray  # [n_box] face id of the box's first (-x) face
    width: float
    depth: float
    height: float
    floor_face: int        # face id of the first floor tile
    ceil_face: int         # face id of the first ceiling tile
    tiles: tuple = (1, 1)  # floor/ceiling tessellation (nx, ny)

    def tile_face(self, x, y, ceiling) -> np.ndarray:
        nx, ny = self.tiles
        i = np.clip((np.asarray(x) / self.width * nx).astype(np.int64), 0, nx - 1)
        j = np.clip((np.asarray(y) / self.depth * ny).astype(np.int64), 0, ny - 1)
        base = np.where(np.asarray(ceiling), self.ceil_face, self.floor_face)
        return base + j * nx + i

    def wall_segments(self) -> np.ndarray:
        """Vertical wall faces as [axis, c, lo, hi, nsign, mat, face] rows
        (axis 0: face on x = c; the face's outward normal is nsign along
        the axis)."""
        rows = []
        for (x0, y0, x1, y1), m, f0 in zip(self.boxes, self.box_mat, self.box_face0):
            rows.append((0, x0, y0, y1, -1.0, m, f0 + 0))
            rows.append((0, x1, y0, y1, +1.0, m, f0 + 1))
            rows.append((1, y0, x0, x1, -1.0, m, f0 + 2))
            rows.append((1, y1, x0, x1, +1.0, m, f0 + 3))
        return np.asarray(rows, np.float64)

    def free(self, x, y, margin=0.1) -> np.ndarray:
        """True where (x, y) lies in free space (not within margin of a box)."""
        x = np.asarray(x)[..., None]
        y = np.asarray(y)[..., None]
        b = self.boxes
        inside = ((x > b[:, 0] - margin) & (x < b[:, 2] + margin) &
                  (y > b[:, 1] - margin) & (y < b[:, 3] + margin))
        return ~inside.any(-1)

    def sample_points(self, rng, n, zlo, zhi, margin=0.1):
        out = np.zeros((0, 3))
        while len(out) < n:
            k = 2 * (n - len(out)) + 16
            x = rng.uniform(0, self.width, k)
            y = rng.uniform(0, self.depth, k)
            ok = self.free(x, y, margin)
            z = rng.uniform(zlo, zhi, k)
            out = np.concatenate([out, np.stack([x, y, z], 1)[ok]])
        return out[:n]


def indoor_floor(seed, width=60.0, depth=40.0, height=3.0, thickness=0.2, min_room=8.0,
                 max_rooms=6, door_w=(1.5, 4.0), open_frac=0.5, n_pillars=24,
                 pillar_w=(0.4, 0.8), n_interior_types=4, target_tris=5000,
                 grid=None) -> FloorPlan:
    """Seeded floor: exterior walls, up to `max_rooms` rectangular rooms made
    by recursive splits (largest region first, longer side, minimum side
    `min_room`) with interior walls `thickness` thick cut by door gaps
    (about `open_frac` of each wall's length), square pillars, and floor and
    ceiling tessellated into tiles so that the mesh has about `target_tris`
    triangles."""
    rng = np.random.default_rng(seed)
    t = thickness
    boxes, mats = [], []
    boxes += [(0, 0, t, depth), (width - t, 0, width, depth),
              (t, 0, width - t, t), (t, depth - t, width - t, depth)]
    mats += [EXTERIOR, EXTERIOR + 1, EXTERIOR + 2, EXTERIOR + 3]
    first_int = EXTERIOR + N_EXTERIOR

    def interior():
        return first_int + int(rng.integers(n_interior_types))

    def wall_pieces(a, b):
        """Intervals of [a, b] left after cutting door gaps."""
        L = b - a
        n_gaps = max(1, int(round(open_frac * L / np.mean(door_w))))
        gaps = []
        for _ in range(n_gaps * 8):
            if len(gaps) == n_gaps:
                break
            w = rng.uniform(*door_w)
            if w > L - 0.6:
                continue
            s0 = rng.uniform(a + 0.3, b - 0.3 - w)
            if all(s0 + w + 0.3 < g0 or s0 > g1 + 0.3 for g0, g1 in gaps):
                gaps.append((s0, s0 + w))
        gaps.sort()
        pieces, cur = [], a
        for g0, g1 in gaps:
            if g0 - cur > 0.3:
                pieces.append((cur, g0))
            cur = g1
        if b - cur > 0.3:
            pieces.append((cur, b))
        return pieces

    if grid is not None:
        # rooms on a jittered grid of cell size (gx, gy): every cell edge is
        # a wall segment with door gaps
        gx, gy = grid
        xs_w = np.arange(gx, width - gx / 2, gx) + rng.uniform(-0.15, 0.15, 1) * gx
        ys_w = np.arange(gy, depth - gy / 2, gy) + rng.uniform(-0.15, 0.15, 1) * gy
        xe = np.concatenate([[t], xs_w, [width - t]])
        ye = np.concatenate([[t], ys_w, [depth - t]])
        for xw in xs_w:
            for j in range(len(ye) - 1):
                for a, b in wall_pieces(ye[j] + t / 2, ye[j + 1] - t / 2):
                    boxes.append((xw - t / 2, a, xw + t / 2, b))
                    mats.append(interior())
        for yw in ys_w:
            for i in range(len(xe) - 1):
                for a, b in wall_pieces(xe[i] + t / 2, xe[i + 1] - t / 2):
                    boxes.append((a, yw - t / 2, b, yw + t / 2))
                    mats.append(interior())
        max_rooms = 1
    n_rooms = 1
    heap = [(-(width - 2 * t) * (depth - 2 * t), (t, t, width - t, depth - t))]
    while heap and n_rooms < max_rooms:
        _, (x0, y0, x1, y1) = heapq.heappop(heap)
        w, h = x1 - x0, y1 - y0
        split_x = w >= h
        span = w if split_x else h
        if span < 2 * min_room + t:
            continue
        lo = (x0 if split_x else y0) + min_room + t / 2
        hi = (x1 if split_x else y1) - min_room - t / 2
        sp = rng.uniform(lo, hi)
        if split_x:
            new = [(sp - t / 2, a, sp + t / 2, b) for a, b in wall_pieces(y0, y1)]
            kids = [(x0, y0, sp - t / 2, y1), (sp + t / 2, y0, x1, y1)]
        else:
            new = [(a, sp - t / 2, b, sp + t / 2) for a, b in wall_pieces(x0, x1)]
            kids = [(x0, y0, x1, sp - t / 2), (x0, sp + t / 2, x1, y1)]
        boxes += new
        mats += [interior() for _ in new]
        n_rooms += 1
        for k in kids:
            heapq.heappush(heap, (-(k[2] - k[0]) * (k[3] - k[1]), k))
    placed, tries = 0, 0
    while placed < n_pillars and tries < 100000:
        tries += 1
        a = rng.uniform(*pillar_w) / 2
        px, py = rng.uniform(1.0, width - 1.0), rng.uniform(1.0, depth - 1.0)
        p = (px - a, py - a, px + a, py + a)
        b_arr = np.asarray(boxes)
        clear = ~(((p[0] - 1.0) < b_arr[:, 2]) & ((p[2] + 1.0) > b_arr[:, 0]) &
                  ((p[1] - 1.0) < b_arr[:, 3]) & ((p[3] + 1.0) > b_arr[:, 1]))
        if clear.all():
            boxes.append(p)
            mats.append(interior())
            placed += 1
    # tiles for floor and ceiling with the remaining triangle budget
    rest = max(4, target_tris - 12 * len(boxes))
    n_tiles = max(1, rest // 4)  # 2 triangles per tile, floor and ceiling
    nx = max(1, int(round(np.sqrt(n_tiles * width / depth))))
    ny = max(1, n_tiles // nx)
    sb = SceneBuilder()
    face0 = []
    for (x0, y0, x1, y1), m in zip(boxes, mats):
        face0.append(len(sb.normals))
        sb.add_box((x0, y0, 0.0), (x1, y1, height), m)
    xs = np.linspace(0.0, width, nx + 1)
    ys = np.linspace(0.0, depth, ny + 1)
    floor_face = len(sb.normals)
    for j in range(ny):
        for i in range(nx):
            sb.add_quad((xs[i], ys[j], 0), (xs[i + 1], ys[j], 0), (xs[i + 1], ys[j + 1], 0),
                        (xs[i], ys[j + 1], 0), FLOOR)
    ceil_face = len(sb.normals)
    for j in range(ny):
        for i in range(nx):
            sb.add_quad((xs[i], ys[j], height), (xs[i], ys[j + 1], height),
                        (xs[i + 1], ys[j + 1], height), (xs[i + 1], ys[j], height), CEILING)
    scene = sb.build(n_mat=first_int + n_interior_types)
    return FloorPlan(scene=scene, boxes=np.asarray(boxes, np.float64),
                     box_mat=np.asarray(mats, np.int64), box_face0=np.asarray(face0, np.int64),
                     width=width, depth=depth, height=height, floor_face=floor_face,
                     ceil_face=ceil_face, tiles=(nx, ny))

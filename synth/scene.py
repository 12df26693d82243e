"""Triangle scenes.

A scene is a list of triangles, each belonging to a planar *face* (a convex
polygon made of coplanar triangles with one material class).  Reflections are
computed per face: a specular reflection point is valid when it falls inside
any triangle of its face.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Scene:
    tri: np.ndarray          # float64 [T, 3, 3] vertices
    tri_face: np.ndarray     # int32 [T] face id of each triangle
    face_normal: np.ndarray  # float64 [F, 3] unit normal (either orientation)
    face_offset: np.ndarray  # float64 [F] plane offset d: n . x = d
    face_mat: np.ndarray     # int32 [F] material class id
    n_mat: int
    aabb_min: np.ndarray     # float64 [3]
    aabb_max: np.ndarray     # float64 [3]

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_face(self) -> int:
        return int(self.face_normal.shape[0])

    def face_triangles(self, f: int) -> np.ndarray:
        return self.tri[self.tri_face == f]

    def face_area(self) -> np.ndarray:
        e1 = self.tri[:, 1] - self.tri[:, 0]
        e2 = self.tri[:, 2] - self.tri[:, 0]
        a = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
        out = np.zeros(self.n_face)
        np.add.at(out, self.tri_face, a)
        return out


class SceneBuilder:
    """Accumulates axis-aligned or general quads as two triangles each."""

    def __init__(self):
        self.tris = []
        self.tri_face = []
        self.normals = []
        self.offsets = []
        self.mats = []

    def add_quad(self, p0, p1, p2, p3, mat: int) -> int:
        """Planar quad with corners in cyclic order; returns its face id."""
        p0, p1, p2, p3 = (np.asarray(p, np.float64) for p in (p0, p1, p2, p3))
        n = np.cross(p1 - p0, p3 - p0)
        n = n / np.linalg.norm(n)
        f = len(self.normals)
        self.normals.append(n)
        self.offsets.append(float(n @ p0))
        self.mats.append(int(mat))
        self.tris.append(np.stack([p0, p1, p2]))
        self.tris.append(np.stack([p0, p2, p3]))
        self.tri_face += [f, f]
        return f

    def add_box(self, lo, hi, mat: int, skip=()):
        """Axis-aligned box as 6 quads (12 triangles).  `skip` lists faces
        to leave out by name: '-x', '+x', '-y', '+y', '-z', '+z'."""
        x0, y0, z0 = lo
        x1, y1, z1 = hi
        quads = {
            "-x": ((x0, y0, z0), (x0, y1, z0), (x0, y1, z1), (x0, y0, z1)),
            "+x": ((x1, y0, z0), (x1, y0, z1), (x1, y1, z1), (x1, y1, z0)),
            "-y": ((x0, y0, z0), (x0, y0, z1), (x1, y0, z1), (x1, y0, z0)),
            "+y": ((x0, y1, z0), (x1, y1, z0), (x1, y1, z1), (x0, y1, z1)),
            "-z": ((x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0)),
            "+z": ((x0, y0, z1), (x0, y1, z1), (x1, y1, z1), (x1, y0, z1)),
        }
        for name, q in quads.items():
            if name not in skip:
                self.add_quad(*q, mat=mat)

    def build(self, n_mat: int) -> Scene:
        tri = np.asarray(self.tris, np.float64)
        lo = tri.reshape(-1, 3).min(0)
        hi = tri.reshape(-1, 3).max(0)
        return Scene(
            tri=tri,
            tri_face=np.asarray(self.tri_face, np.int32),
            face_normal=np.asarray(self.normals, np.float64),
            face_offset=np.asarray(self.offsets, np.float64),
            face_mat=np.asarray(self.mats, np.int32),
            n_mat=n_mat,
            aabb_min=lo,
            aabb_max=hi,
        )


def box_room(size=(10.0, 8.0, 3.0), mat: int = 0) -> Scene:
    """Axis-aligned box room [0,sx]x[0,sy]x[0,sz]: floor, ceiling and four
    walls, 12 triangles, one material class."""
    b = SceneBuilder()
    b.add_box((0.0, 0.0, 0.0), size, mat)
    return b.build(n_mat=1)


def uniform_points_in_box(rng, n, lo, hi, margin=0.5):
    lo = np.asarray(lo, np.float64) + margin
    hi = np.asarray(hi, np.float64) - margin
    return lo + (hi - lo) * rng.random((n, 3))

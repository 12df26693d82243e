"""Exhaustive image-method path finder for tiny scenes (Sec. II-F).

Every sequence of faces up to `max_depth` (no face twice in a row) is tried:
the Tx is mirrored across the face planes in order, the path is traced back
from the Rx through the images, each reflection point must fall inside its
face and strictly between its neighbours, and every segment must be free of
other triangles.  This is brute force over face sequences and is meant for
scenes of a few dozen faces; large scenes use the native finder.
"""
import itertools

import numpy as np

from .store import KIND_SPECULAR, PathStore, pack

_EPS = 1e-9


def _point_in_tri(p, tri, n):
    """Barycentric inside test for point p on the plane of triangle tri."""
    a, b, c = tri
    v0, v1, v2 = b - a, c - a, p - a
    d00, d01, d11 = v0 @ v0, v0 @ v1, v1 @ v1
    d20, d21 = v2 @ v0, v2 @ v1
    den = d00 * d11 - d01 * d01
    v = (d11 * d20 - d01 * d21) / den
    w = (d00 * d21 - d01 * d20) / den
    u = 1.0 - v - w
    tol = -1e-12
    return u >= tol and v >= tol and w >= tol


def _in_face(scene, f, p):
    n = scene.face_normal[f]
    for tri in scene.face_triangles(f):
        if _point_in_tri(p, tri, n):
            return True
    return False


def _segment_blocked(scene, a, b, skip_faces):
    """True if the open segment a->b crosses any triangle not in skip_faces."""
    d = b - a
    tri = scene.tri
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    h = np.cross(d[None, :], e2)
    det = np.einsum("ij,ij->i", e1, h)
    ok = np.abs(det) > 1e-14
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    s = a[None, :] - tri[:, 0]
    u = inv * np.einsum("ij,ij->i", s, h)
    q = np.cross(s, e1)
    v = inv * np.einsum("j,ij->i", d, q)
    t = inv * np.einsum("ij,ij->i", e2, q)
    hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 1e-7) & (t < 1 - 1e-7)
    if skip_faces:
        hit &= ~np.isin(scene.tri_face, list(skip_faces))
    return bool(hit.any())


def _mirror(p, n, d):
    return p - 2.0 * (n @ p - d) * n


def find_paths(scene, tx, rx, max_depth):
    """All specular paths Tx -> Rx with at most max_depth reflections.

    Returns a list of path records sorted by (depth, face sequence)."""
    tx = np.asarray(tx, np.float64)
    rx = np.asarray(rx, np.float64)
    out = []
    if not _segment_blocked(scene, tx, rx, ()):
        out.append(dict(points=np.zeros((0, 3)), normals=np.zeros((0, 3)),
                        mats=[], faces=[], kinds=[], dA=[],
                        length=float(np.linalg.norm(rx - tx))))
    F = scene.n_face
    for depth in range(1, max_depth + 1):
        for seq in itertools.product(range(F), repeat=depth):
            if any(seq[i] == seq[i + 1] for i in range(depth - 1)):
                continue
            images = [tx]
            for f in seq:
                images.append(_mirror(images[-1], scene.face_normal[f], scene.face_offset[f]))
            pts = [None] * depth
            target = rx
            ok = True
            for k in range(depth, 0, -1):
                f = seq[k - 1]
                n = scene.face_normal[f]
                d = scene.face_offset[f]
                direc = images[k] - target
                den = n @ direc
                if abs(den) < _EPS:
                    ok = False
                    break
                t = (d - n @ target) / den
                if not (1e-9 < t < 1 - 1e-9):
                    ok = False
                    break
                p = target + t * direc
                if not _in_face(scene, f, p):
                    ok = False
                    break
                pts[k - 1] = p
                target = p
            if not ok:
                continue
            chain = [tx] + pts + [rx]
            # the first segment must also leave the Tx towards the first point
            # on the same side as the image construction implies
            blocked = False
            for j in range(len(chain) - 1):
                skip = set()
                if j >= 1:
                    skip.add(seq[j - 1])
                if j < depth:
                    skip.add(seq[j])
                if _segment_blocked(scene, chain[j], chain[j + 1], skip):
                    blocked = True
                    break
            if blocked:
                continue
            length = sum(float(np.linalg.norm(chain[j + 1] - chain[j]))
                         for j in range(len(chain) - 1))
            out.append(dict(points=np.asarray(pts), normals=scene.face_normal[list(seq)],
                            mats=[int(scene.face_mat[f]) for f in seq], faces=list(seq),
                            kinds=[KIND_SPECULAR] * depth, dA=[0.0] * depth,
                            length=length))
    return out


def find_store(scene, tx, rx_list, max_depth, geom_dtype=np.float32) -> PathStore:
    links = [find_paths(scene, tx, rx, max_depth) for rx in rx_list]
    return pack(links, [tx] * len(rx_list), rx_list, max_depth, geom_dtype)

"""ctypes wrapper of the native 2.5-D path finder (synth/pathfind25d.cpp)."""
import ctypes
import os
import subprocess

import numpy as np

from .store import PathStore

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pathfind25d.cpp")
LIB = os.path.join(HERE, "libpathfind25d.so")
C0 = 299792458.0

_lib = None


def build() -> str:
    # a per-process temporary name: parallel test workers may build at once
    tmp = f"{LIB}.tmp{os.getpid()}"
    cmd = ["g++", "-O3", "-march=x86-64-v2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        d, i, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        lib.pf_run.restype = i64
        lib.pf_run.argtypes = [vp, i, d, d, d, d, d, i, i, i, i, vp, vp, i, i, i64, d, i, d]
        lib.pf_fetch.restype = i
        lib.pf_fetch.argtypes = [i, vp, vp, vp, vp, vp, vp, vp]
        lib.pf_free.restype = None
        lib.pd_run.restype = i64
        lib.pd_run.argtypes = [vp, i, d, d, d, d, vp, vp, vp, i, vp, vp, i, i, d]
        lib.pd_fetch.restype = i
        lib.pd_fetch.argtypes = [vp, vp]
        lib.pd_free.restype = None
        _lib = lib
    return _lib


def find_store(plan, tx, rx, max_depth=3, n_rays=1 << 18, recv_factor=2.0,
               n_threads=0, cell=1.0) -> PathStore:
    """Specular paths from one Tx to every Rx in a FloorPlan (all walls span
    floor to ceiling; plan.height <= 0: open sky above walls taller than any
    path, one ground reflection at most).  cell: the plan grid's cell size
    (metres) for ray walks."""
    lib = _load()
    walls = np.ascontiguousarray(plan.wall_segments(), np.float64)
    tx = np.ascontiguousarray(np.asarray(tx, np.float64).reshape(3))
    rx = np.ascontiguousarray(np.asarray(rx, np.float64).reshape(-1, 3))
    n_rx = len(rx)
    fm = int(plan.scene.face_mat[plan.floor_face])
    cm = int(plan.scene.face_mat[plan.ceil_face]) if plan.ceil_face >= 0 else 0
    P = lib.pf_run(walls.ctypes.data, len(walls), 0.0, 0.0, plan.width, plan.depth,
                   plan.height, fm, plan.floor_face, cm, plan.ceil_face, tx.ctypes.data,
                   rx.ctypes.data, n_rx, max_depth, int(n_rays), float(recv_factor),
                   int(n_threads), float(cell))
    if P < 0:
        raise RuntimeError(f"pf_run failed ({P})")
    D = max_depth
    link_off = np.zeros(n_rx + 1, np.int64)
    depth = np.zeros(P, np.uint8)
    pts = np.zeros((3, D * P), np.float32)
    nrm = np.zeros((3, D * P), np.float32)
    mat = np.zeros(D * P, np.uint16)
    face = np.zeros(D * P, np.int32)
    length = np.zeros(P, np.float64)
    st = lib.pf_fetch(D, link_off.ctypes.data, depth.ctypes.data, pts.ctypes.data,
                      nrm.ctypes.data, mat.ctypes.data, face.ctypes.data, length.ctypes.data)
    lib.pf_free()
    if st != 0:
        raise RuntimeError("pf_fetch failed")
    # floor/ceiling reflections: the tile that holds the reflection point
    fm_mask = (face == plan.floor_face) | (face == plan.ceil_face)
    if fm_mask.any():
        idx = np.nonzero(fm_mask)[0]
        ceil = face[idx] == plan.ceil_face
        face[idx] = plan.tile_face(pts[0, idx], pts[1, idx], ceil)
    return PathStore(n_links=n_rx, n_paths=int(P), max_depth=D, link_off=link_off,
                     tx_pos=np.repeat(tx[None].astype(np.float32), n_rx, 0),
                     rx_pos=rx.astype(np.float32), depth=depth,
                     kind=np.zeros(D * P, np.uint8), pts=pts, nrm=nrm, mat=mat,
                     dA=np.zeros(D * P, np.float32), tau=length / C0, face=face)


def visible_samples(plan, tx, rx, pts, nrm, seg, n_threads=0, cell=1.0):
    """Per Rx, the indices of the surface samples (pts, unit normals nrm,
    [n, 3]; seg: the wall segment of plan.wall_segments() each lies on, -1
    for the ground) that both tx and the Rx see from the samples' front side
    in a 2.5-D plan (walls block by their floor-plan footprint).  Returns a
    CSR (off int64 [n_rx + 1], idx int32)."""
    lib = _load()
    walls = np.ascontiguousarray(plan.wall_segments(), np.float64)
    tx = np.ascontiguousarray(np.asarray(tx, np.float64).reshape(3))
    rx = np.ascontiguousarray(np.asarray(rx, np.float64).reshape(-1, 3))
    pts = np.ascontiguousarray(pts, np.float64)
    nrm = np.ascontiguousarray(nrm, np.float64)
    seg = np.ascontiguousarray(seg, np.int32)
    n = lib.pd_run(walls.ctypes.data, len(walls), 0.0, 0.0, plan.width, plan.depth,
                   pts.ctypes.data, nrm.ctypes.data, seg.ctypes.data, len(pts), tx.ctypes.data,
                   rx.ctypes.data, len(rx), int(n_threads), float(cell))
    if n < 0:
        raise RuntimeError(f"pd_run failed ({n})")
    off = np.zeros(len(rx) + 1, np.int64)
    idx = np.zeros(int(n), np.int32)
    st = lib.pd_fetch(off.ctypes.data, idx.ctypes.data)
    lib.pd_free()
    if st != 0:
        raise RuntimeError("pd_fetch failed")
    return off, idx

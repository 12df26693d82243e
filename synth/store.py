"""Path store: interaction-major structure of arrays over all paths.

Paths of all links are concatenated; link l owns paths
link_off[l] .. link_off[l+1]-1 (CSR).  Interaction k (0-based) of path p is
stored at index k*n_paths + p, so that consecutive paths are consecutive in
memory for every interaction slot.  Unused slots (k >= depth[p]) hold zeros.

Geometry is FP32 (points, normals); the delay tau is FP64 because the
subcarrier phase 2*pi*f*tau reaches thousands of radians.
"""
from dataclasses import dataclass

import numpy as np

KIND_SPECULAR = 0
KIND_DIFFUSE = 1


@dataclass
class PathStore:
    n_links: int
    n_paths: int
    max_depth: int
    link_off: np.ndarray   # int64 [n_links+1]
    tx_pos: np.ndarray     # float32 [n_links, 3]
    rx_pos: np.ndarray     # float32 [n_links, 3]
    depth: np.ndarray      # uint8 [n_paths]
    kind: np.ndarray       # uint8 [max_depth*n_paths]
    pts: np.ndarray        # float32 [3, max_depth*n_paths]  (x, y, z rows)
    nrm: np.ndarray        # float32 [3, max_depth*n_paths]
    mat: np.ndarray        # uint16 [max_depth*n_paths]
    dA: np.ndarray         # float32 [max_depth*n_paths] (diffuse area, else 0)
    tau: np.ndarray        # float64 [n_paths] seconds
    face: np.ndarray       # int32 [max_depth*n_paths] face ids (bookkeeping)

    def link_of_path(self) -> np.ndarray:
        cnt = np.diff(self.link_off)
        return np.repeat(np.arange(self.n_links), cnt)

    def paths_per_link(self) -> np.ndarray:
        return np.diff(self.link_off)

    def interaction(self, p: int, k: int):
        idx = k * self.n_paths + p
        return self.pts[:, idx], self.nrm[:, idx], int(self.mat[idx])

    def subset_links(self, links) -> "PathStore":
        """New store holding only the given links (in the given order)."""
        links = np.asarray(links, np.int64)
        cnt = self.paths_per_link()[links]
        new_off = np.zeros(len(links) + 1, np.int64)
        new_off[1:] = np.cumsum(cnt)
        sel = np.concatenate([np.arange(self.link_off[l], self.link_off[l + 1])
                              for l in links]) if len(links) else np.zeros(0, np.int64)
        P, D = int(self.n_paths), self.max_depth
        Pn = int(new_off[-1])
        idx = (np.arange(D)[:, None] * P + sel[None, :]).reshape(-1)
        return PathStore(
            n_links=len(links), n_paths=Pn, max_depth=D, link_off=new_off,
            tx_pos=self.tx_pos[links].copy(), rx_pos=self.rx_pos[links].copy(),
            depth=self.depth[sel].copy(), kind=self.kind[idx].copy(),
            pts=self.pts[:, idx].copy(), nrm=self.nrm[:, idx].copy(),
            mat=self.mat[idx].copy(), dA=self.dA[idx].copy(),
            tau=self.tau[sel].copy(), face=self.face[idx].copy())

    def save(self, path):
        np.savez(path, **{k: getattr(self, k) for k in self.__dataclass_fields__})

    @staticmethod
    def load(path) -> "PathStore":
        z = np.load(path, allow_pickle=False)
        kw = {k: z[k] for k in PathStore.__dataclass_fields__}
        for k in ("n_links", "n_paths", "max_depth"):
            kw[k] = int(kw[k])
        return PathStore(**kw)


def pack(links_paths, tx_list, rx_list, max_depth: int, geom_dtype=np.float32) -> PathStore:
    """Build a store from per-link python lists of path records.

    Each path record is a dict with keys 'points' [Q,3] f64, 'normals' [Q,3],
    'mats' [Q], 'faces' [Q], 'kinds' [Q], 'dA' [Q], 'length' (metres, f64).
    geom_dtype other than float32 is for tests that need exact geometry;
    the GPU library takes float32 only.
    """
    c0 = 299792458.0
    n_links = len(links_paths)
    cnt = np.array([len(p) for p in links_paths], np.int64)
    off = np.zeros(n_links + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    P = int(off[-1])
    D = max_depth
    depth = np.zeros(P, np.uint8)
    kind = np.zeros(D * P, np.uint8)
    pts = np.zeros((3, D * P), geom_dtype)
    nrm = np.zeros((3, D * P), geom_dtype)
    mat = np.zeros(D * P, np.uint16)
    dA = np.zeros(D * P, np.float32)
    face = np.full(D * P, -1, np.int32)
    tau = np.zeros(P, np.float64)
    p = 0
    for lp in links_paths:
        for rec in lp:
            q = len(rec["mats"])
            depth[p] = q
            for k in range(q):
                i = k * P + p
                pts[:, i] = rec["points"][k]
                nrm[:, i] = rec["normals"][k]
                mat[i] = rec["mats"][k]
                face[i] = rec["faces"][k]
                kind[i] = rec["kinds"][k]
                dA[i] = rec["dA"][k]
            tau[p] = rec["length"] / c0
            p += 1
    return PathStore(n_links=n_links, n_paths=P, max_depth=D, link_off=off,
                     tx_pos=np.asarray(tx_list, geom_dtype).reshape(n_links, 3),
                     rx_pos=np.asarray(rx_list, geom_dtype).reshape(n_links, 3),
                     depth=depth, kind=kind, pts=pts, nrm=nrm, mat=mat, dA=dA,
                     tau=tau, face=face)

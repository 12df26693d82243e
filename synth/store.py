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
KIND_DIFFRACTION = 2  # first-order edge diffraction (the path's only interaction)


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
    # first-order diffraction paths (kind 2 in slot 0; their point is on the
    # edge, nrm the normal of face 0 and mat its material): unit edge
    # direction e with n0 x e pointing into face 0, and the wedge's n
    # (exterior angle n pi); the material of face n.  None without such paths.
    edge: np.ndarray = None   # float32 [4, n_paths] (ex, ey, ez, n), zeros elsewhere
    mat_n: np.ndarray = None  # uint16 [n_paths]

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
            tau=self.tau[sel].copy(), face=self.face[idx].copy(),
            edge=None if self.edge is None else self.edge[:, sel].copy(),
            mat_n=None if self.mat_n is None else self.mat_n[sel].copy())

    def save(self, path):
        np.savez(path, **{k: getattr(self, k) for k in self.__dataclass_fields__
                          if getattr(self, k) is not None})

    @staticmethod
    def load(path) -> "PathStore":
        z = np.load(path, allow_pickle=False)
        kw = {k: z[k] for k in PathStore.__dataclass_fields__ if k in z}
        for k in ("n_links", "n_paths", "max_depth"):
            kw[k] = int(kw[k])
        return PathStore(**kw)


def pack(links_paths, tx_list, rx_list, max_depth: int, geom_dtype=np.float32) -> PathStore:
    """Build a store from per-link python lists of path records.

    Each path record is a dict with keys 'points' [Q,3] f64, 'normals' [Q,3],
    'mats' [Q], 'faces' [Q], 'kinds' [Q], 'dA' [Q], 'length' (metres, f64),
    and for a diffraction path 'edge' (ex, ey, ez, n) and 'mat_n'.
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
    has_edge = any("edge" in rec for lp in links_paths for rec in lp)
    edge = np.zeros((4, P), np.float32) if has_edge else None
    mat_n = np.zeros(P, np.uint16) if has_edge else None
    p = 0
    for lp in links_paths:
        for rec in lp:
            q = len(rec["mats"])
            depth[p] = q
            if "edge" in rec:
                edge[:, p] = rec["edge"]
                mat_n[p] = rec["mat_n"]
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
                     tau=tau, face=face, edge=edge, mat_n=mat_n)


def merge_links(a: PathStore, b: PathStore) -> PathStore:
    """A store whose link l holds a's paths of link l followed by b's (the
    two stores describe the same links; interaction slots padded to the
    larger depth)."""
    assert a.n_links == b.n_links
    L = a.n_links
    D = max(int(a.max_depth), int(b.max_depth))
    ca, cb = a.paths_per_link(), b.paths_per_link()
    off = np.zeros(L + 1, np.int64)
    off[1:] = np.cumsum(ca + cb)
    P = int(off[-1])
    la, lb = a.link_of_path(), b.link_of_path()
    dst_a = off[la] + (np.arange(a.n_paths) - a.link_off[la])
    dst_b = off[lb] + ca[lb] + (np.arange(b.n_paths) - b.link_off[lb])
    gd = a.pts.dtype
    out = dict(depth=np.zeros(P, np.uint8), kind=np.zeros(D * P, np.uint8),
               pts=np.zeros((3, D * P), gd), nrm=np.zeros((3, D * P), gd),
               mat=np.zeros(D * P, np.uint16), dA=np.zeros(D * P, np.float32),
               face=np.full(D * P, -1, np.int32), tau=np.zeros(P, np.float64))
    has_edge = a.edge is not None or b.edge is not None
    edge = np.zeros((4, P), np.float32) if has_edge else None
    mat_n = np.zeros(P, np.uint16) if has_edge else None
    for s, dst in ((a, dst_a), (b, dst_b)):
        out["depth"][dst] = s.depth
        out["tau"][dst] = s.tau
        for k in range(int(s.max_depth)):
            src = k * s.n_paths + np.arange(s.n_paths)
            d = k * P + dst
            out["kind"][d] = s.kind[src]
            out["pts"][:, d] = s.pts[:, src]
            out["nrm"][:, d] = s.nrm[:, src]
            out["mat"][d] = s.mat[src]
            out["dA"][d] = s.dA[src]
            out["face"][d] = s.face[src]
        if s.edge is not None:
            edge[:, dst] = s.edge
            mat_n[dst] = s.mat_n
    return PathStore(n_links=L, n_paths=P, max_depth=D, link_off=off, tx_pos=a.tx_pos.copy(),
                     rx_pos=a.rx_pos.copy(), edge=edge, mat_n=mat_n, **out)

"""Single-bounce diffuse scattering paths (Sec. II-D-2 with Sec. II-F).

Surfaces are sampled at stratified points, each standing for an area
element dA (its share of the triangle or face).  A point s on a surface
yields the path Tx -> s -> Rx when the Tx and the Rx lie strictly on the same
side of the surface and both segments are free of other geometry.  The
field of such a path is computed by the library (and the oracle); here only
geometry is produced: point, normal, material, dA and the delay
(|s - tx| + |rx - s|) / c.

Two visibility tests are provided: exact segment-triangle tests for small
triangle scenes, and the 2-D footprint test of the 2.5-D floors (walls span
floor to ceiling, so a segment between interior points is blocked exactly
when its floor-plan projection enters a wall box).
"""
import numpy as np

from .imagemethod import _segment_blocked
from .store import KIND_DIFFUSE, PathStore

C0 = 299792458.0


def sample_triangles(scene, per_tri, rng):
    """per_tri stratified points on every triangle of a Scene: sample k of a
    triangle (A, B, C) is (1 - sqrt(r1)) A + sqrt(r1) (1 - r2) B +
    sqrt(r1) r2 C with r1 in the k-th of per_tri strata.  Returns points
    [S,3], normals [S,3], material ids [S], face ids [S], dA [S]."""
    T = scene.n_tri
    k = np.arange(per_tri)
    r1 = (k[None, :] + rng.uniform(size=(T, per_tri))) / per_tri
    r2 = rng.uniform(size=(T, per_tri))
    a, b, c = scene.tri[:, 0], scene.tri[:, 1], scene.tri[:, 2]
    sq = np.sqrt(r1)[..., None]
    pts = (1 - sq) * a[:, None] + sq * (1 - r2[..., None]) * b[:, None] + sq * r2[..., None] * c[:, None]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    face = np.repeat(scene.tri_face, per_tri)
    return (pts.reshape(-1, 3), scene.face_normal[face], scene.face_mat[face].astype(np.int64),
            face.astype(np.int64), np.repeat(area / per_tri, per_tri))


def sample_triangles_density(scene, density, rng):
    """Stratified points on every triangle of a Scene, about `density` per
    square metre (at least one per triangle); each stands for an equal
    share of its triangle's area.  Same outputs as sample_triangles."""
    a, b, c = scene.tri[:, 0], scene.tri[:, 1], scene.tri[:, 2]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    cnt = np.maximum(1, np.round(area * density).astype(np.int64))
    out_p, out_f, out_dA = [], [], []
    for t in range(scene.n_tri):
        n = int(cnt[t])
        r1 = (np.arange(n) + rng.uniform(size=n)) / n
        r2 = rng.uniform(size=n)
        sq = np.sqrt(r1)[:, None]
        out_p.append((1 - sq) * a[t] + sq * (1 - r2[:, None]) * b[t] + sq * r2[:, None] * c[t])
        out_f.append(np.full(n, scene.tri_face[t], np.int64))
        out_dA.append(np.full(n, area[t] / n))
    face = np.concatenate(out_f)
    return (np.concatenate(out_p), scene.face_normal[face], scene.face_mat[face].astype(np.int64),
            face, np.concatenate(out_dA))


def sample_floor(plan, density, rng):
    """Stratified jittered grid on every face of a FloorPlan (wall box sides,
    floor and ceiling), about `density` points per square metre (at least
    one per face)."""
    H = plan.height
    pts, nrm, mat, face, dA = [], [], [], [], []

    def rect(origin, u, v, n, m, f):
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

    for (x0, y0, x1, y1), m, f0 in zip(plan.boxes, plan.box_mat, plan.box_face0):
        z = np.array([0.0, 0.0, H])
        rect(np.array([x0, y0, 0.0]), np.array([0.0, y1 - y0, 0.0]), z, (-1, 0, 0), m, f0)
        rect(np.array([x1, y0, 0.0]), np.array([0.0, y1 - y0, 0.0]), z, (1, 0, 0), m, f0 + 1)
        rect(np.array([x0, y0, 0.0]), np.array([x1 - x0, 0.0, 0.0]), z, (0, -1, 0), m, f0 + 2)
        rect(np.array([x0, y1, 0.0]), np.array([x1 - x0, 0.0, 0.0]), z, (0, 1, 0), m, f0 + 3)
    nx, ny = plan.tiles
    sc = plan.scene
    for ceiling, z, base in ((False, 0.0, plan.floor_face), (True, H, plan.ceil_face)):
        for j in range(ny):
            for i in range(nx):
                f = base + j * nx + i
                x0, x1 = plan.width * i / nx, plan.width * (i + 1) / nx
                y0, y1 = plan.depth * j / ny, plan.depth * (j + 1) / ny
                rect(np.array([x0, y0, z]), np.array([x1 - x0, 0.0, 0.0]),
                     np.array([0.0, y1 - y0, 0.0]), sc.face_normal[f], sc.face_mat[f], f)
    pts = np.concatenate(pts)
    # keep points that are not inside another box (faces hidden by abutting walls)
    eps = 1e-6
    b = plan.boxes
    inside = ((pts[:, None, 0] > b[:, 0] + eps) & (pts[:, None, 0] < b[:, 2] - eps) &
              (pts[:, None, 1] > b[:, 1] + eps) & (pts[:, None, 1] < b[:, 3] - eps))
    keep = ~inside.any(1)
    cat = lambda xs: np.concatenate(xs)[keep]  # noqa: E731
    return pts[keep], cat(nrm), cat(mat).astype(np.int64), cat(face).astype(np.int64), cat(dA)


def _same_side(pts, nrm, a, b):
    sa = np.einsum("ij,ij->i", a - pts, nrm)
    sb = np.einsum("ij,ij->i", b - pts, nrm)
    return sa * sb > 0


def visible_triangles(scene, pts, face, a):
    """Per point: is the segment a -> point free of triangles of other faces."""
    return np.array([not _segment_blocked(scene, a, p, {int(f)}) for p, f in zip(pts, face)])


def visible_floor(plan, pts, a, eps=1e-6):
    """Per point: does the floor-plan segment a -> point stay out of every
    wall box (open boxes shrunk by eps, so a point on a box face sees out)."""
    a2 = np.asarray(a, np.float64)[:2]
    d = pts[:, :2] - a2[None, :]
    b = plan.boxes
    # Liang-Barsky: parameter interval of the segment inside each box
    t0 = np.zeros((len(pts), len(b)))
    t1 = np.ones((len(pts), len(b)))
    ok = np.ones((len(pts), len(b)), bool)
    for ax, lo, hi in ((0, b[:, 0] + eps, b[:, 2] - eps), (1, b[:, 1] + eps, b[:, 3] - eps)):
        da = d[:, ax][:, None]
        pa = a2[ax]
        par = np.abs(da) < 1e-15
        ok &= ~(par & ((pa < lo[None]) | (pa > hi[None])))
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (lo[None] - pa) / da
            tb = (hi[None] - pa) / da
        tmin = np.where(par, -np.inf, np.minimum(ta, tb))
        tmax = np.where(par, np.inf, np.maximum(ta, tb))
        t0 = np.maximum(t0, tmin)
        t1 = np.minimum(t1, tmax)
    hit = ok & (t0 < t1)
    return ~hit.any(1)


def add_diffuse(store, tx, samples, visible_fn, max_links_chunk=64):
    """A new store with every link's single-bounce diffuse paths appended
    after its specular paths.  samples = (pts, nrm, mat, face, dA) from a
    sampler; visible_fn(pts, endpoint) -> bool per point.  tx: the common
    Tx position of all links, or None to take each link's own."""
    pts, nrm, mat, face, dA = samples
    rx_all = store.rx_pos.astype(np.float64)
    L = store.n_links
    per_tx = tx is None
    if per_tx:
        tx_all = store.tx_pos.astype(np.float64)
    else:
        # Tx side: same for every link
        tx = np.asarray(tx, np.float64)
        tx_all = np.repeat(tx[None], L, 0)
        vis_tx = visible_fn(pts, tx)
    per_link = []
    for l in range(L):
        rx = rx_all[l]
        if per_tx:
            vis_tx = visible_fn(pts, tx_all[l])
        tx_rep = np.repeat(tx_all[l][None], len(pts), 0)
        cand = vis_tx & _same_side(pts, nrm, tx_rep, np.repeat(rx[None], len(pts), 0))
        idx = np.nonzero(cand)[0]
        if len(idx):
            idx = idx[visible_fn(pts[idx], rx)]
        per_link.append(idx)
    return append_diffuse(store, tx_all, samples, per_link)


def append_diffuse(store, tx_all, samples, per_link):
    """A new store with the single-bounce diffuse paths through samples
    per_link[l] (sample indices, in order) appended after link l's specular
    paths; tx_all [L, 3] the links' Tx positions."""
    pts, nrm, mat, face, dA = samples
    rx_all = store.rx_pos.astype(np.float64)
    L = store.n_links
    cnt_d = np.array([len(i) for i in per_link], np.int64)
    cnt_s = store.paths_per_link()
    D = max(int(store.max_depth), 1)
    P0 = int(store.n_paths)
    P = P0 + int(cnt_d.sum())
    off = np.zeros(L + 1, np.int64)
    off[1:] = np.cumsum(cnt_s + cnt_d)
    # destination of the specular paths
    src_link = store.link_of_path()
    rank = np.arange(P0) - store.link_off[src_link]
    dst_s = off[src_link] + rank
    didx = np.concatenate(per_link) if L else np.zeros(0, np.int64)
    dlink = np.repeat(np.arange(L), cnt_d)
    drank = np.arange(len(didx)) - np.repeat(np.cumsum(cnt_d) - cnt_d, cnt_d)
    dst_d = off[dlink] + cnt_s[dlink] + drank

    depth = np.zeros(P, np.uint8)
    kind = np.zeros(D * P, np.uint8)
    gd = store.pts.dtype
    P_pts = np.zeros((3, D * P), gd)
    P_nrm = np.zeros((3, D * P), gd)
    P_mat = np.zeros(D * P, np.uint16)
    P_dA = np.zeros(D * P, np.float32)
    P_face = np.full(D * P, -1, np.int32)
    tau = np.zeros(P, np.float64)
    depth[dst_s] = store.depth
    tau[dst_s] = store.tau
    edge = mat_n = None
    if store.edge is not None:
        edge = np.zeros((4, P), np.float32)
        mat_n = np.zeros(P, np.uint16)
        edge[:, dst_s] = store.edge
        mat_n[dst_s] = store.mat_n
    for k in range(int(store.max_depth)):
        src = k * P0 + np.arange(P0)
        dst = k * P + dst_s
        kind[dst] = store.kind[src]
        P_pts[:, dst] = store.pts[:, src]
        P_nrm[:, dst] = store.nrm[:, src]
        P_mat[dst] = store.mat[src]
        P_dA[dst] = store.dA[src]
        P_face[dst] = store.face[src]
    depth[dst_d] = 1
    kind[dst_d] = KIND_DIFFUSE
    P_pts[:, dst_d] = pts[didx].T
    P_nrm[:, dst_d] = nrm[didx].T
    P_mat[dst_d] = mat[didx]
    P_dA[dst_d] = dA[didx]
    P_face[dst_d] = face[didx]
    s = pts[didx]
    rx_d = rx_all[dlink]
    tx_d = tx_all[dlink]
    tau[dst_d] = (np.linalg.norm(s - tx_d, axis=1) + np.linalg.norm(rx_d - s, axis=1)) / C0
    return PathStore(n_links=L, n_paths=P, max_depth=D, link_off=off, tx_pos=store.tx_pos.copy(),
                     rx_pos=store.rx_pos.copy(), depth=depth, kind=kind, pts=P_pts, nrm=P_nrm,
                     mat=P_mat, dA=P_dA, tau=tau, face=P_face, edge=edge, mat_n=mat_n)

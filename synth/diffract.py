"""First-order edge-diffraction paths (geometry only) for the 2.5-D floors.

The diffracting edges of a floor are the vertical corners of its wall boxes
that stand free (not inside or on another box): door jambs, pillar corners,
wall ends.  Each is a right-angled wedge (exterior angle 3 pi / 2, n = 1.5)
from floor to ceiling.  For a Tx and an Rx the point of diffraction follows
Keller's principle of the shortest path: on a vertical edge at horizontal
distances d_t and d_r it lies at height z_t + (z_r - z_t) d_t / (d_t + d_r),
where the two rays make equal angles with the edge.  The path exists when
both legs are free in the floor plan.  The field (UTD) is computed by the
library and the oracle; here only the point, the wedge's face-0 normal, edge
direction, n and the two faces' materials are produced.
"""
import numpy as np

from .diffuse import visible_floor
from .store import KIND_DIFFRACTION, PathStore, merge_links, pack

C0 = 299792458.0


def floor_edges(plan, eps=1e-6):
    """Free vertical box corners of a FloorPlan: rows of (cx, cy, n0x, n0y,
    ez, mat, face0, bx, by) -- the corner, the outward normal of face 0, the
    sign of the edge direction along z (n0 x e points along face 0, away from
    the corner), the box material (both faces), face 0's id and the
    free-space bisector (bx, by)."""
    rows = []
    boxes = plan.boxes
    for b, ((x0, y0, x1, y1), m, f0) in enumerate(zip(boxes, plan.box_mat, plan.box_face0)):
        # corner, face A (normal, along-face direction, face id), face B direction
        corners = (
            ((x0, y0), (-1.0, 0.0), (0.0, 1.0), f0 + 0, (1.0, 0.0)),
            ((x1, y0), (0.0, -1.0), (-1.0, 0.0), f0 + 2, (0.0, 1.0)),
            ((x1, y1), (1.0, 0.0), (0.0, -1.0), f0 + 1, (-1.0, 0.0)),
            ((x0, y1), (0.0, 1.0), (1.0, 0.0), f0 + 3, (0.0, -1.0)),
        )
        others = np.delete(boxes, b, axis=0)
        for (cx, cy), nA, dA, fA, dB in corners:
            touching = ((cx >= others[:, 0] - eps) & (cx <= others[:, 2] + eps) &
                        (cy >= others[:, 1] - eps) & (cy <= others[:, 3] + eps))
            if touching.any():
                continue
            # n0 x e = dA with e = (0, 0, ez): (nA_y ez, -nA_x ez, 0) = dA
            ez = 1.0 if abs(nA[1] - dA[0]) < 1e-9 and abs(-nA[0] - dA[1]) < 1e-9 else -1.0
            bis = -(np.asarray(dA) + np.asarray(dB))
            bis = bis / np.linalg.norm(bis)
            rows.append((cx, cy, nA[0], nA[1], ez, m, fA, bis[0], bis[1]))
    return np.asarray(rows, np.float64).reshape(-1, 9)


def diffraction_records(plan, edges, tx, rx, offset=1e-4):
    """Diffraction path records (for pack) of one link."""
    tx = np.asarray(tx, np.float64)
    rx = np.asarray(rx, np.float64)
    out = []
    if len(edges) == 0:
        return out
    c = edges[:, :2]
    dt = np.linalg.norm(c - tx[None, :2], axis=1)
    dr = np.linalg.norm(c - rx[None, :2], axis=1)
    z = tx[2] + (rx[2] - tx[2]) * dt / np.maximum(dt + dr, 1e-12)
    q = np.column_stack([c, z])
    # both legs free: test from points nudged off the corner into free space
    probe = q.copy()
    probe[:, :2] += offset * edges[:, 7:9]
    ok = visible_floor(plan, probe, tx) & visible_floor(plan, probe, rx)
    ok &= (dt > 1e-3) & (dr > 1e-3)
    for i in np.nonzero(ok)[0]:
        e = edges[i]
        length = float(np.linalg.norm(q[i] - tx) + np.linalg.norm(rx - q[i]))
        out.append(dict(points=q[i][None], normals=np.array([[e[2], e[3], 0.0]]),
                        mats=[int(e[5])], faces=[int(e[6])], kinds=[KIND_DIFFRACTION],
                        dA=[0.0], length=length, edge=(0.0, 0.0, e[4], 1.5), mat_n=int(e[5])))
    return out


def add_diffraction(store: PathStore, plan, edges=None) -> PathStore:
    """A new store with every link's first-order diffraction paths appended
    after its other paths."""
    edges = floor_edges(plan) if edges is None else edges
    links = [diffraction_records(plan, edges, store.tx_pos[l], store.rx_pos[l])
             for l in range(store.n_links)]
    extra = pack(links, store.tx_pos.astype(np.float64), store.rx_pos.astype(np.float64),
                 max(int(store.max_depth), 1))
    if extra.edge is None:  # no link sees an edge
        extra.edge = np.zeros((4, 0), np.float32)
        extra.mat_n = np.zeros(0, np.uint16)
    return merge_links(store, extra)

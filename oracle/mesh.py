"""RWG and pulse discretisation (Section 2, last paragraph).

The current J is expanded in RWG functions, one per interior edge; n.A is
expanded in pulse functions, one per triangle; N = T + E.

RWG function of edge n with length l, triangles T+ / T- (areas A+, A-) and
free vertices p+ / p-:
    f_n(r) = +l/(2A+) (r - p+)   on T+
    f_n(r) = -l/(2A-) (r - p-)   on T-
    div f_n = +l/A+ on T+, -l/A- on T-.

Edge table convention: an edge is the vertex pair (a, b) with a < b; edges are
listed in ascending (a, b) order; T+ is the triangle whose counter-clockwise
vertex cycle runs a -> b, T- the one that runs b -> a.  Pins: closed-surface
invariants (Euler characteristic, every edge shared by two triangles, total
area, divergence theorem for each RWG) in tests/test_oracle_mesh.py.
"""
from __future__ import annotations

import dataclasses

import numpy as np


class MeshError(ValueError):
    pass


@dataclasses.dataclass
class Mesh:
    V: np.ndarray          # [nv,3] float64
    T: np.ndarray          # [nt,3] int64
    edges: np.ndarray      # [E,2]  (a<b)
    tri: np.ndarray        # [E,2]  (T+, T-)
    free: np.ndarray       # [E,2]  (p+, p-) vertex ids
    length: np.ndarray     # [E]
    area: np.ndarray       # [nt]
    normal: np.ndarray     # [nt,3] unit outward
    centroid: np.ndarray   # [nt,3]
    boundary: np.ndarray   # [nb,2] boundary edges (no RWG), open surfaces

    @property
    def nE(self):
        return self.edges.shape[0]

    @property
    def nT(self):
        return self.T.shape[0]

    @property
    def N(self):
        return self.nE + self.nT


def build(V, T) -> Mesh:
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    nt = T.shape[0]
    if T.min() < 0 or T.max() >= V.shape[0]:
        raise MeshError("triangle index out of range")
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cr = np.cross(b - a, c - a)
    twice = np.linalg.norm(cr, axis=1)
    if np.any(twice <= 0.0) or np.any(np.isnan(twice)):
        raise MeshError("degenerate triangle")
    area = 0.5 * twice
    normal = cr / twice[:, None]
    centroid = (a + b + c) / 3.0

    # directed half-edges: (from, to, triangle, free vertex)
    fr = np.concatenate([T[:, 0], T[:, 1], T[:, 2]])
    to = np.concatenate([T[:, 1], T[:, 2], T[:, 0]])
    fv = np.concatenate([T[:, 2], T[:, 0], T[:, 1]])
    tr = np.concatenate([np.arange(nt)] * 3)
    lo = np.minimum(fr, to)
    hi = np.maximum(fr, to)
    forward = fr < to
    order = np.lexsort((~forward, hi, lo))  # by (lo, hi), forward first
    lo, hi, forward, fv, tr = lo[order], hi[order], forward[order], fv[order], tr[order]
    key = lo * V.shape[0] + hi
    uniq, start, count = np.unique(key, return_index=True, return_counts=True)
    if np.any(count > 2):
        raise MeshError("non-manifold edge (more than two triangles)")
    inner = count == 2
    s = start[inner]
    if np.any(~forward[s]) or np.any(forward[s + 1]):
        raise MeshError("inconsistently oriented triangles")
    edges = np.stack([lo[s], hi[s]], 1)
    tri = np.stack([tr[s], tr[s + 1]], 1)
    free = np.stack([fv[s], fv[s + 1]], 1)
    length = np.linalg.norm(V[edges[:, 1]] - V[edges[:, 0]], axis=1)
    sb = start[~inner]
    boundary = np.stack([lo[sb], hi[sb]], 1)
    return Mesh(V, T, edges, tri, free, length, area, normal, centroid, boundary)

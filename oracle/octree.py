"""Cubic-box clustering, near lists and interaction lists (Section 3).

The object is enclosed in a cubic box that is divided recursively into eight
sub-boxes; level 1 is the root, level l has 2**(l-1) boxes per side and L is
the finest level.  With the one-box-buffer scheme, two finest-level boxes
interact directly (near field) when their integer coordinates differ by at
most one in every direction; the far field of a box at level l >= 3 is its
interaction list: boxes of the same level that are not near it but whose
parents are near its parent.  "Three levels" is the single-level FMM
(Section 4).

Conventions the paper leaves open (stated, and followed by the HIP side):
* root box: lo/hi = vertex bounding box, centre = (lo+hi)/2,
  side = max(hi-lo), origin = centre - side/2;
* basis reference point: RWG edge midpoint (Va+Vb)*0.5, pulse centroid
  ((V0+V1)+V2)/3 in the triangle's vertex order;
* t = (p - origin)/side once per point; finest coordinate
  i = clamp(floor(t * 2**(L-1)), 0, 2**(L-1) - 1); level-l coordinate
  i >> (L-l);
* boxes of a level are the nonempty ones sorted by Morton code
  (bit b of x, y, z goes to bit 3b, 3b+1, 3b+2);
* unknowns are reordered by (finest Morton code, RWG before pulse,
  canonical index);
* far offsets: the 316 integer vectors in [-3,3]^3 with max |component| >= 2,
  numbered in lexicographic (dx, dy, dz) order.

Pins: brute-force all-pairs definitions of near and interaction lists, and
the covering identity near + far = all pairs (tests/test_oracle_octree.py).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def morton(ix, iy, iz, bits=21):
    ix = np.asarray(ix, dtype=np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    iz = np.asarray(iz, dtype=np.int64)
    code = np.zeros(ix.shape, dtype=np.int64)
    for b in range(bits):
        code |= ((ix >> b) & 1) << (3 * b)
        code |= ((iy >> b) & 1) << (3 * b + 1)
        code |= ((iz >> b) & 1) << (3 * b + 2)
    return code


def far_offsets():
    out = []
    for dx in range(-3, 4):
        for dy in range(-3, 4):
            for dz in range(-3, 4):
                if max(abs(dx), abs(dy), abs(dz)) >= 2:
                    out.append((dx, dy, dz))
    return np.array(out, dtype=np.int64)


@dataclasses.dataclass
class Level:
    l: int
    coords: np.ndarray        # [nb,3] integer box coordinates (Morton-sorted)
    parent: np.ndarray        # [nb] index into level l-1 (or -1 at level 1)
    centre: np.ndarray        # [nb,3] float64
    il_ptr: np.ndarray = None  # CSR over boxes: interaction list
    il_src: np.ndarray = None
    il_off: np.ndarray = None  # offset id (0..315) of (obs - src)


@dataclasses.dataclass
class Tree:
    L: int
    origin: np.ndarray
    side: float
    levels: dict              # l -> Level
    box_of: np.ndarray        # [N] finest box of each canonical unknown
    perm: np.ndarray          # [N] canonical index of the unknown at box-order position
    box_ptr: np.ndarray       # [nb_L+1] ranges of box-ordered unknowns
    near_ptr: np.ndarray      # CSR over finest boxes: near boxes (incl. self)
    near_idx: np.ndarray

    def size(self, l):
        """Box side at level l."""
        return self.side / 2 ** (l - 1)


def reference_points(mesh):
    V = mesh.V
    mid = (V[mesh.edges[:, 0]] + V[mesh.edges[:, 1]]) * 0.5
    T = mesh.T
    cen = ((V[T[:, 0]] + V[T[:, 1]]) + V[T[:, 2]]) / 3.0
    return np.concatenate([mid, cen], axis=0)


def build(mesh, L):
    if L < 3:
        raise ValueError("at least three levels (one translation level)")
    V = mesh.V
    lo = V.min(axis=0)
    hi = V.max(axis=0)
    centre = (lo + hi) / 2.0
    side = float(np.max(hi - lo))
    origin = centre - side / 2.0
    pts = reference_points(mesh)
    t = (pts - origin) / side
    nL = 2 ** (L - 1)
    iL = np.clip(np.floor(t * nL).astype(np.int64), 0, nL - 1)
    codeL = morton(iL[:, 0], iL[:, 1], iL[:, 2])
    N = pts.shape[0]
    kind = (np.arange(N) >= mesh.nE).astype(np.int64)
    perm = np.lexsort((np.arange(N), kind, codeL))
    levels = {}
    for l in range(1, L + 1):
        il = iL >> (L - l)
        code = morton(il[:, 0], il[:, 1], il[:, 2])
        uc, first = np.unique(code, return_index=True)
        coords = il[first]
        d = side / 2 ** (l - 1)
        levels[l] = Level(l, coords, None, origin + (coords + 0.5) * d)
    for l in range(1, L + 1):
        lev = levels[l]
        if l == 1:
            lev.parent = -np.ones(lev.coords.shape[0], dtype=np.int64)
            continue
        pc = lev.coords >> 1
        pcode = morton(pc[:, 0], pc[:, 1], pc[:, 2])
        up = levels[l - 1]
        ucode = morton(up.coords[:, 0], up.coords[:, 1], up.coords[:, 2])
        lev.parent = np.searchsorted(ucode, pcode)
    lev = levels[L]
    fcode = morton(lev.coords[:, 0], lev.coords[:, 1], lev.coords[:, 2])
    box_of = np.searchsorted(fcode, codeL)
    counts = np.bincount(box_of, minlength=fcode.size)
    box_ptr = np.concatenate([[0], np.cumsum(counts)])
    # near lists by brute force over all box pairs of the finest level
    C = lev.coords
    near_ptr = [0]
    near_idx = []
    for b0 in range(0, C.shape[0], 512):
        dmax = np.max(np.abs(C[b0:b0 + 512, None, :] - C[None, :, :]), axis=2)
        for r in range(dmax.shape[0]):
            nb = np.nonzero(dmax[r] <= 1)[0]
            near_idx.append(nb)
            near_ptr.append(near_ptr[-1] + nb.size)
    offs = far_offsets()
    okey = np.full(7 * 7 * 7, -1, dtype=np.int64)
    okey[(offs[:, 0] + 3) * 49 + (offs[:, 1] + 3) * 7 + (offs[:, 2] + 3)] = np.arange(offs.shape[0])
    for l in range(3, L + 1):
        lev = levels[l]
        C = lev.coords
        P = levels[l - 1].coords[lev.parent]
        ptr = [0]
        src, off = [], []
        for b0 in range(0, C.shape[0], 512):
            dm = np.max(np.abs(C[b0:b0 + 512, None, :] - C[None, :, :]), axis=2)
            dp = np.max(np.abs(P[b0:b0 + 512, None, :] - P[None, :, :]), axis=2)
            for r in range(dm.shape[0]):
                s_ = np.nonzero((dm[r] >= 2) & (dp[r] <= 1))[0]
                dlt = C[b0 + r] - C[s_]
                src.append(s_)
                off.append(okey[(dlt[:, 0] + 3) * 49 + (dlt[:, 1] + 3) * 7 + (dlt[:, 2] + 3)])
                ptr.append(ptr[-1] + s_.size)
        lev.il_ptr = np.array(ptr, dtype=np.int64)
        lev.il_src = np.concatenate(src) if src else np.zeros(0, np.int64)
        lev.il_off = np.concatenate(off) if off else np.zeros(0, np.int64)
    return Tree(L, origin, side, levels, box_of, perm, box_ptr,
                np.array(near_ptr, dtype=np.int64), np.concatenate(near_idx))

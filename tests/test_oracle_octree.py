"""Pins for the clustering: the one-box-buffer partition of all pairs of
finest boxes -- every pair is either near, or far at exactly one level
(through an interaction list of its ancestors) -- plus box/parent geometry
and the offset numbering."""
import numpy as np
import pytest

import synth
from oracle import mesh, octree


@pytest.mark.parametrize("s,L", [(2, 3), (3, 4), (4, 5), ("patch", 5), ("disk", 4)])
def test_partition_of_pairs(s, L):
    # spheres, and flat open plates lying on box faces (z = 0)
    if s == "patch":
        V, T = synth.patch(12)
    elif s == "disk":
        V, T = synth.disk(8)
    else:
        V, T = synth.icosphere(s, jitter=0.05, seed=3)
    m = mesh.build(V, T)
    tr = octree.build(m, L)
    nb = tr.levels[L].coords.shape[0]
    count = np.zeros((nb, nb), dtype=np.int64)
    for b in range(nb):
        count[b, tr.near_idx[tr.near_ptr[b]:tr.near_ptr[b + 1]]] += 1
    # ancestors of every finest box at each level
    anc = {L: np.arange(nb)}
    for l in range(L - 1, 2, -1):
        anc[l] = tr.levels[l + 1].parent[anc[l + 1]]
    offs = octree.far_offsets()
    for l in range(3, L + 1):
        lev = tr.levels[l]
        pair = np.zeros((lev.coords.shape[0],) * 2, dtype=np.int64)
        for b in range(lev.coords.shape[0]):
            src = lev.il_src[lev.il_ptr[b]:lev.il_ptr[b + 1]]
            off = lev.il_off[lev.il_ptr[b]:lev.il_ptr[b + 1]]
            assert src.size <= 189
            assert np.array_equal(offs[off], lev.coords[b] - lev.coords[src])
            pair[b, src] += 1
        count += pair[np.ix_(anc[l], anc[l])]
    assert np.all(count == 1)


def test_geometry_and_order():
    V, T = synth.icosphere(3)
    m = mesh.build(V, T)
    tr = octree.build(m, 4)
    for l in range(2, 5):
        lev = tr.levels[l]
        up = tr.levels[l - 1]
        assert np.array_equal(up.coords[lev.parent], lev.coords >> 1)
        code = octree.morton(*lev.coords.T)
        assert np.all(np.diff(code) > 0)
        d = tr.size(l)
        dc = lev.centre - up.centre[lev.parent]
        assert np.allclose(np.abs(dc), d / 2, rtol=0, atol=1e-15)
    # every unknown's reference point lies in (or on the boundary of) its box
    pts = octree.reference_points(m)
    C = tr.levels[4].centre[tr.box_of]
    assert np.all(np.abs(pts - C) <= tr.size(4) / 2 * (1 + 1e-12))
    assert np.array_equal(np.sort(tr.perm), np.arange(m.N))
    assert np.all(np.diff(tr.box_of[tr.perm]) >= 0)
    assert octree.far_offsets().shape == (316, 3)

"""Pins for the RWG/pulse tables: Euler characteristic of a closed surface,
E = 1.5 T (so N = T + E as in Section 2), and the defining properties of an
RWG function: unit normal flux through its own edge from both triangles
(continuity) and zero normal component on the other four edges."""
import numpy as np
import pytest

import synth
from oracle import mesh


@pytest.mark.parametrize("s,jit", [(0, 0.0), (2, 0.0), (3, 0.05)])
def test_closed_surface_counts(s, jit):
    V, T = synth.icosphere(s, jitter=jit, seed=2)
    m = mesh.build(V, T)
    assert V.shape[0] - m.nE + m.nT == 2
    assert 2 * m.nE == 3 * m.nT
    assert m.boundary.shape[0] == 0
    assert np.all(m.edges[:, 0] < m.edges[:, 1])
    assert np.all(np.diff(m.edges[:, 0] * V.shape[0] + m.edges[:, 1]) > 0)


def _f(m, n, h, r):
    t = m.tri[n, h]
    sgn = 1.0 if h == 0 else -1.0
    return sgn * m.length[n] / (2.0 * m.area[t]) * (r - m.V[m.free[n, h]])


def test_rwg_flux_and_tangency():
    V, T = synth.icosphere(2, jitter=0.05, seed=7)
    m = mesh.build(V, T)
    for n in range(0, m.nE, 37):
        a, b = m.V[m.edges[n, 0]], m.V[m.edges[n, 1]]
        mid = 0.5 * (a + b)
        ehat = (b - a) / np.linalg.norm(b - a)
        for h in range(2):
            t = m.tri[n, h]
            # in-plane unit normal of the edge pointing from T+ towards T-:
            # T+ runs a->b counter-clockwise, so ehat x n leaves T+; T- runs
            # b->a, so ehat x n enters T-
            u = np.cross(ehat, m.normal[t])
            flux = np.dot(_f(m, n, h, mid), u)
            assert abs(flux - 1.0) < 1e-12
            # other two edges of the triangle: f is along them
            p = m.V[m.free[n, h]]
            for q in (a, b):
                e2 = (q - p) / np.linalg.norm(q - p)
                r = 0.5 * (p + q)
                fv = _f(m, n, h, r)
                assert np.linalg.norm(fv - np.dot(fv, e2) * e2) < 1e-12


def test_mesh_errors():
    V, T = synth.icosphere(1)
    bad = T.copy()
    bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(mesh.MeshError):
        mesh.build(V, bad)
    deg = T.copy()
    deg[0] = [deg[0][0], deg[0][0], deg[0][1]]
    with pytest.raises(mesh.MeshError):
        mesh.build(V, deg)

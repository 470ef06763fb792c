"""Open surfaces (flat PEC plates, boundary edges carry no RWG function),
the scatterers of the paper's first example (Section 4, a 0.6 m patch).

Pins of the oracle on open meshes:
* counts: interior edges = RWG functions, boundary edges none, and the
  Euler characteristic of a disc (V - E + T = 1);
* the exact static polarisability of a thin circular PEC disc of radius a,
  p = (16/3) a^3 eps0 E0 (and no magnetic dipole for a magnetic field in
  its plane): the low-frequency far field of the oracle converges to it as
  the mesh is refined;
* low-frequency stability: the normalised far field at 1e-3 and 1e-5
  wavelengths agrees (the property that distinguishes the potential
  formulation on open surfaces).
The host library's mesh and tree tables are bit-exact with the oracle's on
the same plates."""
import numpy as np
import pytest

import synth
from oracle import mesh as omesh
from oracle import mom
from oracle import octree as ooct

_TH = np.linspace(0.0, np.pi, 13)
DIRS = np.stack([np.sin(_TH), 0 * _TH, np.cos(_TH)], 1)     # z-x plane


def _edges(T):
    e = np.sort(np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]]), axis=1)
    u, c = np.unique(e, axis=0, return_counts=True)
    return u, c


@pytest.mark.parametrize("V_T,nb", [(synth.patch(6), 24), (synth.patch(4, cross=True), 16),
                                    (synth.disk(5), 30)])
def test_open_counts(V_T, nb):
    V, T = V_T
    m = omesh.build(V, T)
    u, c = _edges(T)
    assert m.nT == T.shape[0]
    assert m.boundary.shape[0] == nb == int(np.sum(c == 1))
    assert m.nE == int(np.sum(c == 2))
    assert V.shape[0] - u.shape[0] + T.shape[0] == 1
    # every RWG has two distinct triangles; no boundary edge is a basis
    assert np.all(m.tri[:, 0] != m.tri[:, 1])
    bset = {tuple(e) for e in np.sort(m.boundary, axis=1)}
    assert not any(tuple(e) in bset for e in np.sort(m.edges, axis=1))


def test_paper_patch_size():
    """75 x 75 squares, two triangles each: the paper's 11 250 pulses."""
    V, T = synth.patch(75)
    assert T.shape[0] == 11250
    m = omesh.build(V, T)
    assert m.nE == 3 * 75 * 75 - 2 * 75 and m.boundary.shape[0] == 300


def _disk_farfield(rings, dl):
    V, T = synth.disk(rings)
    p = mom.Problem(V, T, dl * synth.C0 / synth.DIAMETER)
    x = np.linalg.solve(p.dense(), p.rhs(*synth.axial_wave()))
    return p.farfield(x, DIRS)[0] / p.k ** 2


def test_disk_polarisability():
    a = synth.DIAMETER / 2
    p = 16.0 / 3.0 * a ** 3 * np.array([1.0, 0.0, 0.0])      # p / (eps0 E0)
    ref = np.cross(np.cross(DIRS, p), DIRS) / (4.0 * np.pi)   # F / k^2
    errs = []
    for rings in (6, 10):
        F = _disk_farfield(rings, 1e-3)
        errs.append(np.linalg.norm(F - ref) / np.linalg.norm(ref))
    print("disc polarisability errors (6, 10 rings):", errs)
    # first-order convergence in h (the charge is singular at the rim)
    assert errs[0] < 0.06 and errs[1] < 0.035
    assert errs[1] < 0.7 * errs[0]


def test_disk_low_frequency_stability():
    F3 = _disk_farfield(6, 1e-3)
    F5 = _disk_farfield(6, 1e-5)
    assert np.linalg.norm(F3 - F5) / np.linalg.norm(F5) < 1e-4


@pytest.mark.parametrize("gen,L", [(lambda: synth.patch(16), 3), (lambda: synth.patch(16), 6),
                                   (lambda: synth.patch(5, cross=True), 3), (lambda: synth.disk(10), 4)])
def test_open_host_tables_bit_exact(gen, L):
    pie = pytest.importorskip("paper_1806_04164_amd.pie")
    V, T = gen()
    m = pie.Mesh(V, T)
    om = omesh.build(V, T)
    e, t, f = m.edges()
    assert np.array_equal(e, om.edges) and np.array_equal(t, om.tri) and np.array_equal(f, om.free)
    assert m.sizes() == (om.nE, om.nT)
    tr = pie.Tree(m, L)
    ot = ooct.build(om, L)
    assert np.array_equal(tr.query("PERM"), ot.perm)
    assert np.array_equal(tr.query("BOXPTR"), ot.box_ptr)
    assert np.array_equal(tr.query("NEAR_PTR"), ot.near_ptr)
    assert np.array_equal(tr.query("NEAR_IDX"), ot.near_idx)
    for lv in range(3, L + 1):
        assert np.array_equal(tr.query("IL_PTR", lv), ot.levels[lv].il_ptr)
        assert np.array_equal(tr.query("IL_SRC", lv), ot.levels[lv].il_src)
        assert np.array_equal(tr.query("IL_OFF", lv), ot.levels[lv].il_off)

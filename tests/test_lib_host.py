"""Host-side checks of libpie (no GPU): every symbol of include/pie.h is
exported, mesh and tree integer tables are bit-exact with the oracle's
independent implementation, and argument validation happens before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import mesh as omesh
from oracle import octree as ooct

pie = pytest.importorskip("paper_1806_04164_amd.pie")
from paper_1806_04164_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "pie.h")).read()
    declared = set(re.findall(r"\b(pie_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTS)
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert L.pie_version() >= 100


@pytest.mark.parametrize("s,jit,seed", [(1, 0.0, 0), (3, 0.05, 2), (4, 0.0, 0)])
def test_mesh_tables_bit_exact(s, jit, seed):
    V, T = synth.icosphere(s, jitter=jit, seed=seed)
    m = pie.Mesh(V, T)
    om = omesh.build(V, T)
    e, t, f = m.edges()
    assert np.array_equal(e, om.edges)
    assert np.array_equal(t, om.tri)
    assert np.array_equal(f, om.free)
    assert m.sizes() == (om.nE, om.nT)


@pytest.mark.parametrize("s,L,jit", [(3, 3, 0.0), (4, 4, 0.05), (5, 5, 0.05)])
def test_tree_bit_exact(s, L, jit):
    V, T = synth.icosphere(s, jitter=jit, seed=2)
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, L)
    ot = ooct.build(omesh.build(V, T), L)
    assert np.array_equal(tr.query("PERM"), ot.perm)
    assert np.array_equal(tr.query("BOXPTR"), ot.box_ptr)
    assert np.array_equal(tr.query("NEAR_PTR"), ot.near_ptr)
    assert np.array_equal(tr.query("NEAR_IDX"), ot.near_idx)
    for l in range(1, L + 1):
        assert int(tr.query("NBOX", l)) == ot.levels[l].coords.shape[0]
        assert np.array_equal(tr.query("COORDS", l).reshape(-1, 3), ot.levels[l].coords)
        if l >= 2:
            assert np.array_equal(tr.query("PARENT", l), ot.levels[l].parent)
        if l >= 3:
            assert np.array_equal(tr.query("IL_PTR", l), ot.levels[l].il_ptr)
            assert np.array_equal(tr.query("IL_SRC", l), ot.levels[l].il_src)
            assert np.array_equal(tr.query("IL_OFF", l), ot.levels[l].il_off)


@pytest.mark.parametrize("s,jit,seed", [(0, 0.0, 0), (1, 0.0, 0), (3, 0.0, 0), (4, 0.05, 2), (5, 0.05, 2),
                                        (6, 0.0, 0), (2, 0.3, 123456789012345)])
def test_icosphere_bit_exact(s, jit, seed):
    """pie_mesh_icosphere (C++) against the workloads' generator: vertices
    and triangles equal bit for bit, so a mesh built by the library is the
    workload's mesh (the jittered ones included)."""
    m = pie.Mesh.icosphere(s, synth.DIAMETER / 2, jit, seed)
    V, T = synth.icosphere(s, synth.DIAMETER / 2, jit, seed)
    assert m.V.shape == (10 * 4 ** s + 2, 3) and m.T.shape == (20 * 4 ** s, 3)
    assert np.array_equal(m.V, V)
    assert np.array_equal(m.T, T)
    om = omesh.build(V, T)
    assert m.sizes() == (om.nE, om.nT)


def test_icosphere_errors():
    for args in ((-1, 0.3, 0.0, 0), (11, 0.3, 0.0, 0), (2, 0.0, 0.0, 0), (2, float("nan"), 0.0, 0),
                 (2, 0.3, -0.1, 0), (2, 0.3, 0.5, 0)):
        with pytest.raises(_lib.PieError) as ei:
            pie.Mesh.icosphere(*args)
        assert ei.value.status == _lib.PIE_ERR_ARG


def test_mesh_errors():
    V, T = synth.icosphere(1)
    bad = T.copy()
    bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(_lib.PieError) as ei:
        pie.Mesh(V, bad)
    assert ei.value.status == _lib.PIE_ERR_MESH
    Vn = V.copy()
    Vn[3, 1] = np.nan
    with pytest.raises(_lib.PieError) as ei:
        pie.Mesh(Vn, T)
    assert ei.value.status == _lib.PIE_ERR_NONFINITE
    with pytest.raises(_lib.PieError) as ei:
        pie.Mesh(V, T + 1000)
    assert ei.value.status == _lib.PIE_ERR_ARG
    m = pie.Mesh(V, T)
    with pytest.raises(_lib.PieError):
        pie.Tree(m, 2)


def test_operator_argument_validation_without_gpu():
    V, T = synth.icosphere(2)
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, 3)
    L = _lib.lib()
    o = _lib.pie_options()
    L.pie_options_default(ctypes.byref(o))
    h = ctypes.c_void_p()
    cases = [dict(version=2), dict(near_prec=16), dict(max_rhs=0)]
    for c in cases:
        oo = _lib.pie_options()
        L.pie_options_default(ctypes.byref(oo))
        for k, v in c.items():
            setattr(oo, k, v)
        assert L.pie_operator_create(m.h, tr.h, 1e6, ctypes.byref(oo), None, ctypes.byref(h)) == _lib.PIE_ERR_ARG
    assert L.pie_operator_create(m.h, tr.h, -1.0, ctypes.byref(o), None, ctypes.byref(h)) == _lib.PIE_ERR_ARG
    # tau/x combination that would amplify FP32 round-off past 1e-2
    oo = _lib.pie_options()
    L.pie_options_default(ctypes.byref(oo))
    oo.far_prec, oo.tau, oo.x = _lib.PIE_FP32, 7, 0.05
    assert L.pie_operator_create(m.h, tr.h, 1e6, ctypes.byref(oo), None, ctypes.byref(h)) == _lib.PIE_ERR_PRECISION
    # level-3 boxes beyond what the truncation numbers cover: 6 wavelengths
    # (k d_3 = 9.4) by default; 2 wavelengths (k d_3 = 3.1) with the FP32 far
    # field (k d_3 <= 1) or a caller's tau = 7 (k d_3 <= 1.6)
    assert L.pie_operator_create(m.h, tr.h, 3e9, ctypes.byref(o), None, ctypes.byref(h)) == _lib.PIE_ERR_UNSUPPORTED
    for far, tau in ((_lib.PIE_FP32, 0), (_lib.PIE_FP64, 7)):
        oo = _lib.pie_options()
        L.pie_options_default(ctypes.byref(oo))
        oo.far_prec, oo.tau = far, tau
        assert L.pie_operator_create(m.h, tr.h, 1e9, ctypes.byref(oo), None, ctypes.byref(h)) == \
            _lib.PIE_ERR_UNSUPPORTED
    # tree built for another mesh
    m2 = pie.Mesh(V, T)
    assert L.pie_operator_create(m2.h, tr.h, 1e6, ctypes.byref(o), None, ctypes.byref(h)) == _lib.PIE_ERR_ARG
    # null handles on the MVM entry points
    assert L.pie_matvec(None, None, None, 1, 0, None) == _lib.PIE_ERR_ARG
    assert L.pie_solve(None, None, None, None, 1, None, None, None) == _lib.PIE_ERR_ARG
    assert L.pie_charge(None, 1, None, None, None, 0, None, None, None, None, None, None) == _lib.PIE_ERR_ARG

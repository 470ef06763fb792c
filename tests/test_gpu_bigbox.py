"""Finest boxes holding more than 128 RWG functions or triangles (coarse
trees, as in the paper's 3- to 6-level runs of its patch, Section 4).  The
near field is stored over near boxes of at most 128 slots (a finest box's
slots in runs of its box order), so every stored block fits the SpMM's
tiles; the reception joins each unknown's partial sums through the list of
its own run.  Checked on the GPU:
* a 40 x 40 patch at 3 levels (about 300 RWG functions and 200 triangles
  per finest box): FP64 operator against the oracle's MLFMA (tau = 4,
  x = 0.15) per sub-operator to 1e-9, the default mixed operator against
  sampled rows of the dense matrix to 1e-3, and batched passes (16
  columns) bitwise equal across pass widths and within FP64 rounding of
  the single-column path;
* the paper's 75 x 75 patch at 3 and 4 levels (about 1 800 and 460
  unknowns per finest box; at 3 levels the single-column aggregation and
  reception take up to the device's per-workgroup LDS) at 1 MHz and
  100 MHz: sampled dense rows to 1e-3; at 100 MHz the 3- and 4-level
  solves' far fields against the 5-level one (the paper's level sweep,
  Section 4, Fig. 1)."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlfma, mom
from paper_1806_04164_amd import pie
from paper_1806_04164_amd._lib import PIE_FP32, PIE_FP64
from tests.oracle_rows import sampled_rows

pytestmark = pytest.mark.gpu

F100 = 1e8
_TH = np.linspace(0.0, np.pi, 181)
ZX = np.stack([np.sin(_TH), 0 * _TH, np.cos(_TH)], 1)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _blocks(fn, x, E):
    out = {}
    for name, sl in (("J", slice(0, E)), ("A", slice(E, None))):
        xm = np.zeros_like(x)
        xm[sl] = x[sl]
        out[name] = fn(xm)
    return out


def _errs(g, ref, E, rows=None):
    """Per sub-operator relative errors of g (full vectors) against ref (full
    vectors, or the sampled rows `rows` of a single column)."""
    errs = {}
    for name in ("J", "A"):
        idx = np.arange(g[name].shape[0]) if rows is None else rows
        gg = g[name][idx]
        rr = ref[name].reshape(len(idx), -1)[:, 0]
        for rn, rs in (("J", idx < E), ("A", idx >= E)):
            errs[rn + name] = np.linalg.norm(gg[rs] - rr[rs]) / np.linalg.norm(rr[rs])
    return errs


def _box_counts(m, tr):
    ne = m.sizes()[0]
    perm = tr.query("PERM")
    bp = tr.query("BOXPTR")
    nJ = [int(np.sum(perm[bp[b]:bp[b + 1]] < ne)) for b in range(len(bp) - 1)]
    nT = [int(bp[b + 1] - bp[b]) - nJ[b] for b in range(len(bp) - 1)]
    return max(nJ), max(nT)


def test_patch40_three_levels():
    V, T = synth.patch(40)
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, 3)
    mJ, mT = _box_counts(m, tr)
    print("patch 40, 3 levels: most RWG / triangles in a finest box", mJ, mT, flush=True)
    assert mJ > 128 and mT > 128
    E = m.sizes()[0]
    prob = mom.Problem(V, T, F100)
    N = prob.N
    x = synth.complex_gaussian(N, 1, 41)[:, 0]
    # FP64 operator against the oracle's MLFMA with the same tau and x
    op = pie.Operator(m, tr, F100, near_prec=PIE_FP64, far_prec=PIE_FP64, tau=4, x=0.15)
    g = _blocks(lambda v: host(op.matvec(dev(v))), x, E)
    print("GPU done; oracle MLFMA (host)", flush=True)
    M = mlfma.MLFMA(prob, 3, mlfma.Params(tau=4, x=0.15))
    o = _blocks(M.matvec, x, E)
    errs = _errs(g, o, E)
    print("vs oracle MLFMA", errs, flush=True)
    assert max(errs.values()) < 1e-9
    # default mixed operator against sampled dense rows
    mixed = pie.Operator(m, tr, F100, near_prec=PIE_FP32, far_prec=PIE_FP64, max_rhs=20)
    rng = np.random.default_rng(42)
    rows = np.sort(np.concatenate([rng.choice(E, 8, replace=False), E + rng.choice(N - E, 8, replace=False)]))
    ref = sampled_rows([(("patch", 40), F100, rows, 41, 1)])[0]
    g = _blocks(lambda v: host(mixed.matvec(dev(v[:, None])))[:, 0], x, E)
    errs = _errs(g, ref, E, rows)
    print("mixed vs dense rows", errs, flush=True)
    assert max(errs.values()) <= 1e-3
    # batched passes: bitwise across widths, FP64 rounding from one column
    X = synth.complex_gaussian(N, 20, 43)
    y20 = host(mixed.matvec(dev(X)))
    y16 = host(mixed.matvec(dev(X[:, 2:18].copy())))
    assert np.array_equal(y20[:, 2:18], y16)
    for r in (0, 19):
        y1 = host(mixed.matvec(dev(X[:, r:r + 1].copy())))[:, 0]
        d = np.linalg.norm(y20[:, r] - y1) / np.linalg.norm(y1)
        print("batched vs single column", r, d, flush=True)
        assert d < 2e-4


@pytest.fixture(scope="module")
def p75():
    V, T = synth.patch(75)
    m = pie.Mesh(V, T)
    return dict(mesh=m, E=m.sizes()[0], trees={L: pie.Tree(m, L) for L in (3, 4, 5)})


@pytest.mark.parametrize("L", (3, 4))
@pytest.mark.parametrize("f", (1e6, F100), ids=("1MHz", "100MHz"))
def test_paper_patch_coarse_trees_sampled_rows(p75, f, L):
    tr = p75["trees"][L]
    mJ, mT = _box_counts(p75["mesh"], tr)
    op = pie.Operator(p75["mesh"], tr, f, near_prec=PIE_FP32, far_prec=PIE_FP64)
    N, E = op.N, p75["E"]
    print("patch 75,", L, "levels", f, "most RWG / triangles in a finest box", mJ, mT, flush=True)
    rng = np.random.default_rng(44)
    rows = np.sort(np.concatenate([rng.choice(E, 8, replace=False), E + rng.choice(N - E, 8, replace=False)]))
    ref = sampled_rows([(("patch", 75), f, rows, 45, 1)])[0]
    x = synth.complex_gaussian(N, 1, 45)[:, 0]
    g = _blocks(lambda v: host(op.matvec(dev(v[:, None])))[:, 0], x, E)
    errs = _errs(g, ref, E, rows)
    print(L, "-level patch vs dense rows", errs, flush=True)
    assert max(errs.values()) <= 1e-3


def test_paper_patch_level_sweep(p75):
    FF = {}
    for L in (3, 4, 5):
        tr = p75["trees"][L]
        fast = pie.Operator(p75["mesh"], tr, F100, near_prec=PIE_FP32, far_prec=PIE_FP64)
        ref = pie.Operator(p75["mesh"], tr, F100, near_prec=PIE_FP64, far_prec=PIE_FP64)
        b = ref.rhs_planewave(*synth.axial_wave())
        x, info = fast.solve(b, res_op=ref, tol=1e-4, inner_tol=1e-3, refine=40, restart=200, maxit=6000)
        print("patch 75, 100 MHz, levels", L, info, flush=True)
        assert info["converged"]
        FF[L] = host(ref.farfield(x, ZX))[0]
        del fast, ref
        torch.cuda.empty_cache()
    for L in (3, 4):
        rel = np.linalg.norm(FF[L] - FF[5]) / np.linalg.norm(FF[5])
        print(L, "vs 5 levels: relative far-field difference", rel, flush=True)
        assert rel < 2e-3

"""Pins for the FP64 MLFMA model (Section 3, Eqs. (4)-(5)):
* the diagonalised kernel against the exact Green's function at all 316
  one-box-buffer offsets (this fixes the 16 pi^2 constant, the direction of
  w and v, and the sampling), at low frequency (s < 1) and at s = 1;
* the complete MVM against the dense matrix of ``mom`` per sub-operator,
  within the diagonalisation's truncation error (the 1e-3 gate);
* the MLFMA operator's own symmetry u^T Z v = v^T Z u."""
import numpy as np
import pytest

import synth
from oracle import mlfma, mom, octree


@pytest.mark.parametrize("kd", [1e-4, 0.157])
def test_kernel_all_offsets(kd):
    p = mlfma.Params(tau=6, x=0.07)
    d = 1.0
    k = kd / d
    s = mlfma.scale_factor(k, d, p.x)
    rng = np.random.default_rng(4)
    errs = []
    for o in octree.far_offsets():
        cs = np.zeros(3)
        co = o * d
        for _ in range(4):
            r = co + (rng.random(3) - 0.5) * d
            rp = cs + (rng.random(3) - 0.5) * d
            R = np.linalg.norm(r - rp)
            g = np.exp(1j * k * R) / (4 * np.pi * R)
            errs.append(abs(mlfma.kernel(k, s, p, r, rp, co, cs) - g) / abs(g))
    errs = np.array(errs)
    assert np.sqrt(np.mean(errs ** 2)) < 1e-3
    assert errs.max() < 1e-2


@pytest.fixture(scope="module")
def op():
    V, T = synth.icosphere(3, jitter=0.05, seed=2)
    p = mom.Problem(V, T, 1e-3 * synth.C0 / synth.DIAMETER)
    return p, mlfma.MLFMA(p, 3, mlfma.Params(tau=6, x=0.07))


def test_matvec_against_dense_rows(op):
    p, M = op
    E = p.mesh.nE
    rows = np.sort(np.random.default_rng(0).choice(p.N, 200, replace=False))
    Zr = p.zblock(rows, np.arange(p.N))
    nearR = M.near_rows(rows)
    xr = synth.complex_gaussian(p.N, 1, 1)[:, 0]
    for xs, rs in ((slice(0, E), rows < E), (slice(E, None), rows < E),
                   (slice(0, E), rows >= E), (slice(E, None), rows >= E)):
        x = np.zeros_like(xr)
        x[xs] = xr[xs]
        yd = Zr @ x
        ym = nearR @ x + M.far(x, rows)
        assert np.linalg.norm((ym - yd)[rs]) < 1e-3 * np.linalg.norm(yd[rs])


def test_two_levels_against_dense_rows():
    # tree depth matched to the mesh (levels = subdivisions), as for the
    # benchmark workloads
    V, T = synth.icosphere(4)
    p = mom.Problem(V, T, 1e-3 * synth.C0 / synth.DIAMETER)
    M = mlfma.MLFMA(p, 4, mlfma.Params(tau=6, x=0.07))
    rows = np.arange(0, p.N, 61)
    Zr = p.zblock(rows, np.arange(p.N))
    x = synth.complex_gaussian(p.N, 1, 5)[:, 0]
    E = p.mesh.nE
    for rs in (rows < E, rows >= E):
        for xs in (slice(0, E), slice(E, None)):
            xx = np.zeros_like(x)
            xx[xs] = x[xs]
            yd = Zr @ xx
            ym = M.near_rows(rows) @ xx + M.far(xx, rows)
            assert np.linalg.norm((ym - yd)[rs]) < 1e-3 * np.linalg.norm(yd[rs])


def test_mlfma_symmetry(op):
    # exact structural symmetry, checked where round-off amplification of
    # the translation, (2 tau + 1)!!/(2 x)^tau, is small
    p, _ = op
    M = mlfma.MLFMA(p, 3, mlfma.Params(tau=4, x=0.15))
    u = synth.complex_gaussian(p.N, 1, 11)[:, 0]
    v = synth.complex_gaussian(p.N, 1, 12)[:, 0]
    a = u @ M.far(v)
    b = v @ M.far(u)
    assert abs(a - b) < 1e-9 * abs(a)

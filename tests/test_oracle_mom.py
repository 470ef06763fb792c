"""Pins for the dense PIE matrix (the plain definition of the operator):
* complex symmetry Z = Z^T and Z^AJ = (Z^JA)^T (Galerkin + reciprocity);
* the Mie series of a PEC sphere at D = 0.1 lambda, with the error falling
  as the mesh is refined (Section 4 compares against Mie);
* the Rayleigh dipole limit and frequency-independence of the normalised
  far field at D = 1e-3 and 1e-5 lambda (low-frequency stability, Sec. 2);
* gauge invariance: the current J does not depend on the gauge of the
  incident potentials;
* a far triangle pair against a high-order product Gauss rule."""
import numpy as np
import pytest

import synth
from oracle import mie, mom, quad

_TH = np.linspace(0.0, np.pi, 13)
DIRS = np.stack([np.sin(_TH), 0 * _TH, np.cos(_TH)], 1)     # z-x plane


def _solve(subdiv, dl, gauge=0):
    V, T = synth.icosphere(subdiv)
    p = mom.Problem(V, T, dl * synth.C0 / synth.DIAMETER)
    Z = p.dense()
    b = p.rhs(*synth.axial_wave(), gauge=gauge)
    return p, Z, np.linalg.solve(Z, b)


@pytest.fixture(scope="module")
def s2():
    return _solve(2, 0.1)


def test_symmetry(s2):
    p, Z, _ = s2
    E = p.mesh.nE
    assert np.max(np.abs(Z - Z.T)) <= 1e-13 * np.max(np.abs(Z))
    assert np.max(np.abs(Z[E:, :E] - Z[:E, E:].T)) <= 1e-13 * np.max(np.abs(Z[:E, E:]))


def test_mie_and_refinement(s2):
    p2, _, x2 = s2
    F2 = p2.farfield(x2, DIRS)[0]
    ref = mie.farfield(p2.k * synth.DIAMETER / 2, p2.k, DIRS)
    e2 = np.linalg.norm(F2 - ref) / np.linalg.norm(ref)
    p3, _, x3 = _solve(3, 0.1)
    e3 = np.linalg.norm(p3.farfield(x3, DIRS)[0] - ref) / np.linalg.norm(ref)
    assert e2 < 0.05 and e3 < 0.012
    assert e3 < e2 / 3.0          # second-order convergence in h


def test_rayleigh_limit_and_low_frequency_stability():
    out = []
    for dl in (1e-3, 1e-5):
        p, Z, x = _solve(2, dl)
        F = p.farfield(x, DIRS)[0] / p.k ** 2
        ref = mie.dipole_farfield(synth.DIAMETER / 2, p.k, DIRS) / p.k ** 2
        assert np.linalg.norm(F - ref) / np.linalg.norm(ref) < 0.05
        out.append(F)
    assert np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[1]) < 1e-4


def test_gauge_invariance_of_J(s2):
    p, Z, x0 = s2
    b1 = p.rhs(*synth.axial_wave(), gauge=1)
    x1 = np.linalg.solve(Z, b1)
    E = p.mesh.nE
    assert np.linalg.norm(x1[:E] - x0[:E]) < 1e-9 * np.linalg.norm(x0[:E])


def test_far_pair_against_high_order():
    V, T = synth.icosphere(2)
    p = mom.Problem(V, T, 0.1 * synth.C0 / synth.DIAMETER)
    m = p.mesh
    a, b = 0, int(np.argmax(np.linalg.norm(m.centroid - m.centroid[0], axis=1)))
    M0 = p.pair_moments([a], [b])[0][0]
    # Gauss-Legendre collapsed-square rule of high order on both triangles
    x, w = np.polynomial.legendre.leggauss(16)
    u, wu = 0.5 * (x + 1), 0.5 * w
    def pts(t):
        v0, v1, v2 = m.V[m.T[t]]
        P, W = [], []
        for i in range(16):
            for j in range(16):
                s_, t_ = u[i], u[j] * (1 - u[i])
                P.append(v0 + s_ * (v1 - v0) + t_ * (v2 - v0))
                W.append(wu[i] * wu[j] * (1 - u[i]) * 2 * m.area[t])
        return np.array(P), np.array(W)
    Pa, Wa = pts(a)
    Pb, Wb = pts(b)
    R = np.linalg.norm(Pa[:, None] - Pb[None], axis=2)
    ref = np.sum(Wa[:, None] * Wb[None] * np.exp(1j * p.k * R) / (4 * np.pi * R))
    assert abs(M0 - ref) < 1e-7 * abs(ref)

"""Pins for the oracle's near-zone charge density (Section 2: rho =
i w eps0 n.A - eps0 n.grad(Phi), with n.grad(Phi) from Eq. (3) in pulses):
* the static limit on a PEC sphere in a uniform field E0 x_hat: the induced
  surface charge is 3 eps0 E0 cos(theta_x) (theta_x from the x axis), and
  the error falls as the mesh is refined;
* gauge invariance: with Phi^inc = 0 (gauge 1) Eq. (3) gives sigma = 0 and
  rho comes from n.A alone, and must equal the Lorenz-gauge rho in which
  both terms contribute;
* charge neutrality of the sphere (it sits at the incident field's zero
  potential)."""
import numpy as np
import pytest

import synth
from oracle import mom


def _rho(subdiv, dl, gauge):
    V, T = synth.icosphere(subdiv)
    p = mom.Problem(V, T, dl * synth.C0 / synth.DIAMETER)
    x = np.linalg.solve(p.dense(), p.rhs(*synth.axial_wave(), gauge=gauge))
    sigma, rho = p.charge(x, *synth.axial_wave(), gauge=gauge)
    return p, sigma[:, 0], rho[:, 0]


def test_static_sphere_charge():
    a = synth.DIAMETER / 2
    errs = []
    for sub in (2, 3):
        p, sigma, rho = _rho(sub, 1e-4, 0)
        ref = 3.0 * mom.EPS0 * p.mesh.centroid[:, 0] / a
        errs.append(np.linalg.norm(rho - ref) / np.linalg.norm(ref))
        # at low frequency rho is real to O(k a) and n.grad(Phi) carries it
        assert np.linalg.norm(rho.imag) < 1e-3 * np.linalg.norm(rho.real)
        assert np.linalg.norm(-mom.EPS0 * sigma - rho) < 1e-3 * np.linalg.norm(rho)
    print("static sphere charge errors (subdivisions 2, 3):", errs)
    assert errs[0] < 0.025 and errs[1] < 0.008
    assert errs[1] < errs[0] / 2.5


@pytest.mark.parametrize("dl", [0.1, 1e-3])
def test_charge_gauge_invariance(dl):
    p, s0, r0 = _rho(2, dl, 0)
    _, s1, r1 = _rho(2, dl, 1)
    assert np.all(s1 == 0)
    assert np.linalg.norm(s0) > 0
    assert np.linalg.norm(r0 - r1) < 1e-10 * np.linalg.norm(r0)


def test_sphere_neutral():
    p, _, rho = _rho(2, 1e-3, 0)
    q = np.sum(rho * p.mesh.area)
    assert abs(q) < 1e-10 * np.sum(np.abs(rho) * p.mesh.area)

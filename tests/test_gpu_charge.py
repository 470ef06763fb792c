"""Near-zone charge density on the GPU (pie_charge: Eq. (3) in pulses,
solved by GMRES on the MLFMA's pulse-pulse block, then rho = i w eps0 n.A
- eps0 sigma) against the FP64 oracle.

Tolerances: sigma = n.grad(Phi) depends only on the incident potential, so
it is compared with the oracle's dense solve directly.  The MLFMA's
pulse-pulse block differs from the dense one by <= 1.6e-4 (the AA
sub-operator error measured on these meshes), and the equilibrated block
has cond(DSD) = 126 (sphere, 3 200 unknowns) and 73 (16 x 16 patch), so the
solutions may differ by up to cond x error ~ 2e-2; held to 1e-2.  rho is
checked as the stated combination of the GPU's own n.A and sigma (to
rounding), against the static charge of a sphere in a uniform field, and
between gauges.

The charge solve's residual floor is that of the MLFMA pulse block in FP64:
about 1e-7 at 0.1 wavelength and 1.3-2.2e-5 at 1e-3 wavelength and 1 MHz
(the amplified rounding of the sampled translation), so those solves stop
at 1e-6 and 1e-4."""
import numpy as np
import pytest
import torch

import synth
from oracle import mom
from paper_1806_04164_amd import pie
from paper_1806_04164_amd._lib import PIE_FP64

pytestmark = pytest.mark.gpu

CASES = {
    "sphere_0.1lam": (lambda: synth.icosphere(3), 0.1 * synth.C0 / synth.DIAMETER, 3),
    "sphere_1e-3lam": (lambda: synth.icosphere(3), 1e-3 * synth.C0 / synth.DIAMETER, 3),
    "patch_1MHz": (lambda: synth.patch(16), 1e6, 3),
}


def _tol(f):
    return 1e-6 if f > 1e7 else 1e-4


def _gpu(V, T, f, L, gauge=0, pie_tol=1e-7, ctol=None):
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, L)
    op = pie.Operator(m, tr, f, near_prec=PIE_FP64, far_prec=PIE_FP64)
    wave = synth.axial_wave()
    b = op.rhs_planewave(*wave, gauge=gauge)
    x, info = op.solve(b, tol=pie_tol, restart=200, maxit=3000)
    sigma, rho, cinfo = op.charge(*wave, x=x, gauge=gauge, tol=ctol or _tol(f), restart=200, maxit=2000)
    torch.cuda.synchronize()
    return op, x.cpu().numpy()[:, 0], sigma.cpu().numpy()[:, 0], rho.cpu().numpy()[:, 0], info, cinfo, (m, tr)


@pytest.mark.parametrize("case", list(CASES))
def test_charge_against_oracle(case):
    gen, f, L = CASES[case]
    V, T = gen()
    prob = mom.Problem(V, T, f)
    E = prob.mesh.nE
    # sigma does not depend on the PIE solution: any x serves the oracle here
    sigma_d, _ = prob.charge(np.zeros(prob.N), *synth.axial_wave())
    op, x, sigma, rho, info, cinfo, keep = _gpu(V, T, f, L, pie_tol=1e-4 if f < 1e7 else 1e-7)
    print(case, "PIE solve", info, "charge solve", cinfo, flush=True)
    assert cinfo["converged"]
    es = np.linalg.norm(sigma - sigma_d[:, 0]) / np.linalg.norm(sigma_d[:, 0])
    w = 2.0 * np.pi * f
    rho_c = 1j * w * mom.EPS0 * x[E:] - mom.EPS0 * sigma
    ec = np.linalg.norm(rho - rho_c) / np.linalg.norm(rho_c)
    print(case, "sigma vs dense oracle", es, "rho vs its formula", ec, flush=True)
    assert es < 1e-2
    assert ec < 1e-14


def test_static_sphere_charge():
    """12 800 unknowns at 1e-3 wavelength, 4 levels: rho against
    3 eps0 E0 cos(theta_x) (the oracle's own discretisation error is 2.0 %
    and 0.6 % at subdivisions 2 and 3).  The charge solve runs to 3e-5,
    just above its floor on this mesh (1.3e-5).  The PIE solve stalls near
    3.5e-3 at this frequency (the charge mode meets the MVM's rounding
    floor); its n.A enters rho only through i w eps0 n.A, under 1e-3 of rho
    here."""
    V, T = synth.icosphere(4)
    f = 1e-3 * synth.C0 / synth.DIAMETER
    op, x, sigma, rho, info, cinfo, keep = _gpu(V, T, f, 4, pie_tol=1e-4, ctol=3e-5)
    print("static sphere: PIE solve", info, "charge solve", cinfo, flush=True)
    assert cinfo["converged"]
    a = synth.DIAMETER / 2
    C = V[T].mean(axis=1)
    ref = 3.0 * mom.EPS0 * C[:, 0] / a
    err = np.linalg.norm(rho - ref) / np.linalg.norm(ref)
    area = 0.5 * np.linalg.norm(np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]]), axis=1)
    q = abs(np.sum(rho * area)) / np.sum(np.abs(rho) * area)
    print("static sphere charge error", err, "net charge", q, flush=True)
    assert err < 0.005 and q < 1e-3


def test_charge_gauge_invariance():
    """rho from the Lorenz gauge (both terms) and from Phi^inc = 0 (n.A
    alone, sigma = 0) on the 0.1-wavelength sphere."""
    gen, f, L = CASES["sphere_0.1lam"]
    V, T = gen()
    r = {}
    for g in (0, 1):
        op, x, sigma, rho, info, cinfo, keep = _gpu(V, T, f, L, gauge=g)
        assert cinfo["converged"]
        if g == 1:
            assert np.all(sigma == 0)
        r[g] = rho
    d = np.linalg.norm(r[0] - r[1]) / np.linalg.norm(r[0])
    print("charge gauge difference", d, flush=True)
    assert d < 1e-2


def test_charge_several_waves():
    """Three plane waves in one call: each column of sigma equals the
    single-wave call's bit for bit (the MVM computes each column the same
    way for any column count below 16, and GMRES keeps its own Krylov
    coefficients and stopping point per column), and its oracle dense
    solve to 1e-2."""
    V, T = synth.icosphere(3)
    f = 0.1 * synth.C0 / synth.DIAMETER
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, 3)
    op = pie.Operator(m, tr, f, near_prec=PIE_FP64, far_prec=PIE_FP64, max_rhs=3)
    kh, pol, amp = synth.plane_waves(3, 17)
    sigma, _, info = op.charge(kh, pol, amp, tol=1e-6, restart=200, maxit=2000)
    assert info["converged"]
    sigma = sigma.cpu().numpy()
    prob = mom.Problem(V, T, f)
    sigma_d, _ = prob.charge(np.zeros((prob.N, 3)), kh, pol, amp)
    for r in range(3):
        s1, _, i1 = op.charge(kh[r:r + 1], pol[r:r + 1], amp[r:r + 1], tol=1e-6, restart=200, maxit=2000)
        s1 = s1.cpu().numpy()[:, 0]
        d = np.linalg.norm(sigma[:, r] - s1) / np.linalg.norm(s1)
        e = np.linalg.norm(sigma[:, r] - sigma_d[:, r]) / np.linalg.norm(sigma_d[:, r])
        print("wave", r, "batched vs single", d, "vs dense oracle", e, flush=True)
        assert np.array_equal(sigma[:, r], s1) and e < 1e-2

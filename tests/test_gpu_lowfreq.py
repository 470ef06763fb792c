"""Low-frequency solves on the MLFMA path (Section 2: the PIEs stay stable
at arbitrarily low frequencies; Section 3: the approximate diagonalisation
keeps the MVM accurate there).

The 12 800-unknown sphere (icosphere subdivision 4, 0.6 m, 4 levels) under
the paper's plane wave at 1e-3, 1e-4 and 1e-5 wavelength: GMRES on the FP64
operator, and the mixed operator (FP32 near field) with FP64 residual
refinement, reach a relative residual of 1e-6, and the solved far field
matches the dense FP64 oracle's direct solution (tests/golden/
lowfreq_farfield_s4.json, written by make_lowfreq_farfield.py from the
oracle alone) to 1e-3.  The system's conditioning grows like 1/(k h)
(1.2e4 at 1e-3 and 1.2e6 at 1e-5 wavelength on the 3 200-unknown sphere),
so this also checks that the operator keeps the loop/charge structure of
the dense matrix: the far-field error stays at the operator's ~1e-4 instead
of growing with the conditioning.

The gradient of the far-field loss (16 plane waves, 32 directions) with the
default operator against the dense oracle's closed form at 1e-4 wavelength
(tests/golden/gradient_s4_1e-4lam.json)."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from paper_1806_04164_amd import pie
from paper_1806_04164_amd._lib import PIE_FP32, PIE_FP64

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_farfield(dl):
    g = json.load(open(os.path.join(GOLDEN, "lowfreq_farfield_s4.json")))
    for c in g["cases"]:
        if abs(c["d_over_lambda"] - dl) < 1e-3 * dl:
            return np.array(c["F_re"]) + 1j * np.array(c["F_im"])
    raise KeyError(dl)


@pytest.fixture(scope="module")
def s4():
    V, T = synth.icosphere(4)
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, 4)
    return m, tr


@pytest.mark.parametrize("dl", [1e-3, 1e-4, 1e-5])
def test_low_frequency_solve_matches_dense(s4, dl):
    m, tr = s4
    f = dl * synth.C0 / synth.DIAMETER
    op64 = pie.Operator(m, tr, f, near_prec=PIE_FP64, far_prec=PIE_FP64)
    opm = pie.Operator(m, tr, f, near_prec=PIE_FP32, far_prec=PIE_FP64)
    b = op64.rhs_planewave(*synth.axial_wave())
    dirs = synth.sphere_directions(32, 40)
    F0 = _golden_farfield(dl)
    for name, run in (("fp64", lambda: op64.solve(b, tol=1e-6, restart=200, maxit=3000)),
                      ("mixed+refine", lambda: opm.solve(b, res_op=op64, tol=1e-6, inner_tol=1e-4, refine=10,
                                                         restart=200, maxit=3000))):
        x, info = run()
        F = op64.farfield(x, dirs).cpu().numpy()[0]
        err = np.linalg.norm(F - F0) / np.linalg.norm(F0)
        print(f"D/lambda {dl:g} {name}: {info} far field vs dense LU {err:.3e}", flush=True)
        assert info["converged"] and info["rel_residual"] <= 1e-6
        assert err < 1e-3


def test_gradient_against_dense_oracle(s4):
    from paper_1806_04164_amd import autograd as ag
    m, tr = s4
    g = json.load(open(os.path.join(GOLDEN, "gradient_s4_1e-4lam.json")))
    R = 16
    op = pie.Operator(m, tr, g["freq_hz"], near_prec=PIE_FP64, far_prec=PIE_FP64, max_rhs=R)
    kh, pol, _ = synth.plane_waves(R, 4)
    dirs = synth.sphere_directions(32, 40)
    a = torch.ones(R, dtype=torch.complex128, device="cuda", requires_grad=True)
    x = ag.solve(op, ag.plane_wave_rhs(op, kh, pol, a), tol=1e-6, restart=200, maxit=3000)
    loss = (ag.farfield(op, x, dirs).abs() ** 2).sum()
    loss.backward()
    gr = a.grad.cpu().numpy()
    gref = np.array(g["grad_re"]) + 1j * np.array(g["grad_im"])
    err = np.linalg.norm(gr - gref) / np.linalg.norm(gref)
    print("loss", loss.item(), "dense", g["loss"], "gradient vs dense oracle", err, flush=True)
    assert abs(loss.item() - g["loss"]) < 1e-3 * g["loss"]
    assert err < 1e-3

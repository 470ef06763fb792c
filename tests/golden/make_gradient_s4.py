"""Writes gradient_s4_1e-4lam.json: the gradient of the far-field loss
L(a) = sum_r sum_d |F_r(d)|^2 with respect to the complex amplitudes a of
16 seeded plane waves (seed 4) at a = 1, for the 12 800-unknown sphere
(icosphere subdivision 4, 0.6 m diameter) at 1e-4 wavelength, 32 seeded
directions (seed 40).  F_r = a_r F_r(unit) with F_r(unit) the far field of
the dense FP64 oracle's direct (LU) solution for unit amplitude, so L
decouples over r and its gradient (PyTorch convention dL/dRe a + i dL/dIm a)
is 2 a_r ||F_r(unit)||^2.  Only the oracle is called.  Run from the
repository root:  python tests/golden/make_gradient_s4.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import mom  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gradient_s4_1e-4lam.json")


def main():
    V, T = synth.icosphere(4)
    f = 1e-4 * synth.C0 / synth.DIAMETER
    kh, pol, _ = synth.plane_waves(16, 4)
    dirs = synth.sphere_directions(32, 40)
    p = mom.Problem(V, T, f)
    Z = p.dense()
    B = p.rhs(kh, pol, np.ones(16))
    X = np.linalg.solve(Z, B)
    del Z
    F = p.farfield(X, dirs)                       # [R, nd, 3]
    g = 2.0 * np.sum(np.abs(F) ** 2, axis=(1, 2))  # at a = 1
    out = {"mesh": "icosphere subdivision 4, diameter 0.6 m", "d_over_lambda": 1e-4, "freq_hz": f,
           "waves": "16 plane waves, seed 4", "directions_seed": 40, "n_directions": 32, "a": "ones",
           "loss": float(np.sum(np.abs(F) ** 2)), "grad_re": g.tolist(), "grad_im": [0.0] * 16}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("loss", out["loss"], flush=True)


if __name__ == "__main__":
    main()

"""Writes lowfreq_farfield_s4.json: far fields of the dense FP64 oracle's
direct (LU) solution of the PIE system (Section 2, Eqs. (1)-(2)) for the
12 800-unknown sphere (icosphere subdivision 4, 0.6 m diameter) under the
paper's plane wave (travelling along +z, polarised along x) at diameters of
1e-3, 1e-4 and 1e-5 wavelengths, in 32 seeded directions (seed 40).
Only the oracle is called.  Run from the repository root:
    python tests/golden/make_lowfreq_farfield.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import mom  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lowfreq_farfield_s4.json")


def main():
    V, T = synth.icosphere(4)
    dirs = synth.sphere_directions(32, 40)
    out = {"mesh": "icosphere subdivision 4, diameter 0.6 m", "directions_seed": 40, "n_directions": 32,
           "wave": "khat = +z, pol = +x, amplitude 1", "cases": []}
    for dl in (1e-3, 1e-4, 1e-5):
        f = dl * synth.C0 / synth.DIAMETER
        p = mom.Problem(V, T, f)
        Z = p.dense()
        b = p.rhs(*synth.axial_wave())
        x = np.linalg.solve(Z, b)
        del Z
        F = p.farfield(x, dirs)[0]
        out["cases"].append({"d_over_lambda": dl, "freq_hz": f,
                             "F_re": F.real.tolist(), "F_im": F.imag.tolist()})
        print(f"D/lambda {dl:g}: |F| = {np.linalg.norm(F):.6e}", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()

"""Host pin of the translation tables' spherical Bessel functions (the
h_t(k w) of Eq. (5)): the library's recurrences against scipy, including
the arguments z = n pi where j_0 vanishes (the Miller recurrence must not
be normalised by it there), small z (power series) and large z."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("hk") / "hankel_tables")
    subprocess.run([cxx, "-O2", "-ffp-contract=off", "-std=c++17", f"-I{ROOT}/include", "-o", exe,
                    os.path.join(ROOT, "tests", "hankel_tables.cpp"),
                    os.path.join(ROOT, "paper_1806_04164_amd", "csrc", "tables.cpp")], check=True)
    return exe


def test_spherical_bessel_tables(harness):
    zs = [0.05, 0.5, 0.99, 1.0, math.pi, 2 * math.pi, 3 * math.pi, 4 * math.pi, 4.71, 12.0, 20.5]
    out = subprocess.run([harness] + [repr(z) for z in zs], check=True, capture_output=True, text=True).stdout
    t = np.arange(11)
    for line in out.strip().splitlines():
        v = np.array(list(map(float, line.split())))
        z, a = v[0], v[1:].reshape(-1, 2)
        j, y = spherical_jn(t, z), spherical_yn(t, z)
        scale = np.max(np.abs(j))
        assert np.max(np.abs(a[:, 0] - j)) <= 1e-14 * scale, z
        assert np.max(np.abs(a[:, 1] - y) / np.abs(y)) <= 1e-12, z

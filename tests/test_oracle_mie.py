"""Pins for the Mie series of a PEC sphere (the analytic reference of
Section 4's sphere experiment), against results independent of it:
* the small-sphere (Rayleigh) limit: the radiation of the induced electric
  and magnetic dipoles p = 4 pi eps0 a^3 E0 x_hat, m = -2 pi a^3 H0 y_hat,
  approached as (ka)^2 (the next term of the series);
* the optical theorem for a lossless scatterer: the extinction cross
  section from the forward amplitude, (4 pi / k) Im(pol* . F(khat)), equals
  the scattered power integral of |F|^2 over the sphere, at ka where the
  series needs many terms."""
import numpy as np

from oracle import mie


def _dirs(th, ph):
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)


def test_rayleigh_limit():
    a = 0.3
    th = np.linspace(0.0, np.pi, 13)
    for ph in (0.0, 0.7, np.pi / 2):
        d = _dirs(th, np.full_like(th, ph))
        for ka in (1e-1, 1e-2, 1e-3):
            k = ka / a
            F = mie.farfield(ka, k, d)
            D = mie.dipole_farfield(a, k, d)
            err = np.linalg.norm(F - D) / np.linalg.norm(D)
            assert err < 0.5 * ka ** 2, (ph, ka, err)


def test_optical_theorem():
    a = 0.3
    xg, wg = np.polynomial.legendre.leggauss(80)
    nph = 160
    ph = 2.0 * np.pi * np.arange(nph) / nph
    th = np.arccos(xg)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = _dirs(TH.ravel(), PH.ravel())
    w = np.repeat(wg, nph) * (2.0 * np.pi / nph)
    for ka in (0.5, 1.0, 3.0, 6.0):
        k = ka / a
        F = mie.farfield(ka, k, d)
        sca = np.sum(w * np.sum(np.abs(F) ** 2, axis=1))
        fwd = mie.farfield(ka, k, np.array([[0.0, 0.0, 1.0]]))[0]
        ext = 4.0 * np.pi / k * np.imag(fwd[0])     # pol = x_hat, E0 = 1
        assert abs(ext - sca) < 1e-9 * sca, (ka, ext, sca)

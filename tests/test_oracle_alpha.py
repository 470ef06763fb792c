"""Pins for the modified translation function of Eq. (5): the spherical
Hankel terms against mpmath's half-integer Bessel functions at 40 digits, and
the low-frequency limit (2t-1)!!-form, which is what keeps the translation
finite as k -> 0."""
import mpmath
import numpy as np

from oracle import mlfma


def _alpha_mp(k, s, tau, w, khat):
    mpmath.mp.dps = 40
    wn = mpmath.sqrt(sum(mpmath.mpf(c) ** 2 for c in w))
    z = mpmath.mpf(k) * wn
    cosang = sum(mpmath.mpf(a) * mpmath.mpf(b) for a, b in zip(khat, w)) / wn
    tot = mpmath.mpc(0)
    for t in range(tau + 1):
        pref = mpmath.sqrt(mpmath.pi / (2 * z))
        h = pref * (mpmath.besselj(t + 0.5, z) + 1j * mpmath.bessely(t + 0.5, z))
        tot += (1j ** t) * (2 * t + 1) * mpmath.mpf(s) ** t * h * mpmath.legendre(t, cosang)
    return complex(tot)


def test_alpha_against_mpmath():
    kh, _ = mlfma.samples(mlfma.Params(tau=5))
    for k, s, w in ((2.0, 1.0, (0.3, -0.1, 0.2)), (0.05, 0.2, (2.0, 1.0, 0.0)),
                    (1e-3, 0.01, (0.0, -3.0, 2.0))):
        a = mlfma.alpha_tilde(k, s, 5, np.array(w), kh[:7])
        for q in range(7):
            ref = _alpha_mp(k, s, 5, w, kh[q])
            assert abs(a[q] - ref) <= 1e-12 * abs(ref)


def test_low_frequency_limit():
    from scipy.special import eval_legendre
    d, x, tau = 0.01, 0.05, 7
    w = np.array([2.0, 1.0, -1.0]) * d
    wn = np.linalg.norm(w)
    kh, _ = mlfma.samples(mlfma.Params(tau=tau))
    lim = np.zeros(kh.shape[0], dtype=np.complex128)
    for t in range(tau + 1):
        dfact = np.prod(np.arange(2 * t - 1, 0, -2)) if t > 0 else 1.0
        lim += (1j ** t) * (2 * t + 1) * dfact * (d / (x * wn)) ** t / wn * eval_legendre(t, kh @ (w / wn))
    for k in (1e-6, 1e-9):
        s = k * d / x
        got = 1j * k * mlfma.alpha_tilde(k, s, tau, w, kh)
        assert np.max(np.abs(got - lim)) < 1e-6 * np.max(np.abs(lim))

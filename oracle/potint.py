"""Closed-form potential integrals over a flat triangle.

For an observation point r and a triangle with unit normal n, let
d = n.(r - v1) and rho = r - d n (projection onto the triangle's plane).
For each edge i running from a to b (counter-clockwise about n):
    lhat = (b-a)/|b-a|, uhat = lhat x n (in-plane outward edge normal),
    t  = (a - rho).uhat          (signed distance of rho to the edge line),
    s- = (a - rho).lhat, s+ = (b - rho).lhat,
    R- = |r-a|, R+ = |r-b|, R0^2 = t^2 + d^2,
    f  = ln((R+ + s+)/(R- + s-)),
    beta = atan(t s+/(R0^2 + |d| R+)) - atan(t s-/(R0^2 + |d| R-)).
Then
    int_T 1/|r-r'| dr'          = sum_i [ t_i f_i - |d| beta_i ]
    int_T (r'-rho)/|r-r'| dr'   = 1/2 sum_i uhat_i [ R0_i^2 f_i + s+_i R+_i - s-_i R-_i ]
(Wilton et al., IEEE TAP 1984; Graglia, IEEE TAP 1993).  R + s is evaluated
as R0^2/(R - s) when s < 0, which is the same number without cancellation.

These are used for singularity extraction on touching triangle pairs, a
treatment the paper leaves unstated.  Pin: a Duffy-transformed high-order
Gauss rule over the same triangle (tests/test_oracle_potint.py), for points
inside, outside, above and on the edge lines of the triangle.
"""
from __future__ import annotations

import numpy as np


def _rps(R, s, R0sq):
    """R + s without cancellation (R >= |s|, R^2 = s^2 + R0^2)."""
    safe = np.where(R - s > 0.0, R - s, 1.0)
    return np.where(s >= 0.0, R + s, R0sq / safe)


def potentials(r, tri):
    """r [...,3] observation points, tri [...,3,3] triangle vertices
    (broadcast together).  Returns (K0 [...], K1 [...,3]) with
    K0 = int_T 1/|r-r'|, K1 = int_T (r' - rho)/|r-r'|, rho the projection of
    r onto the triangle's plane."""
    r = np.asarray(r, dtype=np.float64)
    v = np.asarray(tri, dtype=np.float64)
    v1, v2, v3 = v[..., 0, :], v[..., 1, :], v[..., 2, :]
    n = np.cross(v2 - v1, v3 - v1)
    n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    d = np.sum(n * (r - v1), axis=-1)
    rho = r - d[..., None] * n
    ad = np.abs(d)
    K0 = np.zeros(np.broadcast_shapes(r.shape[:-1], v.shape[:-2]))
    K1 = np.zeros(K0.shape + (3,))
    for a, b in ((v1, v2), (v2, v3), (v3, v1)):
        e = b - a
        lhat = e / np.linalg.norm(e, axis=-1, keepdims=True)
        uhat = np.cross(lhat, n)
        t = np.sum((a - rho) * uhat, axis=-1)
        sm = np.sum((a - rho) * lhat, axis=-1)
        sp = np.sum((b - rho) * lhat, axis=-1)
        Rm = np.linalg.norm(r - a, axis=-1)
        Rp = np.linalg.norm(r - b, axis=-1)
        R0sq = t * t + d * d
        num = _rps(Rp, sp, R0sq)
        den = _rps(Rm, sm, R0sq)
        ok = (num > 0.0) & (den > 0.0)
        f = np.where(ok, np.log(np.where(ok, num, 1.0) / np.where(ok, den, 1.0)), 0.0)
        beta = (np.arctan2(t * sp, R0sq + ad * Rp) - np.arctan2(t * sm, R0sq + ad * Rm))
        K0 = K0 + t * f - ad * beta
        K1 = K1 + 0.5 * uhat * (R0sq * f + sp * Rp - sm * Rm)[..., None]
    return K0, K1

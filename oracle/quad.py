"""Seven-point, degree-five triangle quadrature (Radon's rule).

The paper does not state its quadrature; this rule is used for every surface
integral on both sides (near-field entries, radiation and receiving patterns,
right-hand sides, far fields), so quadrature error cancels between the HIP
path and this oracle.  Pin: exact integration of all monomials of total
degree <= 5 (tests/test_oracle_quad.py), which a wrong node or weight fails.
"""
from __future__ import annotations

import numpy as np

_s15 = np.sqrt(15.0)
_a1 = (6.0 - _s15) / 21.0
_a2 = (6.0 + _s15) / 21.0
_w1 = (155.0 - _s15) / 1200.0
_w2 = (155.0 + _s15) / 1200.0

# barycentric coordinates (weights of v0, v1, v2) and weights summing to 1
BARY = np.array([
    [1 / 3, 1 / 3, 1 / 3],
    [_a1, _a1, 1 - 2 * _a1],
    [_a1, 1 - 2 * _a1, _a1],
    [1 - 2 * _a1, _a1, _a1],
    [_a2, _a2, 1 - 2 * _a2],
    [_a2, 1 - 2 * _a2, _a2],
    [1 - 2 * _a2, _a2, _a2],
])
WEIGHTS = np.array([9 / 40, _w1, _w1, _w1, _w2, _w2, _w2])


def points(V, T):
    """Quadrature points [nt,7,3] of every triangle."""
    P = V[T]  # [nt,3,3]
    return np.einsum("qk,tkd->tqd", BARY, P)


def weights(area):
    """Quadrature weights [nt,7] (area times rule weight)."""
    return area[:, None] * WEIGHTS[None, :]

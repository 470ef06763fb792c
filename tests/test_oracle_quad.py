"""Pin: the 7-point rule integrates every monomial of degree <= 5 exactly
(closed form over the unit right triangle: int x^a y^b = a! b! / (a+b+2)!),
and fails at degree 6 (so the test would notice a lower-order rule)."""
from math import factorial

import numpy as np

from oracle import quad


def _exact(a, b):
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def test_degree5_exact():
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    T = np.array([[0, 1, 2]])
    P = quad.points(V, T)[0]
    W = quad.weights(np.array([0.5]))[0]
    for a in range(6):
        for b in range(6 - a):
            got = np.sum(W * P[:, 0] ** a * P[:, 1] ** b)
            assert abs(got - _exact(a, b)) < 1e-15, (a, b)
    errs = [abs(np.sum(W * P[:, 0] ** a * P[:, 1] ** (6 - a)) - _exact(a, 6 - a)) for a in range(7)]
    assert max(errs) > 1e-6


def test_weights_affine_invariant():
    rng = np.random.default_rng(0)
    V = rng.standard_normal((3, 3))
    T = np.array([[0, 1, 2]])
    area = 0.5 * np.linalg.norm(np.cross(V[1] - V[0], V[2] - V[0]))
    W = quad.weights(np.array([area]))[0]
    P = quad.points(V, T)[0]
    assert abs(W.sum() - area) < 1e-14
    # integral of a linear function = area * value at centroid
    f = P @ np.array([1.0, -2.0, 0.5]) + 3.0
    c = V.mean(axis=0) @ np.array([1.0, -2.0, 0.5]) + 3.0
    assert abs(np.sum(W * f) - area * c) < 1e-13

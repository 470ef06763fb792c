import numpy as np

from oracle import gmres


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(0)
    n = 80
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, rel = gmres.gmres(lambda v: A @ v, b, tol=1e-12, restart=20, maxit=500)
    assert rel <= 1e-12
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)

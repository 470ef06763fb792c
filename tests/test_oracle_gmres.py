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


def test_gmres_minimises_over_krylov_space():
    """k steps from x0 = 0 without restart reach min ||b - A z|| over
    z in span{b, ..., A^(k-1) b} (least squares on an orthonormal basis of
    the explicit Krylov vectors); full GMRES ends in at most n steps."""
    rng = np.random.default_rng(1)
    n = 24
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n) + (0.5 + 0.8j) * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    K = [b / np.linalg.norm(b)]
    for k in range(1, 11):
        Q, _ = np.linalg.qr(np.stack(K, 1))
        z, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
        best = np.linalg.norm(b - A @ (Q @ z)) / np.linalg.norm(b)
        _, it, rel = gmres.gmres(lambda v: A @ v, b, tol=1e-300, restart=k, maxit=k)
        assert it == k
        assert abs(rel - best) <= 1e-10 * max(best, 1e-3), (k, rel, best)
        v = A @ K[-1]
        K.append(v / np.linalg.norm(v))
    _, it, rel = gmres.gmres(lambda v: A @ v, b, tol=1e-10, restart=n, maxit=n)
    assert rel <= 1e-10 and it <= n

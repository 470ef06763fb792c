"""Plain restarted GMRES (Section 4 solves the PIE system with GMRES; the
paper states neither restart, tolerance nor preconditioner).

Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
matrix, stop when ||b - A x|| <= tol ||b||.  One right-hand side at a time.
Pins (tests/test_oracle_gmres.py): agreement with a direct LU solve, and
the defining property of GMRES: after k steps without restart the residual
is the least-squares minimum of ||b - A z|| over the Krylov space
span{b, A b, ..., A^(k-1) b}, checked by brute force on a small complex
matrix.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, x0=None, tol=1e-8, restart=100, maxit=1000):
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    it = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while it < maxit:
        if beta <= tol * bn:
            break
        m = min(restart, maxit - it)
        Vb = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        Vb[0] = r / beta
        j_used = 0
        for j in range(m):
            w = matvec(Vb[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                Vb[j + 1] = w / H[j + 1, j]
            # rotation i is G = [[conj(c), conj(s)], [-s, c]], which maps
            # (H[i, i], H[i + 1, i]) to (|.|, 0); the same G acts on the
            # later columns and on g
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, c = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            cs[j] = a / den if den else 1.0
            sn[j] = c / den if den else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            it += 1
            j_used = j + 1
            if abs(g[j + 1]) <= tol * bn:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + Vb[:j_used].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, it, beta / bn

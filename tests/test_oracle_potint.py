"""Pin: closed-form triangle potentials against a Duffy-transformed
high-order Gauss rule (the singularity at the projected point is removed by
splitting the triangle at it), for points inside, outside, above the plane
and on an edge's supporting line."""
import numpy as np

from oracle import potint


def _brute(r, tri, n=40, m=40):
    """Split the triangle at the projected point rho into three triangles
    (rho, a, b); split each edge (a, b) into m pieces; Duffy map every piece
    (the radial Jacobian cancels 1/R) and use an n x n Gauss rule."""
    x, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * w
    v1, v2, v3 = tri
    nrm = np.cross(v2 - v1, v3 - v1)
    nrm /= np.linalg.norm(nrm)
    d = np.dot(nrm, r - v1)
    rho = r - d * nrm
    K0 = 0.0
    K1 = np.zeros(3)
    for a0, b0 in ((v1, v2), (v2, v3), (v3, v1)):
        for k in range(m):
            a = a0 + (b0 - a0) * (k / m)
            b = a0 + (b0 - a0) * ((k + 1) / m)
            jac = np.dot(np.cross(a - rho, b - a), nrm)   # signed, twice the area
            p = rho + u[:, None, None] * ((a - rho)[None, None, :] + u[None, :, None] * (b - a)[None, None, :])
            R = np.linalg.norm(r - p, axis=-1)
            ww = (wu[:, None] * wu[None, :]) * u[:, None] * jac
            K0 += np.sum(ww / R)
            K1 += np.einsum("ij,ijd->d", ww / R, p - rho)
    return K0, K1


def test_against_duffy():
    rng = np.random.default_rng(1)
    for trial in range(6):
        tri = rng.standard_normal((3, 3))
        nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        nrm /= np.linalg.norm(nrm)
        cen = tri.mean(axis=0)
        pts = [
            cen,                                              # in plane, inside
            0.6 * tri[0] + 0.3 * tri[1] + 0.1 * tri[2],       # in plane, inside
            cen + 2.0 * (tri[1] - cen),                       # in plane, outside
            cen + 0.3 * nrm,                                  # above
            0.2 * tri[0] + 0.5 * tri[1] + 0.3 * tri[2] - 0.05 * nrm,  # just below
            tri[0] + 1.7 * (tri[1] - tri[0]),                 # on an edge line, outside
        ]
        for r in pts:
            K0, K1 = potint.potentials(r, tri)
            B0, B1 = _brute(r, tri)
            assert abs(K0 - B0) < 1e-10 * abs(B0), (trial, r)
            assert np.linalg.norm(K1 - B1) < 1e-10 * np.linalg.norm(B1), (trial, r)

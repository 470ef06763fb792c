"""Pins for the touching-pair moments of the dense PIE matrix (Section 2,
Eqs. (1)-(2); every entry is built from M0 = int int g, Mo = int int (r-ca) g,
Ms = int int (r'-cb) g and Mos = int int (r-ca).(r'-cb) g of triangle pairs).

For pairs that share a vertex the oracle integrates the inner integral's
static part 1/(4 pi R) in closed form, the smooth remainder with the 7-point
rule, the outer integral with the 7-point rule, and averages the pair with
its swap.  Two independent checks, for a triangle with itself and for
edge-adjacent and vertex-adjacent pairs:
* the same definition evaluated another way: the static part of the inner
  integral by a Duffy-split high-order Gauss rule instead of the closed
  forms, the smooth remainder with the 7-point rule as in the oracle, at the
  same seven outer points, then the same swap average.  For the self pair
  the two agree to rounding (1e-12); for adjacent pairs the Duffy rule
  itself converges slowly (outer points lie close to the shared edge, where
  the integrand is nearly singular; 2e-7 at 40 x 40 points on 40 segments
  per edge), so 1e-6 -- a dropped term, a wrong sign or a swapped operand
  would show at 1e-2 or more.  This checks the closed forms, the centroid
  offsets and the assembly of all four moments;
* the exact double integral (high-order rules on both triangles): agreement
  within the error of the 7-point outer rule (measured 7e-5 ... 6e-3 on
  these pairs, on the scale at which the moments enter the entries),
  which bounds what the outer quadrature costs."""
import numpy as np
import pytest

import synth
from oracle import mom, quad


def _inner(r, tri, k, n=40, m=40):
    """int_T exp(ikR)/(4 pi R) (1, r' - c) dr' for one point r: the triangle is
    split at the projection rho of r into (rho, a, b) pieces, every edge into
    m segments, each piece Duffy-mapped (the radial Jacobian cancels 1/R) and
    integrated with an n x n Gauss rule."""
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (x + 1.0), 0.5 * w
    v1, v2, v3 = tri
    c = (v1 + v2 + v3) / 3.0
    nrm = np.cross(v2 - v1, v3 - v1)
    nrm /= np.linalg.norm(nrm)
    rho = r - np.dot(nrm, r - v1) * nrm
    K0 = 0.0 + 0.0j
    K1 = np.zeros(3, np.complex128)
    for a0, b0 in ((v1, v2), (v2, v3), (v3, v1)):
        for s in range(m):
            a = a0 + (b0 - a0) * (s / m)
            b = a0 + (b0 - a0) * ((s + 1) / m)
            jac = np.dot(np.cross(a - rho, b - a), nrm)
            p = rho + u[:, None, None] * ((a - rho)[None, None, :] + u[None, :, None] * (b - a)[None, None, :])
            R = np.linalg.norm(r - p, axis=-1)
            g = np.exp(1j * k * R) / (4.0 * np.pi * R)
            ww = (wu[:, None] * wu[None, :]) * u[:, None] * jac * g
            K0 += np.sum(ww)
            K1 += np.einsum("ij,ijd->d", ww, p - c)
    return K0, K1


def _inner_split(r, tri, Pb, Wb, k):
    """The oracle's inner rule: static part by the Duffy rule, smooth
    remainder (exp(ikR) - 1)/(4 pi R) at the 7-point rule (Pb, Wb)."""
    S0, S1 = _inner(r, tri, 0.0)
    c = tri.mean(axis=0)
    R = np.linalg.norm(r - Pb, axis=1)
    Rs = np.where(R > 0.0, R, 1.0)
    h = np.where(R > 0.0, (np.exp(1j * k * Rs) - 1.0) / (4.0 * np.pi * Rs), 1j * k / (4.0 * np.pi))
    return S0 + np.sum(Wb * h), S1 + np.einsum("j,jd->d", Wb * h, Pb - c)


def _moments(P, W, ca, tri_b, k, rule_b=None):
    """(M0, Mo, Ms, Mos) with the outer rule (P, W) on triangle a; the inner
    integral exact (rule_b None) or the oracle's split (rule_b = (Pb, Wb))."""
    M0 = 0.0 + 0.0j
    Mo = np.zeros(3, np.complex128)
    Ms = np.zeros(3, np.complex128)
    Mos = 0.0 + 0.0j
    for r, wr in zip(P, W):
        K0, K1 = _inner(r, tri_b, k) if rule_b is None else _inner_split(r, tri_b, *rule_b, k)
        M0 += wr * K0
        Mo += wr * (r - ca) * K0
        Ms += wr * K1
        Mos += wr * np.dot(r - ca, K1)
    return M0, Mo, Ms, Mos


def _sym(mab, mba):
    """The oracle's swap average: M0 and Mos averaged, Mo with the swap's Ms."""
    return (0.5 * (mab[0] + mba[0]), 0.5 * (mab[1] + mba[2]), 0.5 * (mab[2] + mba[1]),
            0.5 * (mab[3] + mba[3]))


def _collapsed(tri, n=14):
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (x + 1), 0.5 * w
    v0, v1, v2 = tri
    A = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    P, W = [], []
    for i in range(n):
        for j in range(n):
            s_, t_ = u[i], u[j] * (1 - u[i])
            P.append(v0 + s_ * (v1 - v0) + t_ * (v2 - v0))
            W.append(wu[i] * wu[j] * (1 - u[i]) * 2 * A)
    return np.array(P), np.array(W)


@pytest.fixture(scope="module")
def pairs():
    V, T = synth.icosphere(2)
    p = mom.Problem(V, T, 0.5 * synth.C0 / synth.DIAMETER)
    m = p.mesh
    a = 7
    shared = np.array([len(set(m.T[a]) & set(m.T[b])) for b in range(m.nT)])
    edge = int(np.nonzero(shared == 2)[0][0])
    vert = int(np.nonzero(shared == 1)[0][0])
    return p, [(a, a), (a, edge), (edge, a), (a, vert)]


def _oracle(p, a, b):
    M0, Mo, Ms, Mos = p.pair_moments([a], [b])
    return M0[0], Mo[0], Ms[0], Mos[0]


def _close(x, y, tol):
    for u, v in zip(x, y):
        assert np.linalg.norm(np.atleast_1d(u - v)) <= tol * np.linalg.norm(np.atleast_1d(v)), (u, v)


def test_touching_moments_same_rule(pairs):
    p, prs = pairs
    m = p.mesh
    for a, b in prs:
        mab = _moments(p.P[a], p.W[a], m.centroid[a], m.V[m.T[b]], p.k, (p.P[b], p.W[b]))
        mba = _moments(p.P[b], p.W[b], m.centroid[b], m.V[m.T[a]], p.k, (p.P[a], p.W[a]))
        _close(_oracle(p, a, b), _sym(mab, mba), 1e-12 if a == b else 1e-6)


def test_touching_moments_exact_double_integral(pairs):
    p, prs = pairs
    m = p.mesh
    for a, b in prs:
        Pa, Wa = _collapsed(m.V[m.T[a]])
        Pb, Wb = _collapsed(m.V[m.T[b]])
        ex = _sym(_moments(Pa, Wa, m.centroid[a], m.V[m.T[b]], p.k),
                  _moments(Pb, Wb, m.centroid[b], m.V[m.T[a]], p.k))
        got = _oracle(p, a, b)
        # the moments enter the entries multiplied by offsets of the size of a
        # triangle (free vertex - centroid), so the first and second moments
        # are measured against |M0| h and |M0| h^2 (they nearly cancel for the
        # self pair, where a relative measure would be meaningless)
        h = max(np.linalg.norm(m.V[m.T[a]][i] - m.V[m.T[a]][j]) for i in range(3) for j in range(3))
        scale = (abs(ex[0]), abs(ex[0]) * h, abs(ex[0]) * h, abs(ex[0]) * h * h)
        errs = [np.linalg.norm(np.atleast_1d(u - v)) / s_ for u, v, s_ in zip(got, ex, scale)]
        print("pair", a, b, "7-point outer rule vs exact:", ["%.1e" % e for e in errs])
        assert max(errs) < 1e-2

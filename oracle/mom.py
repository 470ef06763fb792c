"""Dense Galerkin method of moments for the PIEs (Section 2, Eqs. (1)-(2)).

This is the plain definition the MLFMA approximates: the N x N matrix of
Eqs. (1)-(2) discretised with RWG functions for J and pulse functions for n.A,
Galerkin-tested with the same functions (N = T + E).  Moving the gradient of
the Green's function onto the testing function by parts (Section 3, last
paragraph) leaves g as the only kernel:

    Z^JJ_mn = mu0 <f_m, int f_n g>            (vector potential of J)
    Z^JA_mp = <div f_m, int P_p g>            (= <f_m, int P_p grad' g>)
    Z^AJ_qn = <P_q, int div' f_n g>           (first term of Eq. (2))
    Z^AA_qp = w^2 eps0 <P_q, int P_p g>       (second term of Eq. (2))

with g = exp(i k R)/(4 pi R).  Z is complex symmetric and Z^AJ = (Z^JA)^T.
Unknown order: the E RWG coefficients (edge-table order) then the T pulse
coefficients (triangle order).

Every integral uses the 7-point rule of ``quad`` on both triangles.  For
triangle pairs that share at least one vertex, the static part 1/(4 pi R) of
the inner integral is done in closed form (``potint``) and only the smooth
remainder (exp(ikR)-1)/(4 pi R) uses the rule; the pair's integrals are then
averaged with those of the swapped pair, so Z is exactly symmetric.  (The
paper states neither the rule nor the singular treatment.)

Pins: symmetry, the Mie series and the Rayleigh limit for a PEC sphere,
gauge invariance of J, closed forms on tiny meshes (tests/test_oracle_mom.py).
"""
from __future__ import annotations

import numpy as np

from . import mesh as _mesh
from . import potint, quad

MU0 = 4.0e-7 * np.pi
C0 = 299792458.0
EPS0 = 1.0 / (MU0 * C0 * C0)


class Problem:
    """A mesh at one frequency, with its quadrature."""

    def __init__(self, V, T, freq):
        self.mesh = _mesh.build(V, T)
        self.freq = float(freq)
        self.omega = 2.0 * np.pi * self.freq
        self.k = self.omega / C0
        m = self.mesh
        self.P = quad.points(m.V, m.T)          # [nt,7,3]
        self.W = quad.weights(m.area)           # [nt,7]

    @property
    def N(self):
        return self.mesh.N

    # ------------------------------------------------------------------
    # triangle-pair moments
    # ------------------------------------------------------------------
    def _raw_moments(self, ta, tb, touching):
        """Unsymmetrised moments of triangle pairs (ta obs, tb src):
        M0 = int int g, Mo = int int (r - ca) g, Ms = int int (r' - cb) g,
        Mos = int int (r - ca).(r' - cb) g, with ca, cb the centroids."""
        k = self.k
        m = self.mesh
        Pa, Pb = self.P[ta], self.P[tb]
        Wa, Wb = self.W[ta], self.W[tb]
        ca, cb = m.centroid[ta], m.centroid[tb]
        ra = Pa - ca[:, None, :]
        rb = Pb - cb[:, None, :]
        D = Pa[:, :, None, :] - Pb[:, None, :, :]
        R = np.sqrt(np.sum(D * D, axis=-1))                 # [n,7,7]
        g = np.empty(R.shape, dtype=np.complex128)
        far = ~touching
        Rf = R[far]
        g[far] = np.exp(1j * k * Rf) / (4.0 * np.pi * Rf)
        # touching pairs: smooth remainder (exp(ikR)-1)/(4 pi R)
        #               = (ik/4pi) exp(ikR/2) sinc(kR/2)  (finite at R = 0)
        Rt = R[touching]
        g[touching] = ((1j * k / (4.0 * np.pi)) * np.exp(0.5j * k * Rt)
                       * np.sinc(k * Rt / (2.0 * np.pi)))
        G = (Wa[:, :, None] * Wb[:, None, :]) * g
        Gi = G.sum(axis=2)                                  # [n,7] summed over src
        H = np.matmul(G, rb)                                # [n,7,3] sum_j G_ij rb_j
        M0 = Gi.sum(axis=1)
        Mo = np.einsum("ni,nid->nd", Gi, ra)
        Ms = H.sum(axis=1)
        Mos = np.einsum("nid,nid->n", H, ra)
        if np.any(touching):
            it = np.nonzero(touching)[0]
            tri_b = m.V[m.T[tb[it]]]                        # [nt_,3,3]
            r = Pa[it]                                      # [nt_,7,3]
            K0, K1 = potint.potentials(r, tri_b[:, None, :, :])
            nb = m.normal[tb[it]]
            dist = np.einsum("nqd,nd->nq", r - tri_b[:, None, 0, :], nb)
            rho = r - dist[..., None] * nb[:, None, :]
            K1c = K1 + (rho - cb[it][:, None, :]) * K0[..., None]   # int (r'-cb)/R
            w4 = Wa[it] / (4.0 * np.pi)
            M0[it] += np.sum(w4 * K0, axis=1)
            Mo[it] += np.einsum("nq,nq,nqd->nd", w4, K0, ra[it])
            Ms[it] += np.einsum("nq,nqd->nd", w4, K1c)
            Mos[it] += np.einsum("nq,nqd,nqd->n", w4, ra[it], K1c)
        return M0, Mo, Ms, Mos

    def touching(self, ta, tb):
        Ta, Tb = self.mesh.T[ta], self.mesh.T[tb]
        return np.any(Ta[:, :, None] == Tb[:, None, :], axis=(1, 2))

    def pair_moments(self, ta, tb, chunk=65536):
        """Moments of triangle pairs with touching pairs symmetrised:
        I(a,b) := (I(a,b) + I(b,a)^T)/2."""
        ta = np.asarray(ta, dtype=np.int64)
        tb = np.asarray(tb, dtype=np.int64)
        n = ta.size
        M0 = np.empty(n, np.complex128)
        Mo = np.empty((n, 3), np.complex128)
        Ms = np.empty((n, 3), np.complex128)
        Mos = np.empty(n, np.complex128)
        for s in range(0, n, chunk):
            a, b = ta[s:s + chunk], tb[s:s + chunk]
            touch = self.touching(a, b)
            m0, mo, ms, mos = self._raw_moments(a, b, touch)
            if np.any(touch):
                it = np.nonzero(touch)[0]
                n0, no, ns, nos = self._raw_moments(b[it], a[it], np.ones(it.size, bool))
                m0[it] = 0.5 * (m0[it] + n0)
                mo[it] = 0.5 * (mo[it] + ns)
                ms[it] = 0.5 * (ms[it] + no)
                mos[it] = 0.5 * (mos[it] + nos)
            M0[s:s + chunk], Mo[s:s + chunk], Ms[s:s + chunk], Mos[s:s + chunk] = m0, mo, ms, mos
        return M0, Mo, Ms, Mos

    # ------------------------------------------------------------------
    # basis description
    # ------------------------------------------------------------------
    def _basis_halves(self, idx):
        """RWG unknowns among ``idx`` as two halves (T+ then T-), each with
        its triangle, vector scale +-l/(2A), divergence +-l/A and free
        vertex; pulse unknowns with their triangle."""
        m = self.mesh
        idx = np.asarray(idx, dtype=np.int64)
        isr = idx < m.nE
        pos_r = np.nonzero(isr)[0]
        e = idx[isr]
        pos_p = np.nonzero(~isr)[0]
        p = idx[~isr] - m.nE
        halves = []
        for h, sgn in ((0, 1.0), (1, -1.0)):
            t = m.tri[e, h]
            A = m.area[t]
            halves.append((t, sgn * m.length[e] / (2.0 * A), sgn * m.length[e] / A, m.free[e, h]))
        return pos_r, halves, pos_p, p

    def zblock(self, rows, cols, chunk=2048):
        """Dense block Z[rows][:, cols] (canonical unknown numbering)."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        Z = np.zeros((rows.size, cols.size), dtype=np.complex128)
        R = self._basis_halves(rows)
        for c0 in range(0, cols.size, chunk):
            cc = cols[c0:c0 + chunk]
            C = self._basis_halves(cc)
            Z[:, c0:c0 + cc.size] = self._assemble(R, C, rows.size, cc.size)
        return Z

    def _assemble(self, R, C, nr, nc):
        m = self.mesh
        w2e = self.omega ** 2 * EPS0
        pr, hr, pp_r, tp_r = R
        pc, hc, pp_c, tp_c = C
        tr_all = np.concatenate([hr[0][0], hr[1][0], tp_r])
        tc_all = np.concatenate([hc[0][0], hc[1][0], tp_c])
        ur, ir = np.unique(tr_all, return_inverse=True)
        uc, ic = np.unique(tc_all, return_inverse=True)
        A, B = np.meshgrid(ur, uc, indexing="ij")
        M0, Mo, Ms, Mos = self.pair_moments(A.ravel(), B.ravel())
        shp = (ur.size, uc.size)
        M0 = M0.reshape(shp)
        Mo = Mo.reshape(shp + (3,))
        Ms = Ms.reshape(shp + (3,))
        Mos = Mos.reshape(shp)
        nr_, nc_ = pr.size, pc.size
        iRh = (ir[:nr_], ir[nr_:2 * nr_])
        iCh = (ic[:nc_], ic[nc_:2 * nc_])
        iRp = ir[2 * nr_:]
        iCp = ic[2 * nc_:]
        Z = np.zeros((nr, nc), dtype=np.complex128)
        if nr_ and nc_:
            acc = np.zeros((nr_, nc_), dtype=np.complex128)
            for a in range(2):
                ta, vr, _, fr = hr[a]
                pa = m.V[fr] - m.centroid[ta]                    # p - ca
                for b in range(2):
                    tb, vc, _, fc = hc[b]
                    pb = m.V[fc] - m.centroid[tb]                # q - cb
                    sub = np.ix_(iRh[a], iCh[b])
                    # I1 = Mos + (ca-p).Ms + (cb-q).Mo + (ca-p).(cb-q) M0
                    I1 = (Mos[sub]
                          - np.einsum("id,ijd->ij", pa, Ms[sub])
                          - np.einsum("jd,ijd->ij", pb, Mo[sub])
                          + (pa @ pb.T) * M0[sub])
                    acc += (vr[:, None] * vc[None, :]) * I1
            Z[np.ix_(pr, pc)] = MU0 * acc
        if nr_ and pp_c.size:
            acc = np.zeros((nr_, pp_c.size), dtype=np.complex128)
            for a in range(2):
                acc += hr[a][2][:, None] * M0[np.ix_(iRh[a], iCp)]
            Z[np.ix_(pr, pp_c)] = acc
        if pp_r.size and nc_:
            acc = np.zeros((pp_r.size, nc_), dtype=np.complex128)
            for b in range(2):
                acc += hc[b][2][None, :] * M0[np.ix_(iRp, iCh[b])]
            Z[np.ix_(pp_r, pc)] = acc
        if pp_r.size and pp_c.size:
            Z[np.ix_(pp_r, pp_c)] = w2e * M0[np.ix_(iRp, iCp)]
        return Z

    def dense(self):
        """The full N x N matrix (small meshes only)."""
        idx = np.arange(self.N)
        return self.zblock(idx, idx)

    # ------------------------------------------------------------------
    # right-hand side and far field
    # ------------------------------------------------------------------
    def incident_potentials(self, r, khat, pol, amp, gauge=0):
        """Plane wave E = amp pol exp(i k khat.r) (E0 = 1 V/m).
        gauge 0 (Lorenz, finite at zero frequency):
            Phi = -amp (pol.r) e^{ik khat.r}, A = -(amp/c0)(pol.r) khat e^{ik khat.r};
        gauge 1: Phi = 0, A = E/(i omega).
        Both give E = i omega A - grad Phi.  Returns (A [...,3], Phi [...])."""
        k, w = self.k, self.omega
        ph = np.exp(1j * k * (r @ khat)) * amp
        if gauge == 0:
            pr = r @ pol
            Phi = -pr * ph
            A = (-(pr * ph) / C0)[..., None] * khat
        else:
            Phi = np.zeros(ph.shape, dtype=np.complex128)
            A = (ph / (1j * w))[..., None] * pol
        return A, Phi

    def rhs(self, khat, pol, amp, gauge=0):
        """Right-hand sides [N,R]: b^J_m = -<f_m, A^inc> (Eq. (1)),
        b^A_q = -i w eps0 <P_q, Phi^inc> (Eq. (2))."""
        m = self.mesh
        khat = np.atleast_2d(khat)
        pol = np.atleast_2d(pol)
        amp = np.atleast_1d(amp)
        nR = khat.shape[0]
        b = np.zeros((self.N, nR), dtype=np.complex128)
        for r in range(nR):
            A, Phi = self.incident_potentials(self.P, khat[r], pol[r], amp[r], 0 if gauge == 0 else 1)
            bj = np.zeros(m.nE, dtype=np.complex128)
            for h, sgn in ((0, 1.0), (1, -1.0)):
                t = m.tri[:, h]
                f = (sgn * m.length / (2.0 * m.area[t]))[:, None, None] * (
                    self.P[t] - m.V[m.free[:, h]][:, None, :])
                bj += np.einsum("eqd,eqd,eq->e", f, A[t], self.W[t])
            b[: m.nE, r] = -bj
            b[m.nE:, r] = -1j * self.omega * EPS0 * np.sum(self.W * Phi, axis=1)
        return b

    def charge(self, x, khat, pol, amp, gauge=0):
        """Near-zone charge density per triangle (Section 2, the paragraph
        after Eq. (2)).  sigma = n.grad(Phi) solves Eq. (3),
            int_S sigma(r') g(r, r') dr' = Phi^inc(r)   (r on S),
        with sigma expanded in the pulse functions and tested with them:
            sum_p sigma_p <P_q, int P_p g> = <P_q, Phi^inc>
        (the pulse-pulse matrix is Z^AA / (w^2 eps0)); then
            rho = i w eps0 (n.A) - eps0 sigma,
        with n.A the pulse part of the PIE solution x [N,R].
        Returns (sigma [T,R], rho [T,R])."""
        m = self.mesh
        x = np.asarray(x).reshape(self.N, -1)
        khat = np.atleast_2d(khat)
        pol = np.atleast_2d(pol)
        amp = np.atleast_1d(amp)
        idx = np.arange(m.nE, self.N)
        S = self.zblock(idx, idx) / (self.omega ** 2 * EPS0)
        phi = np.zeros((m.nT, khat.shape[0]), dtype=np.complex128)
        for r in range(khat.shape[0]):
            _, Phi = self.incident_potentials(self.P, khat[r], pol[r], amp[r], 0 if gauge == 0 else 1)
            phi[:, r] = np.sum(self.W * Phi, axis=1)
        sigma = np.linalg.solve(S, phi)
        rho = 1j * self.omega * EPS0 * x[m.nE:] - EPS0 * sigma
        return sigma, rho

    def current_radiation(self, x, dirs):
        """int J(r') exp(-i k rhat.r') dr' for J = sum a_n f_n;
        x [N,R] or [N]; returns [R,nd,3]."""
        m = self.mesh
        x = np.atleast_2d(np.asarray(x).T).T if np.ndim(x) == 1 else np.asarray(x)
        a = x[: m.nE]
        out = np.zeros((x.shape[1], dirs.shape[0], 3), dtype=np.complex128)
        for h, sgn in ((0, 1.0), (1, -1.0)):
            t = m.tri[:, h]
            f = (sgn * m.length / (2.0 * m.area[t]))[:, None, None] * (
                self.P[t] - m.V[m.free[:, h]][:, None, :])           # [E,7,3]
            ph = np.exp(-1j * self.k * np.einsum("eqd,sd->eqs", self.P[t], dirs))
            fw = f * self.W[t][..., None]
            out += np.einsum("er,eqd,eqs->rsd", a, fw, ph)
        return out

    def farfield(self, x, dirs):
        """F(rhat) = lim r e^{-ikr} E^s = (i w mu0/4pi)(I - rhat rhat).int J e^{-ik rhat.r'}."""
        dirs = np.atleast_2d(dirs)
        Jr = self.current_radiation(x, dirs)
        rr = np.einsum("rsd,sd->rs", Jr, dirs)
        Jt = Jr - rr[..., None] * dirs[None, :, :]
        return (1j * self.omega * MU0 / (4.0 * np.pi)) * Jt

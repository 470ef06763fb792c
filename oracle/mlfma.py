"""MLFMA with the approximate stable diagonalisation, in FP64 (Section 3).

Steps, in the paper's order for one MVM:
  near field   y = Z_near x, the exact matrix entries of Eqs. (1)-(2) for
               basis functions (RWG part) and triangles (scalar part) in near
               finest-level boxes;
  aggregation  radiation patterns of every finest box, then shifted up to
               coarser levels (down to level 3);
  translation  at every level l >= 3, diagonal (per direction) products of
               the modified translation function of Eq. (5) with the patterns
               of each box's interaction list, using the scaled plane waves of
               Eq. (4);
  disaggregation  incoming patterns shifted down to the finest level, then
               received by the testing functions and added to y.
How the blocks of Z are split between near and far interactions (the
scalar operator per triangle, the vector part per RWG function) is stated
in the class docstring.

Eq. (4) with r - r' = w + v, w = C_obs - C_src, v = (r - C_obs) - (r' - C_src),
kappa = k/s:
    g(r,r') ~= (ik/(16 pi^2)) sum_q w_q exp(i kappa khat_q . v) alpha~(khat_q)
    alpha~  = sum_{t=0}^{tau} i^t (2t+1) s^t h_t^(1)(k|w|) P_t(khat . what)  (Eq. (5))
(the printed prefactor ik/(4 pi) holds when the k-space integral is the mean
over the unit sphere; with quadrature weights summing to 4 pi the factor is
ik/(16 pi^2) -- reading stated in the design notes and pinned by comparing
with the exact g).

Readings where the paper is silent:
* k-space samples: Gauss-Legendre in cos(theta) (n_theta = tau+1) times
  uniform phi_j = 2 pi j / n_phi (n_phi = 2 tau + 2); symmetric under
  khat -> -khat.
* scale factor per level: s_l = min(1, k d_l / x), so kappa_l d_l = x (the
  scaled box size) wherever s < 1.  The tables of tau and s of the paper's
  reference [jp045] are not available; (tau, x) are chosen by measured error.
* truncation per level: as boxes grow, s -> 1 and Eq. (5) becomes the
  ordinary translation function, which needs more terms; a level may take
  its own tau_l (Params.level_tau), while every level keeps the k-space
  samples of the largest tau (so patterns move between levels without
  interpolation) and the inter-level filter keeps degrees up to the parent
  level's tau_l.
* shifting a pattern from a child (kappa_c) to its parent (kappa_p): the
  degree-l spherical-harmonic content is rescaled by (kappa_p/kappa_c)^l
  (the same small-argument behaviour s^t j_t(k v/s) ~ j_t(k v) that underlies
  Eq. (5)), then phase-shifted to the parent centre:
      S_p = sum_c exp(-i kappa_p khat.(C_c - C_p)) (F S_c),
      F_qq' = w_q' sum_{l<=tau} (2l+1)/(4 pi) (kappa_p/kappa_c)^l P_l(khat_q.khat_q');
  disaggregation applies the transpose: G_c += F^T (exp(+i...) G_p).

Pins: the diagonalised kernel against the exact Green's function at every far
offset, and the full MVM against the dense matrix of ``mom`` to the
diagonalisation's truncation error (tests/test_oracle_mlfma.py); the
translation coefficients against the closed forms of h_0, h_1 and their
small-argument limits (tests/test_oracle_alpha.py).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from numpy.polynomial import legendre as _leg
from scipy.special import eval_legendre, spherical_jn, spherical_yn

from . import mom as _mom
from . import octree as _octree


@dataclasses.dataclass(frozen=True)
class Params:
    tau: int = 6          # truncation number of Eq. (5) (the largest, when per level)
    x: float = 0.07       # scaled box size k d / s where s < 1
    n_theta: int = 0      # 0: tau + 1
    n_phi: int = 0        # 0: 2 tau + 2
    level_tau: tuple = ()  # ((level, tau_l), ...): a smaller truncation at those levels

    def tau_at(self, level):
        return dict(self.level_tau).get(level, self.tau)

    @property
    def nth(self):
        return self.n_theta or self.tau + 1

    @property
    def nph(self):
        return self.n_phi or 2 * self.tau + 2


def samples(p: Params):
    """Directions khat_q [Q,3] and weights w_q [Q] (sum 4 pi);
    q = i_theta * n_phi + j_phi."""
    ct, wt = _leg.leggauss(p.nth)
    ph = 2.0 * np.pi * np.arange(p.nph) / p.nph
    st = np.sqrt(1.0 - ct * ct)
    kh = np.stack([
        (st[:, None] * np.cos(ph)[None, :]).ravel(),
        (st[:, None] * np.sin(ph)[None, :]).ravel(),
        np.repeat(ct, p.nph),
    ], axis=1)
    w = np.repeat(wt, p.nph) * (2.0 * np.pi / p.nph)
    return kh, w


def scale_factor(k, d, x):
    return min(1.0, k * d / x)


def alpha_tilde(k, s, tau, wvec, khat):
    """Eq. (5) at direction(s) khat [Q,3] for the vector w [3]."""
    wn = float(np.linalg.norm(wvec))
    cosang = khat @ (np.asarray(wvec) / wn)
    out = np.zeros(khat.shape[0], dtype=np.complex128)
    for t in range(tau + 1):
        h = spherical_jn(t, k * wn) + 1j * spherical_yn(t, k * wn)
        out += (1j ** t) * (2 * t + 1) * (s ** t) * h * eval_legendre(t, cosang)
    return out


def kernel(k, s, p: Params, r, rp, cobs, csrc):
    """Diagonalised g~(r, r') for observation r in the box centred at cobs and
    source r' in the box centred at csrc (Eq. (4))."""
    kh, w = samples(p)
    kap = k / s
    wv = np.asarray(cobs) - np.asarray(csrc)
    v = (np.asarray(r) - cobs) - (np.asarray(rp) - csrc)
    a = alpha_tilde(k, s, p.tau, wv, kh)
    return (1j * k / (16.0 * np.pi ** 2)) * np.sum(w * np.exp(1j * kap * (kh @ v)) * a)


def interlevel_filter(khat, w, tau, ratio):
    """F_qq' = w_q' sum_{l<=tau} (2l+1)/(4 pi) ratio^l P_l(khat_q . khat_q')."""
    c = np.clip(khat @ khat.T, -1.0, 1.0)
    F = np.zeros(c.shape)
    for l in range(tau + 1):
        F += (2 * l + 1) / (4.0 * np.pi) * ratio ** l * eval_legendre(l, c)
    return F * w[None, :]


class MLFMA:
    """One operator: mesh + frequency + tree + parameters.

    Near/far split.  With S_qp = <P_q, int P_p g> (the pulse-pulse Galerkin
    matrix of g) and the divergence matrix G[m, t] = div f_m on triangle t
    (+-l/A), the blocks of Eqs. (1)-(2) after the by-parts step of Section 3
    are Z^JA = G S, Z^AJ = S G^T and Z^AA = w^2 eps0 S: one scalar operator
    acting on sigma = x_A (for the RWG rows) and on u = G^T x_J + w^2 eps0 x_A
    (for the pulse rows).  The paper does not say how basis functions are
    split between near and far interactions; here the split keeps that
    identity for the approximation too:
      * S is applied per triangle: each triangle radiates and receives at the
        finest box of its centroid (the box of its pulse), and a triangle
        pair is near when those boxes are neighbours;
      * the vector part mu0 <f_m, int f_n g> is applied per RWG function,
        both halves at the finest box of its edge midpoint, near when the
        two RWG boxes are neighbours.
    Then Z_mlfma = [[mu0 L~, G S~], [S~ G^T, w^2 eps0 S~]] exactly, so the
    divergence-free (loop) currents give no scalar source and the charge
    vector with S~ b = const * area is annihilated by the JA block, as for the
    dense matrix; only the 7-point-rule moments and Eqs. (4)-(5) differ."""

    def __init__(self, prob: _mom.Problem, L: int, params: Params = Params()):
        self.prob = prob
        self.p = params
        self.tree = _octree.build(prob.mesh, L)
        self.L = L
        k = prob.k
        self.khat, self.w = samples(params)
        self.Q = self.w.size
        tr = self.tree
        self.s, self.kappa, self.d = {}, {}, {}
        for l in range(2, L + 1):
            d = tr.size(l)
            self.d[l] = d
            self.s[l] = scale_factor(k, d, params.x)
            self.kappa[l] = k / self.s[l]
        offs = _octree.far_offsets()
        self.T = {}
        pref = 1j * k / (16.0 * np.pi ** 2)
        for l in range(3, L + 1):
            tab = np.zeros((offs.shape[0], self.Q), dtype=np.complex128)
            for i, o in enumerate(offs):
                tab[i] = pref * self.w * alpha_tilde(k, self.s[l], params.tau_at(l), o * self.d[l], self.khat)
            self.T[l] = tab
        self.F = {}
        for l in range(3, L):
            self.F[l] = interlevel_filter(self.khat, self.w, params.tau_at(l),
                                          self.kappa[l] / self.kappa[l + 1])
        m = prob.mesh
        self.E = m.nE
        self.tri_box = tr.box_of[m.nE:]      # finest box of each triangle (its pulse's box)
        # G as two entries per RWG row: triangle and divergence +-l/A
        self.g_tri = m.tri                               # [E,2]
        self.g_div = np.stack([m.length / m.area[m.tri[:, 0]],
                               -m.length / m.area[m.tri[:, 1]]], axis=1)
        self._near = None

    # ------------------------------------------------------------------
    # the divergence matrix G and its transpose
    # ------------------------------------------------------------------
    def div_sources(self, xJ):
        """G^T x_J: the divergence of the current on each triangle [T,R]."""
        m = self.prob.mesh
        out = np.zeros((m.nT, xJ.shape[1]), dtype=np.complex128)
        for h in range(2):
            np.add.at(out, self.g_tri[:, h], self.g_div[:, h, None] * xJ)
        return out

    def div_test(self, phi):
        """G phi: the divergence of each RWG tested against a per-triangle
        potential phi [T,R] -> [E,R]."""
        return self.g_div[:, 0, None] * phi[self.g_tri[:, 0]] + self.g_div[:, 1, None] * phi[self.g_tri[:, 1]]

    # ------------------------------------------------------------------
    # radiation patterns at the finest level
    # ------------------------------------------------------------------
    def rwg_patterns(self, e):
        """Vector patterns F_n(q) = int f_n(r') exp(-i kappa khat_q.(r' - C)) dr'
        [n,Q,3] of RWG functions e about their boxes' centres, at kappa_L."""
        pr = self.prob
        m = pr.mesh
        tr = self.tree
        e = np.asarray(e, dtype=np.int64)
        C = tr.levels[self.L].centre[tr.box_of[e]]
        kap = self.kappa[self.L]
        F = np.zeros((e.size, self.Q, 3), dtype=np.complex128)
        for h, sgn in ((0, 1.0), (1, -1.0)):
            t = m.tri[e, h]
            P = pr.P[t]                                            # [n,7,3]
            ph = np.exp(-1j * kap * np.einsum("nid,qd->niq", P - C[:, None, :], self.khat))
            fv = (sgn * m.length[e] / (2.0 * m.area[t]))[:, None, None] * (
                P - m.V[m.free[e, h]][:, None, :])
            F += np.einsum("ni,nid,niq->nqd", pr.W[t], fv, ph)
        return F

    def tri_patterns(self, t):
        """Scalar patterns P_t(q) = int_t exp(-i kappa khat_q.(r' - C)) dr' [n,Q]
        of triangles t about their own boxes' centres, at kappa_L."""
        pr = self.prob
        t = np.asarray(t, dtype=np.int64)
        C = self.tree.levels[self.L].centre[self.tri_box[t]]
        ph = np.exp(-1j * self.kappa[self.L] * np.einsum("nid,qd->niq", pr.P[t] - C[:, None, :], self.khat))
        return np.einsum("ni,niq->nq", pr.W[t], ph)

    # ------------------------------------------------------------------
    # near field
    # ------------------------------------------------------------------
    def near_matrix(self):
        """Near-field blocks per finest box: (RWG rows, RWG cols, mu0 L block)
        and (triangle rows, triangle cols, S block)."""
        if self._near is None:
            pr = self.prob
            tr = self.tree
            E = self.E
            w2e = pr.omega ** 2 * _mom.EPS0
            JJ, SS = [], []
            for b in range(tr.box_ptr.size - 1):
                u = tr.perm[tr.box_ptr[b]:tr.box_ptr[b + 1]]
                nbrs = tr.near_idx[tr.near_ptr[b]:tr.near_ptr[b + 1]]
                cols = np.concatenate([tr.perm[tr.box_ptr[j]:tr.box_ptr[j + 1]] for j in nbrs])
                rj, cj = u[u < E], cols[cols < E]
                rt, ct = u[u >= E], cols[cols >= E]
                JJ.append((rj, cj, pr.zblock(rj, cj)))
                SS.append((rt - E, ct - E, pr.zblock(rt, ct) / w2e))
            self._near = (JJ, SS)
        return self._near

    def near(self, x):
        """Near-field part Z_near x; x [N] or [N,R] canonical order."""
        x = np.asarray(x, dtype=np.complex128)
        one = x.ndim == 1
        if one:
            x = x[:, None]
        E = self.E
        w2e = self.prob.omega ** 2 * _mom.EPS0
        xJ, xA = x[:E], x[E:]
        u = self.div_sources(xJ) + w2e * xA
        JJ, SS = self.near_matrix()
        yJ = np.zeros(xJ.shape, dtype=np.complex128)
        phi = np.zeros(xA.shape, dtype=np.complex128)
        psi = np.zeros(xA.shape, dtype=np.complex128)
        for r, c, blk in JJ:
            yJ[r] += blk @ xJ[c]
        for r, c, blk in SS:
            phi[r] += blk @ xA[c]
            psi[r] += blk @ u[c]
        y = np.concatenate([yJ + self.div_test(phi), psi], axis=0)
        return y[:, 0] if one else y

    def near_rows(self, rows):
        """Near-field rows (canonical indices) as a dense [len(rows), N]."""
        pr = self.prob
        tr = self.tree
        E = self.E
        w2e = pr.omega ** 2 * _mom.EPS0
        out = np.zeros((len(rows), pr.N), dtype=np.complex128)

        def near_cols(unk, kind):
            b = tr.box_of[unk]
            nbrs = tr.near_idx[tr.near_ptr[b]:tr.near_ptr[b + 1]]
            cols = np.concatenate([tr.perm[tr.box_ptr[j]:tr.box_ptr[j + 1]] for j in nbrs])
            return cols[cols < E] if kind == "J" else cols[cols >= E]

        def s_row(t):
            """Near row of S for triangle t: (triangle cols, values)."""
            ct = np.sort(near_cols(E + t, "A"))
            return ct - E, pr.zblock([E + t], ct)[0] / w2e

        for i, r in enumerate(rows):
            if r < E:
                cj = near_cols(r, "J")
                out[i, cj] = pr.zblock([r], cj)[0]
                for h in range(2):                      # G S_near x_A
                    tc, sv = s_row(self.g_tri[r, h])
                    out[i, E + tc] += self.g_div[r, h] * sv
            else:
                tc, sv = s_row(r - E)                   # S_near (G^T x_J + w2e x_A)
                out[i, E + tc] += w2e * sv
                for h in range(2):
                    hit = np.isin(self.g_tri[:, h], tc)
                    e = np.nonzero(hit)[0]
                    pos = np.searchsorted(tc, self.g_tri[e, h])
                    np.add.at(out[i], e, self.g_div[e, h] * sv[pos])
        return out

    # ------------------------------------------------------------------
    # far field
    # ------------------------------------------------------------------
    def far(self, x, rows=None):
        """Far-field part of Z x; x [N] or [N,R] canonical order.  If rows
        is given, only those outputs are returned (the whole upward pass and
        translation are still done)."""
        pr = self.prob
        m = pr.mesh
        tr = self.tree
        L = self.L
        E = self.E
        x = np.asarray(x, dtype=np.complex128)
        one = x.ndim == 1
        if one:
            x = x[:, None]
        R = x.shape[1]
        w2e = pr.omega ** 2 * _mom.EPS0
        xJ, xA = x[:E], x[E:]
        u = self.div_sources(xJ) + w2e * xA
        nbL = tr.levels[L].coords.shape[0]
        # --- aggregation at the finest level: components Jx,Jy,Jz,sigma,u
        S = {L: np.zeros((nbL, self.Q, 5, R), dtype=np.complex128)}
        for c0 in range(0, E, 4096):
            e = np.arange(c0, min(E, c0 + 4096))
            F = self.rwg_patterns(e)
            contrib = np.zeros((e.size, self.Q, 5, R), dtype=np.complex128)
            contrib[:, :, 0:3, :] = np.einsum("nqd,nr->nqdr", F, xJ[e])
            np.add.at(S[L], tr.box_of[e], contrib)
        for c0 in range(0, m.nT, 4096):
            t = np.arange(c0, min(m.nT, c0 + 4096))
            P = self.tri_patterns(t)
            contrib = np.zeros((t.size, self.Q, 5, R), dtype=np.complex128)
            contrib[:, :, 3, :] = np.einsum("nq,nr->nqr", P, xA[t])
            contrib[:, :, 4, :] = np.einsum("nq,nr->nqr", P, u[t])
            np.add.at(S[L], self.tri_box[t], contrib)
        # --- aggregation up the tree
        for l in range(L - 1, 2, -1):
            lev, ch = tr.levels[l], tr.levels[l + 1]
            Sl = np.zeros((lev.coords.shape[0], self.Q, 5, R), dtype=np.complex128)
            filt = np.einsum("qp,bpcr->bqcr", self.F[l], S[l + 1])
            dc = ch.centre - lev.centre[ch.parent]                       # [nc,3]
            ph = np.exp(-1j * self.kappa[l] * (dc @ self.khat.T))        # [nc,Q]
            np.add.at(Sl, ch.parent, ph[:, :, None, None] * filt)
            S[l] = Sl
        # --- translation at every level
        G = {}
        for l in range(3, L + 1):
            lev = tr.levels[l]
            nb = lev.coords.shape[0]
            Gl = np.zeros((nb, self.Q, 5, R), dtype=np.complex128)
            own = np.repeat(np.arange(nb), np.diff(lev.il_ptr))
            for i0 in range(0, own.size, 8192):
                sl = slice(i0, i0 + 8192)
                Tq = self.T[l][lev.il_off[sl]]                           # [n,Q]
                np.add.at(Gl, own[sl], Tq[:, :, None, None] * S[l][lev.il_src[sl]])
            G[l] = Gl
        # --- disaggregation down the tree
        for l in range(3, L):
            lev, ch = tr.levels[l], tr.levels[l + 1]
            dc = ch.centre - lev.centre[ch.parent]
            ph = np.exp(1j * self.kappa[l] * (dc @ self.khat.T))
            H = ph[:, :, None, None] * G[l][ch.parent]
            G[l + 1] += np.einsum("qp,bqcr->bpcr", self.F[l], H)
        # --- receive at the finest level: the scalar potentials of every
        # triangle, then the RWG and pulse rows
        phi = np.zeros((m.nT, R), dtype=np.complex128)
        psi = np.zeros((m.nT, R), dtype=np.complex128)
        for c0 in range(0, m.nT, 4096):
            t = np.arange(c0, min(m.nT, c0 + 4096))
            P = self.tri_patterns(t).conj()
            Gb = G[L][self.tri_box[t]]
            phi[t] = np.einsum("nq,nqr->nr", P, Gb[:, :, 3])
            psi[t] = np.einsum("nq,nqr->nr", P, Gb[:, :, 4])
        if rows is None:
            rows = np.arange(pr.N)
        rows = np.asarray(rows, dtype=np.int64)
        y = np.zeros((rows.size, R), dtype=np.complex128)
        isr = rows < E
        e = rows[isr]
        if e.size:
            F = self.rwg_patterns(e).conj()
            Gb = G[L][tr.box_of[e]]
            y[isr] = (_mom.MU0 * np.einsum("nqd,nqdr->nr", F, Gb[:, :, 0:3])
                      + self.g_div[e, 0, None] * phi[self.g_tri[e, 0]]
                      + self.g_div[e, 1, None] * phi[self.g_tri[e, 1]])
        y[~isr] = psi[rows[~isr] - E]
        return y[:, 0] if one else y

    def matvec(self, x):
        return self.near(x) + self.far(x)

    def matvec_rows(self, x, rows):
        """(Z_mlfma x)[rows] without forming the full near field."""
        x = np.asarray(x, dtype=np.complex128)
        return self.near_rows(rows) @ x + self.far(x, rows)

"""Restricted additive Schwarz preconditioner over finest-box near
neighbourhoods: a reading for the preconditioner the solves of Section 4
leave open (the paper names none).  Closed surfaces at very low frequency
need one, and the self-box block-diagonal one fails there.

For the equilibrated matrix A = D Z D, a finest box b with its own unknowns
O_b and its neighbourhood N_b (the unknowns of b's near boxes, b included):

    M v = sum_b  R_{O_b}^T  [ (A_{N_b, N_b})^{-1} ]_{rows O_b}  v_{N_b}

so each box solves the local problem on its neighbourhood and keeps the rows
of its own unknowns.  The local matrices are the dense blocks of A, or
those blocks restricted to the pairs a near-field store holds (``near``).

Pins (tests/test_oracle_schwarz.py): a single box that holds every unknown
(its neighbourhood listed in another order) gives M = A^{-1}, so A M = I;
neighbourhoods equal to the boxes themselves give block Jacobi, whose
defining property is that each block's own equations are solved exactly;
every unknown is owned by exactly one box; and on the 3 200-unknown sphere
at 1e-5 wavelength, GMRES(200) with M on the right reaches 1e-6 in at most
60 iterations against at least 250 without.
"""
from __future__ import annotations

import numpy as np


def box_neighbourhoods(tree):
    """(members, neighbourhoods) of the finest boxes of an oracle octree:
    members[b] = canonical unknowns of box b, neighbourhoods[b] = the
    unknowns of b's near boxes in near-list order."""
    nb = len(tree.near_ptr) - 1
    order = np.argsort(tree.box_of, kind="stable")
    counts = np.bincount(tree.box_of, minlength=nb)
    starts = np.concatenate([[0], np.cumsum(counts)])
    members = [order[starts[i]:starts[i + 1]] for i in range(nb)]
    nbh = [np.concatenate([members[j] for j in tree.near_idx[tree.near_ptr[i]:tree.near_ptr[i + 1]]])
           for i in range(nb)]
    return members, nbh


def build(A, members, neighbourhoods, near=None):
    """Local operators [(nbh, own, M_b)]: M_b = rows of own of the inverse of
    A restricted to nbh x nbh (entries outside ``near`` set to zero when a
    mask is given).  Every unknown of own must be in nbh."""
    blocks = []
    for own, nbh in zip(members, neighbourhoods):
        own = np.asarray(own)
        nbh = np.asarray(nbh)
        loc = A[np.ix_(nbh, nbh)]
        if near is not None:
            loc = np.where(near[np.ix_(nbh, nbh)], loc, 0.0)
        where = {int(u): i for i, u in enumerate(nbh)}
        pos = np.array([where[int(u)] for u in own], dtype=np.int64)
        blocks.append((nbh, own, np.linalg.inv(loc)[pos]))
    return blocks


def apply(blocks, v):
    """M v (one column)."""
    y = np.zeros(v.shape, dtype=np.complex128)
    for nbh, own, Mb in blocks:
        y[own] = Mb @ v[nbh]
    return y

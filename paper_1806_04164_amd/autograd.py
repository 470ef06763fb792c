"""Differentiation through the PIE solve with hand-written adjoints.

For x = Z^-1 b the vector-Jacobian product is grad_b = Z^-H grad_x: the
backward pass runs the GMRES solve with the adjoint MVM (Z^H, libpie's
adjoint kernels).  The far field F = Phi x is linear; its backward applies
Phi^H with libpie's adjoint far-field kernel.  Gradients follow PyTorch's
convention for complex inputs (dL/dRe z + i dL/dIm z for a real loss L).
"""
from __future__ import annotations

import numpy as np
import torch


class PieSolve(torch.autograd.Function):
    """x = Z^-1 b with GMRES on the operator; backward solves Z^H g = grad_x."""

    @staticmethod
    def forward(ctx, b, op, solve_kw):
        x, info = op.solve(b.contiguous(), **solve_kw)
        ctx.op = op
        ctx.kw = dict(solve_kw)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        kw = dict(ctx.kw)
        kw.pop("adjoint", None)
        g, _ = ctx.op.solve(gx.contiguous(), adjoint=True, **kw)
        return g, None, None


class FarField(torch.autograd.Function):
    """F[r, d, :] = far field of the current of column r in direction d."""

    @staticmethod
    def forward(ctx, x, op, dirs):
        ctx.op = op
        ctx.dirs = np.ascontiguousarray(dirs, np.float64)
        return op.farfield(x.contiguous(), ctx.dirs)

    @staticmethod
    def backward(ctx, gF):
        return ctx.op.farfield_adjoint(gF.contiguous(), ctx.dirs), None, None


def plane_wave_rhs(op, khat, pol, amp):
    """b[:, r] = amp[r] * (unit-amplitude plane-wave right-hand side r);
    amp is a complex128 GPU tensor and may require grad."""
    R = amp.shape[0]
    unit = op.rhs_planewave(khat, pol, np.ones(R, np.complex128))
    return unit * amp[None, :]


def solve(op, b, **solve_kw):
    return PieSolve.apply(b, op, solve_kw)


def farfield(op, x, dirs):
    return FarField.apply(x, op, dirs)

"""Differentiation through the PIE solve with hand-written adjoints.

For x = Z^-1 b the vector-Jacobian product is grad_b = Z^-H grad_x: the
backward pass runs the GMRES solve with the adjoint MVM (Z^H, libpie's
adjoint kernels).  The far field F = Phi x is linear; its backward applies
Phi^H with libpie's adjoint far-field kernel.  Gradients follow PyTorch's
convention for complex inputs (dL/dRe z + i dL/dIm z for a real loss L).
"""
from __future__ import annotations

import warnings

import numpy as np
import torch


def _check(info, what, on_fail):
    if info["converged"]:
        return
    msg = (f"{what} solve stopped at relative residual {info['rel_residual']:.3e} after "
           f"{info['iterations']} iterations (tolerance not met)")
    if on_fail == "warn":
        warnings.warn(msg, RuntimeWarning, stacklevel=3)
    else:
        raise RuntimeError(msg)


class PieSolve(torch.autograd.Function):
    """x = Z^-1 b with GMRES on the operator; backward solves Z^H g = grad_x.
    A forward or adjoint solve that misses its tolerance raises RuntimeError
    (on_fail="raise", the default) or warns (on_fail="warn"); the solve
    reports of the last call are kept in PieSolve.last_info."""

    last_info = {}

    @staticmethod
    def forward(ctx, b, op, solve_kw):
        kw = dict(solve_kw)
        on_fail = kw.pop("on_fail", "raise")
        x, info = op.solve(b.contiguous(), **kw)
        PieSolve.last_info = {"forward": info}
        _check(info, "forward", on_fail)
        ctx.op = op
        ctx.kw = kw
        ctx.on_fail = on_fail
        return x

    @staticmethod
    def backward(ctx, gx):
        kw = dict(ctx.kw)
        kw.pop("adjoint", None)
        kw.pop("x", None)  # the adjoint solve gets a fresh, zero-initialised output
        g, info = ctx.op.solve(gx.contiguous(), adjoint=True, **kw)
        PieSolve.last_info["adjoint"] = info
        _check(info, "adjoint", ctx.on_fail)
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

"""pie_solve_noalloc (the solve for callers that cannot allocate device
memory: its workspace is the library's fixed per-GPU array) against
pie_solve, through the C ABI: two calls in a row, the second with a smaller
input (fewer right-hand sides, shorter restart), each bit for bit equal to
pie_solve's solution and report; and a problem larger than the array is
rejected with PIE_ERR_ARG before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_1806_04164_amd import _lib, pie
from paper_1806_04164_amd._lib import PIE_ERR_ARG, PIE_FP64

pytestmark = pytest.mark.gpu


def _call(fn, op, b, R, restart, maxit=2000, tol=1e-6):
    o = _lib.pie_solve_opts()
    _lib.lib().pie_solve_opts_default(ctypes.byref(o))
    o.restart, o.maxit, o.tol = restart, maxit, tol
    x = torch.full_like(b, 7.0)  # stale contents: the solve must not read them (use_x0 = 0)
    info = _lib.pie_solve_info()
    st = fn(op.h, None, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), R, ctypes.byref(o),
            ctypes.byref(info), None)
    torch.cuda.synchronize()
    return st, x, (info.iterations, info.refinements, info.rel_residual)


def test_noalloc_solve_matches_solve():
    V, T = synth.icosphere(3)
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, 3)
    op = pie.Operator(m, tr, 0.1 * synth.C0 / synth.DIAMETER, near_prec=PIE_FP64, far_prec=PIE_FP64, max_rhs=3)
    L = _lib.lib()
    kh, pol, amp = synth.plane_waves(3, 12)
    b3 = op.rhs_planewave(kh, pol, amp)
    b1 = b3[:, 1:2].contiguous()
    for R, b, restart in ((3, b3, 120), (1, b1, 60)):
        s0, x0, i0 = _call(L.pie_solve, op, b, R, restart)
        s1, x1, i1 = _call(L.pie_solve_noalloc, op, b, R, restart)
        print("R", R, "restart", restart, "pie_solve", s0, i0, "pie_solve_noalloc", s1, i1, flush=True)
        assert s0 == 0 and s1 == 0
        assert i0 == i1
        assert torch.equal(x0, x1)


def test_noalloc_rejects_oversize():
    V, T = synth.icosphere(3)
    m = pie.Mesh(V, T)
    tr = pie.Tree(m, 3)
    op = pie.Operator(m, tr, 0.1 * synth.C0 / synth.DIAMETER, max_rhs=3)
    b = op.rhs_planewave(*synth.plane_waves(3, 12))
    st, _, _ = _call(_lib.lib().pie_solve_noalloc, op, b, 3, 2000)  # 16 N R (m + 7) = 0.3 GB
    assert st == PIE_ERR_ARG
    assert "workspace" in _lib.last_error()

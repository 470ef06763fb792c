"""Launch schedules, the autotuner and graph replays of the MVM (GPU).

Every schedule places the same kernels with the same per-column arithmetic
order on different streams, and every RHS chunking computes each column the
same way, so results must agree bit for bit; a captured graph replays
exactly the eager MVM.
"""
import itertools

import numpy as np
import pytest
import torch

import synth
from paper_1806_04164_amd import pie
from paper_1806_04164_amd._lib import (PIE_FP32, PIE_FP64, PIE_NEAR_FORK_AFTER_AGGREGATE, PIE_NEAR_FORK_START,
                                       PIE_NEAR_SERIAL, PieError)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s4():
    """Sphere subdivision 4 (12800 unknowns), 4 levels: the finest-level
    translation can run on its own stream."""
    V, T = synth.icosphere(4)
    mesh = pie.Mesh(V, T)
    tree = pie.Tree(mesh, 4)
    f = 1e-2 * synth.C0 / synth.DIAMETER
    return dict(mesh=mesh, tree=tree, f=f)


def _op(c, near=PIE_FP32, far=PIE_FP64, max_rhs=3):
    return pie.Operator(c["mesh"], c["tree"], c["f"], near_prec=near, far_prec=far, max_rhs=max_rhs)


def _x(op, R, seed):
    return torch.from_numpy(synth.complex_gaussian(op.N, R, seed)).cuda()


@pytest.mark.parametrize("near,far", [(PIE_FP32, PIE_FP64), (PIE_FP64, PIE_FP64), (PIE_FP32, PIE_FP32)])
def test_schedules_bitwise_equal(s4, near, far):
    op = _op(s4, near, far)
    x = _x(op, 3, 11)
    ref = op.matvec(x).cpu().numpy()
    refa = op.matvec(x, adjoint=True).cpu().numpy()
    for nf, il, ch in itertools.product((PIE_NEAR_SERIAL, PIE_NEAR_FORK_START, PIE_NEAR_FORK_AFTER_AGGREGATE),
                                        (0, 1, 2, 3, 4), (1, 2, 4)):
        op.schedule = dict(near_fork=nf, il_fork=il, max_chunk=ch)
        assert op.schedule == dict(near_fork=nf, il_fork=il, max_chunk=ch)
        y = op.matvec(x).cpu().numpy()
        ya = op.matvec(x, adjoint=True).cpu().numpy()
        print("schedule", nf, il, ch, flush=True)
        assert np.array_equal(y, ref)
        assert np.array_equal(ya, refa)


def test_one_launch_translations_five_levels():
    """With five levels, il_fork 4 runs the translations of levels 3..5 in
    one launch: eager MVMs and graph replays equal the serial schedule bit
    for bit (mixed and FP32 far field, one and three columns, adjoint too)."""
    V, T = synth.icosphere(5)
    mesh = pie.Mesh(V, T)
    tree = pie.Tree(mesh, 5)
    f = 1e-3 * synth.C0 / synth.DIAMETER
    for far, R in ((PIE_FP64, 1), (PIE_FP64, 3), (PIE_FP32, 1)):
        op = pie.Operator(mesh, tree, f, near_prec=PIE_FP32, far_prec=far, max_rhs=R)
        x = _x(op, R, 21)
        op.schedule = dict(near_fork=PIE_NEAR_SERIAL, il_fork=0, max_chunk=1)
        ref = op.matvec(x).cpu().numpy()
        refa = op.matvec(x, adjoint=True).cpu().numpy()
        for nf in (PIE_NEAR_SERIAL, PIE_NEAR_FORK_START, PIE_NEAR_FORK_AFTER_AGGREGATE):
            op.schedule = dict(near_fork=nf, il_fork=4, max_chunk=1)
            assert np.array_equal(op.matvec(x).cpu().numpy(), ref)
            assert np.array_equal(op.matvec(x, adjoint=True).cpu().numpy(), refa)
        y = torch.empty_like(x)
        g = op.graph(x, y)
        for rep in range(3):
            y.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy(), ref), (far, R, rep)
            op.matvec(_x(op, R, 22))
            torch.cuda.synchronize()
        print("il_fork 4, five levels", far, R, flush=True)


def test_schedule_validation(s4):
    op = _op(s4, max_rhs=1)
    for bad in (dict(near_fork=3), dict(il_fork=5), dict(max_chunk=3)):
        with pytest.raises(PieError):
            op.schedule = bad


def test_autotune_keeps_result(s4):
    op = _op(s4)
    x = _x(op, 3, 12)
    ref = op.matvec(x).cpu().numpy()
    sched, ms = op.autotune(x, reps=3)
    print("autotune", sched, ms, flush=True)
    assert ms > 0 and op.schedule == sched
    assert sched["near_fork"] in (PIE_NEAR_SERIAL, PIE_NEAR_FORK_START, PIE_NEAR_FORK_AFTER_AGGREGATE)
    assert np.array_equal(op.matvec(x).cpu().numpy(), ref)


@pytest.mark.parametrize("adjoint", [False, True])
def test_graph_replays_match_eager(s4, adjoint):
    op = _op(s4)
    x = _x(op, 3, 13)
    ref = op.matvec(x, adjoint=adjoint).cpu().numpy()
    y = torch.empty_like(x)
    g = op.graph(x, y, adjoint=adjoint)
    other = _x(op, 3, 14)
    for rep in range(4):
        y.zero_()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), ref), rep
        # eager work on the same operator between replays
        op.matvec(other)
        torch.cuda.synchronize()
    # a graph keeps the schedule it was captured with
    for sch in (dict(near_fork=PIE_NEAR_SERIAL, il_fork=0, max_chunk=1),
                dict(near_fork=PIE_NEAR_FORK_START, il_fork=3, max_chunk=1),
                dict(near_fork=PIE_NEAR_FORK_AFTER_AGGREGATE, il_fork=4, max_chunk=1)):
        op.schedule = sch
        g2 = op.graph(x, y, adjoint=adjoint)
        for rep in range(2):
            y.zero_()
            g2.launch()
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy(), ref), (sch, rep)
            op.matvec(other)
            torch.cuda.synchronize()


def test_batch_graph_matches_each_object():
    """Objects of different sizes, frequencies, precisions and RHS counts in
    one graph: every replay equals each object's own MVM bit for bit."""
    specs = [(2, 1e-1, 3, PIE_FP64, PIE_FP64, 1), (3, 1e-3, 3, PIE_FP32, PIE_FP64, 2),
             (4, 1e-5, 4, PIE_FP32, PIE_FP32, 3)]
    ops, xs, ys, keep = [], [], [], []
    for i, (sub, dl, L, near, far, R) in enumerate(specs):
        V, T = synth.icosphere(sub)
        m = pie.Mesh(V, T)
        tr = pie.Tree(m, L)
        op = pie.Operator(m, tr, dl * synth.C0 / synth.DIAMETER, near_prec=near, far_prec=far, max_rhs=R)
        ops.append(op)
        xs.append(_x(op, R, 30 + i))
        ys.append(torch.empty_like(xs[-1]))
        keep.append((m, tr))
    refs = [op.matvec(x).cpu().numpy() for op, x in zip(ops, xs)]
    g = pie.BatchGraph(ops, xs, ys)
    for rep in range(3):
        for y in ys:
            y.zero_()
        g.launch()
        torch.cuda.synchronize()
        for y, r in zip(ys, refs):
            assert np.array_equal(y.cpu().numpy(), r), rep
        ops[0].matvec(xs[0])  # eager work between replays
        torch.cuda.synchronize()
    with pytest.raises(PieError):
        pie.BatchGraph([ops[0], ops[0]], [xs[0], xs[0]], [ys[0], torch.empty_like(ys[0])])

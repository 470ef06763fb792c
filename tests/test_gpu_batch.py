"""Uneven batch (pie_batch_create / pie_batch_matvec): the MVMs of several
distinct operators in one call, each object on its own stream so that the
objects' kernels run concurrently, joined back into the caller's stream.
Every object's result equals its own pie_matvec bit for bit (the per-column
arithmetic does not depend on the stream), and the eight-sphere batch
(12 800 to 3 276 800 unknowns, 1e-5 to 1e-1 wavelength, 8 plane waves each)
is timed against the sum of the eight MVMs run one after another; its three
smallest objects are checked against sampled rows of the dense FP64 oracle
per sub-operator to 1e-3."""
import numpy as np
import pytest
import torch

import synth
from paper_1806_04164_amd import pie
from paper_1806_04164_amd._lib import PIE_FP32, PIE_FP64, PieError
from tests.oracle_rows import sampled_rows

pytestmark = pytest.mark.gpu


def _x(N, R, seed):
    return torch.from_numpy(synth.complex_gaussian(N, R, seed)).cuda()


def test_batch_matches_each_object():
    specs = [(2, 1e-1, 3, PIE_FP64, PIE_FP64, 1), (3, 1e-3, 3, PIE_FP32, PIE_FP64, 2),
             (4, 1e-5, 4, PIE_FP32, PIE_FP32, 3), (3, 1e-2, 3, PIE_FP32, PIE_FP64, 16)]
    ops, xs, keep = [], [], []
    for i, (sub, dl, L, near, far, R) in enumerate(specs):
        m = pie.Mesh.icosphere(sub, synth.DIAMETER / 2)
        tr = pie.Tree(m, L)
        op = pie.Operator(m, tr, dl * synth.C0 / synth.DIAMETER, near_prec=near, far_prec=far, max_rhs=R)
        ops.append(op)
        xs.append(_x(op.N, R, 30 + i))
        keep.append((m, tr))
    refs = [op.matvec(x).cpu().numpy() for op, x in zip(ops, xs)]
    refa = [op.matvec(x, adjoint=True).cpu().numpy() for op, x in zip(ops, xs)]
    b = pie.Batch(ops)
    for rep in range(3):
        ys = b.matvec(xs)
        torch.cuda.synchronize()
        for y, r in zip(ys, refs):
            assert np.array_equal(y.cpu().numpy(), r), rep
        ya = b.matvec(xs, adjoint=True)
        torch.cuda.synchronize()
        for y, r in zip(ya, refa):
            assert np.array_equal(y.cpu().numpy(), r), rep
        ops[0].matvec(xs[0])  # eager work between calls
    with pytest.raises(PieError):
        pie.Batch([ops[0], ops[0]])
    with pytest.raises(ValueError):
        b.matvec(xs[:2])


def test_uneven_batch_concurrent():
    objs = synth.uneven_batch()
    ops, xs, keep = [], [], []
    for i, w in enumerate(objs):
        m = pie.Mesh.icosphere(w.subdiv, synth.DIAMETER / 2, w.jitter, w.seed)
        tr = pie.Tree(m, w.levels)
        ops.append(pie.Operator(m, tr, w.freq, near_prec=PIE_FP32, far_prec=PIE_FP64, max_rhs=w.nrhs))
        xs.append(_x(ops[-1].N, w.nrhs, 60 + i))
        keep.append((m, tr))
        print("object", i, "N", ops[-1].N, "built", flush=True)
    refs = [op.matvec(x) for op, x in zip(ops, xs)]
    b = pie.Batch(ops)
    ys = [torch.empty_like(x) for x in xs]
    for rep in range(2):
        b.matvec(xs, ys)
        torch.cuda.synchronize()
        for i, (y, r) in enumerate(zip(ys, refs)):
            assert torch.equal(y, r), (rep, i)
    print("batch results equal each object's MVM", flush=True)
    # timing: the eight MVMs one after another against one batch call
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        s0.record()
        for _ in range(reps):
            fn()
        s1.record()
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / reps

    def serial():
        for op, x, y in zip(ops, xs, ys):
            op.matvec(x, y)

    t_serial = timed(serial)
    t_batch = timed(lambda: b.matvec(xs, ys))
    print(f"eight MVMs one after another {t_serial:.3f} ms, one batch call {t_batch:.3f} ms "
          f"(ratio {t_serial / t_batch:.2f})", flush=True)
    # the three smallest objects against sampled dense FP64 rows
    jobs, meta = [], []
    for i in range(3):
        E = keep[i][0].sizes()[0]
        N = ops[i].N
        rng = np.random.default_rng(70 + i)
        rows = np.sort(np.concatenate([rng.choice(E, 4, replace=False), E + rng.choice(N - E, 4, replace=False)]))
        jobs.append((("uneven", i), objs[i].freq, rows, 60 + i, objs[i].nrhs))
        meta.append((i, E, rows))
    refrows = sampled_rows(jobs)
    for (i, E, rows), ref in zip(meta, refrows):
        x = xs[i].cpu().numpy()
        errs = {}
        for name, sl in (("J", slice(0, E)), ("A", slice(E, None))):
            xm = np.zeros_like(x)
            xm[sl] = x[sl]
            xd = [torch.from_numpy(xm).cuda() if j == i else xs[j] for j in range(len(ops))]
            y = b.matvec(xd)[i].cpu().numpy()[rows]
            for rn, rs in (("J", rows < E), ("A", rows >= E)):
                errs[rn + name] = np.linalg.norm(y[rs] - ref[name][rs]) / np.linalg.norm(ref[name][rs])
        print("object", i, "sampled rows", errs, flush=True)
        assert max(errs.values()) <= 1e-3

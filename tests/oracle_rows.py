"""Sampled rows of the dense FP64 oracle operator, y_rows = Z[rows, :] x,
computed in a pool of spawned worker processes (each rebuilds the seeded
mesh and input itself; nothing but the oracle and the input generators runs
in the workers).  Used by the full-size GPU parity tests."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _mesh(spec):
    import synth
    kind, arg = spec
    if kind == "workload":
        return synth.WORKLOADS[arg].mesh()
    if kind == "uneven":
        return synth.uneven_batch()[arg].mesh()
    if kind == "patch":
        return synth.patch(arg)
    if kind == "icosphere":
        return synth.icosphere(arg)
    raise ValueError(kind)


def _rows_job(args):
    spec, freq, rows, xseed, R = args
    import synth
    from oracle import mom
    V, T = _mesh(spec)
    prob = mom.Problem(V, T, freq)
    Zr = prob.zblock(np.asarray(rows), np.arange(prob.N))
    x = synth.complex_gaussian(prob.N, R, xseed)
    xs = {}
    E = prob.mesh.nE
    for name, sl in (("J", slice(0, E)), ("A", slice(E, None))):
        xm = np.zeros_like(x)
        xm[sl] = x[sl]
        xs[name] = Zr @ xm
    return xs


def sampled_rows(jobs, processes=None):
    """jobs: list of (mesh spec, freq, rows, xseed, R); returns, per job, a
    dict {"J": Z[rows] x_J, "A": Z[rows] x_A} with x the seeded complex
    Gaussian input split into its RWG (J) and pulse (A) parts."""
    # one job per row so that large meshes spread over the workers
    flat = []
    for j, (spec, freq, rows, xseed, R) in enumerate(jobs):
        for r in rows:
            flat.append((j, (spec, freq, [int(r)], xseed, R)))
    n = processes or min(16, os.cpu_count() or 1, len(flat))
    ctx = mp.get_context("spawn")
    with ctx.Pool(n) as pool:
        res = pool.map(_rows_job, [a for _, a in flat], chunksize=1)
    out = [{"J": [], "A": []} for _ in jobs]
    for (j, _), r in zip(flat, res):
        out[j]["J"].append(r["J"])
        out[j]["A"].append(r["A"])
    return [{k: np.concatenate(v, axis=0) for k, v in o.items()} for o in out]

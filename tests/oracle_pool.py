"""Oracle runs in worker processes, for the parity tests of large workloads.

The workers import only the input generators and the oracle (no torch, no
GPU): they are started with the "spawn" method so that nothing of a parent
that has initialised the GPU is inherited.  Results come back as plain numpy
arrays.
"""

import concurrent.futures
import multiprocessing
import os


def _rgg_member(b, maxit, tau):
    import numpy as np

    import gen
    import oracle
    from gen.problems import rgg_one, rgg_sizes

    inp = rgg_one(b, int(rgg_sizes()[b]))
    st, res = oracle.solve(inp, maxit=maxit, tau=tau)
    E = oracle.energy(inp.A, st.rowptr, st.colind, res.P, inp.nc)
    return b, np.asarray(res.P), res.iterations, res.status, np.asarray(res.dE), float(E)


def workers():
    """Worker count: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def rgg_members(members, maxit=None, tau=0.0):
    """Oracle solutions of the listed members of the 256-matrix batch:
    {b: (P, iterations, status, dE history, energy)}."""
    ctx = multiprocessing.get_context("spawn")
    out = {}
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers(), mp_context=ctx) as ex:
        futs = [ex.submit(_rgg_member, int(b), maxit, tau) for b in members]
        for f in concurrent.futures.as_completed(futs):
            b, P, it, status, dE, E = f.result()
            out[b] = (P, it, status, dE, E)
    return out

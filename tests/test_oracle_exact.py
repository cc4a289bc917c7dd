"""The oracle's iterate against exact arithmetic, and its block-Jacobi
against the preconditioner's dense definition.

Alg. 2 and Alg. 3 are rational in their inputs, so on small-integer inputs
``tests/rational_ref.py`` runs them exactly (Fractions, Gram solves, no QR);
the FP64 oracle must agree to rounding.  A slip anywhere in the oracle's set-up,
projector, masked product, preconditioner or CG scalars moves its iterate by
far more than that.
"""

import numpy as np
import pytest

import gen
import oracle
from tests import dense_ref as dr
from tests import rational_ref as rr

# (m, preconditioner, node size, seed): seeds whose local blocks G_i all have
# full rank, so every row takes Alg. 2's QR branch
CASES = [
    (1, "jacobi", 1, 0), (1, "jacobi", 1, 3), (2, "jacobi", 1, 2), (2, "jacobi", 1, 4),
    (1, "bjacobi", 2, 0), (1, "bjacobi", 2, 5), (2, "bjacobi", 2, 6), (2, "bjacobi", 2, 8),
]


def _exact_case(m, seed, n=12, nc=4):
    inp = gen.tiny_problem(seed, n=n, nc=nc, m=m, p0_per_row=m, extra_per_row=2, rational=True)
    rowptr, colind = inp.extra["pattern"]
    ex = rr.ExactProblem(inp.A, inp.P0, inp.B, inp.Bc, rowptr, colind)
    return inp, rowptr, colind, ex


@pytest.mark.parametrize("m,precond,bs,seed", CASES)
def test_iterate_matches_exact_arithmetic(m, precond, bs, seed):
    try:
        inp, rowptr, colind, ex = _exact_case(m, seed)
        P_ex, E_ex = ex.rcg(5, precond, bs)
    except rr.RankDeficient:
        pytest.fail("seed chosen for full-rank local blocks")
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    assert not st.used_svd.any()
    # the set-up alone (Alg. 2)
    p0_ex = np.array(rr.flatten(ex.setup()))
    assert np.linalg.norm(st.p0 - p0_ex) <= 1e-14 * np.linalg.norm(p0_ex)
    res = oracle.rcg_solve(inp.A, st, inp.nc, 5, precond, bs=bs, record_energy=True)
    assert res.iterations == 5
    P = np.array(rr.flatten(P_ex))
    assert np.linalg.norm(res.P - P) <= 1e-13 * np.linalg.norm(P)
    E = np.array([float(e) for e in E_ex])
    assert np.max(np.abs(np.array(res.energies) - E)) <= 1e-13 * E[0]


def test_exact_route_detects_a_planted_slip():
    """A Jacobi scaling by the wrong diagonal entry moves the exact iterate far
    beyond the bar above (so agreement to 1e-13 is not vacuous)."""
    inp, rowptr, colind, ex = _exact_case(1, 0)
    P_ok, _ = ex.rcg(3)
    A_diag = [ex.A[i][i] for i in range(ex.n)]
    ex.jacobi = lambda X: [[v / A_diag[(i + 1) % ex.n] for v in X[i]] for i in range(ex.n)]
    P_bad, _ = ex.rcg(3)
    a, b = np.array(rr.flatten(P_ok)), np.array(rr.flatten(P_bad))
    assert np.linalg.norm(a - b) > 1e-6 * np.linalg.norm(a)


@pytest.mark.parametrize("seed,bs", [(0, 2), (3, 2), (5, 3)])
def test_block_jacobi_matches_dense_definition(seed, bs):
    inp = gen.tiny_problem(seed, n=12, nc=5, m=1, p0_per_row=1, extra_per_row=2)
    rowptr, colind = inp.extra["pattern"]
    M = dr.dense_block_jacobi(inp.A, rowptr, colind, bs)
    X = np.random.default_rng(seed).normal(size=colind.shape[0])
    want = np.linalg.solve(M, X)
    got = oracle.block_jacobi(inp.A, rowptr, colind, X, bs)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_block_jacobi_shared_matches_dense_definition():
    """The shared-pattern form on a pattern whose node rows share columns."""
    inp = gen.tiny_problem(17, n=12, nc=5, m=1, p0_per_row=1, extra_per_row=2)
    rowptr, colind = inp.extra["pattern"]
    rows = []
    for a in range(inp.n // 3):
        u = sorted(set(colind[rowptr[3 * a]:rowptr[3 * a + 3]].tolist()))
        rows += [u, u, u]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    M = dr.dense_block_jacobi(inp.A, rp, ci, 3)
    X = np.random.default_rng(2).normal(size=ci.shape[0])
    want = np.linalg.solve(M, X)
    got = oracle.block_jacobi_shared(inp.A, rp, ci, X, 3, inp.nc)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)

"""Pins of the oracle's tentative set-up (Alg. 1, Sec. 3.2) and of the
classical C/F form P = [W; I] (Sec. 2, eqs. CFspl and prol): the fitted
distance against its closed form (the smallest l whose COARSE set spans
v_i), the exact fit, max vol's local maximality, the C/F pattern against
brute force, the initial residual against the W-gradient with the A_FC
term, and the RCG limit against the dense KKT solution."""

import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import gen
import oracle
from oracle import ptent
from tests import dense_ref as dr

CF_CASES = {
    "poisson2d": lambda: gen.cf_poisson2d(16),
    "linear2d": lambda: gen.cf_linear2d(12),
    "random0": lambda: gen.cf_random(0),
    "random1_m3": lambda: gen.cf_random(1, m=3),
    "random2_m1": lambda: gen.cf_random(2, m=1),
}


def _hops(S):
    G = sp.csr_matrix(S, copy=True)
    G.setdiag(0)
    G.eliminate_zeros()
    G.data[:] = 1.0
    return shortest_path(G, unweighted=True, directed=False)


def _spans(Vc_rows, v, tol=1e-9):
    if len(Vc_rows) == 0:
        return not np.any(v)
    M = np.asarray(Vc_rows).T
    w = np.linalg.lstsq(M, v, rcond=None)[0]
    return np.linalg.norm(M @ w - v) <= tol * max(np.linalg.norm(v), 1e-300)


@pytest.mark.parametrize("name", list(CF_CASES))
def test_ptent_level_is_smallest_spanning_distance(name):
    inp = CF_CASES[name]()
    P0, level = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    D = _hops(inp.S)
    Bc = inp.Bc
    for i in range(inp.n):
        if inp.cf[i] >= 0:
            assert level[i] == 0
            assert P0[i].nnz == 1 and P0[i, inp.cf[i]] == 1.0
            continue
        want = -1
        for l in range(1, inp.lmax + 1):
            near = [u for u in range(inp.n) if inp.cf[u] >= 0 and D[i, u] <= l]
            if _spans([Bc[inp.cf[u]] for u in near], inp.V[i]):
                want = l
                break
        assert level[i] == want, (i, level[i], want)
        row = P0[i]
        if want < 0:
            assert row.nnz == 0
            continue
        # an exact fit with at most m entries, all within the fitted distance
        assert row.nnz <= inp.m
        cols = row.indices
        nodes = [int(np.flatnonzero(inp.cf == c)[0]) for c in cols]
        assert all(D[i, u] <= want for u in nodes)
        assert np.linalg.norm(row.toarray() @ Bc - inp.V[i]) <= 1e-10 * np.linalg.norm(inp.V[i])


def test_ptent_ones_picks_first_nearest():
    """V = ones: the fit is a single entry of 1 at the COARSE node of lowest
    coarse index among the nearest ones (max vol on a column of ones is the
    first row)."""
    inp = gen.cf_poisson2d(16)
    P0, level = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    D = _hops(inp.S)
    for i in np.flatnonzero(inp.cf < 0):
        near = [u for u in range(inp.n) if inp.cf[u] >= 0 and D[i, u] <= level[i]]
        c = min(inp.cf[u] for u in near)
        assert P0[i].nnz == 1 and P0[i, c] == 1.0


@pytest.mark.parametrize("seed", range(6))
def test_maxvol_locally_maximal(seed):
    rng = np.random.default_rng(seed)
    k, m = int(rng.integers(3, 9)), int(rng.integers(1, 4))
    M = rng.standard_normal((k, m))
    sel = ptent.maxvol(M.tolist())
    assert len(sel) == m and len(set(sel)) == m
    vol = abs(np.linalg.det(M[sel]))
    # no single swap gains more than the tolerance
    for pos, q in itertools.product(range(m), range(k)):
        if q in sel:
            continue
        s2 = list(sel)
        s2[pos] = q
        assert abs(np.linalg.det(M[s2])) <= ptent.MAXVOL_TOL * vol * (1 + 1e-12)
    # and it is within the dominant-submatrix bound of the global maximum
    best = max(abs(np.linalg.det(M[list(c)])) for c in itertools.combinations(range(k), m))
    assert vol >= best / (ptent.MAXVOL_TOL ** m * m ** (m / 2)) - 1e-12


def test_maxvol_rank_deficient_spans():
    M = [[1.0, 2.0], [2.0, 4.0], [3.0, 6.0]]  # rank 1: the largest pivot row
    assert ptent.maxvol(M) == [2]
    # rank 2 in three columns, the second column empty after one step
    M = [[1.0, 0.0, 0.0], [1.0, 0.0, 2.0], [2.0, 0.0, 2.0]]
    sel = ptent.maxvol(M)
    assert len(sel) == 2 and np.linalg.matrix_rank(np.asarray(M)[sel]) == 2


@pytest.mark.parametrize("name", list(CF_CASES))
@pytest.mark.parametrize("k", [1, 2])
def test_cf_pattern_bruteforce(name, k):
    inp = CF_CASES[name]()
    P0, _ = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    rp, ci = ptent.cf_pattern(inp.A, P0, inp.cf, k)
    # stored structures (explicit zeros count, as in the pattern growth)
    Ab = sp.csr_matrix((np.ones(inp.A.nnz), inp.A.indices, inp.A.indptr), shape=inp.A.shape)
    Ab = Ab.toarray().astype(int)
    Pb = sp.csr_matrix((np.ones(P0.nnz), P0.indices, P0.indptr), shape=P0.shape)
    Pb = Pb.toarray().astype(int)
    for _ in range(k):
        Pb = ((Ab @ Pb) > 0).astype(int)
    for i in range(inp.n):
        got = ci[rp[i]:rp[i + 1]]
        if inp.cf[i] >= 0:
            assert list(got) == [inp.cf[i]]
        else:
            assert list(got) == list(np.flatnonzero(Pb[i]))


def _cf_solve(inp, maxit, **kw):
    P0, _ = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    rp, ci = ptent.cf_pattern(inp.A, P0, inp.cf, inp.pattern_power)
    st = oracle.emin_setup(rp, ci, P0, inp.V, inp.Bc)
    res = oracle.rcg_solve(inp.A, st, inp.nc, maxit, kw.get("precond", "jacobi"))
    return P0, rp, ci, st, res


@pytest.mark.parametrize("name", ["poisson2d", "random0", "random2_m1"])
def test_cf_initial_residual_is_w_gradient(name):
    """In the C/F form the unknowns are W (the FINE rows); the energy
    gradient in W is 2 (K_FF w + f) with f(i, j) = A(i, node of j) (the A_FC
    block acting on P's identity rows).  The first residual must equal
    -Pi (K_FF w0 + f) on FINE rows and vanish on COARSE rows."""
    inp = CF_CASES[name]()
    P0, rp, ci, st, res = _cf_solve(inp, 0)
    rows, cols = dr.entry_rows_cols(rp, ci)
    fine = inp.cf[rows] < 0
    node_of = np.empty(inp.nc, dtype=int)
    node_of[inp.cf[inp.cf >= 0]] = np.flatnonzero(inp.cf >= 0)
    Ad = inp.A.toarray()
    K = dr.dense_K(inp.A, rp, ci)
    Kff = K[np.ix_(fine, fine)]
    f = Ad[rows[fine], node_of[cols[fine]]]
    Pi = dr.dense_projector(rp, ci, inp.Bc)
    g = np.zeros(ci.size)
    g[fine] = Kff @ st.p0[fine] + f
    r_want = -Pi @ g
    r_got = -oracle.project(st, oracle.masked_product(inp.A, rp, ci, st.p0, inp.nc))
    assert np.allclose(r_got, r_want, rtol=1e-12, atol=1e-12 * np.abs(r_want).max())
    assert np.all(np.abs(r_got[~fine]) <= 1e-13 * np.abs(r_want).max())


@pytest.mark.parametrize("name", ["poisson2d", "random0", "random1_m3"])
def test_cf_rcg_limit_is_kkt(name):
    inp = CF_CASES[name]()
    P0, rp, ci, st, res = _cf_solve(inp, 600)
    assert res.status == "converged"
    want = dr.kkt_solution(inp.A, rp, ci, inp.V, inp.Bc)
    rows, _ = dr.entry_rows_cols(rp, ci)
    # COARSE rows stay the identity
    assert np.all(res.P[inp.cf[rows] >= 0] == 1.0)
    fitted = np.linalg.norm(st.p0 - want) > 0  # (a constant guard, see below)
    assert fitted
    assert np.linalg.norm(res.P - want) / np.linalg.norm(want) < 1e-9

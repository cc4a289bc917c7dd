"""Pins of the oracle's projected SGS preconditioner M_2 (Sec. 3.4.1, eq.
SGS_prec without its second term): the colouring against the definition of
Jones-Plassmann rounds, M_SGS^{-1} against its dense definition on K (eq.
11blk) in the sweep order, the Krylov characterisation of the iterates with
the dense M_2, and the KKT limit."""

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from oracle import sgs as osgs
from tests import dense_ref as dr


def _edges(A):
    A = sp.csr_matrix(A)
    r = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    off = r != A.indices
    return r[off], A.indices[off]


def _check_jp(A, rnd, colour):
    """Every row is picked in some round; a row of round r out-ranks every
    neighbour still unpicked at round r (round >= r), and a row left for a
    later round is out-ranked by one of them; its colour is the smallest
    not held by a neighbour picked earlier; no edge joins two rows of one
    colour."""
    n = A.shape[0]
    key = osgs.priorities(n)
    assert np.all(rnd >= 0) and np.all(colour >= 0)
    er, ec = _edges(A)
    assert not np.any(colour[er] == colour[ec])
    nbrs = [[] for _ in range(n)]
    for a, b in zip(er, ec):
        nbrs[a].append(b)
    for i in range(n):
        r = rnd[i]
        live = [k for k in nbrs[i] if rnd[k] >= r]
        assert all(key[i] > key[k] for k in live)
        for rr in range(r):  # not a local maximum in any earlier round
            live = [k for k in nbrs[i] if rnd[k] >= rr]
            assert any(key[k] > key[i] for k in live)
        used = {colour[k] for k in nbrs[i] if rnd[k] < r}
        assert colour[i] == min(set(range(len(used) + 1)) - used)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_colouring_is_jp_rounds(seed):
    inp = gen.tiny_problem(seed, n=40, nc=6)
    _check_jp(inp.A, *osgs.jp_rounds(inp.A))


def test_colouring_poisson():
    A = gen.poisson2d_32().A
    _check_jp(A, *osgs.jp_rounds(A))
    A3 = gen.poisson3d_ln32(N=8).A
    _check_jp(A3, *osgs.jp_rounds(A3))
    # the 5-point grid graph is bipartite, and first fit keeps it to few colours
    assert osgs.jp_colours(A).max() + 1 <= 5


def test_colouring_no_edges_one_round():
    A = sp.identity(17, format="csr") * 3.0
    rnd, colour = osgs.jp_rounds(A)
    assert np.all(rnd == 0) and np.all(colour == 0)


def _dense_sgs(A, rowptr, colind, colour):
    """(L + D)^{-T} D (L + D)^{-1} built densely from K (row-wise entry
    order), L and D taken after ordering the entries by their row's sweep
    position (rows by colour, then index)."""
    K = dr.dense_K(A, rowptr, colind)
    rows, _ = dr.entry_rows_cols(rowptr, colind)
    n = len(rowptr) - 1
    sweep = sorted(range(n), key=lambda i: (colour[i], i))
    pos = np.empty(n, dtype=int)
    pos[sweep] = np.arange(n)
    perm = np.argsort(pos[rows], kind="stable")
    Kp = K[np.ix_(perm, perm)]
    LD = np.tril(Kp)
    Li = np.linalg.inv(LD)
    Mp = Li.T @ np.diag(np.diag(Kp)) @ Li
    M = np.empty_like(Mp)
    M[np.ix_(perm, perm)] = Mp
    return M


@pytest.mark.parametrize("seed,m", [(0, 1), (1, 1), (2, 2), (3, 2)])
def test_sgs_dense_definition(seed, m):
    inp = gen.tiny_problem(seed, n=18, nc=6, m=m, p0_per_row=m, extra_per_row=3)
    rowptr, colind = inp.extra["pattern"]
    colour = osgs.jp_colours(inp.A)
    M = _dense_sgs(inp.A, rowptr, colind, colour)
    X = np.random.default_rng(seed).standard_normal((len(colind), 3))
    for c in range(3):
        got = osgs.sgs(inp.A, rowptr, colind, X[:, c], colour)
        assert np.allclose(got, M @ X[:, c], rtol=1e-12, atol=1e-12 * np.abs(M @ X[:, c]).max())
    # symmetric positive definite, as the CG needs
    assert np.allclose(M, M.T, atol=1e-12 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_sgs_diagonal_A_is_jacobi():
    inp = gen.tiny_problem(4, n=15, nc=5, m=1, extra_per_row=2)
    A = sp.diags(np.linspace(1.0, 3.0, 15)).tocsr()
    rowptr, colind = inp.extra["pattern"]
    X = np.random.default_rng(4).standard_normal(len(colind))
    got = osgs.sgs(A, rowptr, colind, X, osgs.jp_colours(A))
    assert np.allclose(got, oracle.jacobi(A, rowptr, X), rtol=1e-15, atol=0)


def test_sgs_order_within_colour_is_free():
    """Rows of one colour are uncoupled: sweeping them in reverse index order
    gives the same M_SGS^{-1} (dense route with the other tie-break)."""
    inp = gen.tiny_problem(6, n=18, nc=6, m=1, extra_per_row=3)
    rowptr, colind = inp.extra["pattern"]
    colour = osgs.jp_colours(inp.A)
    M1 = _dense_sgs(inp.A, rowptr, colind, colour)
    n = inp.n
    # same colours, reversed index order inside each colour
    colour_rev = colour * n + (n - 1 - np.arange(n))
    M2 = _dense_sgs(inp.A, rowptr, colind, colour_rev)
    assert np.allclose(M1, M2, rtol=1e-13, atol=1e-13 * np.abs(M1).max())


@pytest.mark.parametrize("seed,m", [(0, 1), (1, 2), (2, 1)])
def test_krylov_characterisation_sgs(seed, m):
    inp = gen.tiny_problem(seed, n=14, nc=5, m=m, p0_per_row=m)
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    Minv = _dense_sgs(inp.A, rowptr, colind, osgs.jp_colours(inp.A))
    for k in (1, 2, 3, 4):
        res = oracle.rcg_solve(inp.A, st, inp.nc, k, "sgs")
        want = dr.krylov_iterate(inp.A, rowptr, colind, inp.Bc, st.p0, Minv, k)
        assert np.linalg.norm(res.P - want) / np.linalg.norm(want) < 1e-9


@pytest.mark.parametrize("seed,m", [(0, 1), (6, 2)])
def test_kkt_limit_sgs(seed, m):
    inp = gen.tiny_problem(seed, n=16, nc=6, m=m, p0_per_row=m, extra_per_row=3)
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    res = oracle.rcg_solve(inp.A, st, inp.nc, 400, "sgs")
    assert res.status == "converged"
    want = dr.kkt_solution(inp.A, rowptr, colind, inp.B, inp.Bc)
    assert np.linalg.norm(res.P - want) / np.linalg.norm(want) < 1e-10


def test_sgs_energy_falls_faster_than_jacobi():
    """The paper's observation (Sec. 5, Figs. of energy vs iterations): SGS
    lowers the energy more per iteration than Jacobi; here on 2D Poisson."""
    inp = gen.poisson2d_32()
    _, rj = oracle.solve(inp, maxit=6, precond="jacobi", record_energy=True)
    _, rs = oracle.solve(inp, maxit=6, precond="sgs", record_energy=True)
    assert rs.energies[-1] < rj.energies[-1]
    assert np.all(np.diff(rs.energies) <= 1e-13 * rs.energies[0])

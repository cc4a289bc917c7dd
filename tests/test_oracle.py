"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own route: dense brute force
(pattern), closed forms (pattern counts on box-aggregated grids, the
dense-pattern minimiser, the m = 1 projector), library routines (min-norm
least squares), the saddle-point limit (eq. sadsys), the Krylov
characterisation of PCG (Sec. 3.1), Theorem 3.1 / Corollary 3.2, and the
energy-decrease identity (Sec. 3.3, eq. CG_dEa).  The planted-mistake tests at
the end show that plausible slips in the oracle fail at least one pin.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from oracle import rcg as orc
from tests import dense_ref as dr


# ---------------------------------------------------------------- pattern ---

def _brute_pattern(A, P0, k):
    S = np.zeros(A.shape, bool)
    Ac = A.tocoo()
    S[Ac.row, Ac.col] = True  # stored structure, explicit zeros included
    T = np.zeros(P0.shape, bool)
    Pc = P0.tocoo()
    T[Pc.row, Pc.col] = True
    for _ in range(k):
        U = np.zeros_like(T)
        for i in range(S.shape[0]):
            for l in range(S.shape[1]):
                if S[i, l]:
                    U[i] |= T[l]
        T = U
    return T


@pytest.mark.parametrize("seed,k", [(0, 1), (1, 1), (2, 2), (3, 2)])
def test_pattern_bruteforce(seed, k):
    inp = gen.tiny_problem(seed, n=12, nc=4, p0_per_row=1)
    A = inp.A.copy()
    A.data[::5] = 0.0  # explicit zeros still count as structure
    rowptr, colind = oracle.pattern_expand(A, inp.P0, k)
    T = _brute_pattern(A, inp.P0, k)
    for i in range(T.shape[0]):
        assert list(colind[rowptr[i]:rowptr[i + 1]]) == list(np.nonzero(T[i])[0])
    assert oracle.pattern_contains(rowptr, colind, inp.P0)


def _closed_form_count(N, b, d):
    """Box aggregates of width b on an N^d grid with the (2d+1)-point
    stencil: row i of struct(A P0) holds its own aggregate plus, per axis,
    the aggregate across the nearer aggregate face when the cell touches
    one that is not the grid boundary.  Per axis and grid line that is
    2 N/b - 2 cells."""
    return N ** d + d * N ** (d - 1) * (2 * (N // b) - 2)


@pytest.mark.parametrize("N,b,d", [(32, 2, 2), (12, 3, 3), (32, 2, 3), (96, 3, 3), (30, 3, 2)])
def test_pattern_closed_form_counts(N, b, d):
    A = gen.fd_poisson(N, d)
    from gen.problems import _box_aggregation, _piecewise_constant_P0
    P0 = _piecewise_constant_P0(_box_aggregation(N, d, b), (N // b) ** d)
    rowptr, colind = oracle.pattern_expand(A, P0, 1)
    assert int(rowptr[-1]) == _closed_form_count(N, b, d)
    assert np.diff(rowptr).max() == d + 1


def test_workload_pattern_counts():
    # the 2D and 3D workloads from the closed form above
    assert _closed_form_count(32, 2, 2) == 2944
    assert _closed_form_count(96, 3, 3) == 2598912
    assert _closed_form_count(32, 2, 3) == 124928


# ------------------------------------------------------------------ setup ---

@pytest.mark.parametrize("seed,m", [(0, 1), (1, 1), (2, 2), (3, 2), (4, 3)])
def test_setup_constraint_and_projector(seed, m):
    inp = gen.tiny_problem(seed, n=15, nc=6, m=m, p0_per_row=m, extra_per_row=2)
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    assert np.all(st.rank == m)
    # P0' B_c = B (the range requirement, eq. TSP)
    assert orc.constraint_error(rowptr, colind, st.p0, inp.B, inp.Bc) < 1e-14
    for i in range(inp.n):
        a, b = rowptr[i], rowptr[i + 1]
        G = inp.Bc[colind[a:b]]
        Q = st.Q[a:b]
        assert np.allclose(Q.T @ Q, np.eye(m), atol=1e-14)
        Pi = np.eye(b - a) - Q @ Q.T
        assert np.abs(Pi @ G).max() < 1e-14
        # delta is the min-norm solution of G^T delta = r (library lstsq)
        phat = oracle.values_on_pattern(inp.P0, rowptr, colind)[a:b]
        r = inp.B[i] - G.T @ phat
        d_ref = np.linalg.lstsq(G.T, r, rcond=None)[0]
        assert np.allclose(st.p0[a:b] - phat, d_ref, atol=1e-13)


def test_projector_m1_closed_form():
    inp = gen.tiny_problem(7, n=10, nc=5, m=1, extra_per_row=3)
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    X = np.random.default_rng(0).normal(size=colind.shape[0])
    got = oracle.project(st, X)
    for i in range(inp.n):
        a, b = rowptr[i], rowptr[i + 1]
        g = inp.Bc[colind[a:b], 0]
        want = X[a:b] - g * (g @ X[a:b]) / (g @ g)
        assert np.allclose(got[a:b], want, atol=1e-14)


def test_setup_svd_branch():
    """Rows with l_i < m, and rows whose G_i is rank deficient (two coarse
    columns with identical B_c rows), take the SVD branch: Q spans range(G),
    delta is the min-norm least-squares solution."""
    inp = gen.tiny_problem(11, n=12, nc=5, m=2, p0_per_row=1, extra_per_row=1)
    Bc = inp.Bc.copy()
    Bc[1] = Bc[0]  # columns 0 and 1 indistinguishable
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, Bc)
    phat = oracle.values_on_pattern(inp.P0, rowptr, colind)
    seen_def = False
    for i in range(inp.n):
        a, b = rowptr[i], rowptr[i + 1]
        G = Bc[colind[a:b]]
        rk = np.linalg.matrix_rank(G)
        assert st.rank[i] == rk
        if rk < 2:
            seen_def = True
            assert st.used_svd[i]
        r = inp.B[i] - G.T @ phat[a:b]
        d_ref = np.linalg.lstsq(G.T, r, rcond=None)[0]
        assert np.allclose(st.p0[a:b] - phat[a:b], d_ref, atol=1e-12)
        Q = st.Q[a:b, :rk]
        assert np.allclose(Q @ Q.T @ G, G, atol=1e-13)
    assert seen_def


# ---------------------------------------------------------------- iterate ---

def _tiny(seed, m=1, **kw):
    inp = gen.tiny_problem(seed, n=kw.pop("n", 14), nc=kw.pop("nc", 5), m=m,
                           p0_per_row=kw.pop("p0_per_row", m), **kw)
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    return inp, rowptr, colind, st


def _krylov_error(seed, m, precond, k, bs=1, n=14):
    inp, rowptr, colind, st = _tiny(seed, m=m, n=n)
    res = oracle.rcg_solve(inp.A, st, inp.nc, k, precond, bs=bs)
    if precond == "jacobi":
        Minv = dr.dense_jacobi(inp.A, rowptr, colind)
    elif precond == "none":
        Minv = np.eye(colind.shape[0])
    else:
        # the preconditioner from its dense definition, not from the oracle
        Minv = np.linalg.inv(dr.dense_block_jacobi(inp.A, rowptr, colind, bs))
    want = dr.krylov_iterate(inp.A, rowptr, colind, inp.Bc, st.p0, Minv, k)
    return np.linalg.norm(res.P - want) / np.linalg.norm(want)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("precond", ["jacobi", "none"])
@pytest.mark.parametrize("m", [1, 2])
def test_krylov_characterisation(seed, precond, m):
    for k in (1, 2, 3, 4):
        assert _krylov_error(seed, m, precond, k) < 1e-9


@pytest.mark.parametrize("seed", [3, 4])
def test_krylov_characterisation_block_jacobi(seed):
    for k in (1, 2, 3):
        assert _krylov_error(seed, 2, "bjacobi", k, bs=2) < 1e-9


def _kkt_error(inp, rowptr, colind, st, precond="jacobi", bs=1, maxit=400):
    res = oracle.rcg_solve(inp.A, st, inp.nc, maxit, precond, bs=bs)
    assert res.status == "converged"
    want = dr.kkt_solution(inp.A, rowptr, colind, inp.B, inp.Bc)
    return np.linalg.norm(res.P - want) / np.linalg.norm(want)


@pytest.mark.parametrize("seed,m", [(0, 1), (5, 1), (6, 2), (8, 2)])
def test_kkt_limit(seed, m):
    inp, rowptr, colind, st = _tiny(seed, m=m, n=16, nc=6, extra_per_row=3)
    assert _kkt_error(inp, rowptr, colind, st) < 1e-10


def test_kkt_limit_block_jacobi():
    inp, rowptr, colind, st = _tiny(9, m=2, n=16, nc=6, extra_per_row=3)
    assert _kkt_error(inp, rowptr, colind, st, "bjacobi", bs=2) < 1e-10


def test_kkt_limit_poisson2d():
    inp = gen.poisson2d_32()
    rowptr, colind = oracle.pattern_expand(inp.A, inp.P0, 1)
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    assert _kkt_error(inp, rowptr, colind, st, maxit=2000) < 1e-10


@pytest.mark.parametrize("m", [1, 2])
def test_closed_form_dense_pattern(m):
    """With every entry free the minimiser of tr(P^T A P) subject to
    P B_c = B is B (B_c^T B_c)^{-1} B_c^T, whatever A is (stationarity
    2 A P = L B_c^T with feasibility)."""
    inp = gen.tiny_problem(21 + m, n=9, nc=4, m=m, p0_per_row=m, dense_pattern=True)
    rowptr, colind = inp.extra["pattern"]
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    res = oracle.rcg_solve(inp.A, st, inp.nc, 500, "jacobi")
    assert res.status == "converged"
    Pstar = inp.B @ np.linalg.solve(inp.Bc.T @ inp.Bc, inp.Bc.T)
    got = np.zeros_like(Pstar)
    got[np.repeat(np.arange(inp.n), np.diff(rowptr)), colind] = res.P
    assert np.abs(got - Pstar).max() < 1e-10 * np.abs(Pstar).max()


@pytest.mark.parametrize("seed,m,precond,bs", [(0, 1, "jacobi", 1), (1, 2, "jacobi", 1),
                                               (2, 2, "bjacobi", 2)])
def test_energy_identity_and_invariants(seed, m, precond, bs):
    inp, rowptr, colind, st = _tiny(seed, m=m, n=16, nc=6, extra_per_row=3)
    res = oracle.rcg_solve(inp.A, st, inp.nc, 6, precond, bs=bs, record_energy=True)
    E = np.array(res.energies)
    # energy of each iterate, recomputed densely
    assert abs(E[0] - dr.dense_energy(inp.A, rowptr, colind, st.p0, inp.nc)) < 1e-12 * E[0]
    for k in range(res.iterations):
        assert abs((E[k] - E[k + 1]) - res.dE[k]) < 1e-10 * E[0]   # eq. CG_dEa
        assert E[k + 1] <= E[k] + 1e-13 * E[0]
    assert orc.constraint_error(rowptr, colind, res.P, inp.B, inp.Bc) < 1e-12


def test_theorem_31_and_corollary_32():
    """diag(Z^T K Z) = A(i,i) on row i's block and Z^T D_K Q = 0 for the
    block-diagonal Z, Q of Sec. 3.4 (eqs. diagZKZ, nullZKQ)."""
    inp, rowptr, colind, st = _tiny(4, m=2, n=10, nc=5, extra_per_row=3)
    K = dr.dense_K(inp.A, rowptr, colind)
    DK = np.diag(np.diag(K))
    nnz = colind.shape[0]
    Zcols, Qcols, zrow = [], [], []
    for i in range(inp.n):
        a, b = rowptr[i], rowptr[i + 1]
        G = inp.Bc[colind[a:b]]
        U, s, _ = np.linalg.svd(G, full_matrices=True)
        r = int(np.sum(s > 1e-12))
        for c in range(b - a):
            v = np.zeros(nnz)
            v[a:b] = U[:, c]
            (Qcols if c < r else Zcols).append(v)
            if c >= r:
                zrow.append(i)
    Z = np.stack(Zcols, 1)
    Q = np.stack(Qcols, 1)
    ZKZ = Z.T @ K @ Z
    assert np.allclose(np.diag(ZKZ), inp.A.diagonal()[zrow], atol=1e-13)
    ZDZ = Z.T @ DK @ Z
    assert np.abs(ZDZ - np.diag(np.diag(ZDZ))).max() < 1e-13
    assert np.abs(Z.T @ DK @ Q).max() < 1e-13


def test_gamma_floor_and_zero_residual():
    """A pattern equal to P0's with l_i = m leaves no freedom: gamma_1 = 0 and
    the loop stops at once with P = P0'."""
    inp = gen.tiny_problem(13, n=8, nc=4, m=1, p0_per_row=1, extra_per_row=0)
    rowptr, colind = inp.P0.indptr, inp.P0.indices
    st = oracle.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    res = oracle.rcg_solve(inp.A, st, inp.nc, 5, "jacobi")
    assert res.status == "converged" and res.iterations == 0
    assert np.array_equal(res.P, st.p0)


def test_tau_stop_skips_update():
    inp, rowptr, colind, st = _tiny(2, m=1, n=16, nc=6, extra_per_row=3)
    full = oracle.rcg_solve(inp.A, st, inp.nc, 10, "jacobi")
    ratios = np.array(full.dE) / full.dE[0]
    tau = 0.5 * (ratios[2] + ratios[3]) if ratios[3] < ratios[2] else None
    if tau is None:
        pytest.skip("non-monotone ratios")
    res = oracle.rcg_solve(inp.A, st, inp.nc, 10, "jacobi", tau=tau)
    k_stop = int(np.nonzero(ratios < tau)[0][0])
    assert res.status == "tau" and res.iterations == k_stop
    part = oracle.rcg_solve(inp.A, st, inp.nc, k_stop, "jacobi")
    assert np.array_equal(res.P, part.P)


def test_poisson2d_workload_trend():
    """On the 2D workload the energy drops every iteration and dE_k / dE_1
    decreases (the trend of Tables 1-2; dE_1/dE_1 = 1)."""
    inp = gen.poisson2d_32()
    st, res = oracle.solve(inp, record_energy=True)
    E = np.array(res.energies)
    assert res.iterations == 10
    assert np.all(np.diff(E) < 0)
    assert res.dE[-1] < 0.5 * res.dE[0]
    assert orc.constraint_error(st.rowptr, st.colind, res.P, inp.B, inp.Bc) < 1e-12


# -------------------------------------------------------- planted mistakes ---

def _pins_fail(monkeypatch, target, replacement):
    """Replace one oracle function by a plausible wrong version and report
    which pins notice."""
    monkeypatch.setattr(orc, target, replacement)
    failed = []
    try:
        if _krylov_error(0, 2, "jacobi", 3) > 1e-9:
            failed.append("krylov")
    except Exception:
        failed.append("krylov")
    try:
        inp, rowptr, colind, st = _tiny(5, m=1, n=16, nc=6, extra_per_row=3)
        if _kkt_error(inp, rowptr, colind, st) > 1e-10:
            failed.append("kkt")
    except Exception:
        failed.append("kkt")
    inp, rowptr, colind, st = _tiny(1, m=2, n=16, nc=6, extra_per_row=3)
    try:
        res = oracle.rcg_solve(inp.A, st, inp.nc, 5, "jacobi")
        if orc.constraint_error(rowptr, colind, res.P, inp.B, inp.Bc) > 1e-12:
            failed.append("constraint")
    except Exception:
        failed.append("constraint")
    return failed


def test_planted_wrong_jacobi_diagonal(monkeypatch):
    def bad(A, rowptr, X):
        d = np.asarray(abs(A).sum(axis=1)).ravel()  # row sums instead of A(i,i)
        return X / d[orc.row_ids(rowptr)]
    assert "krylov" in _pins_fail(monkeypatch, "jacobi", bad)


def test_planted_projector_dropped(monkeypatch):
    assert _pins_fail(monkeypatch, "project", lambda st, X: X.copy())


def test_planted_transposed_block(monkeypatch):
    """Using the wrong index set for the product (A^T-like shift via
    unmasked rows) must fail."""
    real = orc.masked_product

    def bad(A, rowptr, colind, Y, nc):
        out = real(A, rowptr, colind, Y, nc)
        return np.roll(out, 1)
    assert _pins_fail(monkeypatch, "masked_product", bad)


def test_planted_setup_sign(monkeypatch):
    real = orc.emin_setup

    def bad(rowptr, colind, P0, B, Bc):
        st = real(rowptr, colind, P0, B, Bc)
        phat = orc.values_on_pattern(P0, np.asarray(rowptr), np.asarray(colind))
        st.p0 = phat - (st.p0 - phat)  # delta with the wrong sign
        return st
    monkeypatch.setattr(orc, "emin_setup", bad)
    inp, rowptr, colind, st = _tiny(0, m=1, n=16, nc=6, extra_per_row=3)
    st = orc.emin_setup(rowptr, colind, inp.P0, inp.B, inp.Bc)
    assert orc.constraint_error(rowptr, colind, st.p0, inp.B, inp.Bc) > 1e-6


def test_planted_beta_inverted(monkeypatch):
    """beta = gamma_old / gamma instead of gamma / gamma_old."""
    src_rcg = orc.rcg

    def bad_rcg(A, st, nc, maxit, precond="jacobi", bs=1, **kw):
        # re-run the loop with the slip, reusing the oracle's pieces
        rowptr, colind = st.rowptr, st.colind
        K = lambda x: orc.masked_product(A, rowptr, colind, x, nc)
        r = -orc.project(st, K(st.p0))
        dw = np.zeros_like(st.p0)
        y = None
        g_old = None
        for k in range(1, maxit + 1):
            z = orc.project(st, orc.jacobi(A, rowptr, r))
            g = np.sum(r * z)
            y = z.copy() if k == 1 else z + (g_old / g) * y
            g_old = g
            yh = orc.project(st, K(y))
            a = g / np.sum(y * yh)
            dw += a * y
            r = r - a * yh
        res = src_rcg(A, st, nc, 0, precond, bs=bs)
        res.P = st.p0 + dw
        res.status = "converged"
        return res
    # the slip moves the 3rd iterate away from the Krylov minimiser
    inp, rowptr, colind, st = _tiny(0, m=2)
    res = bad_rcg(inp.A, st, inp.nc, 3)
    want = dr.krylov_iterate(inp.A, rowptr, colind, inp.Bc, st.p0,
                             dr.dense_jacobi(inp.A, rowptr, colind), 3)
    assert np.linalg.norm(res.P - want) / np.linalg.norm(want) > 1e-6


def test_block_jacobi_shared_matches_general():
    """The vectorised nodal block-Jacobi (rows of a node share J) equals the
    per-column sub-block definition."""
    inp = gen.tiny_problem(17, n=12, nc=5, m=1, p0_per_row=1, extra_per_row=2)
    rowptr, colind = inp.extra["pattern"]
    # make rows 2a and 2a+1 share the union of their columns
    n = inp.n
    rows = []
    for a in range(n // 2):
        u = sorted(set(colind[rowptr[2 * a]:rowptr[2 * a + 2]].tolist()))
        rows += [u, u]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    assert orc.rows_share_pattern(rp, ci, 2)
    X = np.random.default_rng(1).normal(size=ci.shape[0])
    a = orc.block_jacobi(inp.A, rp, ci, X, 2)
    b = orc.block_jacobi_shared(inp.A, rp, ci, X, 2, inp.nc)
    assert np.allclose(a, b, atol=1e-13)

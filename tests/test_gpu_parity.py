"""GPU path vs the CPU oracle, element by element, through the C ABI.

Bars: pattern and index structure bit-exact; FP64 values within 1e-10
relative (Frobenius; max-abs reported); the mixed form within 1e-4 relative
with the energy within 1e-6 relative and the constraint error at FP64 level.
"""

import numpy as np
import pytest

import gen
import oracle
from oracle import rcg as orc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02995_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _run(ctx, inp, **kw):
    from paper_2208_02995_amd import api

    print(f"[case] {inp.name} n={inp.n} m={inp.m} kw={kw}", flush=True)
    prob = api.Problem.from_input(ctx, inp, **kw)
    P, status, hist, st = prob.solve()
    return prob, P, status, hist, st


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check_fp64(ctx, inp, tol=1e-10, ref=None, **kw):
    prob, P, status, hist, st = _run(ctx, inp, **kw)
    if ref is None:
        ref = oracle.solve(inp, maxit=kw.get("maxit"), precond=kw.get("precond"),
                           tau=kw.get("tau", 0.0))
    st_o, res = ref
    rp, ci = prob.pattern()
    assert np.array_equal(rp, st_o.rowptr), "rowptr differs"
    assert np.array_equal(ci, st_o.colind), "colind differs"
    Pg = P[: prob.nnz].cpu().numpy()
    rel = _rel(Pg, res.P)
    mx = np.abs(Pg - res.P).max() / np.abs(res.P).max()
    print(f"  rel={rel:.3e} maxrel={mx:.3e} it={st.iterations} oracle_it={res.iterations}")
    assert st.iterations == res.iterations
    assert rel < tol
    if res.iterations:
        dE = np.array(res.dE)
        assert np.allclose(hist[: res.iterations], dE, rtol=1e-8, atol=1e-12 * abs(dE[0]))
    ce = prob.constraint_error(P)
    ce_o = orc.constraint_error(st_o.rowptr, st_o.colind, res.P, inp.B, inp.Bc)
    assert ce <= max(1e-12, 10 * ce_o)
    E = prob.energy(P)
    E_o = oracle.energy(inp.A, st_o.rowptr, st_o.colind, res.P, inp.nc)
    assert abs(E - E_o) <= 1e-10 * abs(E_o)
    prob.close()
    return Pg, res


# ------------------------------------------------------------- pattern ---

@pytest.mark.parametrize("k", [1, 2])
def test_pattern_bitexact_tiny(ctx, k):
    from paper_2208_02995_amd import api

    for seed in range(4):
        inp = gen.tiny_problem(seed, n=37, nc=7, p0_per_row=1)
        prob = api.Problem(ctx, inp.A, inp.P0, inp.B, inp.Bc, pattern_power=k, maxit=1)
        rp, ci = prob.pattern()
        rp_o, ci_o = oracle.pattern_expand(inp.A, inp.P0, k)
        assert np.array_equal(rp, rp_o) and np.array_equal(ci, ci_o)
        prob.close()


def test_pattern_bitexact_workloads(ctx):
    from paper_2208_02995_amd import api

    for inp in (gen.poisson2d_32(), gen.poisson3d_ln32(), gen.poisson3d_het96(),
                gen.elasticity_q1_40(Ne=6)):
        prob = api.Problem.from_input(ctx, inp, maxit=1)
        rp, ci = prob.pattern()
        rp_o, ci_o = oracle.pattern_expand(inp.A, inp.P0, inp.pattern_power)
        print(f"[pattern] {inp.name} nnz={prob.nnz}", flush=True)
        assert np.array_equal(rp, rp_o) and np.array_equal(ci, ci_o)
        prob.close()


def _structure_case(kind, bs, m, seed, n_nodes=60, nc_groups=40):
    """Small problems whose structure selects each compressed growth path:
    A in full aligned bs x bs node blocks ('node') or a plain random graph
    ('plain'); P0 rows made of whole aligned groups of m columns, or of
    random columns (m = 1, or 'broken' groups with one partial group)."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    base = gen.tiny_problem(seed, n=n_nodes, nc=5)
    if kind == "node":
        M = np.full((bs, bs), 0.25) + np.eye(bs)
        A = sp.csr_matrix(sp.kron(base.A, M))
    else:
        A = gen.tiny_problem(seed, n=n_nodes * bs, nc=5).A
    A.sort_indices()
    n = A.shape[0]
    nc = nc_groups * m
    rows = []
    for i in range(n):
        if m > 1:
            gs = rng.choice(nc_groups, size=int(rng.integers(1, 3)), replace=False)
            cols = sorted(int(g) * m + t for g in gs for t in range(m))
        else:
            cols = sorted(rng.choice(nc, size=int(rng.integers(1, 3)), replace=False).tolist())
        rows.append(cols)
    if kind == "broken":
        rows[n // 2] = [rows[n // 2][0]]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    P0 = sp.csr_matrix((rng.uniform(0.5, 1.5, ci.size), ci, rp), shape=(n, nc))
    B = rng.standard_normal((n, m))
    Bc = rng.standard_normal((nc, m))
    return A, P0, B, Bc


@pytest.mark.parametrize("kind,bs,m", [("node", 2, 1), ("node", 3, 1), ("node", 3, 2),
                                       ("node", 2, 4), ("plain", 2, 2), ("plain", 1, 2),
                                       ("plain", 3, 1), ("broken", 1, 2), ("node", 1, 3)])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_pattern_bitexact_compressed(ctx, kind, bs, m, k):
    """Growth S^k P0 through every compressed path (node rows when A is in
    full aligned blocks, group ids when P0's rows are whole aligned groups,
    both, neither) equals the oracle's row-by-row growth exactly."""
    from paper_2208_02995_amd import api

    for seed in range(3):
        A, P0, B, Bc = _structure_case(kind, bs, m, seed)
        prob = api.Problem(ctx, A, P0, B, Bc, pattern_power=k, maxit=1, block=bs)
        rp, ci = prob.pattern()
        rp_o, ci_o = oracle.pattern_expand(A, P0, k)
        assert np.array_equal(rp, rp_o) and np.array_equal(ci, ci_o), (kind, bs, m, k, seed)
        prob.close()


# ----------------------------------------------------------- FP64 solve ---

# masked-product kernels that short pattern rows can take (emin_opts hints)
K1_KINDS = {"auto": {}, "wide": {"k1_group": -2}, "wide8": {"k1_group": -2, "k1_slots": 8},
            "short": {"k1_group": 2}, "map": {"k1_slots": -1}, "hash": {"k1_slots": -3},
            "deep": {"k1_group": -4}, "nodemap": {"k1_group": -5}}

@pytest.mark.parametrize("kind", list(K1_KINDS))
@pytest.mark.parametrize("seed,m", [(0, 1), (1, 1), (2, 2), (3, 2), (4, 3)])
def test_fp64_tiny(ctx, seed, m, kind):
    inp = gen.tiny_problem(seed, n=41, nc=9, m=m, p0_per_row=m, extra_per_row=3)
    _check_fp64(ctx, inp, maxit=6, **K1_KINDS[kind])


@pytest.mark.parametrize("kind", list(K1_KINDS))
def test_fp64_poisson2d(ctx, kind):
    _check_fp64(ctx, gen.poisson2d_32(), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", list(K1_KINDS))
def test_fp64_poisson3d_ln32(ctx, kind):
    _check_fp64(ctx, gen.poisson3d_ln32(), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", list(K1_KINDS))
def test_fp64_poisson3d_het_small(ctx, kind):
    # 24^3 cells: many tiles plus a ragged last tile
    _check_fp64(ctx, gen.poisson3d_het96(N=24), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", ["auto", "wide"])
def test_fp64_poisson3d_het96_full(ctx, kind):
    _check_fp64(ctx, gen.poisson3d_het96(), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", ["auto", "hash", "deep", "nodemap"])
def test_fp64_elasticity_small_bjacobi(ctx, kind):
    inp = gen.elasticity_q1_40(Ne=6, maxit=4)
    _check_fp64(ctx, inp, **K1_KINDS[kind])


def test_elasticity_full_masked_product(ctx):
    """Full 40^3 elasticity (14.2M pattern entries, m = 6, rows up to 162):
    the node-map masked product with the projector, element by element."""
    import torch

    from paper_2208_02995_amd import api

    inp = gen.elasticity_q1_40()
    prob = api.Problem.from_input(ctx, inp, maxit=0)
    prob.solve()
    rp, ci = prob.pattern()
    st_o = oracle.emin_setup(rp, ci, inp.P0, inp.B, inp.Bc)
    Y = np.random.default_rng(3).normal(size=ci.size)
    Yd = torch.tensor(Y, device="cuda")
    Yh = torch.empty_like(Yd)
    prob.masked_product(Yd, Yh)
    want = oracle.project(st_o, oracle.masked_product(inp.A, rp, ci, Y, inp.nc))
    got = Yh.cpu().numpy()
    print(f"[mprod C3] rel={_rel(got, want):.2e}", flush=True)
    assert _rel(got, want) < 1e-12
    prob.close()


@pytest.fixture(scope="module")
def elasticity_full():
    """The full 40^3 elasticity workload and its oracle solution at the
    configured 10 iterations (about 100 s on one host core), shared by the
    FP64 and mixed tests."""
    inp = gen.elasticity_q1_40()
    print("[oracle] elasticity_q1_40, 10 iterations ...", flush=True)
    return inp, oracle.solve(inp)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_elasticity_full_10_iterations(ctx, elasticity_full, precision):
    """Full 40^3 elasticity, 3x3 block Jacobi, the configured 10 iterations,
    element by element against the oracle."""
    inp, ref = elasticity_full
    assert inp.maxit == 10 and ref[1].iterations == 10
    if precision == "fp64":
        _check_fp64(ctx, inp, ref=ref)
    else:
        _check_mixed(ctx, inp, ref=ref)


NODE_INPUTS = {
    "elasticity_m3": lambda: gen.elasticity_q1_40(Ne=6, maxit=4, modes=3),
    "elasticity_m1": lambda: gen.elasticity_q1_40(Ne=6, maxit=4, modes=1),
    "grid2d_bs2": lambda: gen.node_grid2d(N=12, bs=2, maxit=5),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(NODE_INPUTS))
def test_node_kernels_other_sizes(ctx, name, precision):
    """Node-blocked A with node-shared pattern rows at other near-kernel and
    node sizes: m = 3 (the node projector specialised for three modes),
    m = 1 (row-by-row projection in the node update), and 2-row nodes (the
    node-map product for two rows per node), each against the oracle."""
    inp = NODE_INPUTS[name]()
    if precision == "fp64":
        _check_fp64(ctx, inp)
    else:
        _check_mixed(ctx, inp)


@pytest.mark.parametrize("name", list(NODE_INPUTS))
def test_node_masked_product_other_sizes(ctx, name):
    import torch

    from paper_2208_02995_amd import api

    inp = NODE_INPUTS[name]()
    prob = api.Problem.from_input(ctx, inp, maxit=1)
    prob.solve()
    rp, ci = prob.pattern()
    st_o = oracle.emin_setup(rp, ci, inp.P0, inp.B, inp.Bc)
    Y = np.random.default_rng(5).normal(size=ci.size)
    Yd = torch.tensor(Y, device="cuda")
    Yh = torch.empty_like(Yd)
    prob.masked_product(Yd, Yh)
    want = oracle.project(st_o, oracle.masked_product(inp.A, rp, ci, Y, inp.nc))
    assert _rel(Yh.cpu().numpy(), want) < 1e-12
    prob.close()


PAIR_DEPTHS = {"depth2": -6, "depth3": -7, "depth4": -8}
PAIR_INPUTS = {
    "elasticity_ne6": lambda: gen.elasticity_q1_40(Ne=6, maxit=4),
    "grid2d_bs2": lambda: gen.node_grid2d(N=12, bs=2, maxit=5),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("depth", list(PAIR_DEPTHS))
@pytest.mark.parametrize("name", list(PAIR_INPUTS))
def test_node_pair_depths(ctx, name, depth, precision):
    """The slot-pair node product at two, three and four neighbour blocks in
    flight (one- and two-node waves): against the oracle, and bitwise equal
    to the default depth (every depth sums the blocks in the same order)."""
    inp = PAIR_INPUTS[name]()
    hint = PAIR_DEPTHS[depth]
    if precision == "fp64":
        _check_fp64(ctx, inp, k1_group=hint)
    else:
        _check_mixed(ctx, inp, k1_group=hint)
    P_hint = _run(ctx, inp, precision=precision, k1_group=hint)
    P_def = _run(ctx, inp, precision=precision)
    a = P_hint[1][: P_hint[0].nnz].cpu().numpy()
    b = P_def[1][: P_def[0].nnz].cpu().numpy()
    assert np.array_equal(a, b)
    for x in (P_hint, P_def):
        x[0].close()


def test_fp64_tiny_block_jacobi(ctx):
    """Nodes of 2 rows sharing their pattern row (block-Jacobi, m = 2)."""
    inp = gen.tiny_problem(9, n=40, nc=8, m=2, p0_per_row=2, extra_per_row=2)
    rp, ci = inp.extra["pattern"]
    rows = []
    for a in range(inp.n // 2):
        u = sorted(set(ci[rp[2 * a]:rp[2 * a + 2]].tolist()))
        rows += [u, u]
    rp2 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci2 = np.concatenate(rows).astype(np.int32)
    inp.extra["pattern"] = (rp2, ci2)
    inp.precond, inp.block = "bjacobi", 2
    _check_fp64(ctx, inp, maxit=5)


def _node_pattern(inp, block):
    """Give the `block` rows of each node the union of their pattern rows."""
    rp, ci = inp.extra["pattern"]
    rows = []
    for a in range(inp.n // block):
        u = sorted(set(ci[rp[block * a]:rp[block * a + block]].tolist()))
        rows += [u] * block
    rp2 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    inp.extra["pattern"] = (rp2, np.concatenate(rows).astype(np.int32))


@pytest.mark.parametrize("block,m,dup,precond,seed", [
    (3, 3, False, "bjacobi", 43), (2, 3, False, "bjacobi", 42), (3, 6, False, "bjacobi", 77),
    (3, 6, True, "bjacobi", 77), (3, 3, False, "jacobi", 43)])
def test_node_setup_shared_pattern(ctx, block, m, dup, precond, seed):
    """Nodes of `block` rows sharing one pattern row: Alg. 2 runs once per
    node (one Gram factorization, W written to every row).  Nodes with fewer
    than m columns, or (dup) with two coarse columns sharing their B_c row,
    go whole to the row-wise fallback; the rank-deficient count matches the
    oracle's SVD branch.  The full-rank rows' Gram matrices are kept well
    conditioned (Cholesky and QR differ by about eps * cond(G_i)^2), which
    the seeds do (cond(G_i)^2 below 1e6, asserted here)."""
    inp = gen.tiny_problem(seed, n=60, nc=12, m=m, p0_per_row=1, extra_per_row=2)
    _node_pattern(inp, block)
    if dup:
        inp.Bc[1] = inp.Bc[0]
    inp.precond, inp.block = precond, block
    rp, ci = inp.extra["pattern"]
    conds = []
    for i in range(inp.n):
        sv = np.linalg.svd(inp.Bc[ci[rp[i]:rp[i + 1]]], compute_uv=False)
        if sv.size >= m and sv[-1] > max(sv.size, m) * 1e3 * np.finfo(float).eps * sv[0]:
            conds.append((sv[0] / sv[-1]) ** 2)
    assert max(conds) < 1e6
    prob, P, status, hist, st = _run(ctx, inp, maxit=5)
    st_o, res = oracle.solve(inp, maxit=5)
    n_def = int(np.sum(st_o.rank < m))
    print(f"  rank-deficient rows: gpu {st.rank_deficient_rows} oracle {n_def}")
    assert st.rank_deficient_rows == n_def
    if m == 6:
        assert n_def > 0  # the fallback is exercised
    prob.close()
    _check_fp64(ctx, inp, maxit=5)


def test_tau_stop(ctx):
    inp = gen.poisson3d_het96(N=12)
    _, res_full = oracle.solve(inp, maxit=12)
    r = np.array(res_full.dE) / res_full.dE[0]
    tau = float(np.sqrt(r[3] * r[4]))
    _check_fp64(ctx, inp, maxit=12, tau=tau)


def test_maxit_zero_returns_corrected_p0(ctx):
    inp = gen.tiny_problem(5, n=30, nc=6, m=2, p0_per_row=2, extra_per_row=2)
    Pg, res = _check_fp64(ctx, inp, maxit=0)
    assert res.iterations == 0


def test_rank_deficient_rows_warn(ctx):
    """Two coarse columns with identical B_c rows make some G_i rank
    deficient; the GPU flags them and matches the oracle's SVD branch."""
    from paper_2208_02995_amd import api, emin

    inp = gen.tiny_problem(11, n=24, nc=5, m=2, p0_per_row=1, extra_per_row=1)
    inp.Bc[1] = inp.Bc[0]
    prob = api.Problem.from_input(ctx, inp, maxit=3)
    P, status, hist, st = prob.solve()
    assert status == emin.EMIN_WARN_RANK and st.rank_deficient_rows > 0
    st_o, res = oracle.solve(inp, maxit=3)
    assert int(np.sum(st_o.rank < 2)) == st.rank_deficient_rows
    Pg = P[: prob.nnz].cpu().numpy()
    print(f"  rel={_rel(Pg, res.P):.2e}", flush=True)
    assert _rel(Pg, res.P) < 1e-10
    prob.close()


def test_deterministic(ctx):
    from paper_2208_02995_amd import api

    inp = gen.poisson3d_het96(N=24)
    prob = api.Problem.from_input(ctx, inp)
    P1 = prob.solve()[0].cpu().numpy()
    P2 = prob.solve()[0].cpu().numpy()
    assert np.array_equal(P1, P2)
    prob.close()


# ------------------------------------------------------ masked product ---

@pytest.mark.parametrize("kind", list(K1_KINDS))
def test_masked_product_entry_point(ctx, kind):
    import torch

    from paper_2208_02995_amd import api

    for inp in (gen.poisson3d_ln32(), gen.elasticity_q1_40(Ne=5),
                gen.tiny_problem(3, n=50, nc=9, m=2, p0_per_row=2, extra_per_row=4)):
        prob = api.Problem.from_input(ctx, inp, maxit=1, **K1_KINDS[kind])
        prob.solve()
        rp, ci = prob.pattern()
        st_o = oracle.emin_setup(rp, ci, inp.P0, inp.B, inp.Bc)
        Y = np.random.default_rng(0).normal(size=ci.size)
        Yd = torch.tensor(Y, device="cuda")
        Yh = torch.empty_like(Yd)
        prob.masked_product(Yd, Yh)
        want = oracle.project(st_o, oracle.masked_product(inp.A, rp, ci, Y, inp.nc))
        got = Yh.cpu().numpy()
        print(f"[mprod] {inp.name} rel={_rel(got, want):.2e}", flush=True)
        assert _rel(got, want) < 1e-12
        prob.close()


# ------------------------------------------------------------- mixed -----

def _check_mixed(ctx, inp, ref=None, **kw):
    prob, P, status, hist, st = _run(ctx, inp, precision="mixed", **kw)
    st_o, res = ref if ref is not None else oracle.solve(inp, maxit=kw.get("maxit"))
    Pg = P[: prob.nnz].cpu().numpy()
    rel = _rel(Pg, res.P)
    E = oracle.energy(inp.A, st_o.rowptr, st_o.colind, Pg, inp.nc)
    E_o = oracle.energy(inp.A, st_o.rowptr, st_o.colind, res.P, inp.nc)
    ce = orc.constraint_error(st_o.rowptr, st_o.colind, Pg, inp.B, inp.Bc)
    print(f"  mixed rel={rel:.2e} dE/E={abs(E - E_o) / E_o:.2e} cons={ce:.2e}")
    assert rel < 1e-4
    assert abs(E - E_o) <= 1e-6 * abs(E_o)
    assert ce < 1e-12
    prob.close()


@pytest.mark.parametrize("kind", ["auto", "hash", "deep", "nodemap"])
def test_mixed_elasticity_small_kinds(ctx, kind):
    _check_mixed(ctx, gen.elasticity_q1_40(Ne=6, maxit=4), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", list(K1_KINDS))
def test_mixed_poisson2d(ctx, kind):
    _check_mixed(ctx, gen.poisson2d_32(), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", list(K1_KINDS))
def test_mixed_poisson3d_het_small(ctx, kind):
    _check_mixed(ctx, gen.poisson3d_het96(N=24), **K1_KINDS[kind])


@pytest.mark.parametrize("kind", ["auto", "wide"])
def test_mixed_poisson3d_het96_full(ctx, kind):
    _check_mixed(ctx, gen.poisson3d_het96(), **K1_KINDS[kind])


def test_mixed_elasticity_small(ctx):
    _check_mixed(ctx, gen.elasticity_q1_40(Ne=6, maxit=4))


# ------------------------------------------------------------- errors ----

def test_error_paths(ctx):
    import scipy.sparse as sp

    from paper_2208_02995_amd import api, emin

    inp = gen.tiny_problem(2, n=20, nc=5, m=1, p0_per_row=1, extra_per_row=2)
    # pattern missing an entry of P0
    rp, ci = inp.extra["pattern"]
    P0c = inp.P0
    bad_rows = []
    for i in range(inp.n):
        cols = [c for c in ci[rp[i]:rp[i + 1]] if not (i == 0 and c == P0c.indices[P0c.indptr[0]])]
        bad_rows.append(cols)
    brp = np.concatenate([[0], np.cumsum([len(r) for r in bad_rows])]).astype(np.int32)
    bci = np.concatenate(bad_rows).astype(np.int32)
    with pytest.raises(emin.EminError) as e:
        api.Problem(ctx, inp.A, inp.P0, inp.B, inp.Bc, pattern=(brp, bci))
    assert e.value.status == emin.EMIN_ERR_PATTERN
    # unsorted columns in A
    A = inp.A.copy()
    r0 = A.indptr[0]
    A.indices[r0], A.indices[r0 + 1] = A.indices[r0 + 1], A.indices[r0]
    with pytest.raises(emin.EminError) as e:
        api.Problem(ctx, A, inp.P0, inp.B, inp.Bc)
    assert e.value.status == emin.EMIN_ERR_CSR
    # non-positive diagonal
    A = inp.A.copy()
    d = A.indptr[3] + list(A.indices[A.indptr[3]:A.indptr[4]]).index(3)
    A.data[d] = -1.0
    prob = api.Problem(ctx, A, inp.P0, inp.B, inp.Bc)
    with pytest.raises(emin.EminError) as e:
        prob.solve()
    assert e.value.status == emin.EMIN_ERR_DIAG
    prob.close()
    # missing diagonal
    A = sp.csr_matrix(inp.A.toarray() - np.diag(np.diag(inp.A.toarray())))
    A.sort_indices()
    with pytest.raises(emin.EminError) as e:
        api.Problem(ctx, A, inp.P0, inp.B, inp.Bc)
    assert e.value.status == emin.EMIN_ERR_DIAG
    # m out of range
    with pytest.raises(emin.EminError) as e:
        api.Problem(ctx, inp.A, inp.P0, np.ones((inp.n, 9)), np.ones((inp.nc, 9)))
    assert e.value.status == emin.EMIN_ERR_UNSUPPORTED


# ------------------------------------------------------- edge cases -------

@pytest.mark.parametrize("extra", [12, 25, 70])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_long_rows_each_kernel_shape(ctx, extra, precision):
    """Pattern rows of 13, 26 and 71 entries select the column-matching
    kernel (S = 16), the row-map kernel (17..32) and the LDS-hash kernel
    (> 32, no node structure)."""
    inp = gen.tiny_problem(21, n=300, nc=120, m=1, p0_per_row=1, extra_per_row=extra)
    if precision == "fp64":
        _check_fp64(ctx, inp, maxit=6)
    else:
        _check_mixed(ctx, inp, maxit=6)


def test_max_m(ctx):
    """m = EMIN_MAX_M = 8 near-kernel vectors (8 x 8 Gram factors per row)."""
    inp = gen.tiny_problem(22, n=60, nc=20, m=8, p0_per_row=8, extra_per_row=6)
    _check_fp64(ctx, inp, maxit=5)


def _with_empty_rows(rows, zero_b=True):
    import scipy.sparse as sp

    inp = gen.tiny_problem(23, n=40, nc=8, m=1, p0_per_row=1, extra_per_row=2)
    rp, ci = inp.extra["pattern"]
    pat = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(inp.n, inp.nc)).tolil()
    P0 = inp.P0.tolil()
    B = inp.B.copy()
    for r in rows:
        pat.rows[r] = []
        pat.data[r] = []
        P0.rows[r] = []
        P0.data[r] = []
        if zero_b:
            B[r] = 0.0
    pat = pat.tocsr()
    pat.sort_indices()
    P0 = P0.tocsr()
    P0.sort_indices()
    inp.P0 = P0
    inp.B = B
    inp.extra["pattern"] = (pat.indptr.astype(np.int32), pat.indices.astype(np.int32))
    return inp


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_empty_pattern_rows(ctx, precision):
    """Rows with an empty pattern row (first, middle and last row): they carry
    no unknowns, their G_i has rank 0 (flagged, as in the oracle's SVD
    branch), and every other row is unaffected."""
    from paper_2208_02995_amd import api, emin

    inp = _with_empty_rows((0, 17, 39))
    prob = api.Problem.from_input(ctx, inp, maxit=5, precision=precision)
    P, status, hist, st = prob.solve()
    assert status == emin.EMIN_WARN_RANK and st.rank_deficient_rows == 3
    st_o, res = oracle.solve(inp, maxit=5)
    assert int(np.sum(st_o.rank < 1)) == 3
    rp, ci = prob.pattern()
    assert np.array_equal(rp, st_o.rowptr) and np.array_equal(ci, st_o.colind)
    Pg = P[: prob.nnz].cpu().numpy()
    assert _rel(Pg, res.P) < (1e-10 if precision == "fp64" else 1e-4)
    assert prob.constraint_error(P) < 1e-12
    prob.close()


def test_unsatisfiable_rows_reported(ctx):
    """An empty pattern row whose B row is not zero cannot meet the
    constraint: the row is flagged rank deficient and the constraint error
    reports it; the rest of P still matches the oracle."""
    from paper_2208_02995_amd import api, emin

    inp = _with_empty_rows((5,), zero_b=False)
    prob = api.Problem.from_input(ctx, inp, maxit=4)
    P, status, hist, st = prob.solve()
    assert status == emin.EMIN_WARN_RANK and st.rank_deficient_rows == 1
    st_o, res = oracle.solve(inp, maxit=4)
    Pg = P[: prob.nnz].cpu().numpy()
    assert _rel(Pg, res.P) < 1e-10
    ce = prob.constraint_error(P)
    ce_o = orc.constraint_error(st_o.rowptr, st_o.colind, res.P, inp.B, inp.Bc)
    assert abs(ce - ce_o) <= 1e-12 + 1e-9 * ce_o and ce > 1e-3
    prob.close()


def test_empty_problem(ctx):
    """n = 0: creation, solve, energy and constraint on an empty problem."""
    import scipy.sparse as sp

    from paper_2208_02995_amd import api, emin

    A = sp.csr_matrix((0, 0))
    P0 = sp.csr_matrix((0, 3))
    prob = api.Problem(ctx, A, P0, np.zeros((0, 1)), np.ones((3, 1)), maxit=3)
    assert prob.nnz == 0
    P, status, hist, st = prob.solve()
    assert status == emin.EMIN_OK and st.iterations == 0
    assert prob.energy(P) == 0.0 and prob.constraint_error(P) == 0.0
    prob.close()


def test_empty_pattern(ctx):
    """n > 0 but an empty pattern (P0 without entries, B = 0): nothing to
    minimise; the solve returns at once."""
    import scipy.sparse as sp

    from paper_2208_02995_amd import api, emin

    n = 7
    A = sp.diags(np.full(n, 2.0)).tocsr() - sp.eye(n, k=1).tocsr() - sp.eye(n, k=-1).tocsr()
    A = A.tocsr()
    A.sort_indices()
    P0 = sp.csr_matrix((n, 2))
    prob = api.Problem(ctx, A, P0, np.zeros((n, 1)), np.ones((2, 1)), maxit=4)
    assert prob.nnz == 0
    P, status, hist, st = prob.solve()
    assert status == emin.EMIN_OK and st.iterations == 0
    assert prob.energy(P) == 0.0 and prob.constraint_error(P) == 0.0
    prob.close()

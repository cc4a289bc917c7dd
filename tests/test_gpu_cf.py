"""Alg. 1 (Sec. 3.2) and the C/F form P = [W; I] (Sec. 2) on the GPU
against the oracle: the tentative prolongation's structure and fitted
distances bit-exact and its values to rounding; the RCG on the C/F pattern
element by element (FP64 within 1e-10; mixed within 1e-4, energy 1e-6),
COARSE rows exactly the identity."""

import numpy as np
import pytest

import gen
import oracle
from oracle import ptent
from oracle import rcg as orc

pytestmark = pytest.mark.gpu

CASES = {
    "poisson2d_32": lambda: gen.cf_poisson2d(32),
    "linear2d_24": lambda: gen.cf_linear2d(24),
    "random0": lambda: gen.cf_random(0),
    "random1_m3": lambda: gen.cf_random(1, m=3),
    "random2_m1": lambda: gen.cf_random(2, m=1),
    "random3_m2": lambda: gen.cf_random(3, n=200, m=2, lmax=4),
    "poisson2d_128": lambda: gen.cf_poisson2d(128),
}


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02995_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _gpu_ptent(ctx, inp):
    from paper_2208_02995_amd import api

    P0, level = api.ptent_setup(ctx, inp.S, inp.cf, inp.V, inp.lmax, nc=inp.nc)
    return P0, level


@pytest.mark.parametrize("name", list(CASES))
def test_ptent_matches_oracle(ctx, name):
    inp = CASES[name]()
    print(f"[ptent] {name} n={inp.n} nc={inp.nc} m={inp.m} lmax={inp.lmax}", flush=True)
    P0g, lev_g = _gpu_ptent(ctx, inp)
    P0o, lev_o = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    G = P0g.to_scipy()
    assert np.array_equal(lev_g, lev_o)
    assert np.array_equal(G.indptr, P0o.indptr)
    assert np.array_equal(G.indices, P0o.indices)
    assert np.allclose(G.data, P0o.data, rtol=1e-12, atol=1e-12 * np.abs(P0o.data).max())
    print(f"  nnz={G.nnz} levels={np.bincount(lev_o + 1)} "
          f"max diff={np.abs(G.data - P0o.data).max():.1e}", flush=True)


def _oracle_cf(inp, P0, maxit, precond="jacobi"):
    rp, ci = ptent.cf_pattern(inp.A, P0, inp.cf, inp.pattern_power)
    st = oracle.emin_setup(rp, ci, P0, inp.V, inp.Bc)
    res = oracle.rcg_solve(inp.A, st, inp.nc, maxit, precond)
    return rp, ci, st, res


@pytest.mark.parametrize("name", ["poisson2d_32", "linear2d_24", "random0", "random1_m3",
                                  "random3_m2", "poisson2d_128"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cf_solve_matches_oracle(ctx, name, precision):
    from paper_2208_02995_amd import api

    inp = CASES[name]()
    P0g, _ = _gpu_ptent(ctx, inp)
    P0o, _ = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    rp, ci, st, res = _oracle_cf(inp, P0o, inp.maxit)
    prob = api.Problem(ctx, inp.A, P0g, inp.V, inp.Bc, cf=inp.cf, precision=precision,
                       maxit=inp.maxit, pattern_power=inp.pattern_power)
    rpg, cig = prob.pattern()
    assert np.array_equal(rpg, rp) and np.array_equal(cig, ci)
    P, status, hist, stt = prob.solve()
    Pg = P[: prob.nnz].cpu().numpy()
    rows = np.repeat(np.arange(inp.n), np.diff(rp))
    coarse = inp.cf[rows] >= 0
    assert np.all(Pg[coarse] == 1.0)  # COARSE rows stay the identity
    rel = np.linalg.norm(Pg - res.P) / np.linalg.norm(res.P)
    n_def = int(np.sum((st.rank < inp.m) & (inp.cf < 0)))
    print(f"[cf] {name} {precision} rel={rel:.2e} rank-deficient FINE rows: gpu "
          f"{stt.rank_deficient_rows} oracle {n_def}", flush=True)
    assert stt.rank_deficient_rows == n_def
    assert stt.iterations == res.iterations
    if precision == "fp64":
        assert rel < 1e-10
    else:
        E = oracle.energy(inp.A, rp, ci, Pg, inp.nc)
        E_o = oracle.energy(inp.A, rp, ci, res.P, inp.nc)
        assert rel < 1e-4
        assert abs(E - E_o) <= 1e-6 * abs(E_o)
    ce = orc.constraint_error(rp, ci, Pg, inp.V, inp.Bc)
    ce_o = orc.constraint_error(rp, ci, res.P, inp.V, inp.Bc)
    assert ce <= max(1e-12, 10 * ce_o)
    prob.close()


def test_cf_sgs(ctx):
    from paper_2208_02995_amd import api

    inp = CASES["poisson2d_32"]()
    P0g, _ = _gpu_ptent(ctx, inp)
    P0o, _ = ptent.ptent_setup(inp.S, inp.V, inp.cf, inp.lmax)
    rp, ci, st, res = _oracle_cf(inp, P0o, inp.maxit, precond="sgs")
    prob = api.Problem(ctx, inp.A, P0g, inp.V, inp.Bc, cf=inp.cf, precond="sgs",
                       maxit=inp.maxit)
    Pg = prob.solve()[0][: prob.nnz].cpu().numpy()
    assert np.linalg.norm(Pg - res.P) / np.linalg.norm(res.P) < 1e-10
    prob.close()


def test_cf_rejects_bad_splitting(ctx):
    from paper_2208_02995_amd import api, emin

    inp = CASES["random0"]()
    P0g, _ = _gpu_ptent(ctx, inp)
    bad = inp.cf.copy()
    c0 = np.flatnonzero(bad >= 0)[:2]
    bad[c0[1]] = bad[c0[0]]  # a coarse index held twice
    with pytest.raises(emin.EminError):
        api.Problem(ctx, inp.A, P0g, inp.V, inp.Bc, cf=bad, maxit=2)
    # a COARSE row of P0 that is not its identity row
    P0s = P0g.to_scipy()
    r = c0[0]
    P0s.data[P0s.indptr[r]] = 2.0
    with pytest.raises(emin.EminError):
        api.Problem(ctx, inp.A, P0s, inp.V, inp.Bc, cf=inp.cf, maxit=2)

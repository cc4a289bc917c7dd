"""Projected SGS preconditioner M_2 (Sec. 3.4.1, eq. SGS_prec) on the GPU
against the oracle: the sweep colouring bit-exact, the RCG iterates element
by element (FP64 within 1e-10; mixed within 1e-4, energy within 1e-6)."""

import numpy as np
import pytest

import gen
import oracle
from oracle import sgs as osgs
from tests.test_gpu_parity import _check_fp64, _check_mixed

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


def _sgs(inp, maxit=None):
    inp.precond = "sgs"
    if maxit is not None:
        inp.maxit = maxit
    return inp


CASES = {
    "tiny_m1": lambda: gen.tiny_problem(0, n=41, nc=9, m=1, p0_per_row=1, extra_per_row=3),
    "tiny_m2": lambda: gen.tiny_problem(2, n=41, nc=9, m=2, p0_per_row=2, extra_per_row=3),
    "tiny_m3": lambda: gen.tiny_problem(4, n=41, nc=9, m=3, p0_per_row=3, extra_per_row=3),
    "poisson2d_32": lambda: gen.poisson2d_32(),
    "poisson3d_ln32": lambda: gen.poisson3d_ln32(),
    "het_24": lambda: gen.poisson3d_het96(N=24),
    "elasticity_4": lambda: gen.elasticity_q1_40(Ne=4, maxit=4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sgs_colours_bitexact(ctx, name):
    from paper_2208_02995_amd import api

    inp = _sgs(CASES[name](), maxit=1)
    prob = api.Problem.from_input(ctx, inp)
    nc, col = prob.sgs_colours()
    want = osgs.jp_colours(inp.A)
    print(f"[colours] {name} n={inp.n} colours={nc}", flush=True)
    assert nc == int(want.max()) + 1
    assert np.array_equal(col, want)
    prob.close()


@pytest.mark.parametrize("name", list(CASES))
def test_sgs_fp64(ctx, name):
    inp = _sgs(CASES[name](), maxit=5)
    _check_fp64(ctx, inp, maxit=5, precond="sgs")


@pytest.mark.parametrize("name", ["tiny_m1", "tiny_m2", "poisson2d_32", "poisson3d_ln32",
                                  "elasticity_4"])
def test_sgs_mixed(ctx, name):
    inp = _sgs(CASES[name](), maxit=5)
    _check_mixed(ctx, inp, maxit=5)


def test_sgs_tau_stop(ctx):
    inp = _sgs(gen.poisson3d_het96(N=12), maxit=12)
    _, full = oracle.solve(inp, maxit=12)
    r = np.array(full.dE) / full.dE[0]
    tau = float(np.sqrt(r[3] * r[4]))
    _check_fp64(ctx, inp, maxit=12, precond="sgs", tau=tau)


def test_sgs_deterministic(ctx):
    from paper_2208_02995_amd import api

    inp = _sgs(gen.poisson3d_het96(N=18), maxit=6)
    prob = api.Problem.from_input(ctx, inp)
    a = prob.solve()[0][: prob.nnz].cpu().numpy().copy()
    b = prob.solve()[0][: prob.nnz].cpu().numpy().copy()
    assert np.array_equal(a, b)
    prob.close()


def test_sgs_converges_faster_than_jacobi(ctx):
    """Per iteration, M_2 lowers the energy more than Jacobi (Sec. 5)."""
    from paper_2208_02995_amd import api

    inp = gen.poisson3d_het96(N=18)
    inp.maxit = 6
    E = {}
    for pc in ("jacobi", "sgs"):
        inp.precond = pc
        prob = api.Problem.from_input(ctx, inp)
        E[pc] = prob.energy(prob.solve()[0])
        prob.close()
    assert E["sgs"] < E["jacobi"]

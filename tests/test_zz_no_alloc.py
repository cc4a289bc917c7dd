"""The allocation-free energy entry point against emin_energy, through the
C ABI: two calls in a row on one GPU (the second on a smaller problem, so
the shared scratch array still holds the first call's larger contents), the
kernels that stage P (one lane per row, node map) and the one that does not,
and the clear error for a pattern beyond the scratch array."""

import numpy as np
import pytest

import gen
import oracle

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


def _energies(ctx, inp):
    from paper_2208_02995_amd import api, emin

    prob = api.Problem.from_input(ctx, inp)
    P, status, hist, st = prob.solve()
    E = emin.emin_energy(prob.handle, P)
    E_na = emin.emin_energy_noalloc(prob.handle, P)
    rp, ci = prob.pattern()
    E_o = oracle.energy(inp.A, rp, ci, P[: prob.nnz].cpu().numpy(), inp.nc)
    print(f"[noalloc] {inp.name} nnz(P)={prob.nnz} E={E:.17g} noalloc={E_na:.17g}", flush=True)
    prob.close()
    return E, E_na, E_o


def test_noalloc_energy_two_calls(ctx):
    # larger first, then smaller: the second call must not depend on what the
    # first left in the scratch array
    for inp in (gen.poisson3d_ln32(), gen.poisson2d_32(), gen.elasticity_q1_40(Ne=5, maxit=2),
                gen.tiny_problem(3, n=50, nc=9, m=2, p0_per_row=2, extra_per_row=4)):
        E, E_na, E_o = _energies(ctx, inp)
        assert E_na == E
        assert abs(E_na - E_o) <= 1e-10 * abs(E_o)


def test_noalloc_energy_rejects_large_pattern(ctx):
    from paper_2208_02995_amd import api, emin

    inp = gen.poisson3d_het96()
    prob = api.Problem.from_input(ctx, inp, maxit=0)
    P = prob.new_values()
    P.zero_()
    with pytest.raises(emin.EminError) as e:
        emin.emin_energy_noalloc(prob.handle, P)
    assert e.value.status == emin.EMIN_ERR_UNSUPPORTED
    assert "scratch" in str(e.value)
    # the allocating entry point still works on it
    assert emin.emin_energy(prob.handle, P) == 0.0
    prob.close()

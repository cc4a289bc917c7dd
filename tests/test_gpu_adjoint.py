"""Reverse mode on the GPU (emin_solve_taped / emin_backward / emin_loss and
the torch.autograd wrappers) against the oracle's reverse sweep, which is
itself pinned by complex-step derivatives (tests/test_adjoint_oracle.py),
and against central finite differences of the GPU forward path."""

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from oracle import adjoint as oad

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


def _gpu_grad(ctx, inp, e, wE, wT, maxit=None):
    """(L, dL/dA, dL/dP0, iterations) through the C ABI."""
    import torch

    from paper_2208_02995_amd import api

    kw = {} if maxit is None else {"maxit": maxit}
    prob = api.Problem.from_input(ctx, inp, **kw)
    P, status, tape = prob.solve_taped()
    e_d = torch.tensor(e, dtype=torch.float64, device="cuda") if e is not None else None
    L, gP, gA = prob.loss(P, e_d, wE, wT)
    gA, gP0 = tape.backward(gP, gA)
    out = (L, gA.cpu().numpy(), gP0.cpu().numpy())
    tape.close()
    prob.close()
    return out


def _close(got, ref, tol):
    scale = max(np.abs(ref).max(), 1e-300)
    return np.abs(got - ref).max() <= tol * scale


@pytest.mark.parametrize("seed,m,wE,wT", [(0, 1, 1.0, 0.0), (1, 1, 0.0, 1.0), (2, 2, 1.0, 1.0),
                                          (3, 1, 1.0, 1.0)])
def test_backward_tiny_matches_oracle(ctx, seed, m, wE, wT):
    inp = gen.tiny_problem(seed, n=12, nc=4, m=m, p0_per_row=m, extra_per_row=2)
    e = np.random.default_rng(seed + 100).normal(size=inp.n)
    print(f"[adjoint tiny] seed={seed} m={m} wE={wE} wT={wT}", flush=True)
    L, gA, gP0 = _gpu_grad(ctx, inp, e, wE, wT, maxit=4)
    L_o, gA_o, gP0_o = oad.gradient(inp, maxit=4, e=e, w_energy=wE, w_twogrid=wT)
    assert abs(L - L_o) <= 1e-11 * abs(L_o)
    assert _close(gA, gA_o, 1e-10)
    assert _close(gP0, gP0_o, 1e-10)


@pytest.mark.parametrize("seed", [0, 3])
def test_backward_after_early_stop(ctx, seed):
    """The forward stops on the gamma floor before maxit: the sweep must run
    over the applied iterations only.  Converged, P is the exact minimiser
    over P0' + range(Pi) and P0' moves only inside range(Pi) with P0's values,
    so dL/dP0 vanishes (to rounding) on both sides."""
    inp = gen.tiny_problem(seed, n=12, nc=4, m=1, p0_per_row=1, extra_per_row=1)
    e = np.random.default_rng(seed + 7).normal(size=inp.n)
    print(f"[adjoint early stop] seed={seed}", flush=True)
    L, gA, gP0 = _gpu_grad(ctx, inp, e, 1.0, 1.0, maxit=25)
    L_o, gA_o, gP0_o = oad.gradient(inp, maxit=25, e=e)
    assert abs(L - L_o) <= 1e-11 * abs(L_o)
    assert _close(gA, gA_o, 1e-10)
    scale = np.abs(gA_o).max()
    assert np.abs(gP0).max() <= 1e-12 * scale
    assert np.abs(gP0_o).max() <= 1e-12 * scale


def test_backward_poisson3d_ln32_matches_oracle(ctx):
    """3D log-normal Poisson, 32^3 cells, 5 iterations, energy + two-grid loss."""
    inp = gen.poisson3d_ln32()
    e = inp.extra["e"]
    print("[adjoint C5] poisson3d_ln32", flush=True)
    L, gA, gP0 = _gpu_grad(ctx, inp, e, 1.0, 1.0)
    L_o, gA_o, gP0_o = oad.gradient(inp, e=e)
    print(f"  L={L:.12e} L_o={L_o:.12e}", flush=True)
    assert abs(L - L_o) <= 1e-11 * abs(L_o)
    assert _close(gA, gA_o, 1e-10)
    assert _close(gP0, gP0_o, 1e-10)


def _sym_direction(A, rng):
    """Random direction on A's stored entries with V = V^T (A stays symmetric)."""
    V = sp.csr_matrix((rng.normal(size=A.nnz), A.indices, A.indptr), shape=A.shape)
    S = ((V + V.T) * 0.5).tocsr()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    return np.asarray(S[rows, A.indices]).ravel()


def test_backward_poisson3d_ln32_central_fd(ctx):
    """Central differences (h = 1e-6) of the GPU forward path in 16 random
    directions of (A values, P0 values) agree with the GPU gradient to 1e-5.
    Directions have N(0, 1) entries (not unit length): the loss is ~2e5, so its
    rounding error over 2h must stay well below the directional derivative."""
    import torch

    from paper_2208_02995_amd import api

    inp = gen.poisson3d_ln32()
    e_d = torch.tensor(inp.extra["e"], dtype=torch.float64, device="cuda")
    prob = api.Problem.from_input(ctx, inp)
    a0 = prob.A.vals.clone()
    q0 = prob.P0.vals.clone()
    P, _, tape = prob.solve_taped()
    L0, gP, gA = prob.loss(P, e_d, 1.0, 1.0)
    gA, gP0 = tape.backward(gP, gA)
    tape.close()
    gA = gA.cpu().numpy()
    gP0 = gP0.cpu().numpy()

    def L_at(av, qv):
        prob.A.vals.copy_(torch.tensor(av, device="cuda"))
        prob.P0.vals.copy_(torch.tensor(qv, device="cuda"))
        Pn = prob.solve()[0]
        return prob.loss(Pn, e_d, 1.0, 1.0, grad=False)[0]

    rng = np.random.default_rng(2024)
    h = 1e-6
    a0h = a0.cpu().numpy()
    q0h = q0.cpu().numpy()
    worst = 0.0
    for d in range(16):
        va = _sym_direction(inp.A, rng)
        vq = rng.normal(size=inp.P0.nnz)
        fd = (L_at(a0h + h * va, q0h + h * vq) - L_at(a0h - h * va, q0h - h * vq)) / (2 * h)
        an = gA @ va + gP0 @ vq
        rel = abs(fd - an) / abs(an)
        worst = max(worst, rel)
        print(f"  dir {d}: fd={fd:.10e} adj={an:.10e} rel={rel:.2e}", flush=True)
        assert rel <= 1e-5
    print(f"  worst rel = {worst:.2e}", flush=True)
    prob.A.vals.copy_(a0)
    prob.P0.vals.copy_(q0)
    prob.close()


def test_autograd_functions(ctx):
    """torch.autograd through EminRCG and EminLoss gives the oracle gradient."""
    import torch

    from paper_2208_02995_amd import api, autograd

    inp = gen.tiny_problem(5, n=14, nc=5, m=1, extra_per_row=2)
    e = np.random.default_rng(9).normal(size=inp.n)
    prob = api.Problem.from_input(ctx, inp, maxit=5)
    A_t = prob.A.vals.clone().requires_grad_(True)
    P0_t = prob.P0.vals.clone().requires_grad_(True)
    e_t = torch.tensor(e, dtype=torch.float64, device="cuda")
    P = autograd.rcg(prob, A_t, P0_t)
    L = autograd.loss(prob, P, A_t, e_t, 1.0, 1.0)
    (3.0 * L).backward()
    L_o, gA_o, gP0_o = oad.gradient(inp, maxit=5, e=e)
    assert abs(L.item() - L_o) <= 1e-11 * abs(L_o)
    assert _close(A_t.grad.cpu().numpy(), 3.0 * gA_o, 1e-10)
    assert _close(P0_t.grad.cpu().numpy(), 3.0 * gP0_o, 1e-10)
    prob.close()


def test_backward_twice_on_one_tape(ctx):
    """emin_backward may run twice on one tape; later solves do not disturb it."""
    import torch

    from paper_2208_02995_amd import api

    inp = gen.tiny_problem(6, n=12, nc=4, m=1, extra_per_row=2)
    prob = api.Problem.from_input(ctx, inp, maxit=4)
    P, _, tape = prob.solve_taped()
    _, gP, _ = prob.loss(P, None, 1.0, 0.0)
    gA1, gP01 = tape.backward(gP)
    prob.A.vals.mul_(2.0)
    prob.solve()
    prob.A.vals.mul_(0.5)
    gA2, gP02 = tape.backward(gP)
    assert torch.equal(gA1, gA2) and torch.equal(gP01, gP02)
    tape.close()
    prob.close()


def test_backward_poisson3d_ln32_per_entry_fd(ctx):
    """Per-entry central differences (h = 1e-6) on the 200 entries of A and
    the 200 of P0 with the largest gradients.  An entry of A moves A(i,l) and
    A(l,i) together (A must stay symmetric), so it is compared with
    g(i,l) + g(l,i).  A single-entry difference of a loss of ~2e5 carries the
    rounding of L over 2h, about 1e-10 |L| in absolute terms, so the bound is
    1e-5 |g| plus that floor (the directional test above is the 1e-5
    relative check)."""
    import torch

    from paper_2208_02995_amd import api

    inp = gen.poisson3d_ln32()
    e_d = torch.tensor(inp.extra["e"], dtype=torch.float64, device="cuda")
    prob = api.Problem.from_input(ctx, inp)
    a0 = prob.A.vals.clone()
    q0 = prob.P0.vals.clone()
    P, _, tape = prob.solve_taped()
    _, gP, gA = prob.loss(P, e_d, 1.0, 1.0)
    gA, gP0 = tape.backward(gP, gA)
    tape.close()
    gA = gA.cpu().numpy()
    gP0 = gP0.cpu().numpy()
    A = inp.A
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    # position of the transposed entry (l, i) of every stored (i, l)
    key = rows.astype(np.int64) * A.shape[0] + A.indices
    tkey = A.indices.astype(np.int64) * A.shape[0] + rows
    tpos = np.searchsorted(key, tkey)
    gsym = np.where(rows == A.indices, gA, gA + gA[tpos])

    def L_at(av, qv):
        prob.A.vals.copy_(av)
        prob.P0.vals.copy_(qv)
        Pn = prob.solve()[0]
        return prob.loss(Pn, e_d, 1.0, 1.0, grad=False)[0]

    h = 1e-6
    L0 = abs(L_at(a0, q0))
    floor = 3e-10 * L0
    worst = 0.0
    for j in np.argsort(-np.abs(gsym))[:200]:
        d = torch.zeros_like(a0)
        d[int(j)] = h
        if tpos[j] != j:
            d[int(tpos[j])] = h
        fd = (L_at(a0 + d, q0) - L_at(a0 - d, q0)) / (2 * h)
        rel = abs(fd - gsym[j]) / abs(gsym[j])
        worst = max(worst, rel)
        assert abs(fd - gsym[j]) <= 1e-5 * abs(gsym[j]) + floor, (int(j), fd, gsym[j])
    for j in np.argsort(-np.abs(gP0))[:200]:
        d = torch.zeros_like(q0)
        d[int(j)] = h
        fd = (L_at(a0, q0 + d) - L_at(a0, q0 - d)) / (2 * h)
        rel = abs(fd - gP0[j]) / abs(gP0[j])
        worst = max(worst, rel)
        assert abs(fd - gP0[j]) <= 1e-5 * abs(gP0[j]) + floor, (int(j), fd, gP0[j])
    print(f"  per-entry worst rel = {worst:.2e} (floor {floor:.1e})", flush=True)
    prob.A.vals.copy_(a0)
    prob.P0.vals.copy_(q0)
    prob.close()


def test_loss_forward_backward_pair(ctx):
    """emin_loss_forward / emin_loss_backward give what emin_loss gives."""
    import torch

    from paper_2208_02995_amd import api, emin

    inp = gen.poisson3d_ln32(N=8)
    prob = api.Problem.from_input(ctx, inp, maxit=3)
    P = prob.solve()[0]
    e_d = torch.tensor(np.random.default_rng(3).standard_normal(inp.n), dtype=torch.float64,
                       device="cuda")
    L, gP, gA = prob.loss(P, e_d, 1.0, 1.0)
    L2 = emin.emin_loss_forward(prob.handle, P, e_d, 1.0, 1.0)
    gP2 = prob.new_values()
    gA2 = torch.zeros_like(prob.A.vals)
    emin.emin_loss_backward(prob.handle, P, e_d, 1.0, 1.0, gP2, gA2)
    assert L2 == L
    assert torch.equal(gP2[: prob.nnz], gP[: prob.nnz]) and torch.equal(gA2, gA)
    prob.close()

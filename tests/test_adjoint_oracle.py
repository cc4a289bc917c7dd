"""Pins of the oracle's reverse sweep (oracle/adjoint.py).

With B_c fixed every step of the path is analytic in the values of A and P0,
so the complex-step derivative Im L(theta + i h v) / h (h = 1e-30) equals the
exact directional derivative to rounding: an independent route to every
component of the gradient."""

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from oracle import adjoint as oad


def _cs_A(inp, j, e, maxit, wE, wT, h=1e-30):
    av = inp.A.data.astype(complex)
    av[j] += 1j * h
    L, *_ = oad.forward(inp, A_vals=av, maxit=maxit, e=e, w_energy=wE, w_twogrid=wT)
    return np.imag(L) / h


def _cs_P0(inp, j, e, maxit, wE, wT, h=1e-30):
    pv = inp.P0.data.astype(complex)
    pv[j] += 1j * h
    L, *_ = oad.forward(inp, P0_vals=pv, maxit=maxit, e=e, w_energy=wE, w_twogrid=wT)
    return np.imag(L) / h


@pytest.mark.parametrize("seed,m,wE,wT", [(0, 1, 1.0, 0.0), (1, 1, 0.0, 1.0), (2, 2, 1.0, 1.0),
                                          (3, 1, 1.0, 1.0)])
def test_reverse_sweep_matches_complex_step_every_entry(seed, m, wE, wT):
    inp = gen.tiny_problem(seed, n=12, nc=4, m=m, p0_per_row=m, extra_per_row=2)
    e = np.random.default_rng(seed + 100).normal(size=inp.n)
    maxit = 4
    L, gA, gP0 = oad.gradient(inp, maxit=maxit, e=e, w_energy=wE, w_twogrid=wT)
    for j in range(inp.A.nnz):
        cs = _cs_A(inp, j, e, maxit, wE, wT)
        assert abs(gA[j] - cs) <= 1e-10 * max(1.0, abs(cs)), (j, gA[j], cs)
    for j in range(inp.P0.nnz):
        cs = _cs_P0(inp, j, e, maxit, wE, wT)
        assert abs(gP0[j] - cs) <= 1e-10 * max(1.0, abs(cs)), (j, gP0[j], cs)


def test_reverse_sweep_directional_poisson3d_small():
    """Random directions on a 3D log-normal Poisson case (12^3 cells)."""
    inp = gen.poisson3d_ln32(N=12)
    e = inp.extra["e"]
    L, gA, gP0 = oad.gradient(inp, e=e)
    rng = np.random.default_rng(7)
    for _ in range(3):
        va = rng.normal(size=inp.A.nnz)
        vp = rng.normal(size=inp.P0.nnz)
        h = 1e-30
        Lc, *_ = oad.forward(inp, A_vals=inp.A.data + 1j * h * va,
                             P0_vals=inp.P0.data + 1j * h * vp, e=e)
        cs = np.imag(Lc) / h
        got = gA @ va + gP0 @ vp
        assert abs(got - cs) <= 1e-10 * abs(cs)


def test_loss_gradient_energy_closed_form():
    """dE/dP = 2 mask(A P) and dE/dA_il = (P P^T)_il checked by complex step
    on P directly (the loss alone, P fixed)."""
    from oracle import rcg as orc

    inp = gen.tiny_problem(4, n=10, nc=4, m=1, extra_per_row=2)
    rp, ci = inp.extra["pattern"]
    P = np.random.default_rng(1).normal(size=ci.size)
    gP, gA = oad.loss_grad(inp.A, rp, ci, P, inp.nc, None, 1.0, 0.0)
    for j in range(ci.size):
        Pc = P.astype(complex)
        Pc[j] += 1e-30j
        cs = np.imag(oad.loss(inp.A, rp, ci, Pc, inp.nc, None, 1.0, 0.0)) / 1e-30
        assert abs(gP[j] - cs) <= 1e-12 * max(1, abs(cs))
    for j in range(inp.A.nnz):
        Ac = inp.A.astype(complex)
        Ac.data[j] += 1e-30j
        cs = np.imag(oad.loss(Ac, rp, ci, P, inp.nc, None, 1.0, 0.0)) / 1e-30
        assert abs(gA[j] - cs) <= 1e-12 * max(1, abs(cs))
